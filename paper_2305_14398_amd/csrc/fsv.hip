// Full-state-vector simulation: the per-amplitude gate update of Appendix A
// (Eq. 12), the backend the paper proposes to accelerate next (Section 7).
// The state (planar complex64: re plane then im plane, N = 2^n floats each)
// is updated in place; no 2^n x 2^n operator exists, so n reaches 34 qubits
// (a 128 GiB state) instead of 16.
//
// Design.  Applying gates one launch at a time would stream the whole state
// through HBM once per gate.  Instead the host groups consecutive gates into
// passes; a pass names 12 "local" qubits (the low L qubits 0..L-1 plus up to
// 12 - L others) and contains only gates whose non-diagonal target is local.
// One launch per pass: workgroup w takes the 4096 amplitudes that share w's
// values of the other n - 12 qubits, applies every gate of the pass to them
// in registers and writes them back, so a pass costs 16 bytes of HBM traffic
// per amplitude however many gates it holds.
//
// A workgroup copies the pass's operation records (at most 256 per pass) into
// LDS before it starts.  Inside a workgroup, 256 threads hold 16 amplitudes
// each (16-wide vector registers, so no amplitude ever goes through scratch).
// Of the 12 local
// index bits, 4 live in a thread's registers and 8 in its thread index; three
// layouts put bits 0-3, 4-7 or 8-11 in registers.  A gate whose target bit is
// in the register group updates 8 register pairs per thread with no exchange;
// otherwise the workgroup first changes layout through LDS (32 KiB, XOR
// swizzled so each wave's 64 accesses hit distinct banks in every layout).
// Controls never need to be local: a control on a local bit is a per-register
// predicate, one on any other qubit is the same for the whole workgroup.
// Diagonal gates (Z, S, T, R, RZ, CZ, controlled phases) only scale
// amplitudes, so they need no local target at all; when neither of their
// qubits is a register bit, their factor is the same for a thread's 16
// amplitudes and is folded into one per-thread phase that is applied once.
// SWAP needs both qubits local and is one LDS round trip that reads every
// amplitude back from the index with the two bits exchanged (exact).  A custom
// operation on m qubits (Section 5.2.2) needs its whole range local; it is
// applied through LDS: every amplitude is written out, then each thread forms
// its 16 outputs as sums of 2^m products with the operation's float32 matrix.
//
// Gate entries are the float64 matrices of the unitary path rounded once to
// float32; amplitude arithmetic is float32 with fused multiply-adds.
#include <algorithm>
#include <cmath>
#include <complex>
#include <set>
#include <utility>
#include <vector>

#include "host.h"

namespace qsim {

constexpr int kFsvLocal = 12;     // local qubits per workgroup: 4096 amplitudes
constexpr int kFsvMinLow = 6;     // low qubits always local: 64 lanes x 4 B contiguous per plane
constexpr int kFsvMaxHigh = kFsvLocal - kFsvMinLow;
constexpr int kFsvNormBlocks = 1024;
constexpr int kFsvMaxOps = 256;   // operations per pass (a planning cap)
constexpr int kFsvSeeds = 16;      // alternative first operations tried when a pass is formed
constexpr int kFsvLaneRun = 5;    // longest run of operations applied across lanes instead of a layout change

// A thread's 16 values of one plane: 16 scalars (every index is a compile-time
// constant), so that each register is coalesced on its own.
struct f32x16 {
    float v[16];
    __device__ __forceinline__ float& operator[](int i) { return v[i]; }
    __device__ __forceinline__ const float& operator[](int i) const { return v[i]; }
};

// Calls f(std::integral_constant<int, r>) for r = 0..15: every register index
// is a compile-time constant from the start, so the amplitude vectors never
// need an addressable (scratch) copy.
template <class F, int... Rs>
__device__ __forceinline__ void fsv_for16_impl(F&& f, std::integer_sequence<int, Rs...>) {
    (f(std::integral_constant<int, Rs>{}), ...);
}
template <class F>
__device__ __forceinline__ void fsv_for16(F&& f) {
    fsv_for16_impl(f, std::make_integer_sequence<int, 16>{});
}
template <class F>
__device__ __forceinline__ void fsv_for4(F&& f) {
    fsv_for16_impl(f, std::make_integer_sequence<int, 4>{});
}

enum : int32_t { FSV_GENERAL = 0, FSV_DIAG = 1, FSV_DENSE = 2, FSV_TABLE = 3, FSV_PHASE = 4, FSV_SWAP = 5 };
constexpr int kFsvPhaseBits = 10;    // workgroup-number bits per FSV_PHASE window (up to 2^10 entries)
constexpr int kFsvPhaseWindows = 3;  // windows per FSV_PHASE record

struct FsvGate {
    int32_t kind;
    int32_t tloc;   // local bit of the target (dense: of the range's lowest qubit), or -1 (diagonal only)
    int32_t tglob;  // the target qubit when it is not local (phase: its windows, 10 bits each: lo | w << 5;
                    // table: 1 when it has a per-thread factor P);
                    // general: planned actions before it (bit 0: apply the pending per-lane phase,
                    // bit 1: change to the target's register layout)
    int32_t cloc;   // local bit of the control, or -1 (table: the register bits with a per-thread factor W)
    int32_t cglob;  // a non-local control qubit, or -1
    int32_t width;  // dense: qubits in the range; phase: windows (tables) it multiplies;
                    // table: the registers its uniform factors F apply to (bit mask);
                    // general: 1 + the lane bit its target occupies when it is applied across
                    // lanes in the current layout (0: its target is in the register group)
    int32_t moff;   // dense / table / phase: offset of its float32 data in the plan's pool
    int32_t real;   // general and diagonal: the leaf code of its update (see the host-planned dispatch);
                    // while the host plans, a general record's form (FSV_COMPLEX .. FSV_IPERM)
    float m[8];  // row-major 2x2 (re, im); a diagonal gate uses m[0..1] and m[6..7]
};

// Forms of a non-diagonal 2x2 (after rounding to float32), each applied with
// only the arithmetic it needs:
//   FSV_COMPLEX  any matrix: 16 multiply-adds per amplitude pair;
//   FSV_REAL     every entry real (H, RY): 8;
//   FSV_XSWAP    [[0, 1], [1, 0]] (X, the target of CNOT): an exact exchange;
//   FSV_ANTI     [[0, b], [c, 0]] (Y, phases times X): 8;
//   FSV_IMAGOFF  real diagonal, imaginary off-diagonal (RX): 8;
//   FSV_IPERM    [[0, -i], [i, 0]] (Y): exchanges and sign flips only, exact.
enum : int32_t { FSV_COMPLEX = 0, FSV_REAL = 1, FSV_XSWAP = 2, FSV_ANTI = 3, FSV_IMAGOFF = 4, FSV_IPERM = 5 };

// A pass of pairwise disjoint SWAPs is one permutation sigma of qubit
// positions (an involution): the amplitude at index i moves to sigma(i), the
// index with its bits moved by sigma.  Positions 0-5 (a row of 64 contiguous
// amplitudes), the positions that sigma exchanges with them and further whole
// orbits of sigma, h positions above 5 in all, form a tile of 64 * 2^h
// amplitudes (4 <= h <= 6); the other positions name a group, and sigma maps
// group g's tile onto group sigma(g)'s with the tile bits permuted.  One workgroup per
// pair {g, sigma(g)} reads both tiles (rows of 64 contiguous amplitudes), and
// writes both through LDS in the permuted order, again in contiguous rows: one
// read and one write of every amplitude, in place, with no workgroup writing
// where another reads.
struct FsvPerm {
    int32_t h;           // tile bits 6 .. 5 + h are positions hpos[0 .. h)
    int32_t ng;          // group bits 0 .. ng - 1 are positions gpos[0 .. ng), in the order of max(x, sigma(x))
    int32_t hpos[6];
    int32_t fold[6];     // LDS slot of a tile element: e ^ (fold[j] for each set row bit 6 + j)
    int32_t gpos[QSIM_FSV_MAX_QUBITS];
    int32_t sig_tile[12];                  // tile bit -> tile bit under sigma
    int32_t sig_group[QSIM_FSV_MAX_QUBITS];  // group bit -> group bit under sigma
};

struct FsvPass {
    int32_t L;   // local bits 0..L-1 are qubits 0..L-1
    int32_t nh;  // local bits L..L+nh-1 are qubits high[0..nh-1], ascending
    int32_t high[kFsvMaxHigh];
    int32_t pos[kFsvLocal];  // the qubit of each local bit (bits beyond L + nh: the bit itself)
    int32_t wide;            // the pass holds a dense operation (both planes staged in LDS)
    int32_t g0, g1;  // the pass's records in the plan's table
    int32_t op0, op1;  // the operations the pass covers
    float scale;     // the product of the factors the pass's scaled forms take out
    int32_t tail;    // at the end: 2 apply the pending per-lane phase and the scale, 1 the scale, 0 nothing
    int32_t perm;    // a permutation pass (disjoint SWAPs on any qubits), described by pm
    FsvPerm pm;
};


namespace {

// Bank-spreading map of a local index to its LDS slot (a bijection on 0..4095
// that only changes bits 0-5).
__host__ __device__ constexpr int fsv_swz(int j) { return j ^ ((j >> 6) & 15) ^ (((j >> 8) & 3) << 4); }

// The map is linear over XOR and register bits never overlap a thread's bits,
// so a slot is the thread's part XOR a per-register constant: the byte offset
// 4 fsv_swz(r << 4k) of register r in layout k, read from this table with
// scalar loads (one XOR per LDS access instead of the whole map per access).
struct FsvSwzTable {
    int32_t v[3][16];
};
constexpr FsvSwzTable fsv_make_swz_table() {
    FsvSwzTable t{};
    for (int k = 0; k < 3; ++k)
        for (int r = 0; r < 16; ++r) t.v[k][r] = 4 * fsv_swz(r << (4 * k));
    return t;
}
__constant__ FsvSwzTable kFsvSwzReg = fsv_make_swz_table();

// The local index bits a thread contributes in layout k (its 8 index bits
// around the register nibble 4k..4k+3).
__device__ __forceinline__ int fsv_thread_bits(int t, int k) {
    const int s = 4 * k;
    return (t & ((1 << s) - 1)) | ((t >> s) << (s + 4));
}

// Form of a float32 2x2 (row-major (re, im)); exact tests on the rounded entries.
inline int fsv_form(const float m[8]) {
    const bool real = m[1] == 0.f && m[3] == 0.f && m[5] == 0.f && m[7] == 0.f;
    const bool anti = m[0] == 0.f && m[1] == 0.f && m[6] == 0.f && m[7] == 0.f;
    if (anti && real && m[2] == 1.f && m[4] == 1.f) return FSV_XSWAP;
    if (anti && m[2] == 0.f && m[3] == -1.f && m[4] == 0.f && m[5] == 1.f) return FSV_IPERM;
    if (anti) return FSV_ANTI;
    if (real) return FSV_REAL;
    if (m[1] == 0.f && m[7] == 0.f && m[2] == 0.f && m[4] == 0.f) return FSV_IMAGOFF;
    return FSV_COMPLEX;
}

// ---- In-place amplitude updates ----
// The operation loop keeps a thread's 32 amplitude values (16 re, 16 im) in
// fixed registers, and every update below rewrites its inputs in place.  They
// are short inline-assembly sequences with tied operands: written as plain
// expressions, each branch of the operation dispatch gets fresh result
// registers and the compiler copies the whole state back at the merge, which
// costs more than the arithmetic itself.  Only plain float32 VALU instructions
// appear (v_mul_f32, v_fma_f32, v_fmac_f32, v_cndmask_b32, v_swap_b32, v_mov_b32);
// each sequence keeps the rounding of the expression written beside it.
// Coefficients are SGPRs when they are uniform (VC = false) and VGPRs when a
// control on a lane index bit makes them per lane (VC = true).

// x <- f x (complex):  xr' = fma(fr, xr, -(fi xi)),  xi' = fma(fr, xi, fi xr)
#define FSV_CMUL_ASM                 \
    "v_mul_f32 %0, %5, %3\n\t"      \
    "v_mul_f32 %1, %5, %2\n\t"      \
    "v_fma_f32 %2, %4, %2, -%0\n\t" \
    "v_fma_f32 %3, %4, %3, %1"
template <bool VC>
__device__ __forceinline__ void fsv_cmul(float& xr, float& xi, float fr, float fi) {
    float t, u;
    if constexpr (VC)
        asm(FSV_CMUL_ASM : "=&v"(t), "=&v"(u), "+v"(xr), "+v"(xi) : "v"(fr), "v"(fi));
    else
        asm(FSV_CMUL_ASM : "=&v"(t), "=&v"(u), "+v"(xr), "+v"(xi) : "s"(fr), "s"(fi));
}

// One real plane of a pair under a real 2x2 [[a, b], [c, d]]:
//   x0' = fma(a, x0, b x1),  x1' = fma(c, x0, d x1)
#define FSV_ROT_ASM              \
    "v_mul_f32 %0, %4, %2\n\t"  \
    "v_mul_f32 %2, %6, %2\n\t"  \
    "v_fmac_f32 %2, %5, %1\n\t" \
    "v_fma_f32 %1, %3, %1, %0"
template <bool VC>
__device__ __forceinline__ void fsv_rot(float& x0, float& x1, float a, float b, float c, float d) {
    float t;
    if constexpr (VC)
        asm(FSV_ROT_ASM : "=&v"(t), "+v"(x0), "+v"(x1) : "v"(a), "v"(b), "v"(c), "v"(d));
    else
        asm(FSV_ROT_ASM : "=&v"(t), "+v"(x0), "+v"(x1) : "s"(a), "s"(b), "s"(c), "s"(d));
}

// A pair under [[a, i b], [i c, d]] with a, b, c, d real (RX and its kind):
//   x0r' = fma(a, x0r, -(b x1i)),  x0i' = fma(a, x0i, b x1r)
//   x1r' = fma(d, x1r, -(c x0i)),  x1i' = fma(d, x1i, c x0r)
#define FSV_IMAGOFF_ASM              \
    "v_mul_f32 %0, %9, %7\n\t"       \
    "v_mul_f32 %1, %9, %6\n\t"       \
    "v_mul_f32 %2, %10, %5\n\t"      \
    "v_mul_f32 %3, %10, %4\n\t"      \
    "v_fma_f32 %4, %8, %4, -%0\n\t"  \
    "v_fma_f32 %5, %8, %5, %1\n\t"   \
    "v_fma_f32 %6, %11, %6, -%2\n\t" \
    "v_fma_f32 %7, %11, %7, %3"
template <bool VC>
__device__ __forceinline__ void fsv_imagoff(float& x0r, float& x0i, float& x1r, float& x1i, float a, float b,
                                            float c, float d) {
    float t0, t1, t2, t3;
    if constexpr (VC)
        asm(FSV_IMAGOFF_ASM
            : "=&v"(t0), "=&v"(t1), "=&v"(t2), "=&v"(t3), "+v"(x0r), "+v"(x0i), "+v"(x1r), "+v"(x1i)
            : "v"(a), "v"(b), "v"(c), "v"(d));
    else
        asm(FSV_IMAGOFF_ASM
            : "=&v"(t0), "=&v"(t1), "=&v"(t2), "=&v"(t3), "+v"(x0r), "+v"(x0i), "+v"(x1r), "+v"(x1i)
            : "s"(a), "s"(b), "s"(c), "s"(d));
}

// A pair under any complex 2x2 m (row-major m0 m1 / m2 m3):
//   y0r = fma(m0r, x0r, fma(-m0i, x0i, fma(m1r, x1r, -(m1i x1i))))
//   y0i = fma(m0r, x0i, fma( m0i, x0r, fma(m1r, x1i,   m1i x1r)))
//   y1r = fma(m2r, x0r, fma(-m2i, x0i, fma(m3r, x1r, -(m3i x1i))))
//   y1i = fma(m2r, x0i, fma( m2i, x0r, fma(m3r, x1i,   m3i x1r)))
// The partial sums need x1 last, so y1 lands in x1's registers and y0 in x0's.
#define FSV_CPLX_ASM                   \
    "v_mul_f32 %0, %11, %7\n\t"        \
    "v_fma_f32 %0, %10, %6, -%0\n\t"   \
    "v_fma_f32 %0, -%9, %5, %0\n\t"    \
    "v_mul_f32 %1, %11, %6\n\t"        \
    "v_fmac_f32 %1, %10, %7\n\t"       \
    "v_fmac_f32 %1, %9, %4\n\t"        \
    "v_mul_f32 %2, %15, %7\n\t"        \
    "v_fma_f32 %2, %14, %6, -%2\n\t"   \
    "v_fma_f32 %2, -%13, %5, %2\n\t"   \
    "v_mul_f32 %3, %15, %6\n\t"        \
    "v_fmac_f32 %3, %14, %7\n\t"       \
    "v_fmac_f32 %3, %13, %4\n\t"       \
    "v_fma_f32 %6, %12, %4, %2\n\t"    \
    "v_fma_f32 %7, %12, %5, %3\n\t"    \
    "v_fma_f32 %4, %8, %4, %0\n\t"     \
    "v_fma_f32 %5, %8, %5, %1"
struct Mat2 {
    float m0r, m0i, m1r, m1i, m2r, m2i, m3r, m3i;
};
template <bool VC>
__device__ __forceinline__ void fsv_cplx(float& x0r, float& x0i, float& x1r, float& x1i, const Mat2& M) {
    float a, b, c, d;
    if constexpr (VC)
        asm(FSV_CPLX_ASM
            : "=&v"(a), "=&v"(b), "=&v"(c), "=&v"(d), "+v"(x0r), "+v"(x0i), "+v"(x1r), "+v"(x1i)
            : "v"(M.m0r), "v"(M.m0i), "v"(M.m1r), "v"(M.m1i), "v"(M.m2r), "v"(M.m2i), "v"(M.m3r), "v"(M.m3i));
    else
        asm(FSV_CPLX_ASM
            : "=&v"(a), "=&v"(b), "=&v"(c), "=&v"(d), "+v"(x0r), "+v"(x0i), "+v"(x1r), "+v"(x1i)
            : "s"(M.m0r), "s"(M.m0i), "s"(M.m1r), "s"(M.m1i), "s"(M.m2r), "s"(M.m2i), "s"(M.m3r), "s"(M.m3i));
}

// Scaled forms of common 2x2s, for operations without a control, which act on
// every amplitude: the real factor a that is taken out multiplies the pass's
// scale, applied once when the pass stores (a factor common to all amplitudes
// commutes with every operation).
//   FSV_HADA  a [[1, 1], [1, -1]] (H):  x1' = x0 - x1,  x0' = fma(2, x0, -x1')  (= x0 + x1)
//   FSV_ROTR  a [[1, -t], [t, 1]] (RY with |t| <= 1, k = 1 + t^2):
//             x1' = fma(t, x0, x1),  x0' = fma(-t, x1', k x0)  (= x0 - t x1)
//   FSV_ROTI  a [[1, -i t], [-i t, 1]] (RX with |t| <= 1), per plane as FSV_ROTR
//             with the planes crossed:  x1r' = fma(t, x0i, x1r),  x1i' = fma(-t, x0r, x1i),
//             x0r' = fma(t, x1i', k x0r),  x0i' = fma(-t, x1r', k x0i)
//   FSV_ROTR2 a [[k, -1], [1, k]] (RY whose sine is the larger, |k| < 1), with a temporary:
//             y0 = fma(k, x0, -x1),  x1' = fma(k, x1, x0),  x0' = y0
//   FSV_ROTI2 a [[k, i], [i, k]] (RX likewise):  y0r = fma(k, x0r, -x1i),  y0i = fma(k, x0i, x1r),
//             x1r' = fma(k, x1r, -x0i),  x1i' = fma(k, x1i, x0r)
//   (the last two on register bits only: across lanes they save nothing).
enum : int32_t { FSV_HADA = 0, FSV_ROTR = 1, FSV_ROTI = 2, FSV_ROTR2 = 3, FSV_ROTI2 = 4 };
__device__ __forceinline__ void fsv_hada(float& x0, float& x1) {
    asm("v_sub_f32 %1, %0, %1\n\t"
        "v_fma_f32 %0, 2.0, %0, -%1"
        : "+v"(x0), "+v"(x1));
}
__device__ __forceinline__ void fsv_rotr(float& x0, float& x1, float k, float t) {
    asm("v_fmac_f32 %1, %3, %0\n\t"
        "v_mul_f32 %0, %2, %0\n\t"
        "v_fma_f32 %0, -%3, %1, %0"
        : "+v"(x0), "+v"(x1)
        : "s"(k), "s"(t));
}
__device__ __forceinline__ void fsv_rotr2(float& x0, float& x1, float k) {
    float t;
    asm("v_fma_f32 %2, %3, %0, -%1\n\t"
        "v_fma_f32 %1, %3, %1, %0\n\t"
        "v_mov_b32 %0, %2"
        : "+v"(x0), "+v"(x1), "=&v"(t)
        : "s"(k));
}
__device__ __forceinline__ void fsv_roti2(float& x0r, float& x0i, float& x1r, float& x1i, float k) {
    float t0, t1;
    asm("v_fma_f32 %4, %6, %0, -%3\n\t"
        "v_fma_f32 %5, %6, %1, %2\n\t"
        "v_fma_f32 %2, %6, %2, -%1\n\t"
        "v_fma_f32 %3, %6, %3, %0\n\t"
        "v_mov_b32 %0, %4\n\t"
        "v_mov_b32 %1, %5"
        : "+v"(x0r), "+v"(x0i), "+v"(x1r), "+v"(x1i), "=&v"(t0), "=&v"(t1)
        : "s"(k));
}
__device__ __forceinline__ void fsv_roti(float& x0r, float& x0i, float& x1r, float& x1i, float k, float t) {
    asm("v_fmac_f32 %2, %5, %1\n\t"
        "v_fma_f32 %3, -%5, %0, %3\n\t"
        "v_mul_f32 %0, %4, %0\n\t"
        "v_fmac_f32 %0, %5, %3\n\t"
        "v_mul_f32 %1, %4, %1\n\t"
        "v_fma_f32 %1, -%5, %2, %1"
        : "+v"(x0r), "+v"(x0i), "+v"(x1r), "+v"(x1i)
        : "s"(k), "s"(t));
}

// Exact exchanges: always, or in the lanes whose bit is set in a uniform mask.
__device__ __forceinline__ void fsv_swap(float& x0, float& x1) { asm("v_swap_b32 %0, %1" : "+v"(x0), "+v"(x1)); }
// Exact sign flip.
__device__ __forceinline__ void fsv_neg(float& x) { asm("v_xor_b32 %0, 0x80000000, %0" : "+v"(x)); }
__device__ __forceinline__ void fsv_cswap(float& x0, float& x1, uint64_t mask) {
    float t;
    asm("v_mov_b32 %0, %1\n\t"
        "v_cndmask_b32_e64 %1, %1, %2, %3\n\t"
        "v_cndmask_b32_e64 %2, %2, %0, %3"
        : "=&v"(t), "+v"(x0), "+v"(x1)
        : "s"(mask));
}

// A non-diagonal 2x2 of form FORM on register bit RB; with CP >= 0 only the
// pairs whose register bit CP is set (a control on that bit).
template <int RB, int CP, int FORM, bool VC>
__device__ __forceinline__ void fsv_pairs(f32x16& ar, f32x16& ai, const Mat2& M) {
    fsv_for16([&](auto I_) {
        constexpr int r0 = decltype(I_)::value;
        if constexpr (((r0 >> RB) & 1) == 0 && (CP < 0 || ((r0 >> CP) & 1) == 1)) {
            constexpr int r1 = r0 | (1 << RB);
            float x0r = ar[r0], x0i = ai[r0], x1r = ar[r1], x1i = ai[r1];
            if constexpr (FORM == FSV_REAL) {
                fsv_rot<VC>(x0r, x1r, M.m0r, M.m1r, M.m2r, M.m3r);
                fsv_rot<VC>(x0i, x1i, M.m0r, M.m1r, M.m2r, M.m3r);
            } else if constexpr (FORM == FSV_IMAGOFF) {
                fsv_imagoff<VC>(x0r, x0i, x1r, x1i, M.m0r, M.m1i, M.m2i, M.m3r);
            } else if constexpr (FORM == FSV_ANTI) {  // y0 = m1 x1, y1 = m2 x0
                fsv_swap(x0r, x1r);
                fsv_swap(x0i, x1i);
                fsv_cmul<VC>(x0r, x0i, M.m1r, M.m1i);
                fsv_cmul<VC>(x1r, x1i, M.m2r, M.m2i);
            } else if constexpr (FORM == FSV_XSWAP) {
                fsv_swap(x0r, x1r);
                fsv_swap(x0i, x1i);
            } else if constexpr (FORM == FSV_IPERM) {
                // y0 = -i x1 = (x1i, -x1r),  y1 = i x0 = (-x0i, x0r)
                fsv_swap(x0r, x1i);
                fsv_swap(x0i, x1r);
                fsv_neg(x0i);
                fsv_neg(x1r);
            } else {
                fsv_cplx<VC>(x0r, x0i, x1r, x1i, M);
            }
            ar[r0] = x0r;
            ai[r0] = x0i;
            ar[r1] = x1r;
            ai[r1] = x1i;
        }
    });
}

// A scaled form (FSV_HADA .. FSV_ROTI2) on register bit RB; k and t as above.
template <int RB, int KIND>
__device__ __forceinline__ void fsv_scaled_pairs(f32x16& ar, f32x16& ai, float k, float t) {
    fsv_for16([&](auto I_) {
        constexpr int r0 = decltype(I_)::value;
        if constexpr (((r0 >> RB) & 1) == 0) {
            constexpr int r1 = r0 | (1 << RB);
            float x0r = ar[r0], x0i = ai[r0], x1r = ar[r1], x1i = ai[r1];
            if constexpr (KIND == FSV_HADA) {
                fsv_hada(x0r, x1r);
                fsv_hada(x0i, x1i);
            } else if constexpr (KIND == FSV_ROTR) {
                fsv_rotr(x0r, x1r, k, t);
                fsv_rotr(x0i, x1i, k, t);
            } else if constexpr (KIND == FSV_ROTI) {
                fsv_roti(x0r, x0i, x1r, x1i, k, t);
            } else if constexpr (KIND == FSV_ROTR2) {
                fsv_rotr2(x0r, x1r, k);
                fsv_rotr2(x0i, x1i, k);
            } else {
                fsv_roti2(x0r, x0i, x1r, x1i, k);
            }
            ar[r0] = x0r;
            ai[r0] = x0i;
            ar[r1] = x1r;
            ai[r1] = x1i;
        }
    });
}

// X on register bit RB in the lanes whose bit is set in mask (a control on a
// lane index bit; exact).
template <int RB>
__device__ __forceinline__ void fsv_xswap_lanes(f32x16& ar, f32x16& ai, uint64_t mask) {
    fsv_for16([&](auto I_) {
        constexpr int r0 = decltype(I_)::value;
        if constexpr (((r0 >> RB) & 1) == 0) {
            constexpr int r1 = r0 | (1 << RB);
            float x0r = ar[r0], x0i = ai[r0], x1r = ar[r1], x1i = ai[r1];
            fsv_cswap(x0r, x1r, mask);
            fsv_cswap(x0i, x1i, mask);
            ar[r0] = x0r;
            ai[r0] = x0i;
            ar[r1] = x1r;
            ai[r1] = x1i;
        }
    });
}

// ---- Operations on a lane bit ----
// A non-diagonal 2x2 whose target is one of the six lane bits of the current
// layout is applied across lanes instead of after a layout change: each lane
// holds one amplitude of every pair (its own) and reads the other from the
// partner lane (lane id XOR 2^B), then forms its row of the product with
// per-lane coefficients: lane bit s = 0 keeps y0 = m0 x + m1 p, s = 1 keeps
// y1 = m3 x + m2 p (a lane whose control bit is 0 takes the identity row).

// x in the partner lane: DPP inside a row of 16 lanes (bits 0-3; two moves for
// bits 2 and 3: a mirror composed with a smaller one), ds_swizzle for bit 4,
// ds_bpermute for bit 5.
template <int B>
__device__ __forceinline__ float fsv_partner(float x, int lane) {
    const int v = __builtin_bit_cast(int, x);
    int p;
    if constexpr (B == 0)
        p = __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);  // quad_perm [1,0,3,2]: lane ^ 1
    else if constexpr (B == 1)
        p = __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);  // quad_perm [2,3,0,1]: lane ^ 2
    else if constexpr (B == 2)  // row_half_mirror (lane ^ 7), then quad_perm [3,2,1,0] (lane ^ 3)
        p = __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true), 0x1B, 0xF, 0xF, true);
    else if constexpr (B == 3)  // row_mirror (lane ^ 15), then row_half_mirror (lane ^ 7)
        p = __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true), 0x141, 0xF, 0xF, true);
    else if constexpr (B == 4)
        p = __builtin_amdgcn_ds_swizzle(v, 0x401F);  // bit-mask mode: and 0x1f, or 0, xor 0x10
    else
        p = __builtin_amdgcn_ds_bpermute((lane ^ 32) << 2, v);
    return __builtin_bit_cast(float, p);
}

// x <- a x + b p on one plane, a and b real per lane: x' = fma(a, x, b p)
__device__ __forceinline__ void fsv_axbp(float& x, float p, float a, float b) {
    float t;
    asm("v_mul_f32 %0, %3, %2\n\t"
        "v_fma_f32 %1, %4, %1, %0"
        : "=&v"(t), "+v"(x)
        : "v"(p), "v"(b), "v"(a));
}

// (xr, xi) <- a x + b p, complex a and b per lane:
//   xr' = fma(ar, xr, fma(-ai, xi, fma(-bi, pi, br pr)))
//   xi' = fma(ar, xi, fma( ai, xr, fma( bi, pr, br pi)))
#define FSV_AXBP_C_ASM                 \
    "v_mul_f32 %0, %8, %4\n\t"        \
    "v_fma_f32 %0, -%9, %5, %0\n\t"   \
    "v_fma_f32 %0, -%7, %3, %0\n\t"   \
    "v_mul_f32 %1, %8, %5\n\t"        \
    "v_fmac_f32 %1, %9, %4\n\t"       \
    "v_fmac_f32 %1, %7, %2\n\t"       \
    "v_fma_f32 %2, %6, %2, %0\n\t"    \
    "v_fma_f32 %3, %6, %3, %1"
__device__ __forceinline__ void fsv_axbp_c(float& xr, float& xi, float pr, float pi, const Mat2& c) {
    float t1, t2;
    asm(FSV_AXBP_C_ASM
        : "=&v"(t1), "=&v"(t2), "+v"(xr), "+v"(xi)
        : "v"(pr), "v"(pi), "v"(c.m0r), "v"(c.m0i), "v"(c.m1r), "v"(c.m1i));
}

// FORM FSV_XSWAP: an uncontrolled X (every lane takes its partner's value);
// FSV_REAL: real per-lane coefficients (c.m0r, c.m1r); otherwise complex.
template <int B, int FORM>
__device__ __forceinline__ void fsv_lane_op(f32x16& ar, f32x16& ai, const Mat2& c, int lane) {
    fsv_for16([&](auto I_) {
        constexpr int r = decltype(I_)::value;
        float xr = ar[r], xi = ai[r];
        const float pr = fsv_partner<B>(xr, lane), pi = fsv_partner<B>(xi, lane);
        if constexpr (FORM == FSV_XSWAP) {
            xr = pr;
            xi = pi;
        } else if constexpr (FORM == FSV_REAL) {
            fsv_axbp(xr, pr, c.m0r, c.m1r);
            fsv_axbp(xi, pi, c.m0r, c.m1r);
        } else {
            fsv_axbp_c(xr, xi, pr, pi, c);
        }
        ar[r] = xr;
        ai[r] = xi;
    });
}

// An exchange across lanes on lane bit B in the lanes set in mask `on` (a
// control on a thread bit): one select per value after the partner exchange.
template <int B>
__device__ __forceinline__ void fsv_lane_cswap(f32x16& ar, f32x16& ai, uint64_t on, int lane) {
    fsv_for16([&](auto I_) {
        constexpr int r = decltype(I_)::value;
        float xr = ar[r], xi = ai[r];
        const float pr = fsv_partner<B>(xr, lane), pi = fsv_partner<B>(xi, lane);
        asm("v_cndmask_b32_e64 %0, %0, %2, %4\n\t"
            "v_cndmask_b32_e64 %1, %1, %3, %4"
            : "+v"(xr), "+v"(xi)
            : "v"(pr), "v"(pi), "s"(on));
        ar[r] = xr;
        ai[r] = xi;
    });
}

// A scaled form (FSV_HADA .. FSV_ROTI, no control) applied across lanes on lane
// bit B; each lane keeps its row with its own value's coefficient 1:
//   FSV_HADA  y = fma(s, x, p), s = t (lane bit 0: x0 + x1) or -t (bit 1: x0 - x1), t = 1
//             (read from the record: a constant select would be hoisted out of the
//             operation loop and hold a register per lane bit)
//   FSV_ROTR  y = fma(c, p, x), c = -t (bit 0) or t (bit 1)
//   FSV_ROTI  yr = fma(t, pi, xr),  yi = fma(-t, pr, xi)  (the same in both lanes)
template <int B, int KIND>
__device__ __forceinline__ void fsv_lane_scaled(f32x16& ar, f32x16& ai, float t, int lane) {
    const bool hi = (lane >> B) & 1;
    const float c = KIND == FSV_HADA ? (hi ? -t : t) : (hi ? t : -t);
    fsv_for16([&](auto I_) {
        constexpr int r = decltype(I_)::value;
        float xr = ar[r], xi = ai[r];
        const float pr = fsv_partner<B>(xr, lane), pi = fsv_partner<B>(xi, lane);
        if constexpr (KIND == FSV_HADA) {
            asm("v_fma_f32 %0, %2, %0, %3\n\t"
                "v_fma_f32 %1, %2, %1, %4"
                : "+v"(xr), "+v"(xi)
                : "v"(c), "v"(pr), "v"(pi));
        } else if constexpr (KIND == FSV_ROTR) {
            asm("v_fmac_f32 %0, %2, %3\n\t"
                "v_fmac_f32 %1, %2, %4"
                : "+v"(xr), "+v"(xi)
                : "v"(c), "v"(pr), "v"(pi));
        } else {
            asm("v_fmac_f32 %0, %2, %3\n\t"
                "v_fma_f32 %1, -%2, %4, %1"
                : "+v"(xr), "+v"(xi)
                : "s"(t), "v"(pi), "v"(pr));
        }
        ar[r] = xr;
        ai[r] = xi;
    });
}

// Registers whose bit P is set (or all, P < 0) times the per-lane factor f.
template <int P>
__device__ __forceinline__ void fsv_scale(f32x16& ar, f32x16& ai, float fr, float fi) {
    fsv_for16([&](auto I_) {
        constexpr int r = decltype(I_)::value;
        if constexpr (P < 0 || ((r >> P) & 1) == 1) {
            float xr = ar[r], xi = ai[r];
            fsv_cmul<true>(xr, xi, fr, fi);
            ar[r] = xr;
            ai[r] = xi;
        }
    });
}

// Registers with bit CP set (all if CP < 0) times d1 where bit TP is set, else
// d0 (D0 false: d0 is exactly 1 and is skipped).
template <int TP, int CP, bool D0>
__device__ __forceinline__ void fsv_diag_reg(f32x16& ar, f32x16& ai, float d0r, float d0i, float d1r, float d1i) {
    fsv_for16([&](auto I_) {
        constexpr int r = decltype(I_)::value;
        if constexpr (CP < 0 || ((r >> CP) & 1) == 1) {
            float xr = ar[r], xi = ai[r];
            if constexpr (((r >> TP) & 1) == 1)
                fsv_cmul<true>(xr, xi, d1r, d1i);
            else if constexpr (D0)
                fsv_cmul<true>(xr, xi, d0r, d0i);
            ar[r] = xr;
            ai[r] = xi;
        }
    });
}

// Applies the pending per-lane phase to all 16 registers (unconditionally:
// a phase of exactly 1 leaves every amplitude bit-identical).
__device__ __forceinline__ void fsv_flush(f32x16& ar, f32x16& ai, float& lpr, float& lpi) {
    fsv_scale<-1>(ar, ai, lpr, lpi);
    lpr = 1.f;
    lpi = 0.f;
}

// ---- Host-planned dispatch ----
// The host follows the register layout through each pass and gives every
// general and diagonal record a leaf code (in `real`) that names the exact
// update to run, so the kernel's per-record work is one switch.  General
// leaves:
//   kLeafNC   + form * 4 + RB            no local control (form FSV_COMPLEX .. FSV_IPERM)
//   kLeafCP   + fc * 16 + RB * 4 + cp    control on register bit cp (fc: exchange, real, complex)
//   kLeafLC   + fc * 4 + RB              control on a thread bit (fc: exchange, real, imaginary
//                                        off-diagonal, complex)
//   kLeafLane + fc * 6 + lane bit        target on a lane bit (fc: plain exchange, real, complex,
//                                        exchange under a thread-bit control)
//   kLeafScl  + kind * 4 + RB            no control, a scaled form (kind FSV_HADA .. FSV_ROTI2;
//                                        m[0] = k, m[1] = t)
//   kLeafLaneScl + kind * 6 + lane bit   the same across lanes (kind FSV_HADA .. FSV_ROTI; m[1] = t)
// Diagonal leaves (factors d0, d1 on the target's bit values):
//   kDiagLP   + ts                       target and control off the register group: one factor
//                                        per lane (ts: 0 the target is a workgroup bit, 1 a thread bit)
//   kDiagCP   + ts * 4 + cp              control on register bit cp, target off the group
//   kDiagTP   + (TP * 5 + cp + 1) * 2 + d0   target on register bit TP (cp -1: none or a thread bit);
//                                        d0 = 0 when d0 is exactly 1
constexpr int kLeafNC = 0, kLeafCP = 24, kLeafLC = 72, kLeafLane = 88, kLeafScl = 112, kLeafLaneScl = 132,
              kLeafEnd = 150;
constexpr int kDiagLP = 0, kDiagCP = 2, kDiagTP = 10, kDiagEnd = 50;

template <int C>
__device__ __forceinline__ void fsv_general_leaf(f32x16& ar, f32x16& ai, const Mat2& M, int jt, int cloc,
                                                 int lane) {
    if constexpr (C < kLeafCP) {
        constexpr int form = (C - kLeafNC) / 4, rb = (C - kLeafNC) % 4;
        fsv_pairs<rb, -1, form, false>(ar, ai, M);
    } else if constexpr (C < kLeafLC) {
        constexpr int x = C - kLeafCP, fc = x / 16, rb = (x / 4) % 4, cp = x % 4;
        constexpr int form = fc == 0 ? FSV_XSWAP : (fc == 1 ? FSV_REAL : FSV_COMPLEX);
        if constexpr (cp != rb) fsv_pairs<rb, cp, form, false>(ar, ai, M);
    } else if constexpr (C < kLeafLane) {
        constexpr int x = C - kLeafLC, fc = x / 4, rb = x % 4;
        const bool on = (jt >> cloc) & 1;
        if constexpr (fc == 0) {
            fsv_xswap_lanes<rb>(ar, ai, __builtin_amdgcn_ballot_w64(on));
        } else {
            // lanes whose control bit is 0 apply the identity (exact: products
            // with 1 and 0); the identity is REAL and IMAGOFF, not ANTI or IPERM
            Mat2 L;
            L.m0r = on ? M.m0r : 1.f;
            L.m0i = on ? M.m0i : 0.f;
            L.m1r = on ? M.m1r : 0.f;
            L.m1i = on ? M.m1i : 0.f;
            L.m2r = on ? M.m2r : 0.f;
            L.m2i = on ? M.m2i : 0.f;
            L.m3r = on ? M.m3r : 1.f;
            L.m3i = on ? M.m3i : 0.f;
            constexpr int form = fc == 1 ? FSV_REAL : (fc == 2 ? FSV_IMAGOFF : FSV_COMPLEX);
            fsv_pairs<rb, -1, form, true>(ar, ai, L);
        }
    } else if constexpr (C >= kLeafLaneScl) {
        constexpr int x = C - kLeafLaneScl;
        fsv_lane_scaled<x % 6, x / 6>(ar, ai, M.m0i, lane);
    } else if constexpr (C >= kLeafScl) {
        constexpr int x = C - kLeafScl;
        fsv_scaled_pairs<x % 4, x / 4>(ar, ai, M.m0r, M.m0i);
    } else {
        constexpr int x = C - kLeafLane, fc = x / 6, lb = x % 6;
        if constexpr (fc == 0) {
            fsv_lane_op<lb, FSV_XSWAP>(ar, ai, M, lane);
        } else if constexpr (fc == 3) {
            // the lanes whose control bit is set take their partner's value
            const uint64_t on = __builtin_amdgcn_ballot_w64(((jt >> cloc) & 1) != 0);
            fsv_lane_cswap<lb>(ar, ai, on, lane);
        } else {
            const bool hi = (lane >> lb) & 1;  // this lane holds index bit 1 of the pair
            const bool on = cloc < 0 || ((jt >> cloc) & 1);
            Mat2 c;  // m0: the coefficient of the lane's own value, m1: of its partner's
            c.m0r = on ? (hi ? M.m3r : M.m0r) : 1.f;
            c.m0i = on ? (hi ? M.m3i : M.m0i) : 0.f;
            c.m1r = on ? (hi ? M.m2r : M.m1r) : 0.f;
            c.m1i = on ? (hi ? M.m2i : M.m1i) : 0.f;
            c.m2r = c.m2i = c.m3r = c.m3i = 0.f;
            fsv_lane_op<lb, fc == 1 ? FSV_REAL : FSV_COMPLEX>(ar, ai, c, lane);
        }
    }
}

// d0 = (d0r, d0i) on the target's value 0, d1 on 1; tval: the target bit
// when it is off the register group; on: the thread-bit control holds.
template <int C>
__device__ __forceinline__ void fsv_diag_leaf(f32x16& ar, f32x16& ai, float& lpr, float& lpi, float d0r,
                                              float d0i, float d1r, float d1i, int tval, bool on) {
    if constexpr (C < kDiagCP) {
        // one factor per lane: d_tval where the control holds, else 1
        const float fr = on ? (tval ? d1r : d0r) : 1.f;
        const float fi = on ? (tval ? d1i : d0i) : 0.f;
        const float pr = fmaf(fr, lpr, -fi * lpi), pi = fmaf(fr, lpi, fi * lpr);
        lpr = pr;
        lpi = pi;
    } else if constexpr (C < kDiagTP) {
        // control on register bit cp: those registers times d_tval
        constexpr int cp = (C - kDiagCP) % 4;
        fsv_scale<cp>(ar, ai, tval ? d1r : d0r, tval ? d1i : d0i);
    } else {
        // target on register bit TP; a thread-bit control folds into the factors
        constexpr int x = C - kDiagTP, d0 = x % 2, tp = (x / 2) / 5, cp = (x / 2) % 5 - 1;
        if constexpr (cp != tp) {
            if constexpr (cp >= 0)
                fsv_diag_reg<tp, cp, d0 == 1>(ar, ai, d0r, d0i, d1r, d1i);
            else
                fsv_diag_reg<tp, -1, d0 == 1>(ar, ai, on ? d0r : 1.f, on ? d0i : 0.f, on ? d1r : 1.f,
                                              on ? d1i : 0.f);
        }
    }
}

#define FSV_GEN_LEAF(C) \
    case C: fsv_general_leaf<C>(ar, ai, M, jt, g.cloc, lane); break;
#define FSV_GEN_LEAF2(C) FSV_GEN_LEAF(C) FSV_GEN_LEAF(C + 1)
#define FSV_GEN_LEAF8(C) FSV_GEN_LEAF2(C) FSV_GEN_LEAF2(C + 2) FSV_GEN_LEAF2(C + 4) FSV_GEN_LEAF2(C + 6)
#define FSV_DIAG_LEAF(C) \
    case C: fsv_diag_leaf<C>(ar, ai, lpr, lpi, d0r, d0i, d1r, d1i, tval, on); break;
#define FSV_DIAG_LEAF2(C) FSV_DIAG_LEAF(C) FSV_DIAG_LEAF(C + 1)
#define FSV_DIAG_LEAF10(C) \
    FSV_DIAG_LEAF2(C) FSV_DIAG_LEAF2(C + 2) FSV_DIAG_LEAF2(C + 4) FSV_DIAG_LEAF2(C + 6) FSV_DIAG_LEAF2(C + 8)

// A dense operation on local bits lb .. lb+w-1: out[j] = sum_s M[row(j)][s] in[j with
// those bits = s], through LDS; the register layout is unchanged.
__device__ __forceinline__ void fsv_dense(f32x16& ar_out, f32x16& ai_out, int t, int cur, const FsvGate& g,
                                          const float* __restrict__ pool, float* s_re, float* s_im) {
    f32x16 ar = ar_out, ai = ai_out;  // value copies: the caller sees whole-vector accesses only
    __syncthreads();
    const int jt = fsv_thread_bits(t, cur), sh = 4 * cur;
    fsv_for16([&](auto I_) {
        constexpr int r = decltype(I_)::value;
        const int a = fsv_swz(jt | (r << sh));
        s_re[a] = ar[r];
        s_im[a] = ai[r];
    });
    __syncthreads();
    const int lb = g.tloc, W = 1 << g.width;
    const int field = (W - 1) << lb;
    const float* M = pool + g.moff;
    fsv_for16([&](auto I_) {
        constexpr int r = decltype(I_)::value;
        const int j = jt | (r << sh);
        const int row = (j >> lb) & (W - 1);
        const int rest = j & ~field;
        const float* mr = M + 2 * row * W;
        float yr = 0.f, yi = 0.f;
        for (int c = 0; c < W; ++c) {
            const int a = fsv_swz(rest | (c << lb));
            const float xr = s_re[a], xi = s_im[a];
            const float er = mr[2 * c], ei = mr[2 * c + 1];
            yr = fmaf(er, xr, fmaf(-ei, xi, yr));
            yi = fmaf(er, xi, fmaf(ei, xr, yi));
        }
        ar[r] = yr;
        ai[r] = yi;
    });
    ar_out = ar;
    ai_out = ai;
}

// Layout change cur -> k of one plane through the LDS buffer s (one plane,
// 16 KiB: the two planes go through it in turn, which keeps a workgroup's LDS
// at 16 KiB and lets seven workgroups share a CU).
__device__ __forceinline__ void fsv_relayout_plane(f32x16& x, int t, int cur, int k, float* s) {
    char* sb = reinterpret_cast<char*>(s);
    __syncthreads();  // earlier readers of the buffer are done
    const uint32_t aw = 4 * fsv_swz(fsv_thread_bits(t, cur));
    const int32_t* cw = kFsvSwzReg.v[cur];
    fsv_for16([&](auto I_) {
        constexpr int r = decltype(I_)::value;
        *reinterpret_cast<float*>(sb + (aw ^ cw[r])) = x[r];
    });
    __syncthreads();
    const uint32_t ar_ = 4 * fsv_swz(fsv_thread_bits(t, k));
    const int32_t* cr = kFsvSwzReg.v[k];
    fsv_for16([&](auto I_) {
        constexpr int r = decltype(I_)::value;
        x[r] = *reinterpret_cast<const float*>(sb + (ar_ ^ cr[r]));
    });
}
__device__ __forceinline__ void fsv_relayout(f32x16& ar, f32x16& ai, int t, int cur, int k, float* s) {
    fsv_relayout_plane(ar, t, cur, k, s);
    fsv_relayout_plane(ai, t, cur, k, s);
}

// SWAP of local bits a and b: per plane one LDS round trip in the current
// layout, each amplitude read back from the index with those two bits exchanged.
__device__ __forceinline__ void fsv_swap_plane(f32x16& x, int t, int cur, int a, int b, float* s) {
    __syncthreads();  // earlier readers of the buffer are done
    const int jt = fsv_thread_bits(t, cur), sh = 4 * cur;
    const uint32_t aw = 4 * fsv_swz(jt);
    const int32_t* cw = kFsvSwzReg.v[cur];
    fsv_for16([&](auto I_) {
        constexpr int r = decltype(I_)::value;
        *reinterpret_cast<float*>(reinterpret_cast<char*>(s) + (aw ^ cw[r])) = x[r];
    });
    __syncthreads();
    const int both = (1 << a) | (1 << b);
    fsv_for16([&](auto I_) {
        constexpr int r = decltype(I_)::value;
        int j = jt | (r << sh);
        if (((j >> a) ^ (j >> b)) & 1) j ^= both;
        x[r] = s[fsv_swz(j)];
    });
}
__device__ __forceinline__ void fsv_swap_bits(f32x16& ar, f32x16& ai, int t, int cur, int a, int b, float* s) {
    fsv_swap_plane(ar, t, cur, a, b, s);
    fsv_swap_plane(ai, t, cur, a, b, s);
}

// WIDE: the pass holds a dense operation, whose products need both planes in
// LDS at once (32 KiB); other passes use one 16 KiB plane buffer.
template <bool WIDE>
__global__ __launch_bounds__(256) void fsv_pass_kernel(int n, FsvPass p, const FsvGate* __restrict__ gates,
                                                      const float* __restrict__ pool, float* __restrict__ re,
                                                      float* __restrict__ im) {
    __shared__ float s_buf[(WIDE ? 2 : 1) << kFsvLocal];
    const int t = threadIdx.x;

    // Global index of local index 0: the workgroup number with zero bits
    // inserted at the local positions above the low L qubits.
    uint64_t base = 0;
    if (n > kFsvLocal) {
        base = (uint64_t)blockIdx.x << p.L;
#pragma unroll
        for (int h = 0; h < kFsvMaxHigh; ++h) {
            if (h < p.nh) {
                const uint64_t low = ((uint64_t)1 << p.high[h]) - 1;
                base = ((base & ~low) << 1) | (base & low);
            }
        }
    }
    // Load/store layout 2: local bits 0-7 = thread index, 8-11 = register.
    // A thread's part of the global index is a 32-bit byte offset (local bits
    // 0-7 map to qubits below 30 whenever n <= 34: they are qubits 0-7 or the
    // smallest of the six highest local qubits); each register adds a uniform
    // part, so every access is a scalar base plus this one vector offset.
    uint32_t gt = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b) gt |= (uint32_t)((t >> b) & 1) << p.pos[b];
    const uint32_t off4 = gt << 2;
    const bool full = n >= kFsvLocal;
    const int nloc = full ? (1 << kFsvLocal) : (1 << n);
    auto reg_base = [&](int r) {
        uint64_t u = base;
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if ((r >> b) & 1) u |= (uint64_t)1 << p.pos[8 + b];
        return u;
    };

    f32x16 ar, ai;
    fsv_for16([&](auto I_) {
        constexpr int r = decltype(I_)::value;
        const uint64_t u = reg_base(r);
        float vr = 0.f, vi = 0.f;
        if (full || (t | (r << 8)) < nloc) {
            vr = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(re + u) + off4);
            vi = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(im + u) + off4);
        }
        ar[r] = vr;
        ai[r] = vi;
    });

    // Diagonal factors that depend only on this lane's index bits (and the
    // workgroup's) are gathered into one per-lane phase.  A factor common to a
    // lane's 16 registers commutes with every operation that acts within the
    // current layout (they are linear maps on those 16 values), so the phase is
    // applied only when amplitudes move between lanes (a layout change, SWAP,
    // a dense operation) and when the pass ends.
    float lpr = 1.f, lpi = 0.f;

    // Operation records are read with scalar loads (uniform addresses), so
    // every field and coefficient is an SGPR.  (Requesting the next record
    // ahead costs a 16-register copy per operation; the load latency is
    // instead covered by the other waves on the SIMD.)
    const int nops = p.g1 - p.g0;
    const FsvGate* __restrict__ ops = gates + p.g0;
    int cur = 2;
    for (int gi = 0; gi < nops; ++gi) {
        FsvGate g = ops[gi];
        if (g.kind == FSV_GENERAL) {
            // Planned by the host for every workgroup alike (tglob bit 0: apply
            // the pending per-lane phase; bit 1: change to the target's layout),
            // so they happen even where a non-local control is 0.
            if (g.tglob != 0) {
                if (g.tglob & 1) fsv_flush(ar, ai, lpr, lpi);
                if (g.tglob & 2) {
                    const int k = g.tloc >> 2;
                    fsv_relayout(ar, ai, t, cur, k, s_buf);
                    cur = k;
                }
            }
            if (g.cglob >= 0 && !((base >> g.cglob) & 1)) continue;  // a non-local control is 0 here
            const Mat2 M = {g.m[0], g.m[1], g.m[2], g.m[3], g.m[4], g.m[5], g.m[6], g.m[7]};
            const int jt = fsv_thread_bits(t, cur);  // the thread's local index bits in this layout
            const int lane = t & 63;
            switch (g.real) {
                FSV_GEN_LEAF8(0) FSV_GEN_LEAF8(8) FSV_GEN_LEAF8(16) FSV_GEN_LEAF8(24) FSV_GEN_LEAF8(32)
                FSV_GEN_LEAF8(40) FSV_GEN_LEAF8(48) FSV_GEN_LEAF8(56) FSV_GEN_LEAF8(64) FSV_GEN_LEAF8(72)
                FSV_GEN_LEAF8(80) FSV_GEN_LEAF8(88) FSV_GEN_LEAF8(96) FSV_GEN_LEAF8(104) FSV_GEN_LEAF2(112)
                FSV_GEN_LEAF2(114) FSV_GEN_LEAF2(116) FSV_GEN_LEAF2(118) FSV_GEN_LEAF8(120) FSV_GEN_LEAF8(128)
                FSV_GEN_LEAF8(136) FSV_GEN_LEAF2(144) FSV_GEN_LEAF2(146) FSV_GEN_LEAF2(148)
                default: break;
            }
            continue;
        }
        if (g.cglob >= 0 && !((base >> g.cglob) & 1)) continue;  // a non-local control is 0 here
        if (g.kind == FSV_PHASE) {
            // A grouped-diagonal record holds a table over some non-local
            // qubits: this workgroup's entry makes it a plain diagonal on its
            // local bit (no local bit: d0 = d1, the same factor whatever bit it reads).
            // Entries of its windows (bits lo .. lo + w - 1 of the workgroup
            // number, each window's table after the previous one) multiply.
            const uint32_t wg = blockIdx.x;
            int off = g.moff;
            float4 e = make_float4(1.f, 0.f, 1.f, 0.f);
            for (int k = 0; k < g.width; ++k) {
                const int f = (g.tglob >> (10 * k)) & 1023;
                const int lo = f & 31, w = f >> 5;
                const float4 v = *reinterpret_cast<const float4*>(pool + off + 4 * ((wg >> lo) & ((1u << w) - 1)));
                if (k == 0) {
                    e = v;
                } else {
                    e = make_float4(e.x * v.x - e.y * v.y, e.x * v.y + e.y * v.x,
                                    e.z * v.z - e.w * v.w, e.z * v.w + e.w * v.z);
                }
                off += 4 << w;
            }
            g.m[0] = e.x;
            g.m[1] = e.y;
            g.m[6] = e.z;
            g.m[7] = e.w;
            g.kind = FSV_DIAG;
            if (g.tloc < 0) g.tglob = 0;
        }
        if (g.kind == FSV_TABLE) {
            // Factored diagonal (see the planner): F on the registers named in
            // width, P (tglob bit 0) into the per-lane phase, then W_i on the
            // registers with bit i set for each i in cloc; P and each W_i are
            // tables of 256 entries read at the thread index.
            const float* __restrict__ tb = pool + g.moff;
            fsv_for16([&](auto I_) {
                constexpr int r = decltype(I_)::value;
                if ((g.width >> r) & 1) {
                    float xr = ar[r], xi = ai[r];
                    fsv_cmul<false>(xr, xi, tb[2 * r], tb[2 * r + 1]);
                    ar[r] = xr;
                    ai[r] = xi;
                }
            });
            const float* __restrict__ tt = tb + 32 + 2 * t;
            if (g.tglob & 1) {
                const float2 f = *reinterpret_cast<const float2*>(tt);
                const float nr = lpr * f.x - lpi * f.y;
                lpi = lpr * f.y + lpi * f.x;
                lpr = nr;
                tt += 512;
            }
            fsv_for4([&](auto I_) {
                constexpr int i = decltype(I_)::value;
                if ((g.cloc >> i) & 1) {
                    const float2 w = *reinterpret_cast<const float2*>(tt);
                    tt += 512;
                    fsv_scale<i>(ar, ai, w.x, w.y);
                }
            });
            continue;
        }
        const int jt = fsv_thread_bits(t, cur);
        if (g.kind == FSV_DENSE) {  // only in WIDE passes
            if constexpr (WIDE) {
                fsv_flush(ar, ai, lpr, lpi);
                fsv_dense(ar, ai, t, cur, g, pool, s_buf, s_buf + (1 << kFsvLocal));
            }
            continue;
        }
        if (g.kind == FSV_SWAP) {
            fsv_flush(ar, ai, lpr, lpi);
            fsv_swap_bits(ar, ai, t, cur, g.tloc, g.cloc, s_buf);
            continue;
        }
        // diagonal
        const float d0r = g.m[0], d0i = g.m[1], d1r = g.m[6], d1i = g.m[7];
        const int tval = g.tloc < 0 ? (int)((base >> g.tglob) & 1) : (jt >> g.tloc) & 1;
        const bool on = g.cloc < 0 || ((jt >> g.cloc) & 1);  // used by leaves whose control is a thread bit
        switch (g.real) {
            FSV_DIAG_LEAF10(0) FSV_DIAG_LEAF10(10) FSV_DIAG_LEAF10(20) FSV_DIAG_LEAF10(30) FSV_DIAG_LEAF10(40)
            default: break;
        }
    }
    // The factors the scaled forms took out, and the per-lane phase when one is
    // still pending (the host knows which: tail 2 both, 1 the scale only).
    if (p.tail == 2) {
        lpr *= p.scale;
        lpi *= p.scale;
        fsv_flush(ar, ai, lpr, lpi);
    } else if (p.tail == 1) {
        const float sc = p.scale;
        fsv_for16([&](auto I_) {
            constexpr int r = decltype(I_)::value;
            float xr = ar[r], xi = ai[r];
            asm("v_mul_f32 %0, %2, %0\n\t"
                "v_mul_f32 %1, %2, %1"
                : "+v"(xr), "+v"(xi)
                : "s"(sc));
            ar[r] = xr;
            ai[r] = xi;
        });
    }
    if (cur != 2) fsv_relayout(ar, ai, t, cur, 2, s_buf);

    fsv_for16([&](auto I_) {
        constexpr int r = decltype(I_)::value;
        const uint64_t u = reg_base(r);
        const float vr = ar[r], vi = ai[r];
        if (full || (t | (r << 8)) < nloc) {
            *reinterpret_cast<float*>(reinterpret_cast<char*>(re + u) + off4) = vr;
            *reinterpret_cast<float*>(reinterpret_cast<char*>(im + u) + off4) = vi;
        }
    });
}

// Permutation pass (see FsvPerm): one workgroup per tile pair, planes in turn
// through a 32 KiB LDS buffer (two tiles of 1024 to 4096 floats).  A tile
// element's address, LDS slot and permuted index are linear over XOR in its
// bits, so each splits into a per-thread part and parts uniform over the
// workgroup.
__device__ __forceinline__ uint32_t fsv_tile_perm(uint32_t e, const FsvPerm& q, int tbits) {
    uint32_t o = 0;
    for (int b = 0; b < tbits; ++b) o |= ((e >> b) & 1u) << q.sig_tile[b];
    return o;
}
__device__ __forceinline__ uint64_t fsv_tile_addr(uint32_t e, const FsvPerm& q) {
    uint64_t a = e & 63u;
    for (int j = 0; j < q.h; ++j) a |= (uint64_t)((e >> (6 + j)) & 1u) << q.hpos[j];
    return a;
}
// LDS slot of tile element e: its row bits folded onto its column bits (a
// bijection, linear over XOR), so that a wave reading a permuted row spreads
// over the banks.
__device__ __forceinline__ uint32_t fsv_perm_slot(uint32_t e, const FsvPerm& q) {
    uint32_t s = e;
    for (int j = 0; j < q.h; ++j)
        if ((e >> (6 + j)) & 1u) s ^= (uint32_t)q.fold[j];
    return s;
}

__global__ __launch_bounds__(256) void fsv_perm_kernel(FsvPerm q, float* __restrict__ re, float* __restrict__ im) {
    __shared__ float sa[1 << kFsvLocal], sb[1 << kFsvLocal];
    const uint32_t g = blockIdx.x;
    uint32_t g2 = 0;
    uint64_t base_a = 0, base_b = 0;
    for (int b = 0; b < q.ng; ++b) {
        const uint32_t bit = (g >> b) & 1u;
        g2 |= bit << q.sig_group[b];
        base_a |= (uint64_t)bit << q.gpos[b];
    }
    if (g2 < g) return;  // the pair's other workgroup moves it (uniform exit)
    for (int b = 0; b < q.ng; ++b) base_b |= (uint64_t)((g2 >> b) & 1u) << q.gpos[b];
    const bool pair = g2 != g;
    const int tbits = 6 + q.h;  // 10 to 12
    const int nj = 1 << (tbits - 10);
    // thread t holds elements e0 + c + 1024 j (c < 4): four contiguous
    // amplitudes, 16 threads to a row
    const uint32_t e0 = 4 * threadIdx.x;
    const uint64_t at = fsv_tile_addr(e0, q);
    const uint32_t lt = fsv_perm_slot(e0, q);
    const uint32_t st = fsv_perm_slot(fsv_tile_perm(e0, q, tbits), q);
    uint64_t aj[4];
    uint32_t lj[4], sj[4], sc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t k = (uint32_t)j << 10;
        aj[j] = fsv_tile_addr(k, q) >> 2;
        lj[j] = fsv_perm_slot(k, q);
        sj[j] = fsv_perm_slot(fsv_tile_perm(k, q, tbits), q);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) sc[c] = fsv_perm_slot(fsv_tile_perm((uint32_t)c, q, tbits), q);
    float4 va[4], vb[4];
#pragma unroll
    for (int pl = 0; pl < 2; ++pl) {
        float* __restrict__ P = pl ? im : re;
        float4* pa = reinterpret_cast<float4*>(P + (base_a | at));
        float4* pb = reinterpret_cast<float4*>(P + (base_b | at));
        // every load of the plane in flight before the first LDS write
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j < nj) {
                va[j] = pa[aj[j]];
                if (pair) vb[j] = pb[aj[j]];
            }
        __syncthreads();  // the previous plane's readers of the buffer are done
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j < nj) {
                const uint32_t s0 = lt ^ lj[j];  // slot(e0 + c + 1024 j) = s0 ^ c
                sa[s0] = va[j].x;
                sa[s0 ^ 1] = va[j].y;
                sa[s0 ^ 2] = va[j].z;
                sa[s0 ^ 3] = va[j].w;
                if (pair) {
                    sb[s0] = vb[j].x;
                    sb[s0 ^ 1] = vb[j].y;
                    sb[s0 ^ 2] = vb[j].z;
                    sb[s0 ^ 3] = vb[j].w;
                }
            }
        __syncthreads();
        // output element e of group sigma(g) is input element sigma(e) of group g
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j < nj) {
                const uint32_t s0 = st ^ sj[j];
                va[j] = make_float4(sa[s0 ^ sc[0]], sa[s0 ^ sc[1]], sa[s0 ^ sc[2]], sa[s0 ^ sc[3]]);
                if (pair) vb[j] = make_float4(sb[s0 ^ sc[0]], sb[s0 ^ sc[1]], sb[s0 ^ sc[2]], sb[s0 ^ sc[3]]);
            }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j < nj) {
                pb[aj[j]] = va[j];
                if (pair) pa[aj[j]] = vb[j];
            }
    }
}

// |basis> in planar complex64, written as float4 (2N floats, N >= 2).
__global__ __launch_bounds__(256) void fsv_basis_kernel(uint64_t n4, uint64_t basis, float4* __restrict__ psi) {
    for (uint64_t v = (uint64_t)blockIdx.x * 256 + threadIdx.x; v < n4; v += (uint64_t)gridDim.x * 256) {
        float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
        if (v == (basis >> 2)) {
            const int c = (int)(basis & 3);
            x.x = c == 0 ? 1.f : 0.f;
            x.y = c == 1 ? 1.f : 0.f;
            x.z = c == 2 ? 1.f : 0.f;
            x.w = c == 3 ? 1.f : 0.f;
        }
        psi[v] = x;
    }
}

// sum |psi_i|^2 in float64: fixed-order per-block partials, then one block.
__global__ __launch_bounds__(256) void fsv_norm_partial(uint64_t N, const float* __restrict__ re,
                                                       const float* __restrict__ im, double* __restrict__ part) {
    __shared__ double red[256];
    double s = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (uint64_t)gridDim.x * 256) {
        const double a = re[i], b = im[i];
        s += a * a + b * b;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// ---- measurement of a full state (the collapsing simulator method, Section 5.2.3) ----
// The cumulative distribution is never stored: amplitudes are grouped in
// blocks of 1024 (one wave each: lane l owns amplitudes 16l .. 16l+15 of the
// block), and only the float64 block sums and their prefix are kept.  A shot
// finds its block by binary search over the prefix, its lane by the same
// in-wave scan that produced the block sum (so the two agree exactly), and its
// amplitude by a sequential scan of the lane's 16 values.
constexpr int kSampleBlock = 1024;

__device__ __forceinline__ double lane_prob_sum(const float* __restrict__ re, const float* __restrict__ im, uint64_t N,
                                                uint64_t first) {
    double s = 0.0;
    if (first + 16 <= N) {  // 64-byte aligned runs: vector loads, same summation order
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 a = *reinterpret_cast<const float4*>(re + first + 4 * q);
            const float4 b = *reinterpret_cast<const float4*>(im + first + 4 * q);
            s += (double)a.x * a.x + (double)b.x * b.x;
            s += (double)a.y * a.y + (double)b.y * b.y;
            s += (double)a.z * a.z + (double)b.z * b.z;
            s += (double)a.w * a.w + (double)b.w * b.w;
        }
        return s;
    }
    for (int k = 0; k < 16; ++k) {
        const uint64_t i = first + k;
        if (i < N) {
            const double a = re[i], b = im[i];
            s += a * a + b * b;
        }
    }
    return s;
}

// Inclusive scan over the 64 lanes in a fixed order (Hillis-Steele).
__device__ __forceinline__ double wave_incl_scan(double v, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
    }
    return v;
}

// One wave per block: the block's probability mass.
__global__ __launch_bounds__(256) void fsv_block_sums(uint64_t N, uint64_t nblocks, const float* __restrict__ re,
                                                     const float* __restrict__ im, double* __restrict__ bsum) {
    const uint64_t b = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (b >= nblocks) return;
    const double v = wave_incl_scan(lane_prob_sum(re, im, N, b * kSampleBlock + 16 * lane), lane);
    if (lane == 63) bsum[b] = v;
}

// In place: bsum[b] <- bsum[0] + ... + bsum[b], one 1024-thread block, fixed order
// (each thread a contiguous chunk, chunk totals scanned, chunks re-summed from their offset).
__global__ __launch_bounds__(1024) void fsv_block_prefix(uint64_t nblocks, double* __restrict__ bsum) {
    __shared__ double tot[1024];
    const uint64_t chunk = (nblocks + 1023) / 1024;
    const uint64_t lo = (uint64_t)threadIdx.x * chunk;
    const uint64_t hi = lo + chunk < nblocks ? lo + chunk : nblocks;
    double s = 0.0;
    for (uint64_t i = lo; i < hi; ++i) s += bsum[i];
    tot[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const double v = (int)threadIdx.x >= off ? tot[threadIdx.x - off] : 0.0;
        __syncthreads();
        tot[threadIdx.x] += v;
        __syncthreads();
    }
    double run = threadIdx.x ? tot[threadIdx.x - 1] : 0.0;
    for (uint64_t i = lo; i < hi; ++i) {
        run += bsum[i];
        bsum[i] = run;
    }
}

// One wave per shot.
__global__ __launch_bounds__(256) void fsv_sample_kernel(uint64_t N, uint64_t nblocks, const float* __restrict__ re,
                                                        const float* __restrict__ im, const double* __restrict__ pre,
                                                        const double* __restrict__ u, int shots,
                                                        int64_t* __restrict__ out) {
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (k >= shots) return;
    const double target = u[k] * pre[nblocks - 1];
    // smallest block b with target < pre[b]
    uint64_t lo = 0, hi = nblocks - 1;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (pre[mid] > target)
            hi = mid;
        else
            lo = mid + 1;
    }
    const uint64_t b = lo;
    const double base = b ? pre[b - 1] : 0.0;
    const uint64_t first = b * kSampleBlock + 16 * lane;
    const double L = wave_incl_scan(lane_prob_sum(re, im, N, first), lane);
    const double Lprev = __shfl_up(L, 1, 64);
    // first lane whose chunk ends above the target
    const unsigned long long hit = __ballot(target < base + L);
    const int l = hit ? __ffsll(hit) - 1 : 63;
    if (lane == l) {
        double c = base + (lane ? Lprev : 0.0);
        uint64_t pick = first + 15 < N ? first + 15 : N - 1;
        for (int j = 0; j < 16; ++j) {
            const uint64_t i = first + j;
            if (i >= N) break;
            const double a = re[i], bb = im[i];
            c += a * a + bb * bb;
            if (target < c) {
                pick = i;
                break;
            }
        }
        out[k] = (int64_t)pick;
    }
}

__global__ __launch_bounds__(256) void fsv_norm_final(int parts, const double* __restrict__ part,
                                                     double* __restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < parts; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// --- host planning -------------------------------------------------------------------------

struct LoweredGate {
    int kind;
    int tq, cq;     // target (dense: lowest qubit of the range), control (-1: none)
    int width = 0;  // dense: qubits in the range
    int32_t op = 0; // dense: registered operation
    float m[8];
    double md[8];   // the float64 matrix (diagonal runs are multiplied out from it)
};

void lower(const qsim_gate* gates, int n_gates, std::vector<LoweredGate>& out) {
    out.clear();
    for (int i = 0; i < n_gates; ++i) {
        const qsim_gate& g = gates[i];
        if (g.kind == QSIM_CUSTOM) {
            LoweredGate l{};
            l.kind = FSV_DENSE;
            l.tq = g.target;
            l.cq = -1;
            l.width = custom_qubits(g.op_id);
            l.op = g.op_id;
            out.push_back(l);
            continue;
        }
        if (g.kind == QSIM_SWAP) {  // a permutation of two local bits
            LoweredGate l{};
            l.kind = FSV_SWAP;
            l.tq = g.target;
            l.cq = g.control;
            out.push_back(l);
            continue;
        }
        double m[8];
        gate_matrix(g, m);
        LoweredGate l{};
        l.kind = (m[2] == 0 && m[3] == 0 && m[4] == 0 && m[5] == 0) ? FSV_DIAG : FSV_GENERAL;
        l.tq = g.target;
        l.cq = g.control;
        for (int k = 0; k < 8; ++k) {
            l.m[k] = (float)m[k];
            l.md[k] = m[k];
        }
        out.push_back(l);
    }
}

int popcount64(uint64_t x) { return __builtin_popcountll(x); }

// Largest L in [kFsvMinLow, kFsvLocal] that leaves room for every target at or
// above L among the 12 - L other local slots; -1 if none.
int fit_low(uint64_t targets) {
    for (int L = kFsvLocal; L >= kFsvMinLow; --L)
        if (L + popcount64(targets >> L) <= kFsvLocal) return L;
    return -1;
}

// Qubits a gate needs local: the target of a non-diagonal 2x2, both qubits of a SWAP, the whole range of a
// dense operation.
uint64_t local_need(const LoweredGate& l) {
    if (l.kind == FSV_GENERAL) return (uint64_t)1 << l.tq;
    if (l.kind == FSV_SWAP) return ((uint64_t)1 << l.tq) | ((uint64_t)1 << l.cq);
    if (l.kind == FSV_DENSE) return (((uint64_t)1 << l.width) - 1) << l.tq;
    return 0;
}

// Pool offsets (floats) of each dense operation's float32 matrix, appended to `pool` once per id.
int pool_offset(int32_t op, int width, std::vector<float>& pool, std::vector<std::pair<int32_t, int>>& seen) {
    for (auto& kv : seen)
        if (kv.first == op) return kv.second;
    const int off = (int)pool.size();
    const double* h = custom_host(op);
    const int count = 2 << (2 * width);
    for (int i = 0; i < count; ++i) pool.push_back((float)h[i]);
    seen.emplace_back(op, off);
    return off;
}

// Qubits an operation touches (its whole span for a dense operation).
uint64_t op_qubits(const LoweredGate& l) {
    if (l.kind == FSV_DENSE) return (((uint64_t)1 << l.width) - 1) << l.tq;
    return ((uint64_t)1 << l.tq) | (l.cq >= 0 ? (uint64_t)1 << l.cq : 0);
}

// Passes over a gate list.  An operation must follow every earlier one that
// shares a qubit with it, unless both are diagonal (they commute).  A pass is
// filled by one sweep over the operations whose predecessors are all done, in
// circuit order, taking each one whose local qubits still fit; operations that
// become ready during the sweep are considered in the same sweep.  So a pass may
// take gates from later layers on its local qubits while a gate on a qubit that
// is not local waits for a later pass.  exec_order (optional) receives the
// operations pass by pass, each pass in the order its launch applies them.
// Permutation pass over the ready SWAPs (pairwise disjoint), which it takes
// out of the ready set.  Tile bits: positions 0-5, then the positions sigma
// exchanges with them, then whole orbits of sigma (fixed points first, lowest
// first) up to twelve bits: 10 to 12 bits for any n > 12 (orbits have one or
// two positions, and at least seven positions lie above 5).
FsvPass perm_pass(int n, const std::vector<LoweredGate>& gs, std::set<int>& ready,
                  const std::vector<std::vector<int>>& succ_all, std::vector<int>& indeg_all,
                  std::vector<int>* exec_order, const std::vector<FsvGate>& table, int& executed) {
    FsvPass p{};
    p.perm = 1;
    int sigma[64];
    for (int x = 0; x < n; ++x) sigma[x] = x;
    const std::vector<int> ops(ready.begin(), ready.end());
    for (int b : ops) {
        sigma[gs[b].tq] = gs[b].cq;
        sigma[gs[b].cq] = gs[b].tq;
    }
    for (int b : ops) {
        ready.erase(b);
        for (int c : succ_all[b])
            if (--indeg_all[c] == 0) ready.insert(c);
        if (exec_order) exec_order->push_back(b);
    }
    FsvPerm& q = p.pm;
    int tile_bit[64];
    for (int x = 0; x < n; ++x) tile_bit[x] = x < 6 ? x : -1;
    q.h = 0;
    auto add = [&](int x, int fold) {
        q.hpos[q.h] = x;
        q.fold[q.h] = fold;
        tile_bit[x] = 6 + q.h++;
    };
    // an exchanged row bit folds onto the column bit it came from, so the 64
    // lanes reading a permuted row hit 64 distinct LDS banks
    for (int l = 0; l < 6; ++l)
        if (sigma[l] >= 6) add(sigma[l], 1 << l);
    for (int pairs = 0; pairs < 2; ++pairs)
        for (int x = 6; x < n && q.h < 6; ++x) {
            if (tile_bit[x] >= 0) continue;
            if (sigma[x] == x) {
                add(x, 0);
            } else if (pairs && q.h + 2 <= 6) {  // sigma[x] >= 6 is outside the tile too
                add(x, 0);
                add(sigma[x], 0);
            }
        }
    // Group bits in the order of max(x, sigma(x)): the workgroups resident at
    // once (consecutive indices) then read and write both tiles of their pairs
    // inside one window of the state, not one of them spread over all of it.
    int group_bit[64];
    q.ng = 0;
    for (int x = 6; x < n; ++x)
        if (tile_bit[x] < 0) q.gpos[q.ng++] = x;
    std::sort(q.gpos, q.gpos + q.ng, [&](int a, int b) {
        const int ka = std::max(a, sigma[a]), kb = std::max(b, sigma[b]);
        return ka != kb ? ka < kb : a < b;
    });
    for (int i = 0; i < q.ng; ++i) group_bit[q.gpos[i]] = i;
    for (int x = 0; x < n; ++x) {
        if (tile_bit[x] >= 0)
            q.sig_tile[tile_bit[x]] = tile_bit[sigma[x]];
        else
            q.sig_group[group_bit[x]] = group_bit[sigma[x]];
    }
    p.g0 = p.g1 = (int)table.size();
    p.op0 = executed;
    executed += (int)ops.size();
    p.op1 = executed;
    return p;
}

void fsv_schedule(int n, const std::vector<LoweredGate>& gs, std::vector<FsvPass>& passes,
                  std::vector<FsvGate>& table, std::vector<float>& pool, std::vector<int>* exec_order = nullptr) {
    passes.clear();
    table.clear();
    pool.clear();
    if (exec_order) exec_order->clear();
    std::vector<std::pair<int32_t, int>> seen;
    const int m_all = (int)gs.size();
    std::vector<std::vector<int>> succ_all(m_all);
    std::vector<int> indeg_all(m_all, 0);
    {
        std::vector<int> last_nd(64, -1), mark(m_all, -1);
        std::vector<std::vector<int>> diag_since(64);
        for (int b = 0; b < m_all; ++b) {
            const uint64_t qb = op_qubits(gs[b]);
            const bool dg = gs[b].kind == FSV_DIAG;
            auto dep = [&](int a) {
                if (a >= 0 && mark[a] != b) {
                    mark[a] = b;
                    succ_all[a].push_back(b);
                    ++indeg_all[b];
                }
            };
            for (int x = 0; x < n; ++x) {
                if (!((qb >> x) & 1)) continue;
                dep(last_nd[x]);
                if (!dg)
                    for (int a : diag_since[x]) dep(a);
            }
            for (int x = 0; x < n; ++x) {
                if (!((qb >> x) & 1)) continue;
                if (dg) {
                    diag_since[x].push_back(b);
                } else {
                    last_nd[x] = b;
                    diag_since[x].clear();
                }
            }
        }
    }
    std::set<int> ready;
    for (int b = 0; b < m_all; ++b)
        if (indeg_all[b] == 0) ready.insert(b);
    int executed = 0;
    int nonswap_left = 0;
    for (const LoweredGate& l : gs) nonswap_left += l.kind != FSV_SWAP;
    while (!ready.empty()) {
        // Only SWAPs ready (pairwise disjoint: a later SWAP sharing a qubit
        // waits for the earlier), and either more qubits than one pass holds
        // locally or nothing but SWAPs left: one permutation pass takes them
        // all, whatever their qubits, for one read and write of the state.
        if (n > kFsvLocal) {
            bool swaps = true;
            uint64_t touched = 0;
            for (int b : ready) {
                if (gs[b].kind != FSV_SWAP) swaps = false;
                touched |= op_qubits(gs[b]);
            }
            if (swaps && (__builtin_popcountll(touched) > kFsvLocal || nonswap_left == 0)) {
                passes.push_back(perm_pass(n, gs, ready, succ_all, indeg_all, exec_order, table, executed));
                continue;
            }
        }
        FsvPass p{};
        // One sweep over the ready operations in circuit order, taking each one
        // whose local qubits still fit (operations that become ready join the
        // sweep); with seed >= 0 that operation goes first, so its qubits shape
        // the pass.  Returns the operations taken and leaves rdy / indeg as
        // after them (undo, when given, records the indegrees it changed).
        auto sweep = [&](int seed, std::set<int>& rdy, std::vector<int>* undo, std::vector<int>& ops, uint64_t& T,
                         int& L) {
            T = 0;
            L = n <= kFsvLocal ? n : kFsvLocal;
            auto take = [&](int b) {
                ops.push_back(b);
                rdy.erase(b);
                for (int c : succ_all[b]) {
                    if (undo) undo->push_back(c);
                    if (--indeg_all[c] == 0) rdy.insert(c);
                }
            };
            if (seed >= 0) {
                T = local_need(gs[seed]);
                if (n > kFsvLocal) L = fit_low(T);
                take(seed);
            }
            for (auto it = rdy.begin(); it != rdy.end() && (int)ops.size() < kFsvMaxOps;) {
                const int b = *it;
                const uint64_t T2 = T | local_need(gs[b]);
                if (n > kFsvLocal) {
                    const int L2 = fit_low(T2);
                    if (L2 < 0) {
                        ++it;
                        continue;
                    }
                    L = L2;
                }
                T = T2;
                take(b);
                it = rdy.upper_bound(b);  // successors (larger indices) join this sweep
            }
        };
        // The plain sweep lets the earliest ready operations choose the local
        // qubits; a sweep seeded with one of the next ready operations that
        // needs a qubit above 5 may do better.  Each candidate is scored by the
        // operations it takes plus those the plain sweep after it would take
        // (one pass of look-ahead), and the best is kept (the plain sweep on
        // ties).  20 random layers on 30 qubits: 23-26 passes instead of
        // 25-30 over five seeds.
        int best_seed = -1;
        if (n > kFsvLocal) {
            size_t best = 0;
            std::vector<int> cand;
            cand.push_back(-1);
            for (int b : ready) {
                if ((int)cand.size() > kFsvSeeds) break;
                if (local_need(gs[b]) & ~(((uint64_t)1 << 6) - 1)) cand.push_back(b);
            }
            for (int seed : cand) {
                std::set<int> rdy = ready;
                std::vector<int> undo, ops;
                uint64_t T0;
                int L0;
                sweep(seed, rdy, &undo, ops, T0, L0);
                size_t score = ops.size();
                {
                    std::vector<int> ops2;
                    sweep(-1, rdy, &undo, ops2, T0, L0);
                    score += ops2.size();
                }
                for (int c : undo) ++indeg_all[c];
                if (score > best) {
                    best = score;
                    best_seed = seed;
                }
            }
        }
        uint64_t T = 0;
        int L = 0;
        std::vector<int> pass_ops;
        sweep(best_seed, ready, nullptr, pass_ops, T, L);
        if (n <= kFsvLocal) {
            p.L = n;
            p.nh = 0;
        } else {
            p.L = L;
            p.nh = kFsvLocal - L;
            std::vector<int> hs;
            for (int q = L; q < n; ++q)
                if ((T >> q) & 1) hs.push_back(q);
            for (int q = L; q < n && (int)hs.size() < p.nh; ++q)
                if (!((T >> q) & 1)) hs.push_back(q);
            std::sort(hs.begin(), hs.end());
            for (int h = 0; h < p.nh; ++h) p.high[h] = hs[h];
        }
        // Local bits 6 and 7 are qubits 6, 7 or the two smallest of at least five
        // ascending high qubits below n <= 34, so pos[0..7] < 30 and the kernel's
        // per-thread byte offset fits 32 bits.
        for (int b = 0; b < kFsvLocal; ++b) p.pos[b] = b < p.L ? b : (b < p.L + p.nh ? p.high[b - p.L] : b);
        p.op0 = executed;
        executed += (int)pass_ops.size();
        p.op1 = executed;
        for (int b : pass_ops) nonswap_left -= gs[b].kind != FSV_SWAP;
        auto local_bit = [&](int q) {
            if (q < 0) return -1;
            if (q < p.L) return q;
            for (int h = 0; h < p.nh; ++h)
                if (p.high[h] == q) return p.L + h;
            return -1;
        };
        p.g0 = (int)table.size();
        std::vector<std::vector<size_t>> tab_ops;  // the operations of each FSV_TABLE record
        auto record = [&](const LoweredGate& l) {
            FsvGate d{};
            d.kind = l.kind;
            d.tloc = local_bit(l.tq);
            d.tglob = d.tloc < 0 ? l.tq : -1;
            d.cloc = local_bit(l.cq);
            d.cglob = (l.cq >= 0 && d.cloc < 0) ? l.cq : -1;
            if (l.kind == FSV_DENSE) {
                d.width = l.width;
                d.moff = pool_offset(l.op, l.width, pool, seen);
            }
            d.real = fsv_form(l.m);
            std::copy(l.m, l.m + 8, d.m);
            return d;
        };
        // The thread bit (0-5: a lane bit) that local bit lb occupies in register
        // layout c, or -1 when lb is in the register group or a wave bit.
        auto lane_bit = [](int lb, int c) {
            const int tb = lb < 4 * c ? lb : (lb >= 4 * c + 4 ? lb - 4 : -1);
            return tb >= 0 && tb < 6 ? tb : -1;
        };
        // A non-diagonal operation can run in layout c without a layout change
        // when its target is in the register group, or on a lane bit and its
        // control (if local) is not a register bit.
        auto in_layout = [&](const LoweredGate& l, int c) {
            const int tb = local_bit(l.tq), cb = local_bit(l.cq);
            if ((tb >> 2) == c) return true;
            return lane_bit(tb, c) >= 0 && !(cb >= 0 && (cb >> 2) == c);
        };
        // Reorder the pass's operations where they commute (disjoint qubits, or
        // both diagonal) so that fewer layout changes are needed: ready
        // diagonal and custom operations first, then non-diagonal ones that can
        // run in the current register layout, else the earliest ready one.
        std::vector<size_t> order;
        {
            const size_t m = pass_ops.size();
            std::vector<uint64_t> qm(m);
            std::vector<char> dg(m);
            for (size_t a = 0; a < m; ++a) {
                const LoweredGate& l = gs[pass_ops[a]];
                qm[a] = op_qubits(l);
                dg[a] = l.kind == FSV_DIAG;
            }
            std::vector<std::vector<int>> succ(m);
            std::vector<int> indeg(m, 0);
            for (size_t b = 0; b < m; ++b)
                for (size_t a = 0; a < b; ++a)
                    if ((qm[a] & qm[b]) && !(dg[a] && dg[b])) {
                        succ[a].push_back((int)b);
                        ++indeg[b];
                    }
            std::vector<char> done(m, 0);
            int cur = 2;
            while (order.size() < m) {
                int pick = -1, pick_general = -1;
                for (size_t a = 0; a < m; ++a) {
                    if (done[a] || indeg[a] != 0) continue;
                    const LoweredGate& l = gs[pass_ops[a]];
                    if (l.kind != FSV_GENERAL) {
                        pick = (int)a;
                        break;
                    }
                    if (in_layout(l, cur)) {
                        if (pick < 0) pick = (int)a;
                    } else if (pick_general < 0) {
                        pick_general = (int)a;
                    }
                }
                if (pick < 0) {
                    pick = pick_general;
                    cur = local_bit(gs[pass_ops[pick]].tq) >> 2;
                }
                done[pick] = 1;
                order.push_back((size_t)pass_ops[pick]);
                for (int b : succ[pick]) --indeg[b];
            }
        }
        // the order the kernel runs them in (runs of diagonal operations are
        // multiplied out below, but commute, so any order within a run is this one)
        if (exec_order)
            for (size_t q : order) exec_order->push_back((int)q);
        for (size_t k = 0; k < order.size();) {
            if (gs[order[k]].kind != FSV_DIAG) {
                table.push_back(record(gs[order[k]]));
                ++k;
                continue;
            }
            // A run of diagonal operations (they commute): those whose qubits
            // are all local become one factored table (float64 products
            // rounded once; see the layout planning below); the others follow.
            size_t e = k;
            while (e < order.size() && gs[order[e]].kind == FSV_DIAG) ++e;
            std::vector<size_t> local_ops, other_ops;
            for (size_t x = k; x < e; ++x) {
                const size_t q = order[x];
                const bool local = local_bit(gs[q].tq) >= 0 && (gs[q].cq < 0 || local_bit(gs[q].cq) >= 0);
                (local ? local_ops : other_ops).push_back(q);
            }
            if (local_ops.size() >= 2) {
                // its factors are laid out once the pass's register layout at
                // this point is known (below)
                FsvGate d{};
                d.kind = FSV_TABLE;
                d.tloc = d.tglob = d.cloc = d.cglob = -1;
                d.moff = (int)tab_ops.size();
                tab_ops.push_back(local_ops);
                table.push_back(d);
            } else {
                for (size_t q : local_ops) other_ops.push_back(q);
            }
            // In a workgroup the non-local qubits are fixed, so each remaining operation is a diagonal on one
            // local bit (one local and one non-local qubit) or a single factor (no local qubit).  They are
            // grouped by that local bit and multiplied out on the host in float64 for every value of the
            // non-local qubits they read (tables over windows of the workgroup number): a few table lookups
            // and one update of the amplitudes replace a record per operation.
            std::vector<std::pair<int, std::vector<size_t>>> groups;  // local bit (-1: none), operations
            for (size_t q : other_ops) {
                const LoweredGate& l = gs[q];
                const int tb = local_bit(l.tq), cb = l.cq >= 0 ? local_bit(l.cq) : -1;
                int a;
                if (tb >= 0 && l.cq >= 0 && cb < 0)
                    a = tb;  // local target, non-local control
                else if (tb < 0 && cb >= 0)
                    a = cb;  // local control, non-local target
                else if (tb < 0)
                    a = -1;  // no local qubit
                else {
                    table.push_back(record(l));  // both local (a run with a single such operation)
                    continue;
                }
                size_t gi = 0;
                while (gi < groups.size() && groups[gi].first != a) ++gi;
                if (gi == groups.size()) groups.push_back({a, {}});
                groups[gi].second.push_back(q);
            }
            // The workgroup number holds the non-local qubits in ascending order;
            // a table is indexed by a window of at most kFsvPhaseBits of its bits,
            // and one record multiplies the entries of up to kFsvPhaseWindows
            // windows before it touches the amplitudes.
            auto wg_bit = [&](int q) {
                int below = std::min(q, p.L);
                for (int h = 0; h < p.nh; ++h) below += p.high[h] < q;
                return q - below;
            };
            for (auto& grp : groups) {
                const int a = grp.first;
                auto nonlocal = [&](const LoweredGate& l) {
                    std::vector<int> v;
                    if (local_bit(l.tq) < 0) v.push_back(wg_bit(l.tq));
                    if (l.cq >= 0 && local_bit(l.cq) < 0) v.push_back(wg_bit(l.cq));
                    return v;
                };
                std::vector<int> bits;
                for (size_t q : grp.second)
                    for (int bb : nonlocal(gs[q])) bits.push_back(bb);
                std::sort(bits.begin(), bits.end());
                bits.erase(std::unique(bits.begin(), bits.end()), bits.end());
                std::vector<std::pair<int, int>> wins;  // [lo, hi] over workgroup-number bits
                for (size_t i = 0; i < bits.size();) {
                    size_t j = i;
                    while (j + 1 < bits.size() && bits[j + 1] - bits[i] < kFsvPhaseBits) ++j;
                    wins.push_back({bits[i], bits[j]});
                    i = j + 1;
                }
                std::vector<std::vector<size_t>> in_win(wins.size());
                for (size_t q : grp.second) {
                    const std::vector<int> v = nonlocal(gs[q]);
                    size_t w = 0;
                    while (w < wins.size() && !(v[0] >= wins[w].first && v[0] <= wins[w].second)) ++w;
                    bool fits = true;
                    for (int bb : v) fits = fits && bb >= wins[w].first && bb <= wins[w].second;
                    if (fits)
                        in_win[w].push_back(q);
                    else
                        table.push_back(record(gs[q]));  // two non-local qubits in different windows
                }
                std::vector<size_t> used;
                for (size_t w = 0; w < wins.size(); ++w)
                    if (!in_win[w].empty()) used.push_back(w);
                for (size_t r0 = 0; r0 < used.size(); r0 += kFsvPhaseWindows) {
                    FsvGate d{};
                    d.kind = FSV_PHASE;
                    d.tloc = a;
                    d.tglob = 0;
                    d.cloc = d.cglob = -1;
                    d.width = 0;
                    d.moff = (int)pool.size();
                    for (size_t r = r0; r < used.size() && r < r0 + kFsvPhaseWindows; ++r) {
                        const int lo = wins[used[r]].first, w = wins[used[r]].second - lo + 1;
                        d.tglob |= (lo | (w << 5)) << (10 * d.width);
                        ++d.width;
                        for (int idx = 0; idx < (1 << w); ++idx) {
                            auto bit_of = [&](int q) { return (idx >> (wg_bit(q) - lo)) & 1; };
                            double u0r = 1.0, u0i = 0.0, u1r = 1.0, u1i = 0.0;  // diag(u0, u1) on bit a
                            auto mul = [](double& xr, double& xi, double fr, double fi) {
                                const double t = xr * fr - xi * fi;
                                xi = xr * fi + xi * fr;
                                xr = t;
                            };
                            for (size_t q : in_win[used[r]]) {
                                const LoweredGate& l = gs[q];
                                const double d0r = l.md[0], d0i = l.md[1], d1r = l.md[6], d1i = l.md[7];
                                if (local_bit(l.tq) >= 0) {  // local target, non-local control: where it is 1
                                    if (bit_of(l.cq)) {
                                        mul(u0r, u0i, d0r, d0i);
                                        mul(u1r, u1i, d1r, d1i);
                                    }
                                } else {
                                    const int tv = bit_of(l.tq);
                                    const double fr = tv ? d1r : d0r, fi = tv ? d1i : d0i;
                                    if (l.cq >= 0 && local_bit(l.cq) >= 0) {  // local control: where it is 1
                                        mul(u1r, u1i, fr, fi);
                                    } else if (l.cq < 0 || bit_of(l.cq)) {  // no local qubit: one factor
                                        mul(u0r, u0i, fr, fi);
                                        mul(u1r, u1i, fr, fi);
                                    }
                                }
                            }
                            pool.push_back((float)u0r);
                            pool.push_back((float)u0i);
                            pool.push_back((float)u1r);
                            pool.push_back((float)u1i);
                        }
                    }
                    table.push_back(d);
                }
            }
            k = e;
        }
        p.g1 = (int)table.size();
        // Follow the kernel's register layout through the pass.  The order above
        // groups operations into runs whose targets share a register group; a
        // run of at most kFsvLaneRun operations that can all be applied across
        // lanes in the current layout (targets on lane bits, no control in the
        // register group) is, and keeps the layout, since a layout change costs
        // about as much as five such operations; a longer run changes the layout.
        {
            int c = 2;
            int i = p.g0;
            while (i < p.g1) {
                FsvGate& d = table[i];
                if (d.kind != FSV_GENERAL || (d.tloc >> 2) == c) {
                    ++i;
                    continue;
                }
                const int k = d.tloc >> 2;
                int e = i, count = 0;
                bool lanes = true;
                for (; e < p.g1; ++e) {
                    const FsvGate& x = table[e];
                    if (x.kind != FSV_GENERAL) continue;
                    if ((x.tloc >> 2) != k) break;
                    ++count;
                    if (lane_bit(x.tloc, c) < 0 || (x.cloc >= 0 && (x.cloc >> 2) == c)) lanes = false;
                }
                if (lanes && count <= kFsvLaneRun) {
                    for (int x = i; x < e; ++x)
                        if (table[x].kind == FSV_GENERAL) table[x].width = lane_bit(table[x].tloc, c) + 1;
                } else {
                    c = k;
                }
                i = e;
            }
            // Leaf codes and planned actions.  A general record changes the
            // layout (tglob bit 1) when its target is outside the register
            // group and it is not applied across lanes; it and a lane operation
            // first apply the pending per-lane phase (bit 0) when a diagonal
            // that the kernel folds into it (target and control off the register
            // group) came since the last application.
            c = 2;
            bool dirty = false;
            double scale = 1.0, growth = 1.0;
            for (int x = p.g0; x < p.g1; ++x) {
                FsvGate& d = table[x];
                if (d.kind == FSV_TABLE) {
                    // A run of diagonal operations on local qubits, factored for
                    // register layout c: every factor reads at most two bits, so
                    //   D(r, t) = P(t) * F[r] * prod over set bits i of r of W_i(t)
                    // (r: register index, t: thread index).  A factor on thread
                    // bits only goes to P, on register bits only to F; one on
                    // register bit i and thread bit k, f(b_i, b_k), gives
                    // f(0, b_k) to P and f(1, b_k) / f(0, b_k) to W_i.  The
                    // kernel reads one entry of P and of each W_i per thread, and
                    // P joins the per-lane phase.
                    using cd = std::complex<double>;
                    std::vector<cd> F(16, 1.0), Pt(256, 1.0), Wt(4 * 256, 1.0);
                    int wmask = 0;
                    auto reg_of = [&](int lb) { return (lb >> 2) == c ? (lb & 3) : -1; };
                    auto tbit_of = [&](int lb) { return lb < 4 * c ? lb : lb - 4; };
                    for (size_t q : tab_ops[d.moff]) {
                        const LoweredGate& l = gs[q];
                        const int tb = local_bit(l.tq), cb = l.cq >= 0 ? local_bit(l.cq) : -1;
                        const cd d0(l.md[0], l.md[1]), d1(l.md[6], l.md[7]);
                        auto f = [&](int bc, int bt) { return (cb < 0 || bc) ? (bt ? d1 : d0) : cd(1.0); };
                        const int tr = reg_of(tb), cr = cb >= 0 ? reg_of(cb) : -1;
                        if (cb < 0) {
                            if (tr >= 0)
                                for (int r = 0; r < 16; ++r) F[r] *= f(1, (r >> tr) & 1);
                            else
                                for (int t = 0; t < 256; ++t) Pt[t] *= f(1, (t >> tbit_of(tb)) & 1);
                        } else if (tr >= 0 && cr >= 0) {
                            for (int r = 0; r < 16; ++r) F[r] *= f((r >> cr) & 1, (r >> tr) & 1);
                        } else if (tr < 0 && cr < 0) {
                            for (int t = 0; t < 256; ++t) Pt[t] *= f((t >> tbit_of(cb)) & 1, (t >> tbit_of(tb)) & 1);
                        } else {
                            const int i = tr >= 0 ? tr : cr, k = tr >= 0 ? tbit_of(cb) : tbit_of(tb);
                            for (int t = 0; t < 256; ++t) {
                                const int bk = (t >> k) & 1;
                                const cd a = tr >= 0 ? f(bk, 0) : f(0, bk), b = tr >= 0 ? f(bk, 1) : f(1, bk);
                                Pt[t] *= a;
                                Wt[i * 256 + t] *= b / a;
                            }
                            wmask |= 1 << i;
                        }
                    }
                    auto one = [](cd z) { return (float)z.real() == 1.f && (float)z.imag() == 0.f; };
                    int fmask = 0;
                    bool pt = false;
                    for (int r = 0; r < 16; ++r) fmask |= one(F[r]) ? 0 : 1 << r;
                    for (int t = 0; t < 256; ++t) pt = pt || !one(Pt[t]);
                    d.moff = (int)pool.size();
                    for (int r = 0; r < 16; ++r) {
                        pool.push_back((float)F[r].real());
                        pool.push_back((float)F[r].imag());
                    }
                    auto push256 = [&](const cd* v) {
                        for (int t = 0; t < 256; ++t) {
                            pool.push_back((float)v[t].real());
                            pool.push_back((float)v[t].imag());
                        }
                    };
                    if (pt) push256(Pt.data());
                    for (int i = 0; i < 4; ++i)
                        if ((wmask >> i) & 1) push256(Wt.data() + i * 256);
                    d.width = fmask;
                    d.tglob = pt ? 1 : 0;
                    d.cloc = wmask;
                    if (pt) dirty = true;
                } else if (d.kind == FSV_DIAG || d.kind == FSV_PHASE) {
                    const int tp = d.tloc >= 0 && (d.tloc >> 2) == c ? d.tloc & 3 : -1;
                    const int cp = d.cloc >= 0 && (d.cloc >> 2) == c ? d.cloc & 3 : -1;
                    const int ts = d.tloc >= 0 ? 1 : 0;
                    if (tp < 0 && cp < 0) {
                        dirty = true;
                        d.real = kDiagLP + ts;
                    } else if (tp < 0) {
                        d.real = kDiagCP + ts * 4 + cp;
                    } else {
                        // d0 is applied unless it is exactly 1 (for a grouped record: in
                        // every workgroup's entry of its table)
                        bool d0 = !(d.m[0] == 1.f && d.m[1] == 0.f);
                        if (d.kind == FSV_PHASE) {
                            d0 = false;
                            int off = d.moff;
                            for (int w = 0; w < d.width; ++w) {
                                const int entries = 1 << ((d.tglob >> (10 * w + 5)) & 15);
                                for (int e = 0; e < entries; ++e, off += 4)
                                    if (pool[off] != 1.f || pool[off + 1] != 0.f) d0 = true;
                            }
                        }
                        d.real = kDiagTP + (tp * 5 + cp + 1) * 2 + (d0 ? 1 : 0);
                    }
                } else if (d.kind == FSV_SWAP || d.kind == FSV_DENSE) {
                    dirty = false;  // always applied before these
                } else if (d.kind == FSV_GENERAL) {
                    const int form = d.real;
                    int flags = 0;
                    if (d.width > 0 || (d.tloc >> 2) != c) {
                        if (dirty) flags |= 1;
                        dirty = false;
                        if (d.width == 0) {
                            flags |= 2;
                            c = d.tloc >> 2;
                        }
                    }
                    d.tglob = flags;
                    d.moff = 0;
                    const int rb = d.tloc & 3;
                    // H, RX and RY take a scaled form when no control gates them
                    // (the factor then multiplies every amplitude), while the
                    // values' growth by the factors taken out stays below 2^32;
                    // RX / RY whose sine is the larger only on register bits
                    int kind = -1;
                    double a = 1.0, tt = 0.0;
                    if (d.cloc < 0 && d.cglob < 0) {
                        const float* m = d.m;
                        if (form == FSV_REAL) {
                            if (m[0] == m[2] && m[0] == m[4] && m[6] == -m[0]) {
                                kind = FSV_HADA;
                                a = m[0];
                                tt = 1.0;
                            } else if (m[0] == m[6] && m[4] == -m[2] && std::fabs(m[2]) <= std::fabs(m[0])) {
                                kind = FSV_ROTR;
                                a = m[0];
                                tt = -(double)m[2] / m[0];
                            } else if (m[0] == m[6] && m[4] == -m[2] && d.width == 0) {
                                kind = FSV_ROTR2;
                                a = m[4];
                                tt = (double)m[0] / m[4];
                            }
                        } else if (form == FSV_IMAGOFF) {
                            if (m[0] == m[6] && m[3] == m[5] && std::fabs(m[3]) <= std::fabs(m[0])) {
                                kind = FSV_ROTI;
                                a = m[0];
                                tt = -(double)m[3] / m[0];
                            } else if (m[0] == m[6] && m[3] == m[5] && d.width == 0) {
                                kind = FSV_ROTI2;
                                a = m[3];
                                tt = (double)m[0] / m[3];
                            }
                        }
                        if (kind >= 0 && (a == 0.0 || growth / std::fabs(a) > 4294967296.0)) kind = -1;
                    }
                    if (kind >= 0) {
                        growth /= std::fabs(a);
                        scale *= a;
                        d.real = d.width > 0 ? kLeafLaneScl + kind * 6 + (d.width - 1) : kLeafScl + kind * 4 + rb;
                        d.m[0] = kind >= FSV_ROTR2 ? (float)tt : (float)(1.0 + tt * tt);
                        d.m[1] = kind >= FSV_ROTR2 ? 0.f : (float)tt;
                    } else if (d.width > 0) {
                        const int fc = form == FSV_XSWAP ? (d.cloc < 0 ? 0 : 3) : form == FSV_REAL ? 1 : 2;
                        d.real = kLeafLane + fc * 6 + (d.width - 1);
                    } else if (d.cloc >= 0 && (d.cloc >> 2) == c) {
                        const int fc = form == FSV_XSWAP ? 0 : (form == FSV_REAL ? 1 : 2);
                        d.real = kLeafCP + fc * 16 + rb * 4 + (d.cloc & 3);
                    } else if (d.cloc >= 0) {
                        const int fc = form == FSV_XSWAP ? 0 : form == FSV_REAL ? 1 : form == FSV_IMAGOFF ? 2 : 3;
                        d.real = kLeafLC + fc * 4 + rb;
                    } else {
                        d.real = kLeafNC + form * 4 + rb;
                    }
                }
            }
            p.scale = (float)scale;
            p.tail = dirty ? 2 : (p.scale != 1.f ? 1 : 0);
        }
        p.wide = 0;
        for (int i = p.g0; i < p.g1; ++i)
            if (table[i].kind == FSV_DENSE) p.wide = 1;
        passes.push_back(p);
    }
}

}  // namespace
}  // namespace qsim

struct qsim_fsv_plan {
    int n = 0;
    int device = 0;
    int n_ops = 0;
    std::vector<qsim::FsvPass> passes;
    qsim::FsvGate* d_gates = nullptr;
    float* d_pool = nullptr;  // float32 matrices of the plan's custom operations
};

using namespace qsim;

namespace {

qsim_status fsv_check(int n_qubits, const qsim_gate* gates, int n_gates) {
    if (n_qubits < 1 || n_qubits > QSIM_FSV_MAX_QUBITS)
        return fail(QSIM_E_RANGE, "n_qubits %d outside 1..%d", n_qubits, QSIM_FSV_MAX_QUBITS);
    return check_gates(n_qubits, gates, n_gates);
}

}  // namespace

extern "C" {

qsim_status qsim_fsv_schedule(int n_qubits, const qsim_gate* gates, int n_gates, qsim_fsv_pass_info* passes,
                              int capacity, int* n_passes, int32_t* order) {
    qsim_status s = fsv_check(n_qubits, gates, n_gates);
    if (s != QSIM_OK) return s;
    if (n_passes == nullptr) return fail(QSIM_E_INVALID, "n_passes is NULL");
    if (capacity < 0 || (capacity > 0 && passes == nullptr)) return fail(QSIM_E_INVALID, "bad pass buffer");
    std::vector<LoweredGate> gs;
    lower(gates, n_gates, gs);
    std::vector<FsvPass> ps;
    std::vector<FsvGate> table;
    std::vector<float> pool;
    std::vector<int> exec;
    fsv_schedule(n_qubits, gs, ps, table, pool, &exec);
    *n_passes = (int)ps.size();
    if (order)
        for (size_t i = 0; i < exec.size(); ++i) order[i] = exec[i];
    if ((int)ps.size() > capacity && capacity > 0)
        return fail(QSIM_E_RANGE, "%d passes do not fit the buffer of %d", (int)ps.size(), capacity);
    for (int i = 0; i < (int)ps.size() && i < capacity; ++i) {
        qsim_fsv_pass_info& o = passes[i];
        o.low_qubits = ps[i].L;
        o.n_high = ps[i].nh;
        for (int h = 0; h < QSIM_FSV_MAX_HIGH; ++h) o.high[h] = h < ps[i].nh ? ps[i].high[h] : -1;
        o.first_op = ps[i].op0;
        o.n_ops = ps[i].op1 - ps[i].op0;
        o.permutation = ps[i].perm;
    }
    return ok();
}

qsim_status qsim_fsv_plan_create(qsim_ctx* ctx, int n_qubits, const qsim_gate* gates, int n_gates,
                                 qsim_fsv_plan** out) {
    if (out == nullptr) return fail(QSIM_E_INVALID, "out is NULL");
    *out = nullptr;
    qsim_status s = fsv_check(n_qubits, gates, n_gates);
    if (s != QSIM_OK) return s;
    s = check_ctx(ctx);
    if (s != QSIM_OK) return s;
    auto* plan = new qsim_fsv_plan();
    plan->n = n_qubits;
    plan->device = ctx->device;
    std::vector<LoweredGate> gs;
    lower(gates, n_gates, gs);
    std::vector<FsvGate> table;
    std::vector<float> pool;
    fsv_schedule(n_qubits, gs, plan->passes, table, pool);
    plan->n_ops = (int)gs.size();
    for (const FsvPass& p : plan->passes)
        if (p.perm && (p.pm.h < 4 || p.pm.h > 6)) {  // the permutation kernel's tiles are 2^10 to 2^12
            delete plan;
            return fail(QSIM_E_INVALID, "permutation pass with a %d-bit tile", 6 + p.pm.h);
        }
    if (!table.empty()) {
        DeviceGuard g(ctx->device);
        hipError_t e = g.err;
        if (e == hipSuccess) e = hipMalloc(&plan->d_gates, table.size() * sizeof(FsvGate));
        if (e == hipSuccess)
            e = hipMemcpy(plan->d_gates, table.data(), table.size() * sizeof(FsvGate), hipMemcpyHostToDevice);
        if (e == hipSuccess && !pool.empty()) e = hipMalloc(&plan->d_pool, pool.size() * sizeof(float));
        if (e == hipSuccess && !pool.empty())
            e = hipMemcpy(plan->d_pool, pool.data(), pool.size() * sizeof(float), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            if (plan->d_gates) (void)hipFree(plan->d_gates);
            if (plan->d_pool) (void)hipFree(plan->d_pool);
            delete plan;
            return e == hipErrorOutOfMemory ? fail(QSIM_E_OOM, "gate table: out of device memory")
                                            : device_fail("gate table upload", e);
        }
    }
    *out = plan;
    return ok();
}

qsim_status qsim_fsv_plan_info(const qsim_fsv_plan* plan, int* n_qubits, int* n_passes, int* n_ops) {
    if (plan == nullptr) return fail(QSIM_E_INVALID, "plan is NULL");
    if (n_qubits) *n_qubits = plan->n;
    if (n_passes) *n_passes = (int)plan->passes.size();
    if (n_ops) *n_ops = plan->n_ops;
    return ok();
}

qsim_status qsim_fsv_plan_destroy(qsim_fsv_plan* plan) {
    if (plan == nullptr) return ok();
    if (plan->d_gates || plan->d_pool) {
        DeviceGuard g(plan->device);
        if (plan->d_gates) (void)hipFree(plan->d_gates);
        if (plan->d_pool) (void)hipFree(plan->d_pool);
    }
    delete plan;
    return ok();
}

qsim_status qsim_fsv_run(qsim_ctx* ctx, const qsim_fsv_plan* plan, void* d_psi, void* stream) {
    if (plan == nullptr) return fail(QSIM_E_INVALID, "plan is NULL");
    if (d_psi == nullptr || !aligned(d_psi)) return fail(QSIM_E_INVALID, "d_psi is NULL or not 256-byte aligned");
    qsim_status s = check_ctx(ctx);
    if (s != QSIM_OK) return s;
    if (ctx->device != plan->device) return fail(QSIM_E_INVALID, "plan was made for device %d", plan->device);
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const int n = plan->n;
    const uint64_t N = (uint64_t)1 << n;
    float* re = static_cast<float*>(d_psi);
    float* im = re + N;
    const unsigned blocks = n > kFsvLocal ? 1u << (n - kFsvLocal) : 1u;
    for (const FsvPass& p : plan->passes) {
        hipError_t e = timed(ctx->prof, QSIM_PROFILE_FSV, hs, [&] {
            if (p.perm)
                hipLaunchKernelGGL(fsv_perm_kernel, dim3(1u << p.pm.ng), dim3(256), 0, hs, p.pm, re, im);
            else if (p.wide)
                hipLaunchKernelGGL(fsv_pass_kernel<true>, dim3(blocks), dim3(256), 0, hs, n, p, plan->d_gates,
                                   plan->d_pool, re, im);
            else
                hipLaunchKernelGGL(fsv_pass_kernel<false>, dim3(blocks), dim3(256), 0, hs, n, p, plan->d_gates,
                                   plan->d_pool, re, im);
            return hipGetLastError();
        });
        if (e != hipSuccess) return device_fail("full-state pass launch", e);
    }
    return ok();
}

qsim_status qsim_fsv_init_basis(qsim_ctx* ctx, int n_qubits, int64_t basis, void* d_psi, void* stream) {
    if (n_qubits < 1 || n_qubits > QSIM_FSV_MAX_QUBITS)
        return fail(QSIM_E_RANGE, "n_qubits %d outside 1..%d", n_qubits, QSIM_FSV_MAX_QUBITS);
    if (basis < 0 || basis >= ((int64_t)1 << n_qubits))
        return fail(QSIM_E_RANGE, "basis index %lld outside 0..2^%d-1", (long long)basis, n_qubits);
    if (d_psi == nullptr || !aligned(d_psi)) return fail(QSIM_E_INVALID, "d_psi is NULL or not 256-byte aligned");
    qsim_status s = check_ctx(ctx);
    if (s != QSIM_OK) return s;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const uint64_t n4 = ((uint64_t)2 << n_qubits) / 4;
    const uint64_t want = (n4 + 255) / 256;
    const unsigned blocks = (unsigned)std::min<uint64_t>(want, 65536);
    hipLaunchKernelGGL(fsv_basis_kernel, dim3(blocks), dim3(256), 0, hs, n4, (uint64_t)basis,
                       static_cast<float4*>(d_psi));
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : device_fail("basis-state launch", e);
}

size_t qsim_fsv_sample_workspace_bytes(int n_qubits) {
    if (n_qubits < 1 || n_qubits > QSIM_FSV_MAX_QUBITS) return 0;
    const uint64_t N = (uint64_t)1 << n_qubits;
    return (size_t)(((N + kSampleBlock - 1) / kSampleBlock) * sizeof(double));
}

qsim_status qsim_fsv_sample(qsim_ctx* ctx, int n_qubits, const void* d_psi, const double* d_uniform, int shots,
                            int64_t* d_out, void* d_ws, size_t ws_bytes, void* stream) {
    if (n_qubits < 1 || n_qubits > QSIM_FSV_MAX_QUBITS)
        return fail(QSIM_E_RANGE, "n_qubits %d outside 1..%d", n_qubits, QSIM_FSV_MAX_QUBITS);
    if (shots < 0) return fail(QSIM_E_INVALID, "negative shot count");
    if (d_psi == nullptr || !aligned(d_psi)) return fail(QSIM_E_INVALID, "d_psi is NULL or not 256-byte aligned");
    if (shots > 0 && (!d_uniform || !d_out || !aligned(d_uniform) || !aligned(d_out)))
        return fail(QSIM_E_INVALID, "d_uniform / d_out is NULL or not 256-byte aligned");
    const size_t need = qsim_fsv_sample_workspace_bytes(n_qubits);
    if (d_ws == nullptr || !aligned(d_ws)) return fail(QSIM_E_INVALID, "d_ws is NULL or not 256-byte aligned");
    if (ws_bytes < need) return fail(QSIM_E_RANGE, "workspace %zu bytes, need %zu", ws_bytes, need);
    qsim_status s = check_ctx(ctx);
    if (s != QSIM_OK) return s;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const uint64_t N = (uint64_t)1 << n_qubits;
    const uint64_t nb = (N + kSampleBlock - 1) / kSampleBlock;
    const float* re = static_cast<const float*>(d_psi);
    double* pre = static_cast<double*>(d_ws);
    hipLaunchKernelGGL(fsv_block_sums, dim3((unsigned)((nb + 3) / 4)), dim3(256), 0, hs, N, nb, re, re + N, pre);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(fsv_block_prefix, dim3(1), dim3(1024), 0, hs, nb, pre);
        e = hipGetLastError();
    }
    if (e == hipSuccess && shots > 0) {
        hipLaunchKernelGGL(fsv_sample_kernel, dim3((unsigned)((shots + 3) / 4)), dim3(256), 0, hs, N, nb, re, re + N,
                           pre, d_uniform, shots, d_out);
        e = hipGetLastError();
    }
    return e == hipSuccess ? ok() : device_fail("full-state sampling launch", e);
}

qsim_status qsim_fsv_norm2(qsim_ctx* ctx, int n_qubits, const void* d_psi, double* h_norm2, void* stream) {
    if (n_qubits < 1 || n_qubits > QSIM_FSV_MAX_QUBITS)
        return fail(QSIM_E_RANGE, "n_qubits %d outside 1..%d", n_qubits, QSIM_FSV_MAX_QUBITS);
    if (d_psi == nullptr || !aligned(d_psi)) return fail(QSIM_E_INVALID, "d_psi is NULL or not 256-byte aligned");
    if (h_norm2 == nullptr) return fail(QSIM_E_INVALID, "h_norm2 is NULL");
    qsim_status s = check_ctx(ctx);
    if (s != QSIM_OK) return s;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const uint64_t N = (uint64_t)1 << n_qubits;
    const float* re = static_cast<const float*>(d_psi);
    const int parts = (int)std::min<uint64_t>(kFsvNormBlocks, (N + 255) / 256);
    double* part = ctx->d_scratch + 8;
    double* res = ctx->d_scratch + 6;
    hipLaunchKernelGGL(fsv_norm_partial, dim3(parts), dim3(256), 0, hs, N, re, re + N, part);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(fsv_norm_final, dim3(1), dim3(256), 0, hs, parts, part, res);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(h_norm2, res, sizeof(double), hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    return e == hipSuccess ? ok() : device_fail("norm", e);
}

}  // extern "C"
