// Per-entry form of stage 4 of the unitary method (Section 5.3; Algorithm 2;
// Eq. 9s1), shared by the single-step kernel (expand.hip) and the grouped
// expansion kernel (grouped.hip).
//
// The Kronecker product of the step's gates with identities on idle qubits has
// the per-entry form (little-endian, r_q = bit q of the row index r, s_q of
// the column index s):
//   idle qubit q            : [r_q == s_q]
//   one-qubit gate G on q   : G[r_q][s_q]
//   controlled-U (c -> t)   : [r_c == s_c] * (s_c == 0 ? [r_t == s_t] : U[r_t][s_t])   (Eq. 7)
//   SWAP(a, b)              : [r_a == s_b] * [r_b == s_a]
//   custom M on a..a+m-1    : M[r_{a..a+m-1}][s_{a..a+m-1}]   (a registered unitary, Section 5.2.2)
// and the entry is the product of these factors.  Every entry is computed in
// float64 and rounded once to the output format, so the kernel is a streaming
// writer: 8 bytes of HBM traffic per entry, and no reads beyond the (cached)
// matrices of custom operations.
#pragma once

#include "common.h"

namespace qsim {

__device__ __forceinline__ double sel4(int idx, double a, double b, double c, double d) {
    return idx == 0 ? a : idx == 1 ? b : idx == 2 ? c : d;
}

// Multiply the running entry (pr, pi) by gate G's factor at (r, s), or set
// `zero` where the factor is a structural zero.  Reads of G use a wave-uniform
// gate index, so they stay scalar loads from the kernel argument segment; the
// per-lane choice of matrix entry is a select.
__device__ __forceinline__ void gate_factor(const DevGate& G, uint32_t r, uint32_t s, double& pr, double& pi,
                                            bool& zero) {
    const int type = G.type;
    const int q0 = G.q0, q1 = G.q1;
    if (type == GATE_CUSTOM) {
        const uint32_t mask = (1u << q1) - 1u;
        const uint32_t e = (((r >> q0) & mask) << q1) | ((s >> q0) & mask);
        const double ar = G.ext[2 * e], ai = G.ext[2 * e + 1];
        const double t = pr * ar - pi * ai;
        pi = pr * ai + pi * ar;
        pr = t;
        return;
    }
    int idx = 0;
    bool use = true;
    if (type == GATE_ONE) {
        idx = (((r >> q0) & 1u) << 1) | ((s >> q0) & 1u);
    } else if (type == GATE_CTRL) {
        const uint32_t rc = (r >> q0) & 1u, sc = (s >> q0) & 1u;
        const uint32_t rt = (r >> q1) & 1u, stt = (s >> q1) & 1u;
        zero |= rc != sc;
        if (sc == 0) {
            zero |= rt != stt;
            use = false;
        }
        idx = (int)((rt << 1) | stt);
    } else {  // GATE_SWAP
        zero |= ((r >> q0) & 1u) != ((s >> q1) & 1u);
        zero |= ((r >> q1) & 1u) != ((s >> q0) & 1u);
        use = false;
    }
    if (use) {
        const double* m = G.m;
        const double ar = sel4(idx, m[0], m[2], m[4], m[6]);
        const double ai = sel4(idx, m[1], m[3], m[5], m[7]);
        const double t = pr * ar - pi * ai;
        pi = pr * ai + pi * ar;
        pr = t;
    }
}

// Entry (r, s) of the step operator in float64: the gate factors multiplied
// in the descriptor's order, starting from 1.
__device__ __forceinline__ void step_entry(const DevStep& st, uint32_t r, uint32_t s, double& out_re,
                                           double& out_im) {
    double pr = 1.0, pi = 0.0;
    bool zero = ((r ^ s) & st.idle_mask) != 0;
    if (zero) {  // most entries of a sparse step: no gate factor is needed
        out_re = 0.0;
        out_im = 0.0;
        return;
    }
    for (int g = 0; g < st.n_gates; ++g) gate_factor(st.g[g], r, s, pr, pi, zero);
    out_re = zero ? 0.0 : pr;
    out_im = zero ? 0.0 : pi;
}

// Entries (r + c, s), c = 0..3, for r a multiple of 4 (ALONG_S: (r, s + c),
// s a multiple of 4): the same values as step_entry, with the descriptor's
// leading gates (those whose spans leave out qubits 0 and 1, so whose factors
// do not depend on c) multiplied once.
template <bool ALONG_S = false>
__device__ __forceinline__ void step_entries4(const DevStep& st, uint32_t r, uint32_t s, double (&out_re)[4],
                                              double (&out_im)[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) out_re[c] = out_im[c] = 0.0;
    bool zhi = ((r ^ s) & st.idle_mask & ~3u) != 0;
    if (!zhi) {  // otherwise all four entries are structural zeros (most of a sparse step)
        double pr = 1.0, pi = 0.0;
        for (int g = 0; g < st.n_prefix; ++g) gate_factor(st.g[g], r, s, pr, pi, zhi);
        const uint32_t low = (ALONG_S ? r : s) & 3u;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double qr = pr, qi = pi;
            bool zero = zhi || ((((uint32_t)c ^ low) & st.idle_mask & 3u) != 0);
            const uint32_t rc = ALONG_S ? r : r + c, sc = ALONG_S ? s + c : s;
            if (!zero)
                for (int g = st.n_prefix; g < st.n_gates; ++g) gate_factor(st.g[g], rc, sc, qr, qi, zero);
            out_re[c] = zero ? 0.0 : qr;
            out_im[c] = zero ? 0.0 : qi;
        }
    }
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Split a float64 value into 16-bit hi + lo with value ~= hi + lo * 2^-shift.
template <int FMT>
__device__ __forceinline__ void split16(double v, uint16_t& hi, uint16_t& lo) {
    if (fmt_elem(FMT) == FMT_BF16) {
        hi = bf16_rne((float)v);
        lo = bf16_rne((float)(v - (double)bf16_to_f32(hi)));
    } else {
        _Float16 h = (_Float16)(float)v;
        _Float16 l = (_Float16)(float)((v - (double)(float)h) * (double)(1 << QSIM_LO_SCALE_LOG2));
        hi = __builtin_bit_cast(uint16_t, h);
        lo = __builtin_bit_cast(uint16_t, l);
    }
}

// Work item `it` of the three-product split formats from n = 6 on, whose
// operands are fragment-blocked (32 x 16 blocks of six 1 KiB fragments, see
// tile_split_gauss.h): item it writes 8 bytes per plane at element 4 it of the
// block order, i.e. storage row a and storage columns b .. b+3, so consecutive
// items write consecutive bytes.
__device__ __forceinline__ void fb_item(uint64_t it, int n, uint32_t& a, uint32_t& b, uint64_t& base) {
    const uint64_t blk = it >> 7;                 // 128 items per 32 x 16 block
    const uint32_t w = (uint32_t)(it & 127);
    const uint32_t fl = w >> 1;                   // fragment lane
    const uint64_t kblocks = (1ull << n) >> 4;
    a = (uint32_t)((blk / kblocks) * 32 + (fl & 31));
    b = (uint32_t)((blk % kblocks) * 16 + (fl >> 5) * 8 + (w & 1) * 4);
    base = blk * 6 * 512 + fl * 8 + (w & 1) * 4;  // element index in plane 0; planes 512 apart
}

__device__ __forceinline__ uint2 pack4(const uint16_t* h) {
    return make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16));
}

// Four entries in the six-plane three-product format: re, im and the float32
// sum of the rounded parts (what the products' epilogue splits), each split
// into hi + lo; element `o` of plane 0, planes `ps` elements apart.
template <int FMT>
__device__ __forceinline__ void store_planes6(const double (&vr)[4], const double (&vi)[4], uint16_t* o, uint64_t e,
                                              uint64_t ps) {
    uint16_t h[6][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        split16<FMT>(vr[c], h[0][c], h[1][c]);
        split16<FMT>(vi[c], h[2][c], h[3][c]);
        split16<FMT>((double)((float)vr[c] + (float)vi[c]), h[4][c], h[5][c]);
    }
#pragma unroll
    for (int p = 0; p < 6; ++p) *reinterpret_cast<uint2*>(o + p * ps + e) = pack4(h[p]);
}

// Entries e0 .. e0+3 of the storage order (row-major storage index; logical
// (r, s) = (a, b) for row-major output and (b, a) for column-major), computed
// and stored in the output format.  Fragment-blocked formats (three-product
// split, n >= 6) take e0 / 4 as a block-order item instead (fb_item).
template <int FMT>
__device__ __forceinline__ void expand_four(const DevStep& st, int n, int layout_col, void* out, uint64_t e0) {
    const uint64_t N = 1ull << n;
    const uint64_t NN = N * N;
    double vr[4], vi[4];
    if constexpr (fmt_gauss(FMT)) {
        if (n >= 6) {
            uint32_t a, b;
            uint64_t base;
            fb_item(e0 >> 2, n, a, b, base);
            if (layout_col)
                step_entries4<false>(st, b, a, vr, vi);
            else
                step_entries4<true>(st, a, b, vr, vi);
            store_planes6<FMT>(vr, vi, reinterpret_cast<uint16_t*>(out), base, 512);
            return;
        }
    }
    if (n >= 2) {  // the four entries share a storage row
        const uint32_t a = (uint32_t)(e0 >> n);
        const uint32_t b = (uint32_t)(e0 & (N - 1));
        if (layout_col)
            step_entries4<false>(st, b, a, vr, vi);
        else
            step_entries4<true>(st, a, b, vr, vi);
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint32_t a = (uint32_t)((e0 + c) >> n);
            const uint32_t b = (uint32_t)((e0 + c) & (N - 1));
            const uint32_t r = layout_col ? b : a;
            const uint32_t s = layout_col ? a : b;
            step_entry(st, r, s, vr[c], vi[c]);
        }
    }
    if (FMT == FMT_F32) {
        float* o = reinterpret_cast<float*>(out);
        *reinterpret_cast<float4*>(o + e0) = make_float4((float)vr[0], (float)vr[1], (float)vr[2], (float)vr[3]);
        *reinterpret_cast<float4*>(o + NN + e0) = make_float4((float)vi[0], (float)vi[1], (float)vi[2], (float)vi[3]);
    } else if constexpr (fmt_gauss(FMT)) {
        store_planes6<FMT>(vr, vi, reinterpret_cast<uint16_t*>(out), e0, NN);
    } else {
        uint16_t rh[4], rl[4], ih[4], il[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            split16<FMT>(vr[c], rh[c], rl[c]);
            split16<FMT>(vi[c], ih[c], il[c]);
        }
        uint16_t* o = reinterpret_cast<uint16_t*>(out);
        *reinterpret_cast<uint2*>(o + e0) = pack4(rh);
        *reinterpret_cast<uint2*>(o + NN + e0) = pack4(rl);
        *reinterpret_cast<uint2*>(o + 2 * NN + e0) = pack4(ih);
        *reinterpret_cast<uint2*>(o + 3 * NN + e0) = pack4(il);
    }
}

}  // namespace qsim
