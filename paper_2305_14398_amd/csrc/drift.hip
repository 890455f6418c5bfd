// Unitarity drift of a computed circuit unitary U (Section 2.3: a gate matrix
// is unitary iff its adjoint is its inverse, so any product of step operators
// is unitary and U^H U - I measures the rounding accumulated by the chain).
//
// G = U^H U is formed on float64 MFMA (v_mfma_f64_16x16x4f64) from the float32
// planes, and D = G - I is reduced on the fly to max |D_ij| and sum |D_ij|^2:
// no N x N float64 matrix is written.  G is Hermitian, so only tiles on or
// above the diagonal are computed; off-diagonal tiles count twice in the sum.
//   Re G_ij = sum_k Ur_ki Ur_kj + Ui_ki Ui_kj
//   Im G_ij = sum_k Ur_ki Ui_kj - Ui_ki Ur_kj
// taken in Gauss's three-product form (as the 3M chain products), with
// a = Ur_ki, b = Ui_ki, c = Ur_kj, d = Ui_kj:
//   K1 = sum (a - b) c,  K2 = sum a (d - c),  K3 = sum (-b)(c + d),
//   Re G = K1 - K3,      Im G = K1 + K2,
// three float64 MFMA products instead of four.  Each operand sum of two float32
// values is rounded once in float64 (relative error <= 2^-53; exact unless the
// exponents differ by more than 29), so the result differs from the
// four-product form by rounding of that order and by the accumulation order.
// Both operands are rows k of U, read as contiguous 16-byte vectors.
#include <mutex>

#include "common.h"

namespace qsim {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int DBK = 16;  // k rows per LDS tile

__device__ __forceinline__ void tile_of(int t, int T, int& tm, int& tn) {
    // t-th upper-triangular tile in row order: row tm holds T - tm tiles.
    tm = 0;
    while (t >= T - tm) {
        t -= T - tm;
        ++tm;
    }
    tn = tm + t;
}

// A workgroup of 2 x 2 waves computes a DT x DT tile of G, DT = 32 * BX; each
// wave owns BX x BX blocks of 16 x 16.  The tile edge sets the granularity of
// the work split: at 11 qubits 64-wide tiles give 528 tiles for 256 CUs (16 CUs
// take a third tile while the rest idle), 32-wide ones 2080.  The 32-wide
// tile waits on its operand loads, so it is held to 96 registers: five
// workgroups per CU (the compiler's own choice, 98 registers, allows four).
template <int BX>
__global__ __launch_bounds__(256, BX == 1 ? 5 : 3) void drift_mfma_kernel(int n, const float* __restrict__ U,
                                                            double* __restrict__ partials) {
    constexpr int DT = 32 * BX;
    constexpr int DLD = DT + 16;  // padded row stride (floats): the 4 k-rows of one MFMA land on distinct banks
    constexpr int LOADS = DBK * DT / 4;  // float4 per plane per operand and K-tile: 256 (BX 2) or 128 (BX 1)
    const int N = 1 << n;
    const size_t NN = (size_t)N * N;
    const int T = N / DT;
    const int ntiles = T * (T + 1) / 2;

    __shared__ float As[2][2][DBK][DLD];
    __shared__ float Bs[2][2][DBK][DLD];
    __shared__ double red_max[4], red_sum[4];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int l16 = lane & 15, kq = lane >> 4;
    // loader: float4 number f of a plane covers row f / (DT/4), columns 4*(f % (DT/4)); with 128 per operand,
    // threads 0..127 load A and 128..255 load B
    const int f = tid % LOADS;
    const int lrow = f / (DT / 4), lcol = (f % (DT / 4)) * 4;
    const bool load_a = LOADS == 256 || tid < 128, load_b = LOADS == 256 || tid >= 128;

    double tmax = 0.0, tsum = 0.0;

    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int tm, tn;
        tile_of(t, T, tm, tn);
        const int i0 = tm * DT, j0 = tn * DT;
        doublex4 acc[BX][BX][3];
#pragma unroll
        for (int x = 0; x < BX; ++x)
#pragma unroll
            for (int y = 0; y < BX; ++y)
#pragma unroll
                for (int z = 0; z < 3; ++z) acc[x][y][z] = doublex4{0.0, 0.0, 0.0, 0.0};

        floatx4 ra[2], rb[2];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            if (load_a) ra[p] = *reinterpret_cast<const floatx4*>(U + p * NN + (size_t)lrow * N + i0 + lcol);
            if (load_b) rb[p] = *reinterpret_cast<const floatx4*>(U + p * NN + (size_t)lrow * N + j0 + lcol);
        }
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            if (load_a) *reinterpret_cast<floatx4*>(&As[0][p][lrow][lcol]) = ra[p];
            if (load_b) *reinterpret_cast<floatx4*>(&Bs[0][p][lrow][lcol]) = rb[p];
        }
        __syncthreads();

        const int KT = N / DBK;
        for (int kt = 0; kt < KT; ++kt) {
            const int cur = kt & 1;
            if (kt + 1 < KT) {
                const size_t r = (size_t)((kt + 1) * DBK + lrow) * N;
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    if (load_a) ra[p] = *reinterpret_cast<const floatx4*>(U + p * NN + r + i0 + lcol);
                    if (load_b) rb[p] = *reinterpret_cast<const floatx4*>(U + p * NN + r + j0 + lcol);
                }
            }
#pragma unroll
            for (int s = 0; s < DBK / 4; ++s) {
                const int k = 4 * s + kq;
                double ar[BX], ai[BX], br[BX], bi[BX];
#pragma unroll
                for (int x = 0; x < BX; ++x) {
                    ar[x] = (double)As[cur][0][k][wm * 16 * BX + x * 16 + l16];
                    ai[x] = (double)As[cur][1][k][wm * 16 * BX + x * 16 + l16];
                    br[x] = (double)Bs[cur][0][k][wn * 16 * BX + x * 16 + l16];
                    bi[x] = (double)Bs[cur][1][k][wn * 16 * BX + x * 16 + l16];
                }
#pragma unroll
                for (int x = 0; x < BX; ++x) {
                    const double amb = ar[x] - ai[x];  // exact: float32 operands
#pragma unroll
                    for (int y = 0; y < BX; ++y) {
                        const double dmc = bi[y] - br[y], cpd = br[y] + bi[y];
                        acc[x][y][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(amb, br[y], acc[x][y][0], 0, 0, 0);
                        acc[x][y][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[x], dmc, acc[x][y][1], 0, 0, 0);
                        acc[x][y][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[x], cpd, acc[x][y][2], 0, 0, 0);
                    }
                }
            }
            if (kt + 1 < KT) {
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    if (load_a) *reinterpret_cast<floatx4*>(&As[cur ^ 1][p][lrow][lcol]) = ra[p];
                    if (load_b) *reinterpret_cast<floatx4*>(&Bs[cur ^ 1][p][lrow][lcol]) = rb[p];
                }
            }
            __syncthreads();
        }

        // 16x16 float64 accumulator layout: register r of lane l is row l/16 + 4*r, column l%16.
        const double w = (tm == tn) ? 1.0 : 2.0;
#pragma unroll
        for (int x = 0; x < BX; ++x) {
#pragma unroll
            for (int y = 0; y < BX; ++y) {
                const int j = j0 + wn * 16 * BX + y * 16 + l16;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = i0 + wm * 16 * BX + x * 16 + kq + 4 * r;
                    const double dr = (acc[x][y][0][r] - acc[x][y][2][r]) - (i == j ? 1.0 : 0.0);
                    const double di = acc[x][y][0][r] + acc[x][y][1][r];
                    const double m2 = dr * dr + di * di;
                    tmax = fmax(tmax, sqrt(m2));
                    tsum += w * m2;
                }
            }
        }
    }

#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        tmax = fmax(tmax, __shfl_xor(tmax, off, 64));
        tsum += __shfl_xor(tsum, off, 64);
    }
    if (lane == 0) {
        red_max[wave] = tmax;
        red_sum[wave] = tsum;
    }
    __syncthreads();
    if (tid == 0) {
        partials[2 * blockIdx.x] = fmax(fmax(red_max[0], red_max[1]), fmax(red_max[2], red_max[3]));
        partials[2 * blockIdx.x + 1] = (red_sum[0] + red_sum[1]) + (red_sum[2] + red_sum[3]);
    }
}

// N < 32: one block, one thread per entry of G, plain float64 arithmetic.
__global__ __launch_bounds__(256) void drift_small_kernel(int n, const float* __restrict__ U, double* __restrict__ partials) {
    const int N = 1 << n;
    const size_t NN = (size_t)N * N;
    __shared__ double smax[256], ssum[256];
    double tmax = 0.0, tsum = 0.0;
    for (int e = threadIdx.x; e < N * N; e += 256) {
        const int i = e / N, j = e % N;
        double gr = 0.0, gi = 0.0;
        for (int k = 0; k < N; ++k) {
            const double ar = U[(size_t)k * N + i], ai = U[NN + (size_t)k * N + i];
            const double br = U[(size_t)k * N + j], bi = U[NN + (size_t)k * N + j];
            gr += ar * br + ai * bi;
            gi += ar * bi - ai * br;
        }
        const double dr = gr - (i == j ? 1.0 : 0.0);
        const double m2 = dr * dr + gi * gi;
        tmax = fmax(tmax, sqrt(m2));
        tsum += m2;
    }
    smax[threadIdx.x] = tmax;
    ssum[threadIdx.x] = tsum;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
            ssum[threadIdx.x] += ssum[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[0] = smax[0];
        partials[1] = ssum[0];
    }
}

__global__ __launch_bounds__(256) void drift_final_kernel(int n, int count, const double* __restrict__ partials,
                                                          double* __restrict__ out) {
    __shared__ double smax[256], ssum[256];
    double tmax = 0.0, tsum = 0.0;
    for (int i = threadIdx.x; i < count; i += 256) {
        tmax = fmax(tmax, partials[2 * i]);
        tsum += partials[2 * i + 1];
    }
    smax[threadIdx.x] = tmax;
    ssum[threadIdx.x] = tsum;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
            ssum[threadIdx.x] += ssum[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = smax[0];
        out[1] = sqrt(ssum[0] / (double)(1 << n));
    }
}


// ---- probe variant: | U^H (U x) - x | for one fixed unit vector x ----
// x_j = exp(2 pi i frac(j * g)) / sqrt(N) with g the golden-ratio conjugate
// (unit-modulus entries, so |x| = 1).  y = U x and z = U^H y are accumulated in
// float64 (products of float32 entries are exact in float64); the cost is two
// passes over U instead of the 3 N^3 float64 flops of the full check.
constexpr double kGolden = 0.61803398874989484820;

__device__ __forceinline__ void probe_x(uint32_t j, double inv_sqrt_n, double& xr, double& xi) {
    double t = (double)j * kGolden;
    t -= floor(t);
    double sn, cs;
    sincospi(2.0 * t, &sn, &cs);
    xr = cs * inv_sqrt_n;
    xi = sn * inv_sqrt_n;
}

// y = U x, one wave per row.
__global__ __launch_bounds__(256) void probe_y_kernel(int n, const float* __restrict__ U, double* __restrict__ y) {
    const int N = 1 << n;
    const size_t NN = (size_t)N * N;
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= N) return;
    const double inv = rsqrt((double)N);
    double sr = 0.0, si = 0.0;
    for (int k = lane; k < N; k += 64) {
        const double ar = U[(size_t)row * N + k], ai = U[NN + (size_t)row * N + k];
        double xr, xi;
        probe_x((uint32_t)k, inv, xr, xi);
        sr += ar * xr - ai * xi;
        si += ar * xi + ai * xr;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        sr += __shfl_xor(sr, off, 64);
        si += __shfl_xor(si, off, 64);
    }
    if (lane == 0) {
        y[2 * row] = sr;
        y[2 * row + 1] = si;
    }
}

// Partial z_j over one chunk of rows: zpart[chunk][j] = sum_{i in chunk} conj(U_ij) y_i.
__global__ __launch_bounds__(256) void probe_z_kernel(int n, int rows_per_chunk, const float* __restrict__ U,
                                                      const double* __restrict__ y, double* __restrict__ zpart) {
    const int N = 1 << n;
    const size_t NN = (size_t)N * N;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    const int i0 = blockIdx.y * rows_per_chunk;
    double zr = 0.0, zi = 0.0;
    for (int i = i0; i < i0 + rows_per_chunk; ++i) {
        const double ur = U[(size_t)i * N + j], ui = U[NN + (size_t)i * N + j];
        const double yr = y[2 * i], yi = y[2 * i + 1];
        zr += ur * yr + ui * yi;
        zi += ur * yi - ui * yr;
    }
    zpart[2 * ((size_t)blockIdx.y * N + j)] = zr;
    zpart[2 * ((size_t)blockIdx.y * N + j) + 1] = zi;
}

// Sum the chunks in a fixed order, subtract x, reduce to max |d| and |d|_2.
__global__ __launch_bounds__(1024) void probe_final_kernel(int n, int chunks, const double* __restrict__ zpart,
                                                          double* __restrict__ out) {
    const int N = 1 << n;
    const double inv = rsqrt((double)N);
    __shared__ double smax[1024], ssum[1024];
    double tmax = 0.0, tsum = 0.0;
    for (int j = threadIdx.x; j < N; j += 1024) {
        double zr = 0.0, zi = 0.0;
        for (int c = 0; c < chunks; ++c) {
            zr += zpart[2 * ((size_t)c * N + j)];
            zi += zpart[2 * ((size_t)c * N + j) + 1];
        }
        double xr, xi;
        probe_x((uint32_t)j, inv, xr, xi);
        const double dr = zr - xr, di = zi - xi;
        const double m2 = dr * dr + di * di;
        tmax = fmax(tmax, sqrt(m2));
        tsum += m2;
    }
    smax[threadIdx.x] = tmax;
    ssum[threadIdx.x] = tsum;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
            ssum[threadIdx.x] += ssum[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = smax[0];
        out[1] = sqrt(ssum[0]);
    }
}

}  // namespace

hipError_t launch_drift_probe(int n, const float* U_row, double* scratch, double* d_out, hipStream_t stream) {
    const int N = 1 << n;
    double* y = scratch;
    double* zpart = scratch + 2 * (size_t)N;
    // chunks * N <= kProbeChunkEntries keeps the partials inside the scratch.
    int chunks = kProbeChunkEntries / N;
    if (chunks > N) chunks = N;
    if (chunks < 1) chunks = 1;
    const int rows = N / chunks;
    hipLaunchKernelGGL(probe_y_kernel, dim3((N + 3) / 4), dim3(256), 0, stream, n, U_row, y);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(probe_z_kernel, dim3((N + 255) / 256, chunks), dim3(256), 0, stream, n, rows, U_row, y, zpart);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(probe_final_kernel, dim3(1), dim3(1024), 0, stream, n, chunks, zpart, d_out);
    return hipGetLastError();
}

// Partial sums of the allocation-free entry point (qsim_unitarity_drift_noalloc):
// one (max, sum of squares) pair per workgroup of the persistent drift grid,
// whose size launch_drift caps at kDriftMaxPartials: 32 KiB per device, held
// until the process ends.  Every launch writes all the pairs it later reads, so
// nothing needs clearing between calls; calls that overlap on one device race
// on it.  In host code `scratch` is only a handle: its device address comes
// from hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) double scratch[2 * kDriftMaxPartials];

constexpr int kMaxDevices = 64;

hipError_t drift_static_scratch(double** out, size_t* bytes) {
    static std::mutex mu;
    static double* ptr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (ptr[dev] == nullptr) {
        double* p = nullptr;
        e = hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (p == nullptr) return hipErrorInvalidSymbol;
        ptr[dev] = p;
    }
    *out = ptr[dev];
    *bytes = sizeof(scratch);
    return hipSuccess;
}

hipError_t launch_drift(int n, const float* U_row, double* partials, int max_partials, double* d_out,
                        hipStream_t stream) {
    const int N = 1 << n;
    int count = 1;
    if (N < 32) {
        hipLaunchKernelGGL(drift_small_kernel, dim3(1), dim3(256), 0, stream, n, U_row, partials);
    } else {
        // 64-wide tiles once there are enough of them to spread evenly over the CUs (n >= 12: 2080 tiles)
        const bool wide = n >= 12;
        const int T = N / (wide ? 64 : 32);
        const int ntiles = T * (T + 1) / 2;
        count = ntiles < max_partials ? ntiles : max_partials;
        if (wide)
            hipLaunchKernelGGL(drift_mfma_kernel<2>, dim3(count), dim3(256), 0, stream, n, U_row, partials);
        else
            hipLaunchKernelGGL(drift_mfma_kernel<1>, dim3(count), dim3(256), 0, stream, n, U_row, partials);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(drift_final_kernel, dim3(1), dim3(256), 0, stream, n, count, partials, d_out);
    return hipGetLastError();
}

}  // namespace qsim
