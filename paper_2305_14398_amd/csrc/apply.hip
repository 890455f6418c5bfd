// Stage 6 of the unitary method (Section 5.3; Algorithm 1, return value):
// psi = U . psi0, a complex64 matrix-vector product over the full row-major U
// (8 bytes of HBM reads per matrix entry, so the kernel is bandwidth bound),
// followed by the float64 normalisation sum |psi_i|^2 and, optionally, the
// measurement probabilities |psi_i|^2 / sum (Section 2.2, Eq. 1-3).
#include "common.h"

namespace qsim {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One wave per row; VEC = 4 uses 16-byte loads (N >= 256), VEC = 1 scalar loads.
// psi0 == nullptr stands for |0...0>, i.e. x[k] = (k == 0).
template <int VEC>
__global__ __launch_bounds__(256) void gemv_kernel(int n, const float* __restrict__ U, const float* __restrict__ psi0,
                                                   float* __restrict__ psi) {
    const int N = 1 << n;
    const size_t NN = (size_t)N * N;
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= N) return;
    const float* ur = U + (size_t)row * N;
    const float* ui = U + NN + (size_t)row * N;
    float sr = 0.f, si = 0.f;
    if (VEC == 4) {
        for (int k = lane * 4; k < N; k += 256) {
            const floatx4 a = *reinterpret_cast<const floatx4*>(ur + k);
            const floatx4 b = *reinterpret_cast<const floatx4*>(ui + k);
            floatx4 xr, xi;
            if (psi0) {
                xr = *reinterpret_cast<const floatx4*>(psi0 + k);
                xi = *reinterpret_cast<const floatx4*>(psi0 + N + k);
            } else {
                xr = floatx4{k == 0 ? 1.f : 0.f, 0.f, 0.f, 0.f};
                xi = floatx4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                sr = fmaf(a[c], xr[c], sr);
                sr = fmaf(-b[c], xi[c], sr);
                si = fmaf(a[c], xi[c], si);
                si = fmaf(b[c], xr[c], si);
            }
        }
    } else {
        for (int k = lane; k < N; k += 64) {
            const float a = ur[k], b = ui[k];
            const float xr = psi0 ? psi0[k] : (k == 0 ? 1.f : 0.f);
            const float xi = psi0 ? psi0[N + k] : 0.f;
            sr = fmaf(a, xr, sr);
            sr = fmaf(-b, xi, sr);
            si = fmaf(a, xi, si);
            si = fmaf(b, xr, si);
        }
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) {
        psi[row] = sr;
        psi[N + row] = si;
    }
}

// Single-block float64 reduction of sum |psi_i|^2 with a fixed summation order.
__global__ __launch_bounds__(1024) void norm_kernel(int n, const float* __restrict__ psi, double* __restrict__ out) {
    const int N = 1 << n;
    __shared__ double part[1024];
    double s = 0.0;
    for (int i = threadIdx.x; i < N; i += 1024) {
        const double re = psi[i], im = psi[N + i];
        s += re * re + im * im;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = part[0];
}

__global__ __launch_bounds__(256) void prob_kernel(int n, const float* __restrict__ psi, const double* __restrict__ norm2,
                                                   double* __restrict__ prob) {
    const int N = 1 << n;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const double re = psi[i], im = psi[N + i];
    prob[i] = (re * re + im * im) / norm2[0];
}

// Measurement (the paper's simulateAndCollapse, Section 5.2.3): the
// cumulative distribution of the float64 probabilities in a fixed order (each
// of 1024 threads sums a contiguous chunk, then an exclusive scan of the chunk
// totals), then one binary search per shot.
__global__ __launch_bounds__(1024) void cdf_kernel(int n, const double* __restrict__ prob, double* __restrict__ cdf) {
    const int N = 1 << n;
    const int chunk = (N + 1023) / 1024;
    const int lo = threadIdx.x * chunk;
    const int hi = min(lo + chunk, N);
    __shared__ double tot[1024];
    double s = 0.0;
    for (int i = lo; i < hi; ++i) s += prob[i];
    tot[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the chunk totals (fixed order)
    for (int off = 1; off < 1024; off <<= 1) {
        const double v = (int)threadIdx.x >= off ? tot[threadIdx.x - off] : 0.0;
        __syncthreads();
        tot[threadIdx.x] += v;
        __syncthreads();
    }
    double run = threadIdx.x ? tot[threadIdx.x - 1] : 0.0;
    for (int i = lo; i < hi; ++i) {
        run += prob[i];
        cdf[i] = run;
    }
}

// Shot k: the smallest index i with u_k * cdf[N-1] < cdf[i].
__global__ __launch_bounds__(256) void sample_kernel(int n, const double* __restrict__ cdf, const double* __restrict__ u,
                                                     int shots, int64_t* __restrict__ out) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= shots) return;
    const int N = 1 << n;
    const double target = u[k] * cdf[N - 1];
    int lo = 0, hi = N - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cdf[mid] > target)
            hi = mid;
        else
            lo = mid + 1;
    }
    out[k] = lo;
}

}  // namespace

hipError_t launch_sample(int n, const double* prob, const double* uniforms, int shots, int64_t* out, double* cdf,
                         hipStream_t stream) {
    hipLaunchKernelGGL(cdf_kernel, dim3(1), dim3(1024), 0, stream, n, prob, cdf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || shots == 0) return e;
    hipLaunchKernelGGL(sample_kernel, dim3((shots + 255) / 256), dim3(256), 0, stream, n, cdf, uniforms, shots, out);
    return hipGetLastError();
}

hipError_t launch_apply_state(int n, const float* U_row, const float* psi0, float* psi, double* prob, double* d_norm2,
                              hipStream_t stream) {
    const int N = 1 << n;
    const unsigned rows_blocks = (unsigned)((N + 3) / 4);
    if (N >= 256)
        hipLaunchKernelGGL(gemv_kernel<4>, dim3(rows_blocks), dim3(256), 0, stream, n, U_row, psi0, psi);
    else
        hipLaunchKernelGGL(gemv_kernel<1>, dim3(rows_blocks), dim3(256), 0, stream, n, U_row, psi0, psi);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(norm_kernel, dim3(1), dim3(1024), 0, stream, n, psi, d_norm2);
    e = hipGetLastError();
    if (e != hipSuccess || prob == nullptr) return e;
    hipLaunchKernelGGL(prob_kernel, dim3((N + 255) / 256), dim3(256), 0, stream, n, psi, d_norm2, prob);
    return hipGetLastError();
}

}  // namespace qsim
