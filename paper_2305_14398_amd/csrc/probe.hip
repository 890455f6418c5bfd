// Throughput probes of the device the roofline fractions are quoted against:
// MFMA issue rate per operand type (independent accumulator chains, so no
// dependency stalls) and HBM streaming copy bandwidth.  Vendor peaks are
// nominal; these give what one MI355X sustains for the instruction mixes the
// chain products use, with operands that toggle (random bits) or stay
// constant, since the clock the chip holds depends on switching power.
#include "host.h"

namespace qsim {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// independent accumulators per wave: four for the 32x32 shapes; the 16x16x4
// float64 MFMA needs eight to keep its pipeline full
template <int KIND>
constexpr int chains() { return KIND == 3 ? 8 : 4; }
constexpr int kProbeBlocks = 2048;
constexpr int kProbeThreads = 256;

__device__ __forceinline__ uint32_t mix(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Operand bits: pseudo-random per lane and chain (kept small in magnitude so
// accumulators stay finite), or the constant 1/64.
__device__ __forceinline__ float probe_f32(bool rnd, uint32_t seed) {
    if (!rnd) return 1.0f / 64.0f;
    return __uint_as_float(0x3c000000u | (mix(seed) & 0x007fffffu));  // [2^-7, 2^-6)
}

template <int KIND>
__global__ __launch_bounds__(kProbeThreads) void mfma_probe_kernel(int iters, int rnd, float* __restrict__ sink) {
    constexpr int kChains = chains<KIND>();
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    float total = 0.f;
    if constexpr (KIND == 0) {  // v_mfma_f32_32x32x2f32
        float a[kChains], b[kChains];
        floatx16 acc[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            a[c] = probe_f32(rnd, gid * 8 + c);
            b[c] = probe_f32(rnd, gid * 8 + 4 + c);
            for (int e = 0; e < 16; ++e) acc[c][e] = 0.f;
        }
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[c], b[c], acc[c], 0, 0, 0);
#pragma unroll
        for (int c = 0; c < kChains; ++c) total += acc[c][c];
    } else if constexpr (KIND == 1 || KIND == 2) {  // v_mfma_f32_32x32x16_{bf16,f16}
        u32x4 a[kChains], b[kChains];
        floatx16 acc[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            for (int q = 0; q < 4; ++q) {
                // two 16-bit values per word: a random mantissa under a fixed small exponent
                const uint32_t ra = mix(gid * 64 + c * 8 + q), rb = mix(gid * 64 + c * 8 + 4 + q);
                const uint32_t one = KIND == 1 ? 0x3c003c00u : 0x24002400u;  // bf16 2^-7 / fp16 2^-6
                const uint32_t mant = KIND == 1 ? 0x007f007fu : 0x03ff03ffu;
                a[c][q] = rnd ? (one | (ra & mant)) : one;
                b[c][q] = rnd ? (one | (rb & mant)) : one;
            }
            for (int e = 0; e < 16; ++e) acc[c][e] = 0.f;
        }
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                if constexpr (KIND == 1)
                    acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[c]),
                                                                     __builtin_bit_cast(bf16x8, b[c]), acc[c], 0, 0, 0);
                else
                    acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(halfx8, a[c]),
                                                                    __builtin_bit_cast(halfx8, b[c]), acc[c], 0, 0, 0);
            }
#pragma unroll
        for (int c = 0; c < kChains; ++c) total += acc[c][c];
    } else {  // v_mfma_f64_16x16x4f64
        double a[kChains], b[kChains];
        doublex4 acc[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            a[c] = (double)probe_f32(rnd, gid * 16 + c);
            b[c] = (double)probe_f32(rnd, gid * 16 + 8 + c);
            for (int e = 0; e < 4; ++e) acc[c][e] = 0.0;
        }
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c], b[c], acc[c], 0, 0, 0);
#pragma unroll
        for (int c = 0; c < kChains; ++c) total += (float)acc[c][c & 3];
    }
    if (threadIdx.x == 0) sink[blockIdx.x] = total;  // keeps the work live
}

// Streaming copy, 16 bytes per load and store, grid-stride; each thread has
// up to four loads in flight before it stores (non-temporal: the copy streams
// through and should not displace cached data; measured fastest with 128
// workgroups per CU).
__global__ __launch_bounds__(256) void copy_probe_kernel(const floatx4* __restrict__ src, floatx4* __restrict__ dst,
                                                         size_t n16) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += 4 * stride) {
        floatx4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i + u * stride < n16) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i + u * stride < n16) __builtin_nontemporal_store(v[u], dst + i + u * stride);
    }
}

// flops of one MFMA of each probe kind
constexpr double kMfmaFlops[4] = {2.0 * 32 * 32 * 2, 2.0 * 32 * 32 * 16, 2.0 * 32 * 32 * 16, 2.0 * 16 * 16 * 4};

template <class Launch>
hipError_t time_ms(hipStream_t s, int reps, Launch&& launch, float* ms) {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = launch();  // warm-up
    if (e == hipSuccess) e = hipEventRecord(a, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e == hipSuccess) *ms /= (float)reps;
    return e;
}

}  // namespace
}  // namespace qsim

using namespace qsim;

extern "C" {

qsim_status qsim_probe_mfma(qsim_ctx* ctx, int kind, int random_operands, double* tflops_out) {
    if (kind < 0 || kind > 3) return fail(QSIM_E_INVALID, "unknown probe kind %d", kind);
    if (tflops_out == nullptr) return fail(QSIM_E_INVALID, "tflops_out is NULL");
    qsim_status s = check_ctx(ctx);
    if (s != QSIM_OK) return s;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    const int iters = kind == 0 ? 512 : kind == 3 ? 512 : 1024;
    const int rnd = random_operands ? 1 : 0;
    // one float per workgroup, in the context's scratch (far larger than kProbeBlocks floats)
    float* sink = reinterpret_cast<float*>(ctx->d_scratch);
    static_assert(kProbeBlocks <= 2 * (int)kScratchDoubles, "probe sink exceeds the context scratch");
    float ms = 0.f;
    if (e == hipSuccess) {
        e = time_ms(st, 3, [&] {
            switch (kind) {
                case 0: hipLaunchKernelGGL(mfma_probe_kernel<0>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, st, iters, rnd, sink); break;
                case 1: hipLaunchKernelGGL(mfma_probe_kernel<1>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, st, iters, rnd, sink); break;
                case 2: hipLaunchKernelGGL(mfma_probe_kernel<2>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, st, iters, rnd, sink); break;
                default: hipLaunchKernelGGL(mfma_probe_kernel<3>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, st, iters, rnd, sink); break;
            }
            return hipGetLastError();
        }, &ms);
    }
    if (st) (void)hipStreamDestroy(st);
    if (e != hipSuccess) return device_fail("mfma probe", e);
    const double waves = (double)kProbeBlocks * kProbeThreads / 64.0;
    const int nchains = kind == 3 ? chains<3>() : chains<0>();
    *tflops_out = waves * iters * nchains * kMfmaFlops[kind] / (ms * 1e-3) / 1e12;
    return ok();
}

qsim_status qsim_probe_copy(qsim_ctx* ctx, const void* d_src, void* d_dst, size_t bytes, double* gbs_out) {
    if (!d_src || !d_dst || !aligned(d_src) || !aligned(d_dst)) return fail(QSIM_E_INVALID, "NULL or unaligned buffer");
    if (bytes < (64u << 20) || (bytes & ((64u << 20) - 1)))
        return fail(QSIM_E_RANGE, "bytes must be a multiple of 64 MiB");
    if (gbs_out == nullptr) return fail(QSIM_E_INVALID, "gbs_out is NULL");
    const char* a = static_cast<const char*>(d_src);
    const char* b = static_cast<const char*>(d_dst);
    if (a < b + bytes && b < a + bytes) return fail(QSIM_E_INVALID, "source and destination overlap");
    qsim_status s = check_ctx(ctx);
    if (s != QSIM_OK) return s;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return device_fail("hipSetDevice", g.err);
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    const size_t n16 = bytes / 16;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus <= 0)
        cus = 256;
    float ms = 0.f;
    if (e == hipSuccess) {
        e = time_ms(st, 10, [&] {
            hipLaunchKernelGGL(copy_probe_kernel, dim3(cus * 128), dim3(256), 0, st,
                               static_cast<const floatx4*>(d_src), static_cast<floatx4*>(d_dst), n16);
            return hipGetLastError();
        }, &ms);
    }
    if (st) (void)hipStreamDestroy(st);
    if (e != hipSuccess) return device_fail("copy probe", e);
    *gbs_out = 2.0 * (double)bytes / (ms * 1e-3) / 1e9;
    return ok();
}

}  // extern "C"
