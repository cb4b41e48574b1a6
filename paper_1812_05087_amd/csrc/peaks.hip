// Measured device peaks, the denominators reported beside the vendor
// figures: an FP64 FMA loop on the vector ALUs, an FP64 MFMA loop and a
// device-to-device stream copy.  Each kernel keeps its operands in
// registers and stores one value per thread at the end (so the work is not
// removed); the copy reads and writes a buffer it owns.
#include "internal.h"

namespace fmddm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int PT = 256, PCHAIN = 8;

// 8 independent FMA chains per thread, `iters` rounds: 16 flops per round
__global__ __launch_bounds__(PT) void k_fma_loop(int iters, double a, double b, double *__restrict__ out)
{
    double x[PCHAIN];
#pragma unroll
    for (int c = 0; c < PCHAIN; ++c) x[c] = threadIdx.x * 1e-3 + c;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < PCHAIN; ++c) x[c] = fma(x[c], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < PCHAIN; ++c) s += x[c];
    out[blockIdx.x * PT + threadIdx.x] = s;
}

// MACC independent 16x16x4 FP64 MFMA accumulators per wave, `iters`
// rounds: MACC x 2048 flops per wave and round
constexpr int MACC = 8;

__global__ __launch_bounds__(PT) void k_mfma_loop(int iters, double a, double b, double *__restrict__ out)
{
    d4 acc[MACC];
#pragma unroll
    for (int c = 0; c < MACC; ++c) acc[c] = d4{0.0, 0.0, 0.0, 0.0};
    double x = a + threadIdx.x * 1e-6, y = b - threadIdx.x * 1e-6;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < MACC; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc[c], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < MACC; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[blockIdx.x * PT + threadIdx.x] = s;
}

// grid-stride copy with CU loads in flight per thread (n a multiple of the
// grid's stride times CU is not required: the tail is guarded)
constexpr int CU = 4;

__global__ __launch_bounds__(PT) void k_copy(int64_t n, const double2 *__restrict__ src, double2 *__restrict__ dst)
{
    const int64_t stride = (int64_t)gridDim.x * PT;
    for (int64_t i = (int64_t)blockIdx.x * PT + threadIdx.x; i < n; i += CU * stride) {
        double2 v[CU];
#pragma unroll
        for (int u = 0; u < CU; ++u)
            if (i + u * stride < n) v[u] = src[i + u * stride];
#pragma unroll
        for (int u = 0; u < CU; ++u)
            if (i + u * stride < n) dst[i + u * stride] = v[u];
    }
}

}  // namespace
}  // namespace fmddm

using namespace fmddm;

extern "C" fmddm_status fmddm_measure_peaks(fmddm_peaks *out)
{
    if (!out) return FMDDM_EINVAL;
    try {
        hipStream_t s = nullptr;
        FM_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        struct Guard {
            hipStream_t s;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            ~Guard()
            {
                if (e0) (void)hipEventDestroy(e0);
                if (e1) (void)hipEventDestroy(e1);
                (void)hipStreamDestroy(s);
            }
        } g{s};
        FM_HIP(hipEventCreate(&g.e0));
        FM_HIP(hipEventCreate(&g.e1));
        int dev = 0, ncu = 0;
        FM_HIP(hipGetDevice(&dev));
        FM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        const int nblk = ncu * 16;  // 16 blocks (64 waves) per CU
        DBuf<double> sink;
        sink.alloc((size_t)nblk * PT);
        auto timed = [&](auto launch) {
            launch();  // warm-up
            FM_HIP(hipEventRecord(g.e0, s));
            launch();
            FM_HIP(hipEventRecord(g.e1, s));
            FM_HIP(hipEventSynchronize(g.e1));
            float ms = 0.f;
            FM_HIP(hipEventElapsedTime(&ms, g.e0, g.e1));
            return (double)ms * 1e-3;
        };
        const int it_fma = 4096, it_mfma = 2048;
        double t = timed([&] {
            hipLaunchKernelGGL(k_fma_loop, dim3(nblk), dim3(PT), 0, s, it_fma, 0.999999, 1e-7, sink.p);
            FM_CHECK_LAUNCH();
        });
        out->fp64_vector_tflops = (double)nblk * PT * it_fma * PCHAIN * 2.0 / t * 1e-12;
        t = timed([&] {
            hipLaunchKernelGGL(k_mfma_loop, dim3(nblk), dim3(PT), 0, s, it_mfma, 0.999999, 1e-7, sink.p);
            FM_CHECK_LAUNCH();
        });
        out->fp64_mfma_tflops = (double)nblk * (PT / 64) * it_mfma * MACC * 2048.0 / t * 1e-12;
        const int64_t bytes = (int64_t)1 << 30;
        DBuf<double> a, b;
        a.alloc(bytes / 8);
        b.alloc(bytes / 8);
        FM_HIP(hipMemsetAsync(a.p, 0, bytes, s));
        const int64_t n2 = bytes / 16;
        t = timed([&] {
            hipLaunchKernelGGL(k_copy, dim3(ncu * 32), dim3(PT), 0, s, n2, (const double2 *)a.p, (double2 *)b.p);
            FM_CHECK_LAUNCH();
        });
        out->copy_gbps = 2.0 * (double)bytes / t * 1e-9;
        FM_HIP(hipStreamSynchronize(s));
        return FMDDM_OK;
    } catch (const Error &e) {
        return e.code;
    } catch (...) {
        return FMDDM_EDEVICE;
    }
}
