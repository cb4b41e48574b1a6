// Exact products of the single-step elastic influence operator
// (eqs. 2.3-2.5 with constant elements): on the fly ("direct") and with the
// stored dense matrix.  These are the comparison paths for the FMM and the
// paper's conventional method.
#include "elem.h"
#include "internal.h"

namespace fmddm {
namespace {

constexpr int DT = 256, DTPT = 8, DTGT = DT / DTPT, DTILE = 256;

// One block per 32 receivers, 8 lanes per receiver; sources staged in LDS.
// Each lane sums a fixed subset of sources in order, lanes are combined in
// a fixed order: the result does not depend on the launch.
__global__ __launch_bounds__(DT) void k_direct(int n, const double *__restrict__ cx,
                                               const double *__restrict__ cy,
                                               const double *__restrict__ cb,
                                               const double *__restrict__ sb,
                                               const double *__restrict__ a,
                                               const double *__restrict__ D, double gc,
                                               double *__restrict__ out)
{
    __shared__ double s_cx[DTILE], s_cy[DTILE], s_cb[DTILE], s_sb[DTILE], s_c2[DTILE], s_s2[DTILE], s_a[DTILE],
        s_ds[DTILE], s_dn[DTILE];
    int tid = threadIdx.x, sub = tid & (DTPT - 1);
    int i = blockIdx.x * DTGT + tid / DTPT;
    bool act = i < n;
    double X = act ? cx[i] : 0.0, Y = act ? cy[i] : 0.0;
    double sxx = 0.0, syy = 0.0, sxy = 0.0;
    for (int base = 0; base < n; base += DTILE) {
        __syncthreads();
        int j = base + tid;
        if (j < n) {
            const double c = cb[j], sn = sb[j];
            s_cx[tid] = cx[j]; s_cy[tid] = cy[j]; s_cb[tid] = c; s_sb[tid] = sn;
            s_c2[tid] = c * c - sn * sn; s_s2[tid] = 2.0 * c * sn;
            s_a[tid] = a[j]; s_ds[tid] = D[2 * j]; s_dn[tid] = D[2 * j + 1];
        }
        __syncthreads();
        int cnt = min(DTILE, n - base);
        if (act)
            for (int k = sub; k < cnt; k += DTPT)
                elem_stress_unit(X, Y, s_cx[k], s_cy[k], s_cb[k], s_sb[k], s_c2[k], s_s2[k], s_a[k], s_ds[k], s_dn[k],
                                 sxx, syy, sxy);
    }
    sxx *= -gc;
    syy *= -gc;
    sxy *= -gc;
#pragma unroll
    for (int w = 1; w < DTPT; w <<= 1) {
        sxx += __shfl_xor(sxx, w);
        syy += __shfl_xor(syy, w);
        sxy += __shfl_xor(sxy, w);
    }
    if (act && sub == 0) {
        double ts, tn;
        traction(cb[i], sb[i], sxx, syy, sxy, ts, tn);
        out[2 * i] = ts;
        out[2 * i + 1] = tn;
    }
}

// Dense matrix, row-major (2n x 2n): A[(2i+r)][2j+c] = traction r at i from
// unit DD c on j.  One thread per (i, j).
__global__ void k_dense_assemble(int n, const double *__restrict__ cx, const double *__restrict__ cy,
                                 const double *__restrict__ cb, const double *__restrict__ sb,
                                 const double *__restrict__ a, double gc, double *__restrict__ A)
{
    int i = blockIdx.x;
    int j = blockIdx.y * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double X = cx[i], Y = cy[i];
    size_t ld = 2 * (size_t)n;
    for (int c = 0; c < 2; ++c) {
        double sxx = 0.0, syy = 0.0, sxy = 0.0;
        elem_stress_add(X, Y, cx[j], cy[j], cb[j], sb[j], a[j], c == 0 ? 1.0 : 0.0, c == 1 ? 1.0 : 0.0, gc,
                        sxx, syy, sxy);
        double ts, tn;
        traction(cb[i], sb[i], sxx, syy, sxy, ts, tn);
        A[(2 * i) * ld + 2 * j + c] = ts;
        A[(2 * i + 1) * ld + 2 * j + c] = tn;
    }
}

// y = A x, one 256-thread block per row, 16-byte loads (m even), fixed-order
// reduction.  Streams the matrix once: HBM bound.
__global__ __launch_bounds__(256) void k_gemv(int m, const double *__restrict__ A,
                                              const double *__restrict__ x, double *__restrict__ y)
{
    __shared__ double red[256];
    int row = blockIdx.x;
    typedef double dv2 __attribute__((ext_vector_type(2)));
    const dv2 *Ar = reinterpret_cast<const dv2 *>(A + (size_t)row * m);
    const dv2 *x2 = reinterpret_cast<const dv2 *>(x);
    double s = 0.0;
    if ((m & 1) == 0) {  // rows 16-byte aligned: pairs
        int m2 = m / 2;
        for (int k = threadIdx.x; k < m2; k += 256) {
            dv2 av = __builtin_nontemporal_load(&Ar[k]);
            dv2 xv = x2[k];
            s += av.x * xv.x + av.y * xv.y;
        }
    } else {
        const double *a1 = A + (size_t)row * m;
        for (int k = threadIdx.x; k < m; k += 256) s += __builtin_nontemporal_load(&a1[k]) * x[k];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) y[row] = red[0];
}

}  // namespace

void direct_apply(fmddm_ctx *ctx, fmddm_tree *t, const double *D, double *out)
{
    int n = (int)t->n;
    hipLaunchKernelGGL(k_direct, dim3(cdiv(n, DTGT)), dim3(DT), 0, ctx->stream, n, t->ocx.p, t->ocy.p,
                       t->ocb.p, t->osb.p, t->oa.p, D, ctx->gc, out);
    FM_CHECK_LAUNCH();
}

void dense_gemv(hipStream_t s, int m, const double *A, const double *x, double *y)
{
    hipLaunchKernelGGL(k_gemv, dim3((unsigned)m), dim3(256), 0, s, m, A, x, y);
    FM_CHECK_LAUNCH();
}

void dense_apply(fmddm_ctx *ctx, fmddm_tree *t, const double *D, double *out)
{
    int n = (int)t->n;
    size_t m = 2 * (size_t)n;
    if (!t->Adense.p) {
        size_t freeb = 0, totalb = 0;
        FM_HIP(hipMemGetInfo(&freeb, &totalb));
        if (m * m * 8 + ((size_t)1 << 30) > freeb) throw Error{FMDDM_ENOMEM, "dense matrix does not fit"};
        t->Adense.alloc(m * m);
        hipLaunchKernelGGL(k_dense_assemble, dim3(n, cdiv(n, 256)), dim3(256), 0, ctx->stream, n,
                           t->ocx.p, t->ocy.p, t->ocb.p, t->osb.p, t->oa.p, ctx->gc, t->Adense.p);
        FM_CHECK_LAUNCH();
        t->bytes += (int64_t)(m * m * 8);
    }
    hipLaunchKernelGGL(k_gemv, dim3((unsigned)m), dim3(256), 0, ctx->stream, (int)m, t->Adense.p, D, out);
    FM_CHECK_LAUNCH();
}

}  // namespace fmddm
