// Block-Jacobi preconditioner for GMRES on the elastic system (Section 4).
//
// The paper solves with plain GMRES; this optional right preconditioner
// only changes the iteration count, not the solution.  The influence
// matrix's largest entries couple nearby elements of one fracture (the
// self term falls like 1/a, the kernel like 1/r^2), so the exact inverse
// of the matrix restricted to small groups of neighbouring elements removes
// most of the spread of its spectrum.  Groups: runs of at most PCB elements
// in tree (Morton) order that stay within one leaf, so each group is
// spatially compact.  Each group's 2m x 2m block (traction components of
// its elements from their shear/normal DDs, the exact element formulas) is
// assembled and inverted by one workgroup in LDS (Gauss-Jordan with
// partial pivoting) once per tree; a product with M^-1 is then one small
// dense product per group.  The poroelastic system's blocks (3 unknowns per
// element) are built in poro.hip and applied here.
#include "elem.h"
#include "gj.h"
#include "internal.h"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <cmath>
#include <vector>

namespace fmddm {
namespace {

constexpr int PCB = GJN / 2;  // elements per elastic group

// One workgroup per group: assemble the block, invert in place, write the
// inverse column-major at inv + off[b].  bad[0] is set when a pivot
// vanishes.
__global__ __launch_bounds__(256) void k_pc_build(int nblk, const int *__restrict__ beg,
                                                  const int *__restrict__ cnt, const int64_t *__restrict__ off,
                                                  const double *__restrict__ cx, const double *__restrict__ cy,
                                                  const double *__restrict__ cb, const double *__restrict__ sb,
                                                  const double *__restrict__ a, double gc,
                                                  double *__restrict__ inv, int *__restrict__ bad)
{
    __shared__ double A[GJN][GJN + 1];
    __shared__ double colk[GJN];
    __shared__ int piv[GJN];
    __shared__ double e_cx[PCB], e_cy[PCB], e_cb[PCB], e_sb[PCB], e_a[PCB];
    int b = blockIdx.x, tid = threadIdx.x;
    int s0 = beg[b], m = cnt[b], nb = 2 * m;
    if (tid < m) {
        e_cx[tid] = cx[s0 + tid]; e_cy[tid] = cy[s0 + tid]; e_cb[tid] = cb[s0 + tid];
        e_sb[tid] = sb[s0 + tid]; e_a[tid] = a[s0 + tid];
    }
    __syncthreads();
    // A[2i + r][2j + c]: traction r (0 shear, 1 normal) at element i from a
    // unit DD c (0 shear, 1 normal) on element j
    for (int e = tid; e < m * m; e += 256) {
        int i = e / m, j = e % m;
        for (int c = 0; c < 2; ++c) {
            double sxx = 0.0, syy = 0.0, sxy = 0.0, ts, tn;
            elem_stress_add(e_cx[i], e_cy[i], e_cx[j], e_cy[j], e_cb[j], e_sb[j], e_a[j], c == 0 ? 1.0 : 0.0,
                            c == 1 ? 1.0 : 0.0, gc, sxx, syy, sxy);
            traction(e_cb[i], e_sb[i], sxx, syy, sxy, ts, tn);
            A[2 * i][2 * j + c] = ts;
            A[2 * i + 1][2 * j + c] = tn;
        }
    }
    __syncthreads();
    gj_invert(A, nb, colk, piv, bad);
    double *o = inv + off[b];
    for (int e = tid; e < nb * nb; e += 256) {
        int c = e / nb, r = e % nb;
        o[e] = A[r][c];
    }
}

// out = M^-1 in (acc = 0) or out += M^-1 in (acc = 1); vectors in caller
// order, nc entries per element.  One 64-lane workgroup per group.
__global__ __launch_bounds__(64) void k_pc_apply(int nblk, int nc, const int *__restrict__ beg,
                                                 const int *__restrict__ cnt, const int64_t *__restrict__ off,
                                                 const int *__restrict__ perm, const double *__restrict__ inv,
                                                 const double *__restrict__ in, int acc, double *__restrict__ out)
{
    __shared__ double xs[GJN];
    int b = blockIdx.x, tid = threadIdx.x;
    int s0 = beg[b], nb = nc * cnt[b];
    int idx = 0;
    if (tid < nb) {
        int el = tid / nc;
        idx = nc * perm[s0 + el] + (tid - nc * el);
        xs[tid] = in[idx];
    }
    __syncthreads();
    if (tid < nb) {
        const double *col = inv + off[b] + tid;
        double y = 0.0;
        for (int c = 0; c < nb; ++c) y += col[(size_t)c * nb] * xs[c];
        out[idx] = acc ? out[idx] + y : y;
    }
}

// Coarse matrix R A P, one thread per (receiver aggregate I, source
// aggregate J): A[2I + r][2J + c] = mean over I's elements of traction r
// (0 shear, 1 normal) at their midpoints from a unit DD c on all of J's
// elements.  J is a straight run, so that DD is one long element's; I's
// elements share its direction, so the mean of their tractions is the
// traction of the mean stress.  gc of the modulus the coarse scale sees.
__global__ void k_coarse_build(int nc, const int *__restrict__ abeg, const double *__restrict__ ex,
                               const double *__restrict__ ey, const double *__restrict__ ccx,
                               const double *__restrict__ ccy, const double *__restrict__ ccb,
                               const double *__restrict__ csb, const double *__restrict__ ca, double gc,
                               double *__restrict__ A)
{
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)nc * nc) return;
    int I = (int)(g / nc), J = (int)(g - (int64_t)I * nc);
    const int e0 = abeg[I], e1 = abeg[I + 1];
    const size_t ld = 2 * (size_t)nc;
    for (int c = 0; c < 2; ++c) {
        double sxx = 0.0, syy = 0.0, sxy = 0.0, ts, tn;
        for (int e = e0; e < e1; ++e)
            elem_stress_add(ex[e], ey[e], ccx[J], ccy[J], ccb[J], csb[J], ca[J], c == 0 ? 1.0 : 0.0,
                            c == 1 ? 1.0 : 0.0, gc, sxx, syy, sxy);
        traction(ccb[I], csb[I], sxx, syy, sxy, ts, tn);
        A[(2 * (size_t)I) * ld + 2 * J + c] = ts / (e1 - e0);
        A[(2 * (size_t)I + 1) * ld + 2 * J + c] = tn / (e1 - e0);
    }
}

// rc[2I + r] = mean over aggregate I's elements of in[ncomp e + r], r < 2
__global__ void k_coarse_restrict(int nc, int ncomp, const int *__restrict__ abeg, const double *__restrict__ in,
                                  double *__restrict__ rc)
{
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= 2 * nc) return;
    int I = g >> 1, r = g & 1, e0 = abeg[I], e1 = abeg[I + 1];
    double s = 0.0;
    for (int e = e0; e < e1; ++e) s += in[(size_t)ncomp * e + r];
    rc[g] = s / (e1 - e0);
}

// y = Ainv rc, Ainv row-major (m x m): one wave per row
__global__ __launch_bounds__(256) void k_coarse_gemv(int m, const double *__restrict__ Ainv,
                                                     const double *__restrict__ rc, double *__restrict__ y)
{
    int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (row >= m) return;
    const double *a = Ainv + (size_t)row * m;
    double s = 0.0;
    for (int c = lane; c < m; c += 64) s += a[c] * rc[c];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) y[row] = s;
}

// out[ncomp e + r] += y[2 agg(e) + r], r < 2; one thread per aggregate and
// component, over its elements
__global__ void k_coarse_prolong(int nc, int ncomp, const int *__restrict__ abeg, const double *__restrict__ y,
                                 double *__restrict__ out)
{
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= 2 * nc) return;
    int I = g >> 1, r = g & 1;
    double v = y[g];
    for (int e = abeg[I]; e < abeg[I + 1]; ++e) out[(size_t)ncomp * e + r] += v;
}

template <typename T>
void up(hipStream_t s, DBuf<T> &d, const std::vector<T> &h)
{
    d.alloc(std::max<size_t>(h.size(), 1));
    if (!h.empty()) FM_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

}  // namespace

void pc_groups(fmddm_ctx *ctx, fmddm_tree *t, int maxm, int nc, PcBlocks &B)
{
    hipStream_t s = ctx->stream;
    int ncell = t->ncell;
    std::vector<int> hb(ncell), he(ncell);
    FM_HIP(hipMemcpyAsync(hb.data(), t->cpbeg.p, ncell * 4, hipMemcpyDeviceToHost, s));
    FM_HIP(hipMemcpyAsync(he.data(), t->cpend.p, ncell * 4, hipMemcpyDeviceToHost, s));
    FM_HIP(hipStreamSynchronize(s));
    std::vector<int> beg, cnt;
    std::vector<int64_t> off;
    int64_t tot = 0;
    for (int c : t->leaves)
        for (int q = hb[c]; q < he[c]; q += maxm) {
            int m = std::min(maxm, he[c] - q);
            beg.push_back(q);
            cnt.push_back(m);
            off.push_back(tot);
            tot += (int64_t)(nc * m) * (nc * m);
        }
    int nblk = (int)beg.size();
    B.beg.alloc(nblk);
    B.cnt.alloc(nblk);
    B.off.alloc(nblk);
    B.inv.alloc(tot);
    FM_HIP(hipMemcpyAsync(B.beg.p, beg.data(), nblk * 4, hipMemcpyHostToDevice, s));
    FM_HIP(hipMemcpyAsync(B.cnt.p, cnt.data(), nblk * 4, hipMemcpyHostToDevice, s));
    FM_HIP(hipMemcpyAsync(B.off.p, off.data(), nblk * 8, hipMemcpyHostToDevice, s));
    FM_HIP(hipStreamSynchronize(s));
    B.nblk = nblk;
    B.nc = nc;
}

void pc_setup(fmddm_ctx *ctx, fmddm_tree *t)
{
    PcBlocks &B = t->pc;
    if (B.nblk > 0) return;
    hipStream_t s = ctx->stream;
    pc_groups(ctx, t, PCB, 2, B);
    DBuf<int> bad;
    bad.alloc(1);
    bad.zero(s);
    hipLaunchKernelGGL(k_pc_build, dim3(B.nblk), dim3(256), 0, s, B.nblk, B.beg.p, B.cnt.p, B.off.p, t->scx.p,
                       t->scy.p, t->scb.p, t->ssb.p, t->sa.p, ctx->gc, B.inv.p, bad.p);
    FM_CHECK_LAUNCH();
    int hbad = 0;
    FM_HIP(hipMemcpyAsync(&hbad, bad.p, 4, hipMemcpyDeviceToHost, s));
    FM_HIP(hipStreamSynchronize(s));
    if (hbad) {
        B.nblk = 0;
        throw Error{FMDDM_EGEOM, "singular preconditioner block (coincident elements?)"};
    }
    t->bytes += (int64_t)B.inv.bytes() + (int64_t)B.nblk * 16;
}

void pc_apply(fmddm_ctx *ctx, fmddm_tree *t, const PcBlocks &B, const double *in, int acc, double *out)
{
    hipLaunchKernelGGL(k_pc_apply, dim3(B.nblk), dim3(64), 0, ctx->stream, B.nblk, B.nc, B.beg.p, B.cnt.p,
                       B.off.p, t->perm.p, B.inv.p, in, acc, out);
    FM_CHECK_LAUNCH();
}

// Two-level preconditioning (an addition to the paper's plain GMRES): the
// block-Jacobi groups span a few metres, so the long-wavelength modes of
// long fractures (and of parallel fractures that shield each other) keep
// the Krylov iteration long.  The coarse level represents them with
// piecewise-constant DDs over aggregates of consecutive collinear elements
// of one fracture; an aggregate is a straight run, so the constant-element
// formulas give the coarse operator A_c = R A P exactly (up to the
// medium, below).  M^-1 r = B^-1 r + P A_c^-1 R r, with R the mean over an
// aggregate of the traction residuals and P the constant extension of the
// coarse DDs: the coarse term alone makes the aggregate means of the
// residual vanish.  For the
// poroelastic left-hand side the coarse scale sees the undrained medium
// (nu_u): the diffusion length of one step is far below an aggregate.
constexpr int AGG_MIN = 16;      // elements per aggregate, at least
constexpr int COARSE_MAX = 1024;  // aggregates aimed at by default (runs end at fracture ends)
constexpr int COARSE_CAP = 2048;  // above this many aggregates the coarse level is left out

void pc_coarse_setup(fmddm_ctx *ctx, fmddm_tree *t, bool poro)
{
    PcCoarse &C = poro ? t->ppcc : t->pcc;
    const double nu_eff = poro ? ctx->poro.nu_u : ctx->prm.nu;
    const double key[6] = {ctx->prm.E, ctx->prm.nu, nu_eff, (double)ctx->prm.coarse_aggregates, 0, 0};
    bool same = C.nc > 0 || C.off;
    for (int k = 0; k < 6; ++k) same = same && C.key[k] == key[k];
    if (same) return;
    ++t->poro_gen;  // captured steps read the coarse level
    // unbuilt until the new level is complete (a failed rebuild leaves none)
    if (C.nc > 0) t->bytes -= (int64_t)C.ainv.bytes();
    C.nc = 0;
    C.off = 0;
    hipStream_t s = ctx->stream;
    const int n = (int)t->n;
    std::vector<double> x(n), y(n), cb(n), sb(n), a(n);
    FM_HIP(hipMemcpyAsync(x.data(), t->ocx.p, n * 8, hipMemcpyDeviceToHost, s));
    FM_HIP(hipMemcpyAsync(y.data(), t->ocy.p, n * 8, hipMemcpyDeviceToHost, s));
    FM_HIP(hipMemcpyAsync(cb.data(), t->ocb.p, n * 8, hipMemcpyDeviceToHost, s));
    FM_HIP(hipMemcpyAsync(sb.data(), t->osb.p, n * 8, hipMemcpyDeviceToHost, s));
    FM_HIP(hipMemcpyAsync(a.data(), t->oa.p, n * 8, hipMemcpyDeviceToHost, s));
    FM_HIP(hipStreamSynchronize(s));
    // aggregates: runs in caller order of at most `ag` elements where each
    // element starts at the previous one's end, in the same direction
    const int target = ctx->prm.coarse_aggregates > 0 ? ctx->prm.coarse_aggregates : COARSE_MAX;
    const int ag = std::max(AGG_MIN, (n + target - 1) / target);
    std::vector<int> abeg;
    std::vector<double> hx, hy, hcb, hsb, ha;
    auto close_run = [&](int b, int e) {  // elements [b, e)
        double x0 = x[b] - a[b] * cb[b], y0 = y[b] - a[b] * sb[b];
        double x1 = x[e - 1] + a[e - 1] * cb[e - 1], y1 = y[e - 1] + a[e - 1] * sb[e - 1];
        abeg.push_back(b);
        hx.push_back(0.5 * (x0 + x1));
        hy.push_back(0.5 * (y0 + y1));
        hcb.push_back(cb[b]);
        hsb.push_back(sb[b]);
        ha.push_back(0.5 * std::hypot(x1 - x0, y1 - y0));
    };
    int b = 0;
    for (int e = 1; e <= n; ++e) {
        bool cont = e < n && e - b < ag;
        if (cont) {
            double ex = x[e - 1] + a[e - 1] * cb[e - 1], ey = y[e - 1] + a[e - 1] * sb[e - 1];
            double sx = x[e] - a[e] * cb[e], sy = y[e] - a[e] * sb[e];
            double tol = 1e-9 * (a[e - 1] + a[e]);
            cont = std::hypot(ex - sx, ey - sy) <= tol && std::fabs(cb[e] - cb[e - 1]) <= 1e-9 &&
                   std::fabs(sb[e] - sb[e - 1]) <= 1e-9;
        }
        if (!cont) {
            close_run(b, e);
            b = e;
        }
    }
    const int nc = (int)hx.size();
    if (nc > COARSE_CAP) {  // few collinear runs: block-Jacobi alone
        C.off = 1;
        for (int k = 0; k < 6; ++k) C.key[k] = key[k];
        return;
    }
    abeg.push_back(n);
    const int m = 2 * nc;
    up(s, C.abeg, abeg);
    DBuf<double> dx, dy, dcb, dsb, da;
    up(s, dx, hx);
    up(s, dy, hy);
    up(s, dcb, hcb);
    up(s, dsb, hsb);
    up(s, da, ha);
    C.ainv.alloc((size_t)m * m);
    C.rc.alloc(m);
    C.yc.alloc(m);
    const double G = ctx->prm.E / (2.0 * (1.0 + ctx->prm.nu));
    const double gc = G / (2.0 * M_PI * (1.0 - nu_eff));
    hipLaunchKernelGGL(k_coarse_build, dim3(cdiv((int64_t)nc * nc, 256)), dim3(256), 0, s, nc, C.abeg.p, t->ocx.p,
                       t->ocy.p, dx.p, dy.p, dcb.p, dsb.p, da.p, gc, C.ainv.p);
    FM_CHECK_LAUNCH();
    // the row-major matrix is its transpose column-major; inverting that in
    // place leaves the inverse row-major
    DBuf<int> ipiv, info;
    ipiv.alloc(m);
    info.alloc(2);
    info.zero(s);
    if (!ctx->blas) {
        rocblas_handle h;
        if (rocblas_create_handle(&h) != rocblas_status_success) throw Error{FMDDM_EDEVICE, "rocblas handle"};
        ctx->blas = h;
    }
    rocblas_handle h = (rocblas_handle)ctx->blas;
    rocblas_set_stream(h, s);
    rocblas_status st = rocsolver_dgetrf(h, m, m, C.ainv.p, m, ipiv.p, info.p);
    if (st == rocblas_status_success) st = rocsolver_dgetri(h, m, C.ainv.p, m, ipiv.p, info.p + 1);
    FM_HIP(hipStreamSynchronize(s));
    if (st != rocblas_status_success) throw Error{FMDDM_EDEVICE, "coarse LU failed"};
    int hinfo[2] = {0, 0};
    FM_HIP(hipMemcpy(hinfo, info.p, 8, hipMemcpyDeviceToHost));
    if (hinfo[0] != 0 || hinfo[1] != 0) throw Error{FMDDM_EGEOM, "singular coarse matrix (coincident fractures?)"};
    C.nc = nc;
    for (int k = 0; k < 6; ++k) C.key[k] = key[k];
    t->bytes += (int64_t)C.ainv.bytes();
}

void pc_coarse_add(fmddm_ctx *ctx, fmddm_tree *t, const PcCoarse &C, int ncomp, const double *in, double *out)
{
    (void)t;
    if (C.nc == 0) return;  // left out (too few collinear runs)
    hipStream_t s = ctx->stream;
    const int m = 2 * C.nc;
    hipLaunchKernelGGL(k_coarse_restrict, dim3(cdiv(m, 256)), dim3(256), 0, s, C.nc, ncomp, C.abeg.p, in, C.rc.p);
    hipLaunchKernelGGL(k_coarse_gemv, dim3(cdiv(m, 4)), dim3(256), 0, s, m, C.ainv.p, C.rc.p, C.yc.p);
    hipLaunchKernelGGL(k_coarse_prolong, dim3(cdiv(m, 256)), dim3(256), 0, s, C.nc, ncomp, C.abeg.p, C.yc.p, out);
    FM_CHECK_LAUNCH();
}

}  // namespace fmddm

// The context's destructor lives here, beside the one user of its rocBLAS
// handle (the coarse factorisation), so that no other file needs rocBLAS.
fmddm_ctx::~fmddm_ctx()
{
    if (blas) (void)rocblas_destroy_handle((rocblas_handle)blas);
    release();
}
