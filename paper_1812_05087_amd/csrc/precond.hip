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

}  // namespace fmddm
