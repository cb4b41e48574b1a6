// Right-hand side, restarted GMRES and stress intensity factors on the
// device (Section 4; eq. 2.6).
//
// GMRES(m) with x0 taken from the caller, classical Gram-Schmidt applied
// twice (two passes of V^T w and w -= V h), Givens rotations on the
// Hessenberg column, all in FP64 on the device.  The host only reads the
// running residual estimate after each Arnoldi step to decide when to stop.
// At every restart the residual is recomputed from b - A x.
#include "elem.h"
#include "internal.h"

#include <cmath>

namespace fmddm {
namespace {

__global__ void k_rhs(int n, const double *__restrict__ cb, const double *__restrict__ sb,
                      const double *__restrict__ pf, double pscale, double SH, double Sh,
                      double *__restrict__ rhs)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double ts, tn;
    traction(cb[i], sb[i], -SH, -Sh, 0.0, ts, tn);
    rhs[2 * i] = -ts;
    rhs[2 * i + 1] = -pscale * pf[i] - tn;
}

__global__ void k_fill(int n, double v, double *__restrict__ x)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

constexpr int RT = 256;

// Block-level fixed-order sum.
__device__ double block_sum(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = RT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

// Dot products V_i . w (i < k) in two fixed-order stages.  Stage 1: block
// (c, g) takes the chunk [c DCH, (c+1) DCH) of vectors g DKG .. g DKG +
// DKG - 1, stages w's chunk in LDS, and each of its four waves forms the
// chunk's partial dot for i = g DKG + wave, + 4, ... (lanes stride the
// chunk, then a shuffle tree); part[i * nchunk + c].  Stage 2: one block
// per i sums the partials in chunk order.  The vectors are read once in
// total, over (m / DCH) x (k / DKG) blocks.
constexpr int DCH = 1024, DKG = 8;

__global__ __launch_bounds__(RT) void k_dots_part(int m, int k, const double *__restrict__ V, int ldv,
                                                  const double *__restrict__ w, int nchunk,
                                                  double *__restrict__ part)
{
    __shared__ double ws[DCH];
    int c = blockIdx.x, t0 = c * DCH, len = min(DCH, m - t0);
    for (int t = threadIdx.x; t < DCH; t += RT) ws[t] = t < len ? w[t0 + t] : 0.0;
    __syncthreads();
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i1 = min(k, (int)(blockIdx.y + 1) * DKG);
    for (int i = blockIdx.y * DKG + wave; i < i1; i += RT / 64) {
        const double *v = V + (size_t)i * ldv + t0;
        double s = 0.0;
#pragma unroll 4
        for (int t = lane; t < len; t += 64) s += v[t] * ws[t];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
        if (lane == 0) part[(size_t)i * nchunk + c] = s;
    }
}

// out[i] = sum over chunks of part[i * nchunk + c]; sqrt of it if `root`
__global__ __launch_bounds__(RT) void k_dots_sum(int nchunk, const double *__restrict__ part, int root,
                                                 double *__restrict__ out)
{
    __shared__ double red[RT];
    int i = blockIdx.x;
    double s = 0.0;
    for (int c = threadIdx.x; c < nchunk; c += RT) s += part[(size_t)i * nchunk + c];
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[i] = root ? sqrt(s) : s;
}

// sum_{i<k} h[i] V_i[t] in index order, with VU loads in flight
constexpr int VU = 8;

__device__ __forceinline__ double vcomb(int k, const double *__restrict__ h, const double *__restrict__ V,
                                        int ldv, int t)
{
    double s = 0.0;
    int i = 0;
    for (; i + VU <= k; i += VU) {
        double v[VU];
#pragma unroll
        for (int u = 0; u < VU; ++u) v[u] = V[(size_t)(i + u) * ldv + t];
#pragma unroll
        for (int u = 0; u < VU; ++u) s += h[i + u] * v[u];
    }
    for (; i < k; ++i) s += h[i] * V[(size_t)i * ldv + t];
    return s;
}

// w += sign * sum_{i<k} h[i] V_i
__global__ void k_vupdate(int m, int k, const double *__restrict__ V, int ldv,
                          const double *__restrict__ h, double sign, double *__restrict__ w)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    w[t] += sign * vcomb(k, h, V, ldv, t);
}


// v = src / *nrm (v = 0 when the norm vanishes)
__global__ void k_scale(int m, const double *__restrict__ src, const double *__restrict__ nrm,
                        double *__restrict__ v)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    double d = *nrm;
    v[t] = d != 0.0 ? src[t] / d : 0.0;
}

__global__ void k_residual(int m, const double *__restrict__ b, const double *__restrict__ Ax,
                           double *__restrict__ r)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < m) r[t] = b[t] - Ax[t];
}

// Scalar workspace layout (doubles): g[m+1] | cs[m] | sn[m] | H[(m+1) x m]
// column-major | h1[m+1] | h2[m+1] | y[m] | nrm | est
struct SW {
    int m;
    __host__ __device__ int g() const { return 0; }
    __host__ __device__ int cs() const { return m + 1; }
    __host__ __device__ int sn() const { return 2 * m + 1; }
    __host__ __device__ int H() const { return 3 * m + 1; }
    __host__ __device__ int h1() const { return 3 * m + 1 + (m + 1) * m; }
    __host__ __device__ int h2() const { return h1() + m + 1; }
    __host__ __device__ int y() const { return h2() + m + 1; }
    __host__ __device__ int nrm() const { return y() + m; }
    __host__ __device__ int est() const { return nrm() + 1; }
    __host__ __device__ int size() const { return est() + 1; }
};

// g = (beta, 0, ...), est = beta
__global__ void k_cycle_start(SW s, double *__restrict__ sc)
{
    double beta = sc[s.nrm()];
    for (int i = 0; i <= s.m; ++i) sc[s.g() + i] = 0.0;
    sc[s.g()] = beta;
    sc[s.est()] = beta;
}

// Column j of the Hessenberg matrix from the two Gram-Schmidt passes and the
// new norm; previous rotations applied, new rotation formed, residual
// estimate |g_{j+1}| updated.
// The whole block calls it: the column and the earlier rotations are staged
// in LDS by all threads, then one thread runs the (serial) recurrence out
// of LDS instead of through dependent global loads.
constexpr int MAXRS = 1001;  // restart + 1, at most

__device__ void givens_block(SW s, int j, double nrm, double *__restrict__ sc)
{
    __shared__ double Hc[MAXRS + 1], cs_s[MAXRS], sn_s[MAXRS];
    double *H = sc + s.H() + (size_t)j * (s.m + 1);
    double *cs = sc + s.cs(), *sn = sc + s.sn(), *g = sc + s.g();
    for (int i = threadIdx.x; i <= j; i += blockDim.x) Hc[i] = sc[s.h1() + i] + sc[s.h2() + i];
    for (int i = threadIdx.x; i < j; i += blockDim.x) {
        cs_s[i] = cs[i];
        sn_s[i] = sn[i];
    }
    if (threadIdx.x == 0) Hc[j + 1] = nrm;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < j; ++i) {
            double h0 = Hc[i], hh = Hc[i + 1];
            Hc[i] = cs_s[i] * h0 + sn_s[i] * hh;
            Hc[i + 1] = -sn_s[i] * h0 + cs_s[i] * hh;
        }
        double h0 = Hc[j], hh = Hc[j + 1];
        double den = sqrt(h0 * h0 + hh * hh);
        double c = den == 0.0 ? 1.0 : h0 / den, sv = den == 0.0 ? 0.0 : hh / den;
        cs[j] = c;
        sn[j] = sv;
        Hc[j] = den;
        Hc[j + 1] = 0.0;
        double gj = g[j];
        g[j + 1] = -sv * gj;
        g[j] = c * gj;
        sc[s.est()] = fabs(g[j + 1]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) H[i] = Hc[i];
}

__global__ __launch_bounds__(64) void k_givens(SW s, int j, double *__restrict__ sc)
{
    givens_block(s, j, sc[s.nrm()], sc);
}

// Fused Arnoldi pieces for short vectors (few dot-product chunks), where
// launches, not bytes, set the time.  k_vupdate_sum: every block forms the
// k dot products from the chunk partials (same fixed order in every block,
// so all blocks agree bit for bit; block 0 stores them for the rotation),
// then w += sign * sum_i h_i V_i over its 256 entries; with `npart`, also
// the block's partial of ||w||^2 after the update.
constexpr int FCH = 32;  // most chunks summed per dot product in the fused path

__global__ __launch_bounds__(256) void k_vupdate_sum(int m, int k, const double *__restrict__ V, int ldv,
                                                     const double *__restrict__ part, int nchunk, double sign,
                                                     double *__restrict__ w, double *__restrict__ hout,
                                                     double *__restrict__ npart)
{
    extern __shared__ double hs[];  // k
    __shared__ double red[RT];
    for (int i = threadIdx.x; i < k; i += RT) {
        double s = 0.0;
        for (int c = 0; c < nchunk; ++c) s += part[(size_t)i * nchunk + c];
        hs[i] = s;
        if (blockIdx.x == 0) hout[i] = s;
    }
    __syncthreads();
    int t = blockIdx.x * RT + threadIdx.x;
    double wt = 0.0;
    if (t < m) {
        wt = w[t] + sign * vcomb(k, hs, V, ldv, t);
        w[t] = wt;
    }
    if (npart) {
        double q = block_sum(wt * wt, red);
        if (threadIdx.x == 0) npart[blockIdx.x] = q;
    }
}

// ||w|| from the update blocks' partials (every block sums them the same
// way), v = w / ||w||, and in block 0 the Hessenberg column and rotation.
__global__ __launch_bounds__(256) void k_scale_givens(int m, const double *__restrict__ w,
                                                      const double *__restrict__ npart, int nnp,
                                                      double *__restrict__ v, SW s, int j,
                                                      double *__restrict__ sc)
{
    __shared__ double red[RT];
    double q = 0.0;
    for (int b = threadIdx.x; b < nnp; b += RT) q += npart[b];
    double nrm = sqrt(block_sum(q, red));
    for (int t = blockIdx.x * RT + threadIdx.x; t < m; t += gridDim.x * RT) v[t] = nrm != 0.0 ? w[t] / nrm : 0.0;
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) sc[s.nrm()] = nrm;
        givens_block(s, j, nrm, sc);
    }
}

// y = R^{-1} g over the first k columns, by one block: column sweep from
// the last unknown, the remaining right-hand side in LDS (each column of R
// is read once, its entries spread over the threads).
__global__ __launch_bounds__(RT) void k_backsolve(SW s, int k, double *__restrict__ sc)
{
    __shared__ double v[MAXRS];
    const double *H = sc + s.H();
    double *y = sc + s.y();
    for (int r = threadIdx.x; r < k; r += RT) v[r] = sc[s.g() + r];
    __syncthreads();
    for (int i = k - 1; i >= 0; --i) {
        const double *col = H + (size_t)i * (s.m + 1);
        const double yi = v[i] / col[i];
        for (int r = threadIdx.x; r < i; r += RT) v[r] -= col[r] * yi;
        if (threadIdx.x == 0) y[i] = yi;
        __syncthreads();
    }
}

__global__ void k_sif(const double *__restrict__ D, const double *__restrict__ a, int64_t e, double E,
                      double nu, double *__restrict__ out)
{
    double f = 0.806 * E / (4.0 * (1.0 - nu * nu)) * sqrt(M_PI / (2.0 * a[e]));
    out[0] = f * D[2 * e + 1];
    out[1] = f * D[2 * e];
}

// out[0..k) = V_i . w, with the partials in `part` (k * nchunk doubles)
void dots(hipStream_t st, int m, int k, const double *V, int ldv, const double *w, double *part, double *out)
{
    int nchunk = cdiv(m, DCH);
    hipLaunchKernelGGL(k_dots_part, dim3(nchunk, cdiv(k, DKG)), dim3(RT), 0, st, m, k, V, ldv, w, nchunk, part);
    hipLaunchKernelGGL(k_dots_sum, dim3(k), dim3(RT), 0, st, nchunk, part, 0, out);
    FM_CHECK_LAUNCH();
}

// *out = ||w||
void norm2(hipStream_t st, int m, const double *w, double *part, double *out)
{
    int nchunk = cdiv(m, DCH);
    hipLaunchKernelGGL(k_dots_part, dim3(nchunk), dim3(RT), 0, st, m, 1, w, 0, w, nchunk, part);
    hipLaunchKernelGGL(k_dots_sum, dim3(1), dim3(RT), 0, st, nchunk, part, 1, out);
    FM_CHECK_LAUNCH();
}

}  // namespace

void rhs_build(fmddm_ctx *ctx, fmddm_tree *t, const double *pf, double SH, double Sh, double *rhs,
               double pscale)
{
    int n = (int)t->n;
    hipLaunchKernelGGL(k_rhs, dim3(cdiv(n, 256)), dim3(256), 0, ctx->stream, n, t->ocb.p, t->osb.p, pf,
                       pscale, SH, Sh, rhs);
    FM_CHECK_LAUNCH();
}

void apply_mode(fmddm_ctx *ctx, fmddm_tree *t, int mode, const double *D, double *out)
{
    switch (mode) {
    case FMDDM_APPLY_FMM: fmm_apply(ctx, t, D, out, ctx->prm.precision); break;
    case APPLY_FMM_FP64: fmm_apply(ctx, t, D, out, FMDDM_PREC_FP64); break;
    case FMDDM_APPLY_DIRECT: direct_apply(ctx, t, D, out); break;
    case FMDDM_APPLY_DENSE: dense_apply(ctx, t, D, out); break;
    case APPLY_PORO: poro_apply(ctx, t, 0, D, out); break;
    default: throw Error{FMDDM_EINVAL, "unknown apply mode"};
    }
}

void sif_eval(fmddm_ctx *ctx, fmddm_tree *t, const double *D, int64_t e, double *KI, double *KII)
{
    DBuf<double> o;
    o.alloc(2);
    hipLaunchKernelGGL(k_sif, dim3(1), dim3(1), 0, ctx->stream, D, t->oa.p, e, ctx->prm.E, ctx->prm.nu, o.p);
    FM_CHECK_LAUNCH();
    double h[2];
    FM_HIP(hipMemcpyAsync(h, o.p, 16, hipMemcpyDeviceToHost, ctx->stream));
    FM_HIP(hipStreamSynchronize(ctx->stream));
    *KI = h[0];
    *KII = h[1];
}

static void gmres_workspace(fmddm_tree *t, int m, int n2)
{
    const int ldv = (n2 + 63) / 64 * 64;
    SW s{m};
    if (t->gm_restart != m || t->gm_len != n2 || !t->gm_V.p) {
        t->gm_V.alloc((size_t)(m + 1) * ldv);
        t->gm_w.alloc(ldv);
        t->gm_r.alloc(ldv);
        t->gm_sc.alloc(s.size());
        t->gm_part.alloc((size_t)(m + 1) * cdiv(n2, DCH) + cdiv(n2, 256));
        t->drop_graphs();
        t->gm_restart = m;
        t->gm_len = n2;
    }
    if (!t->gm_host) FM_HIP(hipHostMalloc((void **)&t->gm_host, 4 * sizeof(double), hipHostMallocDefault));
    for (int k = 0; k < 2; ++k)
        if (!t->gm_ev[k]) FM_HIP(hipEventCreateWithFlags(&t->gm_ev[k], hipEventDisableTiming));
}

// Host slots: the norm of b and of residuals arrive in slot 0; Arnoldi step
// j's (new norm, residual estimate) in slot j % 2, so that step j + 1 can be
// in flight while step j's scalars are read.
void GmresRun::post(int slot, int count)
{
    SW s{ctx->prm.restart};
    FM_HIP(hipMemcpyAsync(t->gm_host + 2 * slot, t->gm_sc.p + s.nrm(), 8 * count, hipMemcpyDeviceToHost,
                          ctx->stream));
    FM_HIP(hipEventRecord(t->gm_ev[slot], ctx->stream));
}

void GmresRun::start(fmddm_ctx *c, fmddm_tree *tr, int md, const double *rhs, double *x0, double tl, int mx,
                     int rmd)
{
    ctx = c;
    t = tr;
    mode = md;
    rmode = rmd < 0 ? md : rmd;
    residuals = 0;
    prev_beta = INFINITY;
    b = rhs;
    x = x0;
    tol = tl;
    maxit = mx;
    j = next = it = restarts = 0;
    eager_done = false;
    pc = ctx->prm.precond != FMDDM_PRECOND_NONE;
    pc2 = ctx->prm.precond == FMDDM_PRECOND_TWO_LEVEL;
    bnorm = relres = 0.0;
    converged = false;
    gmres_workspace(t, ctx->prm.restart, (int)vec_len(t, mode));
    if (pc) {
        if (mode == APPLY_PORO) pc_setup_poro(ctx, t);
        else pc_setup(ctx, t);
        if (pc2) pc_coarse_setup(ctx, t, mode == APPLY_PORO);
        if (!t->gm_z.p || t->gm_z.n < (size_t)vec_len(t, mode)) t->gm_z.alloc(vec_len(t, mode));
    }
    SW s{ctx->prm.restart};
    const int n2 = (int)vec_len(t, mode);
    norm2(ctx->stream, n2, b, t->gm_part.p, t->gm_sc.p + s.nrm());
    post(0, 1);
    state = BNORM;
}

// r = b - A x and its norm
void GmresRun::enqueue_residual()
{
    SW s{ctx->prm.restart};
    hipStream_t st = ctx->stream;
    const int n2 = (int)vec_len(t, mode);
    apply_mode(ctx, t, rmode, x, t->gm_w.p);
    ++residuals;
    hipLaunchKernelGGL(k_residual, dim3(cdiv(n2, 256)), dim3(256), 0, st, n2, b, t->gm_w.p, t->gm_r.p);
    norm2(st, n2, t->gm_r.p, t->gm_part.p, t->gm_sc.p + s.nrm());
    post(0, 1);
}

// Arnoldi step `next`: w = A v_j, two classical Gram-Schmidt passes, the new
// basis vector, the Hessenberg column and its Givens rotation, its scalars
// copied to the host slot.  Every step index has a fixed set of launches
// over fixed buffers (the basis, the work vector, the scalars; b and x are
// not touched), so after one uncaptured step has done the product's lazy
// set-up, step jj is captured once as a graph and replayed in later cycles
// and later solves on the tree.  The poroelastic products are captured too:
// whatever they build on first use (operators, near blocks, preconditioner
// blocks) bumps the tree's generation, which drops the captured steps and
// runs the next step uncaptured.  Profiled products stay uncaptured.
void GmresRun::enqueue_step()
{
    const int m = ctx->prm.restart, jj = next++;
    hipStream_t st = ctx->stream;
    ++it;
    if (ctx->prm.use_graphs && t->gm_graph_gen != t->poro_gen) {
        // something the captured steps read was rebuilt: drop them (after
        // any replay still in flight), and let one step run uncaptured
        // first (it may finish lazy set-up)
        FM_HIP(hipStreamSynchronize(st));
        t->drop_graphs();
        t->gm_graph_gen = t->poro_gen;
        eager_done = false;
    }
    bool graph = ctx->prm.use_graphs && eager_done && ctx->prof.mask == 0 &&
                 (mode == FMDDM_APPLY_FMM || mode == FMDDM_APPLY_DIRECT || mode == FMDDM_APPLY_DENSE ||
                  mode == APPLY_PORO);
    if (graph) {
        if (t->gm_graph_ctx != ctx || t->gm_graph_mode != mode || (int)t->gm_graph.size() != m) {
            t->drop_graphs();
            t->gm_graph.assign(m, nullptr);
            t->gm_graph_ctx = ctx;
            t->gm_graph_mode = mode;
        }
        hipGraphExec_t &ge = t->gm_graph[jj];
        if (!ge) {
            // the step's launches follow ctx->stream: point it at the
            // capture stream for the duration
            hipGraph_t g = nullptr;
            hipStream_t cs = ctx->cap;
            FM_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            ctx->stream = cs;
            try {
                step_body(jj);
            } catch (...) {
                ctx->stream = st;
                (void)hipStreamEndCapture(cs, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            ctx->stream = st;
            FM_HIP(hipStreamEndCapture(cs, &g));
            hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            FM_HIP(e);
        }
        FM_HIP(hipGraphLaunch(ge, st));
    } else {
        step_body(jj);
        eager_done = true;
    }
    FM_HIP(hipEventRecord(t->gm_ev[jj & 1], st));
}

void GmresRun::precond(const double *in, int acc, double *out)
{
    const bool poro = mode == APPLY_PORO;
    pc_apply(ctx, t, poro ? t->ppc : t->pc, in, acc, out);
    if (pc2) pc_coarse_add(ctx, t, poro ? t->ppcc : t->pcc, poro ? 3 : 2, in, out);
}

void GmresRun::step_body(int jj)
{
    const int m = ctx->prm.restart;
    SW s{m};
    hipStream_t st = ctx->stream;
    const int n2 = (int)vec_len(t, mode), ldv = (n2 + 63) / 64 * 64, gb = cdiv(n2, 256);
    double *V = t->gm_V.p, *w = t->gm_w.p, *sc = t->gm_sc.p;
    double *vj = V + (size_t)jj * ldv, *vn = V + (size_t)(jj + 1) * ldv;
    if (pc) {
        precond(vj, 0, t->gm_z.p);
        apply_mode(ctx, t, mode, t->gm_z.p, w);
    } else {
        apply_mode(ctx, t, mode, vj, w);
    }
    const int nchunk = cdiv(n2, DCH);
    if (nchunk <= FCH) {
        // five launches: two (partial dots, update) passes, then norm,
        // scaling and rotation
        const size_t hsm = (size_t)(jj + 1) * 8;
        double *np = t->gm_part.p + (size_t)(m + 1) * nchunk;  // gb norm partials after the dot partials
        hipLaunchKernelGGL(k_dots_part, dim3(nchunk, cdiv(jj + 1, DKG)), dim3(RT), 0, st, n2, jj + 1, V, ldv, w,
                           nchunk, t->gm_part.p);
        hipLaunchKernelGGL(k_vupdate_sum, dim3(gb), dim3(RT), hsm, st, n2, jj + 1, V, ldv, t->gm_part.p, nchunk,
                           -1.0, w, sc + s.h1(), (double *)nullptr);
        hipLaunchKernelGGL(k_dots_part, dim3(nchunk, cdiv(jj + 1, DKG)), dim3(RT), 0, st, n2, jj + 1, V, ldv, w,
                           nchunk, t->gm_part.p);
        hipLaunchKernelGGL(k_vupdate_sum, dim3(gb), dim3(RT), hsm, st, n2, jj + 1, V, ldv, t->gm_part.p, nchunk,
                           -1.0, w, sc + s.h2(), np);
        hipLaunchKernelGGL(k_scale_givens, dim3(std::min(gb, 64)), dim3(RT), 0, st, n2, w, np, gb, vn, s, jj, sc);
    } else {
        dots(st, n2, jj + 1, V, ldv, w, t->gm_part.p, sc + s.h1());
        hipLaunchKernelGGL(k_vupdate, dim3(gb), dim3(256), 0, st, n2, jj + 1, V, ldv, sc + s.h1(), -1.0, w);
        dots(st, n2, jj + 1, V, ldv, w, t->gm_part.p, sc + s.h2());
        hipLaunchKernelGGL(k_vupdate, dim3(gb), dim3(256), 0, st, n2, jj + 1, V, ldv, sc + s.h2(), -1.0, w);
        norm2(st, n2, w, t->gm_part.p, sc + s.nrm());
        hipLaunchKernelGGL(k_scale, dim3(gb), dim3(256), 0, st, n2, w, sc + s.nrm(), vn);
        hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, st, s, jj, sc);
    }
    FM_CHECK_LAUNCH();
    FM_HIP(hipMemcpyAsync(t->gm_host + 2 * (jj & 1), sc + s.nrm(), 16, hipMemcpyDeviceToHost, st));
}

bool GmresRun::advance(bool block)
{
    if (state == DONE || state == IDLE) return true;
    // the oldest result not yet read: slot 0 for norms, step j's otherwise
    int slot = state == ITER ? (j & 1) : 0;
    hipEvent_t ev = t->gm_ev[slot];
    if (block) {
        FM_HIP(hipEventSynchronize(ev));
    } else {
        hipError_t q = hipEventQuery(ev);
        if (q == hipErrorNotReady) return false;
        FM_HIP(q);
    }
    const int m = ctx->prm.restart;
    SW s{m};
    hipStream_t st = ctx->stream;
    const int n2 = (int)vec_len(t, mode), ldv = (n2 + 63) / 64 * 64, gb = cdiv(n2, 256);
    double *V = t->gm_V.p, *sc = t->gm_sc.p;
    const double *h = t->gm_host + 2 * slot;
    switch (state) {
    case BNORM:
        bnorm = h[0];
        if (!std::isfinite(bnorm)) throw Error{FMDDM_EINVAL, "non-finite right-hand side"};
        if (bnorm == 0.0) {
            hipLaunchKernelGGL(k_fill, dim3(cdiv(n2, 256)), dim3(256), 0, st, n2, 0.0, x);
            FM_CHECK_LAUNCH();
            FM_HIP(hipStreamSynchronize(st));
            converged = true;
            state = DONE;
            return true;
        }
        enqueue_residual();
        state = RESID;
        return false;
    case RESID: {
        double beta = h[0];
        relres = beta / bnorm;
        if (!std::isfinite(beta)) throw Error{FMDDM_EDEVICE, "non-finite residual"};
        // a refinement cycle that did not reduce the residual: the Arnoldi
        // product is too far from the residual product for this system
        bool stalled = rmode != mode && beta >= prev_beta;
        prev_beta = beta;
        if (beta <= tol * bnorm || it >= maxit || stalled) {
            converged = beta <= tol * bnorm;
            state = DONE;
            return true;
        }
        ++restarts;
        hipLaunchKernelGGL(k_scale, dim3(gb), dim3(256), 0, st, n2, t->gm_r.p, sc + s.nrm(), V);
        hipLaunchKernelGGL(k_cycle_start, dim3(1), dim3(1), 0, st, s, sc);
        FM_CHECK_LAUNCH();
        j = next = 0;
        enqueue_step();
        if (next < m && it < maxit) enqueue_step();  // one step ahead
        state = ITER;
        return false;
    }
    case ITER: {
        double nrm = h[0], est = h[1];
        int k = j + 1;
        bool ahead = next > k;  // step j + 1 already enqueued
        if (est <= tol * bnorm || nrm == 0.0 || k == m || (!ahead && it >= maxit)) {
            // a step enqueued ahead leaves H's first k columns and g[0..k)
            // as they were: the update uses the first k only
            hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(RT), 0, st, s, k, sc);
            if (pc) {  // x += M^-1 V y
                double *u = t->gm_w.p;
                hipLaunchKernelGGL(k_fill, dim3(gb), dim3(256), 0, st, n2, 0.0, u);
                hipLaunchKernelGGL(k_vupdate, dim3(gb), dim3(256), 0, st, n2, k, V, ldv, sc + s.y(), 1.0, u);
                FM_CHECK_LAUNCH();
                precond(u, 1, x);
            } else {
                hipLaunchKernelGGL(k_vupdate, dim3(gb), dim3(256), 0, st, n2, k, V, ldv, sc + s.y(), 1.0, x);
            }
            FM_CHECK_LAUNCH();
            enqueue_residual();
            state = RESID;
        } else {
            ++j;
            if (next < m && it < maxit) enqueue_step();
        }
        return false;
    }
    default: return true;
    }
}

fmddm_status gmres_solve(fmddm_ctx *ctx, fmddm_tree *t, int mode, const double *b, double *x,
                         fmddm_solve_info *info)
{
    // reduced-precision FMM: Arnoldi on it, residuals with the FP64 product
    bool mixed = mode == FMDDM_APPLY_FMM && ctx->prm.precision != FMDDM_PREC_FP64;
    GmresRun g;
    g.start(ctx, t, mode, b, x, ctx->prm.tol, ctx->prm.maxit, mixed ? APPLY_FMM_FP64 : -1);
    while (!g.advance(true)) {
    }
    info->iters = g.it;
    info->restarts = g.restarts;
    info->relres = g.relres;
    info->converged = g.converged;
    info->refinements = mixed ? g.residuals : 0;
    FM_HIP(hipStreamSynchronize(ctx->stream));
    return g.converged ? FMDDM_OK : FMDDM_ENOTCONV;
}

}  // namespace fmddm
