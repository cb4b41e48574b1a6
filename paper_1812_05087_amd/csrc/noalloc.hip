// The FMM product with every per-product intermediate in one static device
// workspace (fmddm_apply_static): the variant of fmddm_apply's FMM mode for
// callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).  It
// launches the same kernels in the same order as fmddm_apply, so the two
// give the same result bit for bit.
#include "internal.h"

#include <algorithm>
#include <mutex>
#include <string>

using fmddm::Error;

namespace {
constexpr size_t STATIC_BYTES = (size_t)96 << 20;  // 96 MiB: the C2 product at p = 20 needs 72 MB
constexpr int MAX_DEVICES = 64;
}  // namespace

// One copy on every device the library runs on, held until the process
// ends.  In host code this name is only a handle for hipGetSymbolAddress:
// kernels get the device address kept in workspace_on().
static __device__ __align__(256) double scratch[STATIC_BYTES / sizeof(double)];

namespace {
std::mutex g_mu;
double *g_addr[MAX_DEVICES] = {};

// Doubles of each buffer one product writes and reads again, in the order
// of FmmBufs, each padded to a multiple of 32 (256 bytes).
void buf_sizes(fmddm_ctx *ctx, const fmddm_tree *t, size_t *sz)
{
    const fmddm::M2LOps &M = *ctx->m2l;
    const bool svd = M.mode == FMDDM_M2L_SVD;
    const size_t n = (size_t)t->n, nc = (size_t)t->ncell;
    const size_t raw[10] = {2 * n,                                                // sorted DDs
                            3 * n,                                                // charges
                            3 * (size_t)t->npartial,                              // near partials
                            nc * M.Mp,                                            // weights
                            svd ? (size_t)fmddm::fmm_ksplit(ctx) * nc * M.rp : 0,  // split-K partials
                            svd ? nc * M.rp : 0,                                  // compressed weights
                            (size_t)std::max<int64_t>(t->nV, 1) * M.rp,           // pair products
                            svd ? nc * M.rp : 0,                                  // compressed fields
                            nc * M.Mp,                                            // fields at the nodes
                            3 * (size_t)std::max(t->nfarlev, 1) * n};             // far stress per level
    for (int i = 0; i < 10; ++i) sz[i] = (raw[i] + 31) / 32 * 32;
}

size_t static_bytes(fmddm_ctx *ctx, const fmddm_tree *t)
{
    size_t sz[10], tot = 0;
    buf_sizes(ctx, t, sz);
    for (size_t v : sz) tot += v;
    return tot * sizeof(double);
}

fmddm::FmmBufs carve(fmddm_ctx *ctx, const fmddm_tree *t, double *base)
{
    size_t sz[10];
    buf_sizes(ctx, t, sz);
    double *p[10];
    for (int i = 0; i < 10; ++i) {
        p[i] = base;
        base += sz[i];
    }
    return fmddm::FmmBufs{p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7], p[8], p[9]};
}

// The workspace keeps the last call's contents.  A product writes every
// element it reads except the padding columns [3 p^2, Mp) of the multipole
// weights, which the M2L GEMMs multiply by zero operator columns: they are
// cleared (by a kernel, so the call can be captured in a graph).
__global__ void k_zero_pad(int ncell, int n3, int Mp, double *__restrict__ W)
{
    const int w = Mp - n3;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)ncell * w) return;
    const int64_t c = i / w;
    W[c * Mp + n3 + (i - c * w)] = 0.0;
}

void clear_pad(fmddm_ctx *ctx, const fmddm_tree *t, const fmddm::FmmBufs &B)
{
    const int n3 = 3 * ctx->prm.p * ctx->prm.p, Mp = ctx->m2l->Mp;
    const int64_t cnt = (int64_t)t->ncell * (Mp - n3);
    if (cnt > 0) {
        hipLaunchKernelGGL(k_zero_pad, dim3(fmddm::cdiv(cnt, 256)), dim3(256), 0, ctx->stream, t->ncell, n3, Mp,
                           B.Wexp);
        FM_CHECK_LAUNCH();
    }
}

// The workspace's device address on `dev` (which must be current), looked
// up once per device.
double *workspace_on(int dev)
{
    if (dev < 0 || dev >= MAX_DEVICES) throw Error{FMDDM_EDEVICE, "device index out of range"};
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[dev]) {
        void *p = nullptr;
        FM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error{FMDDM_EDEVICE, "static workspace has no device address"};
        g_addr[dev] = static_cast<double *>(p);
    }
    return g_addr[dev];
}
}  // namespace

extern "C" fmddm_status fmddm_apply_static(fmddm_ctx *ctx, fmddm_tree *t, const double *D, double *out)
{
    if (!ctx || !t || !D || !out || D == out) return FMDDM_EINVAL;
    return fmddm::guarded(ctx, [&] {
        if (ctx->prm.precision != FMDDM_PREC_FP64)
            throw Error{FMDDM_EUNSUPPORTED, "fmddm_apply_static computes FP64 products only"};
        if (!t->Wexp.p || !ctx->m2l->ready)
            throw Error{FMDDM_EINVAL, "fmddm_apply_static: the tree's schedules and operators are not built; "
                                      "run one fmddm_apply FMM product on it first"};
        const size_t need = static_bytes(ctx, t);
        if (need > STATIC_BYTES)
            throw Error{FMDDM_EINVAL, "fmddm_apply_static: the product needs " + std::to_string(need) +
                                          " bytes of workspace, the static workspace holds " +
                                          std::to_string(STATIC_BYTES)};
        const fmddm::FmmBufs B = carve(ctx, t, workspace_on(ctx->device));
        clear_pad(ctx, t, B);
        fmddm::fmm_apply_bufs(ctx, t, D, out, FMDDM_PREC_FP64, B);
        return FMDDM_OK;
    });
}
