// C ABI entry points (declared and documented in include/fmddm.h).  Each
// call validates its arguments, runs on the context's stream, and turns
// any internal error into a status code plus a message.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

namespace fmddm {
void sif_eval(fmddm_ctx *ctx, fmddm_tree *t, const double *D, int64_t e, double *KI, double *KII);
}

using fmddm::Error;
using fmddm::guarded;

namespace {


const char *check_params(const fmddm_params *p)
{
    if (!(p->E > 0.0) || !std::isfinite(p->E)) return "E must be positive";
    if (!(p->nu > -1.0 && p->nu < 0.5)) return "nu must lie in (-1, 0.5)";
    if (p->leaf < 1) return "leaf must be >= 1";
    if (p->p < 1 || p->p > fmddm::MAXP) return "p must lie in [1, 32]";
    if (p->max_level < 0 || p->max_level > 30) return "max_level must lie in [0, 30]";
    if (!(p->kappa >= 0.0)) return "kappa must be >= 0";
    if (p->m2l != FMDDM_M2L_DENSE && p->m2l != FMDDM_M2L_SVD) return "unknown m2l mode";
    if (p->m2l == FMDDM_M2L_SVD && !(p->m2l_tol > 0.0 && p->m2l_tol < 1.0)) return "m2l_tol must lie in (0, 1)";
    if (p->use_root_box && !(p->root_L > 0.0)) return "root box side must be positive";
    if (p->restart < 1 || p->restart > 1000) return "restart must lie in [1, 1000]";
    if (p->maxit < 0) return "maxit must be >= 0";
    if (!(p->tol >= 0.0)) return "tol must be >= 0";
    if (p->precision < FMDDM_PREC_FP64 || p->precision > FMDDM_PREC_BF16) return "unknown precision";
    if (p->use_graphs != 0 && p->use_graphs != 1) return "use_graphs must be 0 or 1";
    if (p->precond != FMDDM_PRECOND_NONE && p->precond != FMDDM_PRECOND_BLOCK &&
        p->precond != FMDDM_PRECOND_TWO_LEVEL)
        return "unknown precond";
    if (p->m2l_tiles < 0 || p->m2l_tiles > 3) return "m2l_tiles must lie in [0, 3]";
    if (p->direct_below < 0) return "direct_below must be >= 0";
    if (p->coarse_aggregates < 0 || p->coarse_aggregates > 2048) return "coarse_aggregates must lie in [0, 2048]";
    return nullptr;
}

}  // namespace

extern "C" {

void fmddm_default_params(fmddm_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->E = 20e9;
    p->nu = 0.25;
    p->leaf = 32;
    p->p = 20;
    p->max_level = 24;
    p->kappa = 8.0;
    p->m2l = FMDDM_M2L_DENSE;
    p->m2l_tol = 1e-12;
    p->restart = 50;
    p->maxit = 10000;
    p->tol = 1e-10;
    p->use_graphs = 0;
}

fmddm_status fmddm_create(const fmddm_params *p, void *hip_stream, fmddm_ctx **out)
{
    if (!out) return FMDDM_EINVAL;
    *out = nullptr;
    if (!p) return FMDDM_EINVAL;
    if (check_params(p)) return FMDDM_EINVAL;
    fmddm_ctx *ctx = new (std::nothrow) fmddm_ctx();
    if (!ctx) return FMDDM_ENOMEM;
    ctx->prm = *p;
    ctx->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        delete ctx;
        return FMDDM_EDEVICE;
    }
    double G = p->E / (2.0 * (1.0 + p->nu));
    ctx->gc = G / (2.0 * M_PI * (1.0 - p->nu));
    fmddm_status st = guarded(ctx, [&] {
        fmddm::init_streams(ctx);
        ctx->cheb = std::make_shared<fmddm::Cheb>();
        ctx->m2l = std::make_shared<fmddm::M2LOps>();
        ctx->pcache = std::make_shared<fmddm::PoroLhsCache>();
        fmddm::setup_cheb(ctx);
        return FMDDM_OK;
    });
    if (st != FMDDM_OK) {
        delete ctx;
        return st;
    }
    *out = ctx;
    return FMDDM_OK;
}

void fmddm_destroy(fmddm_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    // the caller may destroy the stream next: its work ends here, and the
    // blocks released on it become idle
    (void)hipStreamSynchronize(ctx->stream);
    fmddm::dev_stream_idle(ctx->stream);
    delete ctx;
}

const char *fmddm_last_error(const fmddm_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

fmddm_status fmddm_build_tree(fmddm_ctx *ctx, int64_t n, const double *x1, const double *y1,
                              const double *x2, const double *y2, int on_device, fmddm_tree **out)
{
    if (!ctx || !out) return FMDDM_EINVAL;
    *out = nullptr;
    if (n <= 0 || !x1 || !y1 || !x2 || !y2) {
        ctx->err = "empty geometry or null pointer";
        return FMDDM_EINVAL;
    }
    fmddm_tree *t = new (std::nothrow) fmddm_tree();
    if (!t) return FMDDM_ENOMEM;
    fmddm_status st = guarded(ctx, [&] {
        fmddm::build_tree(ctx, t, n, x1, y1, x2, y2, on_device);
        return FMDDM_OK;
    });
    if (st != FMDDM_OK) {
        fmddm::StreamScope scope(ctx->stream);  // its blocks may be in use by enqueued work
        delete t;
        return st;
    }
    *out = t;
    return FMDDM_OK;
}

void fmddm_tree_free(fmddm_tree *t)
{
    if (!t) return;
    // the tree's blocks go back to the allocator cache: no work that uses
    // them may still be running
    (void)hipDeviceSynchronize();
    delete t;
}

fmddm_status fmddm_tree_get_info(fmddm_ctx *ctx, const fmddm_tree *t, fmddm_tree_info *info)
{
    if (!ctx || !t || !info) return FMDDM_EINVAL;
    std::memset(info, 0, sizeof(*info));
    info->n = t->n;
    info->ncell = t->ncell;
    info->nleaf = t->nleaf;
    info->nlevel = t->nlevel;
    info->nU = t->h_loff[0].empty() ? 0 : t->h_loff[0].back();
    info->nV = t->h_loff[1].empty() ? 0 : t->h_loff[1].back();
    info->nW = t->h_loff[2].empty() ? 0 : t->h_loff[2].back();
    info->nX = t->h_loff[3].empty() ? 0 : t->h_loff[3].back();
    info->near_pairs = t->near_pairs;
    info->l2p_pairs = t->l2p_pairs;
    info->m2m_pairs = t->m2m_pairs;
    for (int c = 0; c < t->ncell; ++c) info->nfar += t->h_level[c] >= 2;
    info->m2l_rank = ctx->m2l->ready ? ctx->m2l->r : 0;
    info->root_x0 = t->x0;
    info->root_y0 = t->y0;
    info->root_L = t->L;
    int64_t b = 0;
    auto add = [&](size_t x) { b += (int64_t)x; };
    add(t->ocx.bytes() * 5); add(t->scx.bytes() * 5); add(t->perm.bytes()); add(t->key.bytes());
    add(t->clevel.bytes() * 8); add(t->cmk.bytes()); add(t->ccx.bytes() * 3);
    for (int w = 0; w < 4; ++w) { add(t->loff[w].bytes()); add(t->lidx[w].bytes()); }
    add(t->noff.bytes()); add(t->nsrc.bytes()); add(t->Wexp.bytes()); add(t->Gexp.bytes());
    add(t->What.bytes()); add(t->Ghat.bytes()); add(t->p2m_mat.bytes());
    add(t->Zm2l.bytes()); add(t->q.bytes()); add(t->Dsort.bytes()); add(t->Adense.bytes());
    add(t->gm_V.bytes()); add(t->gm_w.bytes()); add(t->gm_r.bytes());
    info->device_bytes = b;
    info->m2m_launches = (int64_t)t->m2m_launch.size();
    info->m2m_cut = t->m2m_cut;
    if (t->pc_ok == 1)
        for (int r : t->pc_rank) info->poro_m2l_rank = std::max(info->poro_m2l_rank, (int32_t)r);
    return FMDDM_OK;
}

fmddm_status fmddm_tree_export(fmddm_ctx *ctx, const fmddm_tree *t, int64_t *perm, uint64_t *key,
                               int32_t *level, uint32_t *ix, uint32_t *iy, int32_t *parent,
                               int32_t *child, int64_t *pbeg, int64_t *pend, int32_t *isleaf,
                               double *root)
{
    if (!ctx || !t) return FMDDM_EINVAL;
    return guarded(ctx, [&] {
        hipStream_t s = ctx->stream;
        int n = (int)t->n, nc = t->ncell;
        std::vector<int> tmp;
        auto widen = [&](const int *dsrc, int cnt, int64_t *dst) {
            tmp.resize(cnt);
            FM_HIP(hipMemcpyAsync(tmp.data(), dsrc, cnt * 4, hipMemcpyDeviceToHost, s));
            FM_HIP(hipStreamSynchronize(s));
            for (int i = 0; i < cnt; ++i) dst[i] = tmp[i];
        };
        if (perm) widen(t->perm.p, n, perm);
        if (pbeg) widen(t->cpbeg.p, nc, pbeg);
        if (pend) widen(t->cpend.p, nc, pend);
        if (key) FM_HIP(hipMemcpyAsync(key, t->key.p, n * 8, hipMemcpyDeviceToHost, s));
        if (level) FM_HIP(hipMemcpyAsync(level, t->clevel.p, nc * 4, hipMemcpyDeviceToHost, s));
        if (ix) FM_HIP(hipMemcpyAsync(ix, t->cix.p, nc * 4, hipMemcpyDeviceToHost, s));
        if (iy) FM_HIP(hipMemcpyAsync(iy, t->ciy.p, nc * 4, hipMemcpyDeviceToHost, s));
        if (parent) FM_HIP(hipMemcpyAsync(parent, t->cparent.p, nc * 4, hipMemcpyDeviceToHost, s));
        if (child) FM_HIP(hipMemcpyAsync(child, t->cchild.p, (size_t)nc * 16, hipMemcpyDeviceToHost, s));
        if (isleaf) FM_HIP(hipMemcpyAsync(isleaf, t->cleaf.p, nc * 4, hipMemcpyDeviceToHost, s));
        FM_HIP(hipStreamSynchronize(s));
        if (root) { root[0] = t->x0; root[1] = t->y0; root[2] = t->L; }
        return FMDDM_OK;
    });
}

fmddm_status fmddm_tree_export_list(fmddm_ctx *ctx, const fmddm_tree *t, int which, int64_t *off,
                                    int32_t *idx)
{
    if (!ctx || !t || which < 0 || which > 3) return FMDDM_EINVAL;
    return guarded(ctx, [&] {
        const std::vector<int> &o = t->h_loff[which];
        if (off)
            for (size_t i = 0; i < o.size(); ++i) off[i] = o[i];
        if (idx && o.back() > 0) {
            FM_HIP(hipMemcpyAsync(idx, t->lidx[which].p, (size_t)o.back() * 4, hipMemcpyDeviceToHost,
                                  ctx->stream));
            FM_HIP(hipStreamSynchronize(ctx->stream));
        }
        return FMDDM_OK;
    });
}

fmddm_status fmddm_apply(fmddm_ctx *ctx, fmddm_tree *t, int mode, const double *D, double *out)
{
    if (!ctx || !t || !D || !out || D == out) return FMDDM_EINVAL;
    if (mode < FMDDM_APPLY_FMM || mode > FMDDM_APPLY_DENSE) return FMDDM_EINVAL;
    return guarded(ctx, [&] {
        fmddm::apply_mode(ctx, t, mode, D, out);
        return FMDDM_OK;
    });
}

fmddm_status fmddm_rhs(fmddm_ctx *ctx, fmddm_tree *t, const double *pf, double SH, double Sh, double *rhs)
{
    if (!ctx || !t || !pf || !rhs) return FMDDM_EINVAL;
    return guarded(ctx, [&] {
        fmddm::rhs_build(ctx, t, pf, SH, Sh, rhs);
        return FMDDM_OK;
    });
}

fmddm_status fmddm_solve(fmddm_ctx *ctx, fmddm_tree *t, int mode, const double *rhs, double *D,
                         fmddm_solve_info *info)
{
    if (!ctx || !t || !rhs || !D || rhs == D) return FMDDM_EINVAL;
    if (mode < FMDDM_APPLY_FMM || mode > FMDDM_APPLY_DENSE) return FMDDM_EINVAL;
    fmddm_solve_info local;
    if (!info) info = &local;
    return guarded(ctx, [&] { return fmddm::gmres_solve(ctx, t, mode, rhs, D, info); });
}

fmddm_status fmddm_poro_set(fmddm_ctx *ctx, const fmddm_poro_params *pp)
{
    if (!ctx || !pp) return FMDDM_EINVAL;
    const double nu = ctx->prm.nu;
    if (!(pp->nu_u > nu && pp->nu_u < 0.5) || !(pp->alpha > 0.0 && pp->alpha <= 1.0) || !(pp->perm > 0.0) ||
        !(pp->visc > 0.0) || !(pp->dt > 0.0) || !std::isfinite(pp->p0) ||
        (pp->mode != FMDDM_APPLY_DIRECT && pp->mode != FMDDM_APPLY_FMM && pp->mode != FMDDM_APPLY_DENSE) ||
        (pp->m2l != FMDDM_M2L_DENSE && pp->m2l != FMDDM_M2L_SVD) ||
        (pp->exact_far_levels != 0 && pp->exact_far_levels != 1)) {
        ctx->err = "poroelastic parameters: need nu < nu_u < 0.5, 0 < alpha <= 1, perm, visc, dt > 0, "
                   "mode DIRECT, FMM or DENSE, m2l DENSE or SVD, exact_far_levels 0 or 1";
        return FMDDM_EINVAL;
    }
    if (ctx->prm.precision != FMDDM_PREC_FP64) {
        ctx->err = "the poroelastic operators are FP64 only";
        return FMDDM_EUNSUPPORTED;
    }
    if (pp->mode != FMDDM_APPLY_DIRECT && (ctx->prm.p < 2 || ctx->prm.p > 16)) {
        ctx->err = "poroelastic FMM needs 2 <= p <= 16";
        return FMDDM_EUNSUPPORTED;
    }
    ctx->poro = *pp;
    ctx->poro_set = 1;
    return FMDDM_OK;
}

fmddm_status fmddm_poro_apply(fmddm_ctx *ctx, fmddm_tree *t, int lag, const double *D, double *out)
{
    if (!ctx || !t || !D || !out || D == out || lag < 0) return FMDDM_EINVAL;
    return guarded(ctx, [&] {
        fmddm::poro_apply(ctx, t, lag, D, out);
        return FMDDM_OK;
    });
}

fmddm_status fmddm_add_history(fmddm_ctx *ctx, fmddm_tree *t, int h, const double *Dhist, double *rhs)
{
    if (!ctx || !t || !rhs || h < 1 || (h > 1 && !Dhist)) return FMDDM_EINVAL;
    if (h > 1 && rhs + 3 * t->n > Dhist && Dhist + 3 * t->n * (h - 1) > rhs) return FMDDM_EINVAL;
    return guarded(ctx, [&] {
        fmddm::poro_history(ctx, t, h, Dhist, rhs);
        return FMDDM_OK;
    });
}

fmddm_status fmddm_poro_rhs(fmddm_ctx *ctx, fmddm_tree *t, const double *pf, double SH, double Sh, double *rhs)
{
    if (!ctx || !t || !pf || !rhs) return FMDDM_EINVAL;
    if (!ctx->poro_set) {
        ctx->err = "poroelastic parameters not set (fmddm_poro_set)";
        return FMDDM_EINVAL;
    }
    return guarded(ctx, [&] {
        fmddm::poro_rhs(ctx, t, pf, SH, Sh, rhs);
        return FMDDM_OK;
    });
}

fmddm_status fmddm_poro_solve(fmddm_ctx *ctx, fmddm_tree *t, const double *rhs, double *D,
                              fmddm_solve_info *info)
{
    if (!ctx || !t || !rhs || !D || rhs == D) return FMDDM_EINVAL;
    fmddm_solve_info local;
    if (!info) info = &local;
    return guarded(ctx, [&] { return fmddm::gmres_solve(ctx, t, fmddm::APPLY_PORO, rhs, D, info); });
}

fmddm_status fmddm_sif(fmddm_ctx *ctx, fmddm_tree *t, const double *D, int64_t elem, double *KI,
                       double *KII)
{
    if (!ctx || !t || !D || !KI || !KII || elem < 0 || elem >= t->n) return FMDDM_EINVAL;
    return guarded(ctx, [&] {
        fmddm::sif_eval(ctx, t, D, elem, KI, KII);
        return FMDDM_OK;
    });
}

fmddm_status fmddm_profile(fmddm_ctx *ctx, unsigned mask)
{
    if (!ctx || mask >= (1u << FMDDM_PH_COUNT)) return FMDDM_EINVAL;
    ctx->prof.mask = mask;
    return FMDDM_OK;
}

fmddm_status fmddm_profile_read(fmddm_ctx *ctx, double *ms, int64_t *count)
{
    if (!ctx || !ms) return FMDDM_EINVAL;
    return guarded(ctx, [&] {
        ctx->prof.read(ctx->stream, ms, count);
        return FMDDM_OK;
    });
}

}  // extern "C"
