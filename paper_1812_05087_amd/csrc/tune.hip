// Autotuner of the FMM product's tree and expansion parameters.
//
// The paper fixes the number of Chebyshev nodes by hand (Section 5 uses 3
// and 6 per dimension) and gives no rule for the leaf size.  Both trade
// accuracy against time in ways that depend on the geometry and the chip:
// p sets the far-field error and the M2L/P2M cost, the leaf size the split
// between the near field (P2P, grows with the leaf) and the far field (tree
// depth, list lengths).  The tuner measures both on the geometry at hand:
// for each leaf size it walks p upwards until the product's error against
// the exact product meets the target -- a larger p would only be slower --
// times that configuration, and keeps the fastest.  The test vector is a
// uniform opening: smooth like the DDs of loaded fractures, so the error
// is the far field's, as it is for a solution (the near field is exact).
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <vector>

namespace fmddm {
namespace {

struct Stream {
    hipStream_t s = nullptr;
    ~Stream() { if (s) (void)hipStreamDestroy(s); }
};

struct Ctx {
    fmddm_ctx *c = nullptr;
    ~Ctx() { if (c) fmddm_destroy(c); }
};

struct Tree {
    fmddm_tree *t = nullptr;
    ~Tree() { if (t) fmddm_tree_free(t); }
};

void check(fmddm_status st, fmddm_ctx *c, const char *what)
{
    if (st != FMDDM_OK)
        throw Error{st, std::string(what) + (c ? std::string(": ") + fmddm_last_error(c) : std::string())};
}

}  // namespace
}  // namespace fmddm

using namespace fmddm;

extern "C" fmddm_status fmddm_autotune(const fmddm_params *base, int64_t n, const double *x1, const double *y1,
                                       const double *x2, const double *y2, const int32_t *leaves,
                                       int32_t nleaves, const int32_t *ps, int32_t nps, double target_err,
                                       int32_t reps, fmddm_params *best, fmddm_tune_entry *log,
                                       int32_t log_cap, int32_t *nlog)
{
    if (!base || !x1 || !y1 || !x2 || !y2 || !leaves || !ps || !best || n < 1 || nleaves < 1 || nps < 1 ||
        !(target_err > 0.0) || reps < 1 || log_cap < 0 || (log_cap > 0 && !log))
        return FMDDM_EINVAL;
    for (int i = 0; i < nleaves; ++i)
        if (leaves[i] < 1) return FMDDM_EINVAL;
    for (int i = 0; i < nps; ++i)
        if (ps[i] < 1 || ps[i] > MAXP) return FMDDM_EINVAL;
    if (nlog) *nlog = 0;
    try {
        std::vector<int> P(ps, ps + nps);
        std::sort(P.begin(), P.end());
        P.erase(std::unique(P.begin(), P.end()), P.end());
        Stream st;
        FM_HIP(hipStreamCreateWithFlags(&st.s, hipStreamNonBlocking));
        // uniform opening and its exact product, once
        std::vector<double> hD(2 * n);
        for (int64_t i = 0; i < n; ++i) {
            hD[2 * i] = 0.0;
            hD[2 * i + 1] = 1e-3;
        }
        DBuf<double> dD, dy, dex;
        dD.alloc(2 * n);
        dy.alloc(2 * n);
        dex.alloc(2 * n);
        FM_HIP(hipMemcpyAsync(dD.p, hD.data(), 16 * n, hipMemcpyHostToDevice, st.s));
        std::vector<double> ex(2 * n), y(2 * n);
        {
            Ctx c;
            fmddm_params q = *base;
            q.leaf = leaves[0];
            q.p = P[0];
            check(fmddm_create(&q, st.s, &c.c), nullptr, "autotune: parameters");
            Tree t;
            check(fmddm_build_tree(c.c, n, x1, y1, x2, y2, 0, &t.t), c.c, "autotune: tree");
            check(fmddm_apply(c.c, t.t, FMDDM_APPLY_DIRECT, dD.p, dex.p), c.c, "autotune: exact product");
            FM_HIP(hipMemcpyAsync(ex.data(), dex.p, 16 * n, hipMemcpyDeviceToHost, st.s));
            FM_HIP(hipStreamSynchronize(st.s));
        }
        double exn = 0.0;
        for (double v : ex) exn += v * v;
        exn = std::max(std::sqrt(exn), 1e-300);
        // operator sets shared per p across leaf sizes
        std::map<int, std::unique_ptr<Ctx>> opsets;
        hipEvent_t e0, e1;
        FM_HIP(hipEventCreate(&e0));
        FM_HIP(hipEventCreate(&e1));
        struct Ev {
            hipEvent_t a, b;
            ~Ev() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
        } evs{e0, e1};
        int count = 0;
        double best_ms = INFINITY, best_err = INFINITY;
        fmddm_params bestp = *base, accp = *base;
        bool met = false;
        for (int li = 0; li < nleaves; ++li) {
            for (int p : P) {
                fmddm_params q = *base;
                q.leaf = leaves[li];
                q.p = p;
                Ctx c;
                check(fmddm_create(&q, st.s, &c.c), nullptr, "autotune: parameters");
                auto &os = opsets[p];
                if (!os) {
                    os.reset(new Ctx);
                    check(fmddm_create(&q, st.s, &os->c), nullptr, "autotune: parameters");
                }
                c.c->cheb = os->c->cheb;
                c.c->m2l = os->c->m2l;
                Tree t;
                check(fmddm_build_tree(c.c, n, x1, y1, x2, y2, 0, &t.t), c.c, "autotune: tree");
                check(fmddm_apply(c.c, t.t, FMDDM_APPLY_FMM, dD.p, dy.p), c.c, "autotune: product");
                FM_HIP(hipMemcpyAsync(y.data(), dy.p, 16 * n, hipMemcpyDeviceToHost, st.s));
                FM_HIP(hipStreamSynchronize(st.s));
                double err = 0.0;
                for (int64_t i = 0; i < 2 * n; ++i) err += (y[i] - ex[i]) * (y[i] - ex[i]);
                err = std::sqrt(err) / exn;
                double ms = -1.0;
                bool ok = err <= target_err;
                if (ok) {
                    check(fmddm_apply(c.c, t.t, FMDDM_APPLY_FMM, dD.p, dy.p), c.c, "autotune: product");
                    FM_HIP(hipEventRecord(e0, st.s));
                    for (int k = 0; k < reps; ++k)
                        check(fmddm_apply(c.c, t.t, FMDDM_APPLY_FMM, dD.p, dy.p), c.c, "autotune: product");
                    FM_HIP(hipEventRecord(e1, st.s));
                    FM_HIP(hipEventSynchronize(e1));
                    float t_ms = 0.f;
                    FM_HIP(hipEventElapsedTime(&t_ms, e0, e1));
                    ms = t_ms / reps;
                    if (ms < best_ms) {
                        best_ms = ms;
                        bestp = q;
                        met = true;
                    }
                }
                if (err < best_err) {
                    best_err = err;
                    accp = q;
                }
                if (count < log_cap) log[count] = fmddm_tune_entry{q.leaf, q.p, ms, err, q.m2l_tiles};
                ++count;
                if (ok) break;  // a larger p only costs more
            }
        }
        if (met) {
            // M2L tile sets on the chosen configuration (the error does not
            // depend on them beyond rounding)
            double best_err_m = 0.0;
            for (int i = 0; i < count && i < log_cap; ++i)
                if (log[i].leaf == bestp.leaf && log[i].p == bestp.p && log[i].ms >= 0) best_err_m = log[i].err;
            Ctx c;
            fmddm_params q = bestp;
            check(fmddm_create(&q, st.s, &c.c), nullptr, "autotune: parameters");
            c.c->cheb = opsets[q.p]->c->cheb;
            c.c->m2l = opsets[q.p]->c->m2l;
            Tree t;
            check(fmddm_build_tree(c.c, n, x1, y1, x2, y2, 0, &t.t), c.c, "autotune: tree");
            double best_t = INFINITY;
            for (int ts = 0; ts < 4; ++ts) {
                c.c->prm.m2l_tiles = ts;
                check(fmddm_apply(c.c, t.t, FMDDM_APPLY_FMM, dD.p, dy.p), c.c, "autotune: product");
                FM_HIP(hipEventRecord(e0, st.s));
                for (int k = 0; k < reps; ++k)
                    check(fmddm_apply(c.c, t.t, FMDDM_APPLY_FMM, dD.p, dy.p), c.c, "autotune: product");
                FM_HIP(hipEventRecord(e1, st.s));
                FM_HIP(hipEventSynchronize(e1));
                float t_ms = 0.f;
                FM_HIP(hipEventElapsedTime(&t_ms, e0, e1));
                double ms = t_ms / reps;
                if (count < log_cap) log[count] = fmddm_tune_entry{q.leaf, q.p, ms, best_err_m, ts};
                ++count;
                if (ms < best_t) {
                    best_t = ms;
                    bestp.m2l_tiles = ts;
                }
            }
        }
        if (nlog) *nlog = count;
        *best = met ? bestp : accp;
        return met ? FMDDM_OK : FMDDM_ENOTCONV;
    } catch (const Error &e) {
        return e.code;
    } catch (...) {
        return FMDDM_EDEVICE;
    }
}
