// Serving engine: many fracture solves of different sizes on one device,
// batched continuously.
//
// A request is the problem of Section 4 for its own geometry (tree, right-
// hand side, GMRES with FMM products), repeated over `steps` steps, each
// warm-started from the previous DDs.  Elastic servers ramp the fluid
// pressure linearly over the steps (quasi-static load steps).  A server
// given a poroelastic medium (fmddm_server_set_poro) marches in time
// instead (Section 2, eqs. 2.3-2.5): step h solves F(dt) D^h = b - sum over
// k < h of K_{h-k} D^k with the multipole form on both the product and the
// history sum.
//
// The engine keeps up to max_slots requests admitted.  Each slot owns a
// context with its own pair of streams (default priority) and shares the
// M2L operators and Chebyshev tables built once for the server.  One engine
// step polls every slot's last enqueued work without blocking and enqueues
// its next unit (a GMRES residual or Arnoldi step), so the kernels of
// different requests run side by side on the device; then it admits at
// most one queued request if a slot is free and its footprint estimate
// fits the memory budget (first come, first served).  An admitted
// request's set-up (tree, schedules, operators, near blocks,
// preconditioner), which waits on its stream several times, runs on a host
// thread of its own, so the other slots keep receiving work meanwhile.  A
// request's buffers are its own and every kernel is deterministic, so its
// result does not depend on what runs beside it.
#include "internal.h"

#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <future>
#include <unordered_map>

using fmddm::DBuf;
using fmddm::Error;

namespace {

struct Req {
    fmddm_request r{};
    std::vector<double> geo;  // x1 | y1 | x2 | y2 | pf, n each
    std::vector<double> D;    // result, caller order
    fmddm_result res{};
};

struct Slot {
    fmddm_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    int64_t req = 0;          // 0: free
    int phase = 0;            // 1 solving, 2 copying the result out, 3 setting up (host thread)
    std::future<void> setup;  // the set-up of phase 3
    int step = 0;
    fmddm_tree *t = nullptr;
    DBuf<double> pf, b, x;
    DBuf<double> b0, hist;    // poroelastic: right-hand side, DDs of the steps so far
    fmddm::GmresRun g;
    double *hostD = nullptr;  // pinned
    size_t host_cap = 0;
    hipEvent_t ev = nullptr;
    int64_t charged = 0;
    int mode = FMDDM_APPLY_FMM;  // product of the current request
};

double seconds_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct fmddm_server {
    fmddm_params prm{};
    fmddm_poro_params poro{};  // poroelastic medium (poro_set)
    int poro_set = 0;
    int max_slots = 0;
    int64_t budget = 0, used = 0;
    int device = 0;
    std::string err;
    fmddm_ctx *base = nullptr;  // owns the shared operator sets
    hipStream_t base_stream = nullptr;
    std::unordered_map<int64_t, Req> reqs;
    std::deque<int64_t> queue;
    int64_t next = 1;
    std::deque<Slot> slots;  // never relocated: slots hold device buffers
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    ~fmddm_server();
};

fmddm_server::~fmddm_server()
{
    for (Slot &s : slots)
        if (s.setup.valid()) s.setup.wait();  // set-ups still running
    (void)hipSetDevice(device);
    (void)hipDeviceSynchronize();
    for (Slot &s : slots) {
        delete s.t;
        s.pf.reset();
        s.b.reset();
        s.x.reset();
        s.b0.reset();
        s.hist.reset();
        if (s.hostD) (void)hipHostFree(s.hostD);
        if (s.ev) (void)hipEventDestroy(s.ev);
        delete s.ctx;
        if (s.stream) {
            fmddm::dev_stream_idle(s.stream);
            (void)hipStreamDestroy(s.stream);
        }
    }
    delete base;
    if (base_stream) {
        fmddm::dev_stream_idle(base_stream);
        (void)hipStreamDestroy(base_stream);
    }
}

namespace {

// Footprint estimate of a request of n elements: per element the geometry
// copies, keys and permutation, near-field partials, the P2M matrices and
// the vectors of GMRES(m); per cell (at most 4n/leaf cells) the weight and
// field vectors, their compressed forms, split-K partials, the M2L pair
// results (up to 27 interaction pairs per cell) and the upward-pass
// partials; with block-Jacobi preconditioning the group inverses (at most
// (2 x 32)^2 doubles per 32 elements) and one more vector, with the two-level
// one also the coarse inverse.  Sizes are
// rounded up by the allocator, hence the final 25 %.
int64_t footprint(const fmddm_params &p, int rank_pad, int64_t n, int steps = 0, int64_t near_cap = 0)
{
    const int64_t M = 3LL * p.p * p.p, Mp = (M + 63) / 64 * 64;
    const int64_t rp = p.m2l == FMDDM_M2L_SVD ? rank_pad : Mp;
    const int64_t cells = 4 * n / std::max(1, p.leaf) + 64;
    int64_t per_elem = 8LL * p.p * p.p + 8 * 2 * (p.restart + 4) + 8 * 48;
    if (p.precond != FMDDM_PRECOND_NONE) per_elem += 8 * 128 + 8 * 2 + 16;
    int64_t per_cell = 8 * (3 * Mp + 2 * rp + 4 * rp + 27 * rp) + 4 * 64;
    if (p.precision != FMDDM_PREC_FP64) per_cell += 4 * (2 * rp + 4 * rp + 27 * rp);  // FP32 intermediates
    int64_t b = n * per_elem + cells * per_cell + (4 << 20);
    if (p.precond == FMDDM_PRECOND_TWO_LEVEL) {  // coarse inverse: at most 2048 aggregates, else left out
        const int64_t nc = std::min<int64_t>(n, 2048);
        b += 8 * (2 * nc) * (2 * nc) + 8 * 6 * nc;
    }
    if (steps > 0) {
        // poroelastic march of `steps` steps (3 unknowns, 4 charges): the
        // Krylov basis and vectors at 3n, the step history and its terms,
        // per time level the four-charge weights and sources; per cell the
        // fields, pair products and far stress; the M2L operators per
        // (level, offset) combination and time level (at most 40 offsets on
        // each of ~log4(n) + 4 levels); the near blocks (96 B per near pair
        // and level, capped by the near-field budget)
        const int64_t Mq = (4LL * p.p * p.p + 63) / 64 * 64;
        const int64_t H = steps, levels = 4 + (int64_t)std::ceil(std::log((double)cells) / std::log(4.0));
        b += n * 8 * (3 * (p.restart + 6) + 6 * H + 7 * H + 4 * levels) + cells * 8 * (2 * Mq + 27 * Mq + H * Mq);
        b += 40 * levels * Mq * Mq * 8 * (H + 1);
        if (p.precond != FMDDM_PRECOND_NONE) b += n * 8 * 3 * 3 * 21;  // 3 x 3 blocks of 21-element groups
        b += std::min<int64_t>(near_cap, 96LL * n * 64 * 4 * (H + 1));
    }
    return b + b / 4;
}

void check_request(const fmddm_request *r)
{
    if (!r || r->n <= 0 || !r->x1 || !r->y1 || !r->x2 || !r->y2 || !r->pf)
        throw Error{FMDDM_EINVAL, "request: empty geometry or null pointer"};
    if (r->steps < 1) throw Error{FMDDM_EINVAL, "request: steps must be >= 1"};
    if (!(r->tol > 0.0 && r->tol < 1.0)) throw Error{FMDDM_EINVAL, "request: tol must be in (0, 1)"};
    if (!std::isfinite(r->SH) || !std::isfinite(r->Sh)) throw Error{FMDDM_EINVAL, "request: non-finite stress"};
}

fmddm_ctx *slot_context(fmddm_server *s, hipStream_t st)
{
    fmddm_ctx *c = new fmddm_ctx();
    c->prm = s->prm;
    c->stream = st;
    c->device = s->device;
    c->gc = s->base->gc;
    c->cheb = s->base->cheb;
    c->m2l = s->base->m2l;
    c->pcache = s->base->pcache;
    fmddm::init_streams(c);
    return c;
}

void retire(fmddm_server *s, Slot &sl)
{
    delete sl.t;  // its work has completed: the slot's event was observed
    sl.t = nullptr;
    s->used -= sl.charged;
    sl.charged = 0;
    sl.req = 0;
    sl.phase = 0;
}

void fail(fmddm_server *s, Slot &sl, fmddm_status st)
{
    Req &q = s->reqs[sl.req];
    q.res.state = FMDDM_REQ_FAILED;
    q.res.status = st;
    q.res.t_done = seconds_since(s->t0);
    (void)hipStreamSynchronize(sl.stream);
    retire(s, sl);
}

// Reduced-precision FMM products: Arnoldi on them, residuals and the
// stopping test with the FP64 product (as fmddm_solve)
int residual_mode(const fmddm_server *s, const Slot &sl)
{
    return sl.mode == FMDDM_APPLY_FMM && s->prm.precision != FMDDM_PREC_FP64 ? fmddm::APPLY_FMM_FP64 : -1;
}

int64_t request_footprint(const fmddm_server *s, const fmddm_request &r)
{
    return s->poro_set ? footprint(s->prm, s->base->m2l->rp, r.n, r.steps, s->poro.near_cache_bytes)
                       : footprint(s->prm, s->base->m2l->rp, r.n);
}

// The set-up of an admitted request: tree, schedules and operators,
// right-hand side, preconditioner and the start of its first solve.  It
// runs on a host thread of its own (admit), on the slot's context and
// stream only, while the engine keeps stepping the other slots; it waits
// on nothing but its own stream.  r and g are copies / stable storage of
// the request.
void admit_work(fmddm_server *s, Slot &sl, const fmddm_request r, const double *g)
{
    FM_HIP(hipSetDevice(s->device));
    fmddm::StreamScope scope(sl.stream);
    const int64_t n = r.n;
    sl.t = new fmddm_tree();
    if (s->poro_set && s->poro.m2l == FMDDM_M2L_SVD && n > 0) {
        // a root square of power-of-two side, centred on the midpoints'
        // bounding box: the cell sizes of all requests of one scale then
        // coincide, and so do their compressed left-hand-side operators,
        // built once per cell size and shared by the slots
        double x0 = HUGE_VAL, x1 = -HUGE_VAL, y0 = HUGE_VAL, y1 = -HUGE_VAL;
        for (int64_t i = 0; i < n; ++i) {
            const double cx = 0.5 * (g[i] + g[2 * n + i]), cy = 0.5 * (g[n + i] + g[3 * n + i]);
            x0 = std::min(x0, cx);
            x1 = std::max(x1, cx);
            y0 = std::min(y0, cy);
            y1 = std::max(y1, cy);
        }
        const double ext = std::max(std::max(x1 - x0, y1 - y0), 1e-300);
        const double L = std::exp2(std::ceil(std::log2(ext * 1.0001)));
        sl.ctx->prm.use_root_box = 1;
        sl.ctx->prm.root_L = L;
        sl.ctx->prm.root_x0 = x0 - 0.5 * (L - (x1 - x0));
        sl.ctx->prm.root_y0 = y0 - 0.5 * (L - (y1 - y0));
    } else {
        sl.ctx->prm.use_root_box = s->base->prm.use_root_box;
        sl.ctx->prm.root_L = s->base->prm.root_L;
        sl.ctx->prm.root_x0 = s->base->prm.root_x0;
        sl.ctx->prm.root_y0 = s->base->prm.root_y0;
    }
    fmddm::build_tree(sl.ctx, sl.t, n, g, g + n, g + 2 * n, g + 3 * n, 0);
    if (s->poro_set) {
        // time march: the multipole form throughout (exact transient
        // integration is far slower at every size); operators and near
        // blocks of all its time levels built now
        const int64_t n3 = 3 * n;
        sl.mode = fmddm::APPLY_PORO;
        fmddm::poro_prepare(sl.ctx, sl.t, r.steps);
        if (sl.pf.n < (size_t)n) sl.pf.alloc(n);
        if (sl.b.n < (size_t)n3) sl.b.alloc(n3);
        if (sl.x.n < (size_t)n3) sl.x.alloc(n3);
        if (sl.b0.n < (size_t)n3) sl.b0.alloc(n3);
        if (sl.hist.n < (size_t)(n3 * r.steps)) sl.hist.alloc(n3 * r.steps);
        FM_HIP(hipMemcpyAsync(sl.pf.p, g + 4 * n, n * 8, hipMemcpyHostToDevice, sl.stream));
        FM_HIP(hipMemsetAsync(sl.x.p, 0, n3 * 8, sl.stream));
        fmddm::poro_rhs(sl.ctx, sl.t, sl.pf.p, r.SH, r.Sh, sl.b0.p);
        FM_HIP(hipMemcpyAsync(sl.b.p, sl.b0.p, n3 * 8, hipMemcpyDeviceToDevice, sl.stream));
        sl.g.start(sl.ctx, sl.t, sl.mode, sl.b.p, sl.x.p, r.tol, s->prm.maxit);
        return;
    }
    // small requests: the exact product, one launch, beats the FMM's chain
    sl.mode = n <= s->prm.direct_below ? FMDDM_APPLY_DIRECT : FMDDM_APPLY_FMM;
    if (sl.mode == FMDDM_APPLY_FMM) fmddm::setup_fmm(sl.ctx, sl.t);
    if (sl.pf.n < (size_t)n) sl.pf.alloc(n);
    if (sl.b.n < (size_t)(2 * n)) sl.b.alloc(2 * n);
    if (sl.x.n < (size_t)(2 * n)) sl.x.alloc(2 * n);
    FM_HIP(hipMemcpyAsync(sl.pf.p, g + 4 * n, n * 8, hipMemcpyHostToDevice, sl.stream));
    FM_HIP(hipMemsetAsync(sl.x.p, 0, 2 * n * 8, sl.stream));
    fmddm::rhs_build(sl.ctx, sl.t, sl.pf.p, r.SH, r.Sh, sl.b.p, 1.0 / r.steps);
    sl.g.start(sl.ctx, sl.t, sl.mode, sl.b.p, sl.x.p, r.tol, s->prm.maxit, residual_mode(s, sl));
}

// Admits request `id` into the free slot: charges its footprint and starts
// its set-up on a host thread (phase 3); the engine moves the slot to
// solving once the set-up has finished.
void admit(fmddm_server *s, Slot &sl, int64_t id)
{
    Req &q = s->reqs[id];
    sl.req = id;
    sl.step = 0;
    sl.charged = q.res.device_bytes = request_footprint(s, q.r);
    s->used += sl.charged;
    q.res.state = FMDDM_REQ_RUNNING;
    q.res.t_admit = seconds_since(s->t0);
    const fmddm_request r = q.r;
    const double *g = q.geo.data();  // not modified while the request exists
    Slot *ps = &sl;
    sl.setup = std::async(std::launch::async, [s, ps, r, g] {
        try {
            admit_work(s, *ps, r, g);
        } catch (const Error &) {
            throw;
        } catch (const std::bad_alloc &) {
            throw Error{FMDDM_ENOMEM, "request set-up: host allocation failed"};
        } catch (...) {
            throw Error{FMDDM_EDEVICE, "request set-up failed"};
        }
    });
    sl.phase = 3;
}

// Moves one slot forward if its last enqueued work has finished.
void advance(fmddm_server *s, Slot &sl)
{
    Req &q = s->reqs[sl.req];
    const int64_t n = q.r.n;
    if (sl.phase == 3) {
        if (sl.setup.wait_for(std::chrono::seconds(0)) != std::future_status::ready) return;
        sl.phase = 1;
        sl.setup.get();  // the set-up's error, if any, fails the request
        return;
    }
    if (sl.phase == 1) {
        if (!sl.g.advance(false)) return;
        q.res.iters += sl.g.it;
        q.res.relres = sl.g.relres;
        if (!sl.g.converged) {
            fail(s, sl, FMDDM_ENOTCONV);
            return;
        }
        q.res.steps_done = ++sl.step;
        const int64_t nv = (s->poro_set ? 3 : 2) * n;
        if (s->poro_set) {
            // D^h joins the history; the next step's right-hand side is b
            // minus the history sum over D^1 .. D^h
            FM_HIP(hipMemcpyAsync(sl.hist.p + (size_t)(sl.step - 1) * nv, sl.x.p, nv * 8, hipMemcpyDeviceToDevice,
                                  sl.stream));
            if (sl.step < q.r.steps) {
                FM_HIP(hipMemcpyAsync(sl.b.p, sl.b0.p, nv * 8, hipMemcpyDeviceToDevice, sl.stream));
                fmddm::poro_history(sl.ctx, sl.t, sl.step + 1, sl.hist.p, sl.b.p);
                sl.g.start(sl.ctx, sl.t, sl.mode, sl.b.p, sl.x.p, q.r.tol, s->prm.maxit);
                return;
            }
        } else if (sl.step < q.r.steps) {
            double scale = (double)(sl.step + 1) / q.r.steps;
            fmddm::rhs_build(sl.ctx, sl.t, sl.pf.p, q.r.SH, q.r.Sh, sl.b.p, scale);
            sl.g.start(sl.ctx, sl.t, sl.mode, sl.b.p, sl.x.p, q.r.tol, s->prm.maxit, residual_mode(s, sl));
            return;
        }
        size_t need = (size_t)nv * 8;
        if (sl.host_cap < need) {
            if (sl.hostD) FM_HIP(hipHostFree(sl.hostD));
            sl.hostD = nullptr;
            FM_HIP(hipHostMalloc((void **)&sl.hostD, need, hipHostMallocDefault));
            sl.host_cap = need;
        }
        FM_HIP(hipMemcpyAsync(sl.hostD, sl.x.p, need, hipMemcpyDeviceToHost, sl.stream));
        FM_HIP(hipEventRecord(sl.ev, sl.stream));
        sl.phase = 2;
        return;
    }
    if (sl.phase == 2) {
        hipError_t e = hipEventQuery(sl.ev);
        if (e == hipErrorNotReady) return;
        FM_HIP(e);
        q.D.assign(sl.hostD, sl.hostD + (s->poro_set ? 3 : 2) * n);
        q.res.state = FMDDM_REQ_DONE;
        q.res.status = FMDDM_OK;
        q.res.t_done = seconds_since(s->t0);
        retire(s, sl);
    }
}

template <class F>
fmddm_status sguard(fmddm_server *s, F &&f)
{
    try {
        (void)hipSetDevice(s->device);
        return f();
    } catch (const Error &e) {
        s->err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        s->err = "host allocation failed";
        return FMDDM_ENOMEM;
    }
}

}  // namespace

extern "C" {

fmddm_status fmddm_server_create(const fmddm_params *p, int max_slots, int64_t hbm_budget, fmddm_server **out)
{
    if (!out) return FMDDM_EINVAL;
    *out = nullptr;
    if (!p || max_slots < 1 || max_slots > 64 || hbm_budget < 0) return FMDDM_EINVAL;
    fmddm_server *s = new (std::nothrow) fmddm_server();
    if (!s) return FMDDM_ENOMEM;
    s->prm = *p;
    s->max_slots = max_slots;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return FMDDM_EDEVICE;
    }
    fmddm_status st = sguard(s, [&] {
        FM_HIP(hipStreamCreateWithFlags(&s->base_stream, hipStreamNonBlocking));
        fmddm_ctx *b = nullptr;
        fmddm_status cs = fmddm_create(p, s->base_stream, &b);
        if (cs != FMDDM_OK) throw Error{cs, "server: invalid parameters"};
        s->base = b;
        fmddm::StreamScope scope(s->base_stream);
        fmddm::build_m2l_ops(b);
        // the slots share the operator set and set up on host threads of
        // their own: its reduced-precision copy is made here, not on use
        if (p->precision != FMDDM_PREC_FP64) fmddm::lowp_ops(b, p->precision);
        if (hbm_budget == 0) {
            // free device memory, counting the blocks the library's cache
            // holds for reuse (earlier servers' requests leave them there)
            size_t fr = 0, tot = 0;
            FM_HIP(hipMemGetInfo(&fr, &tot));
            hbm_budget = (int64_t)(0.9 * (double)(fr + fmddm::dev_bytes(true)));
        }
        s->budget = hbm_budget;
        s->slots.resize(max_slots);
        for (Slot &sl : s->slots) {
            FM_HIP(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
            FM_HIP(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
            sl.ctx = slot_context(s, sl.stream);
        }
        return FMDDM_OK;
    });
    if (st != FMDDM_OK) {
        delete s;
        return st;
    }
    *out = s;
    return FMDDM_OK;
}

fmddm_status fmddm_server_set_poro(fmddm_server *s, const fmddm_poro_params *pp)
{
    if (!s || !pp) return FMDDM_EINVAL;
    return sguard(s, [&] {
        if (!s->queue.empty()) throw Error{FMDDM_EINVAL, "server_set_poro: requests are queued"};
        for (Slot &sl : s->slots)
            if (sl.req) throw Error{FMDDM_EINVAL, "server_set_poro: requests are running"};
        if (pp->mode != FMDDM_APPLY_FMM) throw Error{FMDDM_EUNSUPPORTED, "server_set_poro: mode must be FMM"};
        fmddm_poro_params q = *pp;
        if (q.near_cache_bytes == 0) {
            // stored near blocks: a share of the budget per slot
            q.near_cache_bytes = std::max<int64_t>(1, s->budget / (4 * (int64_t)s->slots.size()));
        }
        fmddm_status st = fmddm_poro_set(s->base, &q);
        if (st != FMDDM_OK) throw Error{st, std::string("server_set_poro: ") + fmddm_last_error(s->base)};
        for (Slot &sl : s->slots) {
            st = fmddm_poro_set(sl.ctx, &q);
            if (st != FMDDM_OK) throw Error{st, std::string("server_set_poro: ") + fmddm_last_error(sl.ctx)};
        }
        s->poro = q;
        s->poro_set = 1;
        return FMDDM_OK;
    });
}

void fmddm_server_destroy(fmddm_server *s) { delete s; }

const char *fmddm_server_last_error(const fmddm_server *s) { return s ? s->err.c_str() : "null server"; }

int64_t fmddm_server_footprint(const fmddm_server *s, int64_t n)
{
    if (!s || n <= 0) return 0;
    // poroelastic servers: a march of the longest length requests use here
    return s->poro_set ? footprint(s->prm, s->base->m2l->rp, n, 10, s->poro.near_cache_bytes)
                       : footprint(s->prm, s->base->m2l->rp, n);
}

fmddm_status fmddm_server_submit(fmddm_server *s, const fmddm_request *r, int64_t *ticket)
{
    if (!s || !ticket) return FMDDM_EINVAL;
    return sguard(s, [&] {
        check_request(r);
        int64_t id = s->next++;
        Req &q = s->reqs[id];
        q.r = *r;
        const int64_t n = r->n;
        q.geo.resize(5 * n);
        std::memcpy(q.geo.data(), r->x1, n * 8);
        std::memcpy(q.geo.data() + n, r->y1, n * 8);
        std::memcpy(q.geo.data() + 2 * n, r->x2, n * 8);
        std::memcpy(q.geo.data() + 3 * n, r->y2, n * 8);
        std::memcpy(q.geo.data() + 4 * n, r->pf, n * 8);
        q.r.x1 = q.r.y1 = q.r.x2 = q.r.y2 = q.r.pf = nullptr;
        q.res.state = FMDDM_REQ_QUEUED;
        q.res.t_submit = seconds_since(s->t0);
        s->queue.push_back(id);
        *ticket = id;
        return FMDDM_OK;
    });
}

fmddm_status fmddm_server_step(fmddm_server *s, int *active, int *queued)
{
    if (!s) return FMDDM_EINVAL;
    return sguard(s, [&] {
        for (Slot &sl : s->slots) {
            if (!sl.req) continue;
            fmddm::StreamScope scope(sl.stream);
            try {
                advance(s, sl);
            } catch (const Error &e) {
                s->err = e.msg;
                fail(s, sl, e.code);
            }
        }
        // admission: first come, first served
        while (!s->queue.empty()) {
            Slot *free_slot = nullptr;
            int busy = 0;
            for (Slot &sl : s->slots) {
                if (sl.req) ++busy;
                else if (!free_slot) free_slot = &sl;
            }
            if (!free_slot) break;
            int64_t id = s->queue.front();
            Req &q = s->reqs[id];
            int64_t est = request_footprint(s, q.r);
            if (est > s->budget) {
                s->queue.pop_front();
                q.res.state = FMDDM_REQ_FAILED;
                q.res.status = FMDDM_ENOMEM;
                q.res.t_done = seconds_since(s->t0);
                continue;
            }
            if (s->used + est > s->budget && busy > 0) break;
            s->queue.pop_front();
            fmddm::StreamScope scope(free_slot->stream);
            try {
                admit(s, *free_slot, id);
            } catch (const Error &e) {
                s->err = e.msg;
                fail(s, *free_slot, e.code);
            }
            break;  // at most one admission per step
        }
        int a = 0;
        for (Slot &sl : s->slots) a += sl.req != 0;
        if (active) *active = a;
        if (queued) *queued = (int)s->queue.size();
        return FMDDM_OK;
    });
}

fmddm_status fmddm_server_poll(fmddm_server *s, int64_t ticket, fmddm_result *res, double *D)
{
    if (!s || !res) return FMDDM_EINVAL;
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) {
        s->err = "unknown ticket";
        return FMDDM_EINVAL;
    }
    *res = it->second.res;
    if (D && it->second.res.state == FMDDM_REQ_DONE)
        std::memcpy(D, it->second.D.data(), it->second.D.size() * 8);
    return FMDDM_OK;
}

fmddm_status fmddm_server_release(fmddm_server *s, int64_t ticket)
{
    if (!s) return FMDDM_EINVAL;
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end() || it->second.res.state < FMDDM_REQ_DONE) {
        s->err = "release: unknown or unfinished ticket";
        return FMDDM_EINVAL;
    }
    s->reqs.erase(it);
    return FMDDM_OK;
}

}  // extern "C"
