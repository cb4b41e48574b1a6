// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <new>
#include <string>
#include <map>
#include <mutex>
#include <type_traits>
#include <vector>

#include "../../include/fmddm.h"

namespace fmddm {

// ---------------------------------------------------------------- errors
struct Error {
    fmddm_status code;
    std::string msg;
};

#define FM_HIP(call)                                                             \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess)                                                    \
            throw ::fmddm::Error{e_ == hipErrorOutOfMemory ? FMDDM_ENOMEM        \
                                                           : FMDDM_EDEVICE,      \
                                 std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define FM_CHECK_LAUNCH() FM_HIP(hipGetLastError())

// ------------------------------------------------------- device buffers
// alloc.hip: caching device allocator; sizes are rounded up and *rounded
// receives the block size that dev_release takes back
void *dev_alloc(size_t bytes, size_t *rounded, bool fp = false);
void dev_release(void *p, size_t rounded);
size_t dev_cache_trim();
size_t dev_bytes(bool cached);
// The work enqueued on s so far has completed (the caller synchronized it):
// the blocks released under a scope on s become idle.  Called before a
// stream is destroyed, and when a context lets go of its stream.
void dev_stream_idle(hipStream_t s);

// The stream whose work uses the buffers that this host thread allocates
// and releases, for the duration of a scope (an entry point on a context,
// a serving slot's set-up or step).  A block released inside the scope is
// handed to allocations on the same stream at once (stream order keeps
// the old work first) and to other streams only once the work enqueued on
// it before the release has completed.  Outside every scope a released
// block is taken to be idle.
class StreamScope {
  public:
    explicit StreamScope(hipStream_t s);
    ~StreamScope();
    StreamScope(const StreamScope &) = delete;
    StreamScope &operator=(const StreamScope &) = delete;

  private:
    hipStream_t prev_;
    bool prev_set_;
};

// Owning device allocation from the cache, returned to it in the destructor.
template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    size_t cap = 0;  // bytes of the cached block
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { reset(); }
    void reset() {
        if (p) dev_release(p, cap);
        p = nullptr;
        n = 0;
        cap = 0;
    }
    void alloc(size_t count) {
        reset();
        if (count == 0) count = 1;
        p = (T *)dev_alloc(count * sizeof(T), &cap, std::is_floating_point<T>::value);
        n = count;
    }
    void zero(hipStream_t s) { FM_HIP(hipMemsetAsync(p, 0, n * sizeof(T), s)); }
    size_t bytes() const { return n * sizeof(T); }
};

constexpr int MAXP = 32;
constexpr int NEAR_CHUNK = 256;  // sources per near-field work item

// ------------------------------------------------------------- context
struct Cheb {
    int p = 0;
    DBuf<double> tnode;     // [l][k] = T_k(xbar_l), p x p
    DBuf<double> xbar;      // p nodes
    DBuf<double> gl_t, gl_w;  // p-point Gauss-Legendre
    DBuf<double> bw;        // barycentric weights of the nodes
    DBuf<double> m2mS;      // child-to-parent transfers S_0, S_1 (eq. 3.7), p x p each, row-major
    std::vector<double> h_xbar, h_tnode, h_glt, h_glw, h_bw, h_m2mS;
};

// Block-Jacobi preconditioner: groups of elements (first tree position,
// count), each with the inverse of its (nc m)^2 block, column-major, at
// inv + off[group]; nc unknowns per element (2 elastic, 3 poroelastic).
// key: the parameters the blocks were built for (poroelastic medium, dt).
struct PcBlocks {
    int nblk = 0, nc = 0;
    DBuf<int> beg, cnt;
    DBuf<int64_t> off;
    DBuf<double> inv;
    double key[6] = {0, 0, 0, 0, 0, 0};
};

// Coarse level of the two-level preconditioner: aggregates of consecutive
// collinear elements (caller order), each taken as one long element; the
// explicit inverse of their coarse matrix R A P (2 nc x 2 nc, row-major,
// traction components from shear/normal DDs).
struct PcCoarse {
    int nc = 0;                // aggregates (0: not built, or left out)
    int off = 0;               // left out: more than a few thousand aggregates
    DBuf<int> abeg;            // first element of each aggregate, nc + 1 entries
    DBuf<double> ainv, rc, yc;
    double key[6] = {0, 0, 0, 0, 0, 0};
};

struct M2LOps {
    int ready = 0;
    int mode = 0;           // fmddm_m2l_mode
    int M = 0;              // 3 p^2
    int Mp = 0;             // expansion stride (3 p^2 padded to a multiple of 64)
    int r = 0;              // retained rank (M when uncompressed)
    int rp = 0;             // operator dimension used by the GEMMs (Mp or r padded to 64)
    DBuf<double> ops;       // 40 offset operators, rp x rp each, row-major
    DBuf<double> Ur;        // compressed mode: Mp x rp, columns = left singular vectors
    DBuf<double> Vt;        // compressed mode: rp x Mp, rows = the same vectors
    std::vector<double> sv; // normalised singular values (compressed mode)
    // reduced-precision copies of ops / Vt / Ur, made on first use
    bool have32 = false, have16 = false;
    DBuf<float> ops32, Vt32, Ur32;
    DBuf<uint16_t> ops16, Vt16, Ur16;   // bf16 bit patterns
};

// One tree level's poroelastic left-hand-side M2L operators in compressed
// form, for all 40 V-list offsets: a cell half-width hw, medium, dt, p and
// cut determine them, so trees whose levels share hw share them.
struct PoroLhsBasis {
    bool ok = false;             // false: the rank is too close to 4p^2 to pay
    int r = 0, rq = 0;           // rank, padded to a multiple of 64
    DBuf<double> Vt, U;          // rq x Mq (row-space vectors as rows), Mq x rq (column-space ones)
    DBuf<double> C;              // 40 x rq x rq, row-major, in v_offsets order
};
struct PoroLhsCache {
    std::mutex mu;
    std::map<std::vector<double>, std::shared_ptr<PoroLhsBasis>> lev;
};

}  // namespace fmddm

namespace fmddm {
// Per-phase HIP-event timing of FMM products.
struct Profiler {
    unsigned mask = 0;
    std::vector<hipEvent_t> pool;                      // free events
    std::vector<std::pair<hipEvent_t, hipEvent_t>> rec[FMDDM_PH_COUNT];
    hipEvent_t take();
    void begin(int ph, hipStream_t s, hipEvent_t &e0);
    void end(int ph, hipStream_t s, hipEvent_t e0);
    void read(hipStream_t s, double *ms, int64_t *count);
    ~Profiler();
};
}  // namespace fmddm

struct fmddm_ctx {
    fmddm_params prm;
    fmddm::Profiler prof;
    hipStream_t stream = nullptr;
    // second stream (default priority) for work independent of the far
    // field, forked from and joined back into `stream` with events
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // idle stream that graphs are captured on (the caller's stream may be
    // the null stream, which cannot capture); graphs launch on `stream`
    hipStream_t cap = nullptr;
    // rocBLAS handle of the coarse-level factorisation, made on first use
    void *blas = nullptr;
    ~fmddm_ctx();
    void release()
    {
        if (cap) (void)hipStreamDestroy(cap);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (side) (void)hipStreamDestroy(side);
    }
    int device = 0;
    std::string err;
    // Chebyshev tables and M2L operators depend only on p, the material and
    // the M2L mode: contexts created by a server share one set
    std::shared_ptr<fmddm::Cheb> cheb;
    std::shared_ptr<fmddm::M2LOps> m2l;
    // compressed poroelastic left-hand-side operators per cell size (shared
    // like the operator set)
    std::shared_ptr<fmddm::PoroLhsCache> pcache;
    fmddm_poro_params poro{};  // poroelastic medium and time step (fmddm_poro_set)
    int poro_set = 0;
    double gc = 0.0;        // G / (2 pi (1 - nu))
};

struct fmddm_tree {
    int64_t n = 0;
    double x0 = 0, y0 = 0, L = 1;
    int ncell = 0, nlevel = 0, nleaf = 0;
    std::vector<int> level_start;     // host: first cell of each level, nlevel+1 entries
    std::vector<int> h_level;         // host copies used for scheduling
    std::vector<int> h_isleaf;
    // elements, caller order
    fmddm::DBuf<double> ocx, ocy, ocb, osb, oa;
    // elements, tree (Morton) order
    fmddm::DBuf<double> scx, scy, scb, ssb, sa;
    fmddm::DBuf<int> perm;            // sorted position -> element
    fmddm::DBuf<uint64_t> key;
    // cells
    fmddm::DBuf<int> clevel, cparent, cchild, cpbeg, cpend, cleaf;
    fmddm::DBuf<uint32_t> cix, ciy;
    fmddm::DBuf<uint64_t> cmk;        // Morton code of (ix, iy) within its level
    fmddm::DBuf<double> ccx, ccy, chw;  // centre, half-width
    // lists (CSR over cells)
    fmddm::DBuf<int> loff[4], lidx[4];
    std::vector<int> h_loff[4];
    // near field: per leaf, source cells whose points act directly
    fmddm::DBuf<int> noff, nsrc;
    fmddm::DBuf<int> nbeg, npre, ntot;  // per near entry: first source, prefix in its leaf; per leaf: total
    fmddm::DBuf<int> nfoff, nflat;      // per leaf: its near source points as one list (offsets, points)
    fmddm::DBuf<int> aoff, aidx;        // per leaf: its ancestors (itself first) at level >= 2
    // near-field work items: a leaf's sources split into chunks of at most
    // NEAR_CHUNK, each item producing partial stresses for the leaf's points
    int nitem = 0;
    int64_t npartial = 0;
    fmddm::DBuf<int> it_leaf, it_s0, it_s1, it_poff, lk_off, tleaf;
    fmddm::DBuf<int64_t> it_coff;  // per item: (target, source) pairs of the items before it
    std::vector<int> leaves;          // host list of leaf cells (tree order)
    fmddm::DBuf<int> dleaves;
    int64_t near_pairs = 0, l2p_pairs = 0, m2m_pairs = 0;
    // M2L schedule: pairs are V-list entries grouped by offset into tiles
    int ntile = 0;
    fmddm::DBuf<int> tile_op, tile_beg, tile_end, pair_src, pair_dst;
    fmddm::DBuf<double> pair_scale;
    int64_t nV = 0;
    // cells at level >= 2 (the only ones with interaction lists), as
    // identity "pairs" for the compress / decompress products
    int nfar = 0, nftile = 0;
    fmddm::DBuf<int> far_cells, ftile_op, ftile_beg, ftile_end;
    // expansions
    fmddm::DBuf<double> p2m_mat;      // per element (tree order): p^2 weights of its anterpolation
    fmddm::DBuf<double> Wexp;         // multipole weights, ncell x Mp
    // upward pass: steps (parent, four children or -1) in m2m_item, grouped
    // into chains (children before parents) and launches; a launch's chain
    // offsets (nchain + 1, from its first step step0) start at m2m_coff +
    // first.  m2m_cut: the level below which each subtree is one chain
    struct M2MLaunch {
        int first = 0, nchain = 0, step0 = 0;
        bool single = false;  // every chain one step: no offsets needed
    };
    std::vector<M2MLaunch> m2m_launch;
    fmddm::DBuf<int> m2m_coff, m2m_item;
    int m2m_cut = 0;
    fmddm::DBuf<double> What;         // compressed weights, ncell x rp
    fmddm::DBuf<double> Zm2l;         // one M2L product per V pair, nV x rp
    fmddm::DBuf<double> Ghat;         // summed compressed M2L fields, ncell x rp
    fmddm::DBuf<double> Gexp;         // M2L field of each cell at its nodes, ncell x Mp
    fmddm::DBuf<double> q;            // charges, tree order, 3 per element
    fmddm::DBuf<double> Dsort;        // D in tree order
    fmddm::DBuf<double> far_s;        // far-field stress per (level >= 2, point), tree order, 3 each
    int nlpitem = 0, nfarlev = 0;     // downward-pass items (far cell, 32 points); levels 2.. in far_s
    fmddm::DBuf<int> lp_cell, lp_p0;
    fmddm::DBuf<double> part_s;       // near-field partial stresses per work item
    fmddm::DBuf<double> ksplit;       // split-K partial products
    // reduced-precision M2L intermediates (FP32), allocated on first use
    fmddm::DBuf<float> What32, Zm2l32, Ghat32, ksplit32;
    // dense operator (built on demand)
    fmddm::DBuf<double> Adense;
    // solver workspace; gm_host is pinned host memory the device writes the
    // residual norm and estimate to, gm_ev marks when they have arrived
    fmddm::DBuf<double> gm_V, gm_w, gm_r, gm_sc, gm_part;
    int gm_restart = 0;
    int64_t gm_len = 0;
    // block-Jacobi preconditioners of the elastic and poroelastic systems
    fmddm::PcBlocks pc, ppc;
    fmddm::PcCoarse pcc, ppcc;  // coarse levels (two-level preconditioning)
    fmddm::DBuf<double> gm_z;          // preconditioned basis vector M^-1 v_j
    // poroelastic workspace: chunk partials, term times, term vectors
    fmddm::DBuf<double> poro_part, poro_times, poro_E;
    // poroelastic FMM: V pairs grouped by (level, offset) "combos", tiles of
    // pairs sharing a combo, operators for time levels dt .. H dt
    int pf_ready = 0, pf_ncombo = 0, pf_ntile = 0, pf_H = 0, pf_p = 0, pf_Mq = 0;
    double pf_dt = 0.0;
    std::vector<int> pf_h_combo_lvl, pf_h_combo_ox, pf_h_combo_oy;
    fmddm::DBuf<int> pf_tile_op, pf_tile_beg, pf_tile_end, pf_psrc, pf_pdst, pf_combo_lvl, pf_combo_ox,
        pf_combo_oy;
    fmddm::DBuf<double> pf_ops, pf_W, pf_Z, pf_G, pf_far, pf_Q, pf_D3, pf_near, pf_D2, pf_o2;
    fmddm::DBuf<double> pf_D3a;  // per-level DDs of a history sum whose far field takes two terms
    double pf_key[8] = {};  // medium the operators were built for
    // poroelastic near field: per time level j (time (j+1) dt), the 4 x 3
    // response blocks of every near (target, source) pair in item order,
    // integrated on first use; pn_ptr holds the levels' device addresses
    std::vector<std::unique_ptr<fmddm::DBuf<double>>> pn_lvl;
    std::vector<double *> pn_hptr;
    fmddm::DBuf<double *> pn_ptr;
    int pn_cap = -1;        // levels that fit the budget (-1: not sized yet)
    // left-hand side F(dt) in one multipole pass: the first level's near
    // blocks and M2L operators with the drained elastic part added
    fmddm::DBuf<double> pn_lhs, pf_ops0;
    fmddm::DBuf<int64_t> pn_close;                 // near pairs within the composite rule's reach
    fmddm::DBuf<unsigned long long> pn_ccount;     // their count
    // the left-hand side's M2L compressed per tree level (poro m2l = SVD):
    // level slot k has row-space basis Vt (rq x Mq), column-space basis U
    // (Mq x rq); each combination's operator becomes C (rq x rq)
    int pc_ok = 0;             // 1 built, -1 not worth it (rank near full)
    double pc_tol = 0.0;
    int pc_rq = 0, pc_nlev = 0, pc_nptile = 0, pc_netile = 0;
    std::vector<int> pc_rank;  // retained rank per level slot
    fmddm::DBuf<double> pc_Vt, pc_U, pc_C, pc_What, pc_Z, pc_Ghat;
    fmddm::DBuf<double> pc_Wsplit;  // split-K partials of the projection (zero where never written)
    int pc_ksplit = 1;
    fmddm::DBuf<int> pc_ptile_op, pc_ptile_beg, pc_ptile_end, pc_pcell, pc_etile_op, pc_etile_beg, pc_etile_end,
        pc_ecell;
    // history-only variant: the left-hand side as a dense 3n x 3n matrix
    fmddm::DBuf<double> pdense;
    int pdense_ok = 0;
    double pdense_key[8] = {};
    fmddm::DBuf<double *> pn_lhs_ptr;
    double *pn_lhs_host = nullptr;  // source of the copy into pn_lhs_ptr
    int pn_lhs_ok = 0, pf_ops0_ok = 0;
    double pn_key[8] = {};  // medium and budget the levels were built for
    // Arnoldi steps captured as graphs, one per step index, valid for the
    // context and apply mode they were captured with
    std::vector<hipGraphExec_t> gm_graph;
    const fmddm_ctx *gm_graph_ctx = nullptr;
    int gm_graph_mode = -1;
    // bumped whenever a buffer or constant that a poroelastic product or
    // its preconditioner reads is (re)built; captured steps of an older
    // generation are dropped
    int64_t poro_gen = 0, gm_graph_gen = 0;
    void drop_graphs()
    {
        for (hipGraphExec_t &g : gm_graph)
            if (g) (void)hipGraphExecDestroy(g);
        gm_graph.clear();
        gm_graph_ctx = nullptr;
        gm_graph_mode = -1;
    }
    double *gm_host = nullptr;        // 2 slots of 2 doubles
    hipEvent_t gm_ev[2] = {nullptr, nullptr};
    int64_t bytes = 0;
    ~fmddm_tree()
    {
        drop_graphs();
        for (hipEvent_t e : gm_ev)
            if (e) (void)hipEventDestroy(e);
        if (gm_host) (void)hipHostFree(gm_host);
    }
};

namespace fmddm {

// tree.hip
void build_tree(fmddm_ctx *ctx, fmddm_tree *t, int64_t n, const double *x1, const double *y1,
                const double *x2, const double *y2, int on_device);
// fmm.hip
void gauss_legendre(int n, std::vector<double> &t, std::vector<double> &w);
void init_streams(fmddm_ctx *ctx);
void setup_cheb(fmddm_ctx *ctx);
void build_m2l_ops(fmddm_ctx *ctx);
void v_offsets(std::vector<int> &dx, std::vector<int> &dy, std::vector<int> &slot2op);
int offset_slot(int x, int y);
void fmm_m2m4(fmddm_ctx *ctx, fmddm_tree *t, int nterm, int ldw, int tstride, double *W);
void fmm_l2p4(fmddm_ctx *ctx, fmddm_tree *t, const double *G, int ldg, double *far);
void fmm_pair_gemm(hipStream_t s, int ntile, int Mrows, const double *ops, size_t op_stride, int lda, int Kd,
                   const double *X, int ldx, const int *tile_op, const int *tile_beg, const int *tile_end,
                   const int *psrc, const int *pdst, double *Z, int ldz);
void fmm_pair_gemm_split(hipStream_t s, int ntile, int Mrows, const double *ops, size_t op_stride, int lda, int Kd,
                         const double *X, int ldx, const int *tile_op, const int *tile_beg, const int *tile_end,
                         const int *psrc, const int *pdst, double *part, int ldz, int nsplit, size_t zsplit,
                         double *Z, int64_t count);
void fmm_sum_pairs(hipStream_t s, fmddm_tree *t, const double *Z, int ldz, int width, double *out, int ldo);
void setup_fmm(fmddm_ctx *ctx, fmddm_tree *t);
// prec: fmddm_precision of the near field and the M2L products
void fmm_apply(fmddm_ctx *ctx, fmddm_tree *t, const double *D, double *out, int prec = FMDDM_PREC_FP64);
// The buffers one FMM product writes and reads again (nothing else in the
// tree changes during a product): sorted DDs, charges, near partials,
// multipole weights, split-K partials, compressed weights, pair products,
// compressed fields, fields at the nodes, far stress per level.
struct FmmBufs {
    double *Dsort, *q, *part_s, *Wexp, *ksplit, *What, *Zm2l, *Ghat, *Gexp, *far_s;
};
FmmBufs tree_bufs(fmddm_tree *t);
// the same product with the given buffers (the tree's, or another set of
// the same sizes); the tree's schedules and operators must be set up
void fmm_apply_bufs(fmddm_ctx *ctx, fmddm_tree *t, const double *D, double *out, int prec, const FmmBufs &B);
// split-K depth of the projection onto the singular vectors (the
// context's M2L tile set)
int fmm_ksplit(const fmddm_ctx *ctx);
// direct.hip
void direct_apply(fmddm_ctx *ctx, fmddm_tree *t, const double *D, double *out);
void dense_apply(fmddm_ctx *ctx, fmddm_tree *t, const double *D, double *out);
// y = A x, A row-major m x m (one block per row, fixed-order sums)
void dense_gemv(hipStream_t s, int m, const double *A, const double *x, double *y);
// solve.hip
void rhs_build(fmddm_ctx *ctx, fmddm_tree *t, const double *pf, double SH, double Sh, double *rhs,
               double pscale = 1.0);
fmddm_status gmres_solve(fmddm_ctx *ctx, fmddm_tree *t, int mode, const double *b, double *x,
                         fmddm_solve_info *info);

// One restarted-GMRES solve advanced in asynchronous steps: every call of
// advance() enqueues the next piece of work (a residual, an Arnoldi step)
// on the context's stream once the scalars it depends on have reached the
// host.  start() needs b and x resident; x is the initial guess and holds
// the iterate.  The work and its order are the same whether the caller
// waits (block = true) or polls.
struct GmresRun {
    fmddm_ctx *ctx = nullptr;
    fmddm_tree *t = nullptr;
    int mode = 0;                  // product of the Arnoldi steps
    int rmode = 0;                 // product of the residuals at the restarts
    double prev_beta = 0.0;        // residual at the previous restart (mixed precision)
    const double *b = nullptr;
    double *x = nullptr;
    double tol = 0.0;
    int maxit = 0;
    enum State { IDLE, BNORM, RESID, ITER, DONE } state = IDLE;
    int j = 0;                     // oldest Arnoldi step whose scalars are unread
    int next = 0;                  // next Arnoldi step to enqueue (at most j + 2)
    int it = 0, restarts = 0, residuals = 0;
    double bnorm = 0.0, relres = 0.0;
    bool converged = false;
    // rmd < 0: residuals with the Arnoldi product.  A different residual
    // product makes each restart cycle a step of iterative refinement: the
    // cycle's Krylov space is built with `md`, the residual it corrects and
    // the stopping test use `rmd`; a cycle that does not reduce that
    // residual ends the solve (not converged).
    void start(fmddm_ctx *c, fmddm_tree *tr, int md, const double *rhs, double *x0, double tl, int mx,
               int rmd = -1);
    bool advance(bool block);  // true once finished
  private:
    void enqueue_residual();
    void enqueue_step();
    void step_body(int jj);
    void precond(const double *in, int acc, double *out);  // out (+)= M^-1 in
    void post(int slot, int count);
    bool eager_done = false;       // a first step ran uncaptured (lazy set-up done)
    bool pc = false;               // right preconditioning by the block-Jacobi inverse
    bool pc2 = false;              // ... plus the coarse level
};
void apply_mode(fmddm_ctx *ctx, fmddm_tree *t, int mode, const double *D, double *out);
// apply mode of the poroelastic left-hand side F(dt) (3 unknowns per element)
constexpr int APPLY_PORO = 100;
// the FP64 FMM product whatever the context's precision (residuals of
// iterative refinement)
constexpr int APPLY_FMM_FP64 = 101;
inline int64_t vec_len(const fmddm_tree *t, int mode) { return (mode == APPLY_PORO ? 3 : 2) * t->n; }
// precond.hip
void pc_setup(fmddm_ctx *ctx, fmddm_tree *t);
// groups of at most maxm elements (runs in tree order within one leaf) and
// the offsets of their (nc m)^2 inverses; allocates B's arrays
void pc_groups(fmddm_ctx *ctx, fmddm_tree *t, int maxm, int nc, PcBlocks &B);
// out = M^-1 in (acc = 0) or out += M^-1 in (acc = 1), caller order
void pc_apply(fmddm_ctx *ctx, fmddm_tree *t, const PcBlocks &B, const double *in, int acc, double *out);
// coarse level for the elastic (poro = false) or poroelastic system
void pc_coarse_setup(fmddm_ctx *ctx, fmddm_tree *t, bool poro);
// out += P A_c^-1 R in: coarse correction added into out (nc unknowns per
// element in caller order)
void pc_coarse_add(fmddm_ctx *ctx, fmddm_tree *t, const PcCoarse &C, int ncomp, const double *in, double *out);
// poro.hip
void poro_apply(fmddm_ctx *ctx, fmddm_tree *t, int lag, const double *D, double *out);
void poro_history(fmddm_ctx *ctx, fmddm_tree *t, int h, const double *Dh, double *rhs);
void poro_rhs(fmddm_ctx *ctx, fmddm_tree *t, const double *pf, double SH, double Sh, double *rhs);
void pc_setup_poro(fmddm_ctx *ctx, fmddm_tree *t);
// fmm.hip: the reduced-precision copies of ctx's operator set for prec
void lowp_ops(fmddm_ctx *ctx, int prec);
// fmm.hip: leading left singular vectors of A (m x N, column-major) down to
// tol of the largest singular value (randomized range finder); U (m x m)
// gets them in its first columns, sv the sampled singular values; returns
// the rank.  h is a rocblas_handle on stream s.
int range_basis(void *h, hipStream_t s, int m, int N, const double *A, double tol, double *U,
                std::vector<double> &sv);
// builds now what a march of H steps would build on first use
void poro_prepare(fmddm_ctx *ctx, fmddm_tree *t, int H);

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Runs an entry point's body on the context's device and turns internal
// errors into a status code, with the message kept in ctx->err.
template <class F>
fmddm_status guarded(fmddm_ctx *ctx, F &&f)
{
    try {
        FM_HIP(hipSetDevice(ctx->device));
        StreamScope scope(ctx->stream);
        fmddm_status st = f();
        if (ctx) ctx->err.clear();
        return st;
    } catch (const Error &e) {
        if (ctx) ctx->err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        if (ctx) ctx->err = "host allocation failed";
        return FMDDM_ENOMEM;
    } catch (...) {
        if (ctx) ctx->err = "unexpected error";
        return FMDDM_EDEVICE;
    }
}

}  // namespace fmddm
