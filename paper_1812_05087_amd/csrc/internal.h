// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
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
// Owning device allocation (hipMalloc), freed in the destructor.
template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { reset(); }
    void reset() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    void alloc(size_t count) {
        reset();
        if (count == 0) count = 1;
        FM_HIP(hipMalloc((void **)&p, count * sizeof(T)));
        n = count;
    }
    void zero(hipStream_t s) { FM_HIP(hipMemsetAsync(p, 0, n * sizeof(T), s)); }
    size_t bytes() const { return n * sizeof(T); }
};

constexpr int MAXP = 32;

// ------------------------------------------------------------- context
struct Cheb {
    int p = 0;
    DBuf<double> tnode;     // [l][k] = T_k(xbar_l), p x p
    DBuf<double> xbar;      // p nodes
    DBuf<double> gl_t, gl_w;  // p-point Gauss-Legendre
    DBuf<double> m2m;       // [side][l_parent][l_child] = S_p(xbar_l, +-1/2 + xbar_l'/2), 2 x p x p
    std::vector<double> h_xbar, h_tnode, h_m2m, h_glt, h_glw;
};

struct M2LOps {
    int ready = 0;
    int M = 0;              // 3 p^2
    int Mp = 0;             // padded row stride (multiple of 64)
    int rank = 0;           // operator dimension used by the GEMM (Mp or compressed)
    DBuf<double> ops;       // 49 offset slots x rank x rank (unused slots unfilled)
    DBuf<double> Ut, Vt;    // SVD bases (compressed mode): rank x Mp each
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
    int device = 0;
    std::string err;
    fmddm::Cheb cheb;
    fmddm::M2LOps m2l;
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
    std::vector<int> leaves;          // host list of leaf cells (tree order)
    fmddm::DBuf<int> dleaves;
    int64_t near_pairs = 0;
    // M2L schedule: pairs are V-list entries grouped by offset into tiles
    int ntile = 0;
    fmddm::DBuf<int> tile_op, tile_beg, tile_end, pair_k, pair_src;
    fmddm::DBuf<double> pair_scale;
    int64_t nV = 0;
    // expansions
    fmddm::DBuf<double> Wexp, Fexp, Zm2l, Wc, Gc;
    fmddm::DBuf<double> q;            // charges, tree order, 3 per element
    fmddm::DBuf<double> Dsort;        // D in tree order
    // dense operator (built on demand)
    fmddm::DBuf<double> Adense;
    // solver workspace
    fmddm::DBuf<double> gm_V, gm_w, gm_r, gm_sc;
    int gm_restart = 0;
    int64_t bytes = 0;
};

namespace fmddm {

// tree.hip
void build_tree(fmddm_ctx *ctx, fmddm_tree *t, int64_t n, const double *x1, const double *y1,
                const double *x2, const double *y2, int on_device);
// fmm.hip
void setup_cheb(fmddm_ctx *ctx);
void setup_fmm(fmddm_ctx *ctx, fmddm_tree *t);
void fmm_apply(fmddm_ctx *ctx, fmddm_tree *t, const double *D, double *out);
// direct.hip
void direct_apply(fmddm_ctx *ctx, fmddm_tree *t, const double *D, double *out);
void dense_apply(fmddm_ctx *ctx, fmddm_tree *t, const double *D, double *out);
// solve.hip
void rhs_build(fmddm_ctx *ctx, fmddm_tree *t, const double *pf, double SH, double Sh, double *rhs);
fmddm_status gmres_solve(fmddm_ctx *ctx, fmddm_tree *t, int mode, const double *b, double *x,
                         fmddm_solve_info *info);
void apply_mode(fmddm_ctx *ctx, fmddm_tree *t, int mode, const double *D, double *out);

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace fmddm
