/*
 * fmddm.h -- C ABI of the MI355X (gfx950) fast-multipole displacement
 * discontinuity library.
 *
 * The operation behind every entry point is the influence operator of the
 * constant-element displacement discontinuity method (DDM): for N straight
 * elements with unknown shear and normal displacement discontinuities
 * (D_s, D_n), it returns the shear and normal tractions that those
 * discontinuities induce at every element midpoint (Section 2, eqs. 2.3-2.5,
 * the A_xx, A_xy, A_yx, A_yy blocks of a single time step).  The product is
 * evaluated by the black-box fast multipole method with Chebyshev
 * interpolation (Section 3: quad-tree, upward pass, M2L over the interaction
 * list, downward pass, direct neighbour interactions), and the system of one
 * time step is solved with GMRES whose matrix-vector products are FMM
 * products (Section 4).
 *
 * Conventions (the paper states none of them):
 *   - plane strain, isotropic, Young's modulus E, Poisson ratio nu;
 *   - SI units (m, Pa);
 *   - stresses and tractions are tension-positive;
 *   - element j runs from (x1[j], y1[j]) to (x2[j], y2[j]); its tangent s
 *     points from the first to the second endpoint and its normal is s
 *     rotated by +90 degrees; a displacement discontinuity is
 *     D = u(+) - u(-), the + face being the side the normal points into,
 *     so D_n > 0 is opening and D_s > 0 is the + face sliding along s;
 *   - all vectors are element-major, in the caller's element order:
 *     D[2j] = D_s, D[2j+1] = D_n; out[2i] = shear traction,
 *     out[2i+1] = normal traction at the midpoint of element i.
 *
 * Memory and ownership: vectors passed to fmddm_apply / fmddm_rhs /
 * fmddm_solve / fmddm_sif are DEVICE pointers on the context's device; they
 * are read or written on the context's stream and stay owned by the caller.
 * Geometry passed to fmddm_build_tree may be host or device memory (flag);
 * it is copied.  A tree owns all its device memory until fmddm_tree_free.
 * A context is not thread-safe; use one context per stream.  Calls are
 * asynchronous with respect to the host unless stated otherwise.
 *
 * Errors: every call returns an fmddm_status; nothing is thrown across the
 * ABI.  On failure fmddm_last_error(ctx) describes the cause.  No entry point
 * falls back to the CPU.
 */
#ifndef FMDDM_H
#define FMDDM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmddm_ctx fmddm_ctx;
typedef struct fmddm_tree fmddm_tree;

typedef enum {
    FMDDM_OK = 0,
    FMDDM_ENOTCONV = 1,       /* GMRES stopped at maxit; best iterate kept */
    FMDDM_EINVAL = -1,        /* bad argument */
    FMDDM_ENOMEM = -2,        /* device allocation failed */
    FMDDM_EDEVICE = -3,       /* HIP runtime error */
    FMDDM_EGEOM = -4,         /* zero-length / non-finite element, point outside root box */
    FMDDM_EUNSUPPORTED = -5   /* parameter combination not built */
} fmddm_status;

typedef enum {
    FMDDM_APPLY_FMM = 0,      /* black-box FMM product (Section 3) */
    FMDDM_APPLY_DIRECT = 1,   /* exact product, influence evaluated on the fly */
    FMDDM_APPLY_DENSE = 2     /* exact product with the stored dense matrix */
} fmddm_apply_mode;

typedef enum {
    FMDDM_M2L_DENSE = 0,      /* per-offset (3p^2 x 3p^2) operators, as in eq. 3.8 */
    FMDDM_M2L_SVD = 1         /* the same operators compressed by a truncated SVD */
} fmddm_m2l_mode;

/* Arithmetic of the FMM product's two heavy passes, the near field (P2P)
 * and the M2L products.  P2M, M2M, L2P, the sums of the far and near parts
 * and everything in GMRES stay FP64. */
typedef enum {
    FMDDM_PREC_FP64 = 0,      /* everything FP64 */
    FMDDM_PREC_FP32 = 1,      /* P2P in FP32; M2L on FP32 MFMA, FP32 sums */
    FMDDM_PREC_BF16 = 2       /* P2P in FP32; M2L on BF16 MFMA (operators and
                                 weights rounded to bf16), FP32 sums */
} fmddm_precision;

/* Preconditioning of the GMRES solves (fmddm_solve, fmddm_poro_solve).
 * The paper's GMRES is unpreconditioned (NONE); BLOCK is right block-Jacobi
 * preconditioning with the exact inverse of the operator restricted to
 * groups of neighbouring elements (runs in tree order within one leaf):
 * at most 32 elements for the elastic system (8 (2m)^2 bytes per group of
 * m), at most 21 for the poroelastic left-hand side F(dt) (8 (3m)^2 bytes;
 * rebuilt when the medium or dt changes).  TWO_LEVEL adds a coarse level
 * for the long-wavelength modes of long fractures (8 (2 nc)^2 bytes for nc
 * aggregates, about 1024 for long fractures; the poroelastic one uses the
 * undrained modulus).  A geometry with more than 2048 aggregates (few
 * collinear runs, e.g. many one-element fractures) gets block-Jacobi alone.  Built once per tree.  It changes the iteration count, not the
 * solution. */
typedef enum {
    FMDDM_PRECOND_NONE = 0,
    FMDDM_PRECOND_BLOCK = 1,
    FMDDM_PRECOND_TWO_LEVEL = 2  /* block-Jacobi plus a coarse level: aggregates of up to
                                    max(16, n / 1024) consecutive collinear elements (caller
                                    order) taken as long elements, their coarse matrix R A P
                                    inverted once per tree; M^-1 r = B^-1 r + P A_c^-1 R r */
} fmddm_precond;

typedef struct {
    double E, nu;             /* material (Pa, -) */
    int leaf;                 /* split a cell holding more than `leaf` points (Section 3.1) */
    int p;                    /* Chebyshev nodes per dimension, 1..32 */
    int max_level;            /* cap on tree depth, 0..30 */
    double kappa;             /* a cell splits only if its children stay at least
                                 kappa x the largest element half-length it holds wide */
    int m2l;                  /* fmddm_m2l_mode */
    double m2l_tol;           /* relative singular-value cut for FMDDM_M2L_SVD */
    int use_root_box;         /* 1: level-0 square given below; 0: bounding square */
    double root_x0, root_y0, root_L;
    int restart, maxit;       /* GMRES(restart), at most maxit matrix-vector products */
    double tol;               /* GMRES relative residual target */
    int precision;            /* fmddm_precision of FMDDM_APPLY_FMM products */
    int use_graphs;           /* 1: GMRES replays each Arnoldi step (product,
                                 orthogonalisation, rotation) as a HIP graph
                                 captured on its first use; 0: plain launches
                                 (default: replays measured no faster, and
                                 capture costs ~1 ms per step index and tree) */
    int precond;              /* fmddm_precond of elastic GMRES solves */
    int m2l_tiles;            /* tile set of the M2L products, 0..3: (split-K of
                                 the projection, row tile of the pair products,
                                 row tile of the expansion) = (4, 64, 64),
                                 (2, 32, 64), (8, 64, 32), (4, 32, 32);
                                 fmddm_autotune picks one */
    int64_t direct_below;     /* server: requests of at most this many elements
                                 are solved with the exact on-the-fly product
                                 instead of the FMM (faster below the size where
                                 the FMM's chain of launches dominates); 0: never */
    int32_t coarse_aggregates; /* TWO_LEVEL: the number of coarse aggregates aimed at
                                 (elements per aggregate max(16, n / this), runs ending
                                 at fracture ends); 0: 1024.  Fewer make the coarse LU
                                 cheaper and the coarse space poorer. */
} fmddm_params;

typedef struct {
    int64_t n;                /* elements */
    int64_t ncell, nleaf;     /* tree cells, leaves */
    int32_t nlevel;           /* deepest level + 1 */
    int64_t nU, nV, nW, nX;   /* list lengths (sum over cells) */
    int64_t near_pairs;       /* directly evaluated point pairs per product */
    int64_t l2p_pairs;        /* (midpoint, ancestor cell) interpolations per product */
    int64_t m2m_pairs;        /* child-to-parent transfers of the upward pass per product (cells
                                 whose parent is at level >= 2); the downward pass has as many */
    int64_t nfar;             /* cells at level >= 2 (those with interaction lists) */
    int64_t m2l_rank;         /* M2L rank (3p^2 when uncompressed; 0 before the first product) */
    double root_x0, root_y0, root_L;
    int64_t device_bytes;     /* device memory held by the tree */
    int64_t m2m_launches;     /* launches of the upward pass per product (0 before the first product) */
    int32_t m2m_cut;          /* level below which each subtree's upward pass runs in one block */
    int32_t poro_m2l_rank;    /* poroelastic left-hand side with m2l = SVD: the largest rank kept
                                 over the tree levels (0: uncompressed or not built yet) */
} fmddm_tree_info;

typedef struct {
    int32_t iters;            /* matrix-vector products inside GMRES */
    int32_t restarts;
    double relres;            /* ||b - A x|| / ||b|| of the returned iterate (true residual;
                                 with the FP64 product under iterative refinement) */
    int32_t converged;
    int32_t refinements;      /* reduced precision: FP64 residual products (one
                                 per restart cycle plus the last); 0 otherwise */
} fmddm_solve_info;

/* Fill *p with defaults: E=20e9, nu=0.25, leaf=32, p=20, max_level=24,
 * kappa=8, m2l=DENSE, m2l_tol=1e-12, no root box, restart=50,
 * maxit=10000, tol=1e-10, precision=FP64, use_graphs=0, precond=NONE,
 * m2l_tiles=0, direct_below=0, coarse_aggregates=0 (1024). */
void fmddm_default_params(fmddm_params *p);

/* Create a context on the current HIP device bound to `hip_stream`
 * (a hipStream_t; NULL = the default stream).  Validates the parameters
 * (EINVAL) and builds the Chebyshev tables.  *out is NULL on failure. */
fmddm_status fmddm_create(const fmddm_params *p, void *hip_stream, fmddm_ctx **out);
void fmddm_destroy(fmddm_ctx *ctx);
/* Message of the last failing call on ctx (static storage owned by ctx). */
const char *fmddm_last_error(const fmddm_ctx *ctx);

/* Build the quad-tree and lists over the element midpoints (Section 3.1).
 * x1,y1,x2,y2 hold n element endpoints; on_device != 0 means they are
 * device pointers.  The level-0 square is the bounding square of the
 * midpoints (or the context's root box), coordinates are quantised to a
 * 2^31 grid and Morton-ordered, and a cell splits into its non-empty
 * children (left-to-right, then bottom-to-top) while it holds more than
 * `leaf` points.  U/V/W/X lists follow.  Synchronises the stream.
 * EGEOM for zero-length or non-finite elements or points outside the
 * root box. */
fmddm_status fmddm_build_tree(fmddm_ctx *ctx, int64_t n, const double *x1,
                              const double *y1, const double *x2, const double *y2,
                              int on_device, fmddm_tree **out);
void fmddm_tree_free(fmddm_tree *t);
fmddm_status fmddm_tree_get_info(fmddm_ctx *ctx, const fmddm_tree *t, fmddm_tree_info *info);

/* Copy the tree to host arrays (any pointer may be NULL to skip it).
 * perm[n]: sorted position -> element index; key[n]: Morton keys in sorted
 * order; per cell (ncell entries, cells ordered by level then Morton key):
 * level, ix, iy, parent (-1 for the root), child[4*ncell] (-1 = absent,
 * order BL, BR, TL, TR), pbeg/pend (sorted point range), isleaf;
 * root[3] = x0, y0, L.  Synchronises the stream. */
fmddm_status fmddm_tree_export(fmddm_ctx *ctx, const fmddm_tree *t, int64_t *perm,
                               uint64_t *key, int32_t *level, uint32_t *ix,
                               uint32_t *iy, int32_t *parent, int32_t *child,
                               int64_t *pbeg, int64_t *pend, int32_t *isleaf,
                               double *root);

/* Copy one list as CSR over cells: which = 0 U, 1 V, 2 W, 3 X; off has
 * ncell+1 entries, idx has off[ncell] entries, sorted by cell index.
 * U(B): leaves adjacent to leaf B (B included); V(B): children of the
 * neighbours of B's parent that are not adjacent to B (the interaction
 * list); W(B): cells finer than leaf B, not adjacent to B, whose parent is
 * adjacent to B; X(A): leaves B with A in W(B).  Synchronises. */
fmddm_status fmddm_tree_export_list(fmddm_ctx *ctx, const fmddm_tree *t, int which,
                                    int64_t *off, int32_t *idx);

/* out = A D for the single-step elastic influence operator (device
 * pointers, 2n doubles each; out may not alias D).  mode selects the FMM
 * (Section 3), the exact on-the-fly product or the stored dense matrix
 * (assembled on first use: 32 n^2 bytes; ENOMEM if it does not fit).
 * The FMM product runs at the context's precision (fmddm_precision); the
 * exact products are always FP64. */
fmddm_status fmddm_apply(fmddm_ctx *ctx, fmddm_tree *t, int mode, const double *D,
                         double *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FMM
 * product of fmddm_apply (FMDDM_APPLY_FMM, FP64 contexts only) with every
 * intermediate it writes and reads again in one static device workspace
 * of 96 MiB, which each device the library runs on holds until the
 * process ends.  The call allocates nothing: no hipMalloc, hipFree or
 * allocating library routine.  D, out: device, 2n doubles each, out may
 * not alias D.  The tree must already have run one fmddm_apply FMM product
 * (that builds its schedules and operators); otherwise FMDDM_EINVAL.  A
 * product whose intermediates exceed the workspace (the message states
 * both sizes; C2, N = 20000 at p = 20, needs 72 MB) returns FMDDM_EINVAL.
 * FMDDM_EUNSUPPORTED for FP32/BF16 contexts.  Same kernels, same order:
 * the result equals fmddm_apply's bit for bit.  Every call on one device
 * shares that device's workspace and leaves its contents behind; calls
 * that overlap on one device (other streams, other threads) race. */
fmddm_status fmddm_apply_static(fmddm_ctx *ctx, fmddm_tree *t, const double *D, double *out);

/* Right-hand side of one elastic step (Section 4): tractions the
 * discontinuities must induce so that the element faces carry the fluid
 * pressure pf[i] (device, n doubles, compression-positive) under the far
 * field SH (along x) and Sh (along y), compression-positive:
 * rhs = -pf n - sigma_inf n, resolved on (s, n).  rhs: device, 2n doubles. */
fmddm_status fmddm_rhs(fmddm_ctx *ctx, fmddm_tree *t, const double *pf, double SH,
                       double Sh, double *rhs);

/* Solve A D = rhs by restarted GMRES(restart) (Section 4) with products by
 * `mode`.  D holds the initial guess on entry and the solution on exit
 * (device, 2n).  Orthogonalisation (classical Gram-Schmidt, applied twice),
 * Givens rotations and the residual checks run on the device in FP64; the
 * final residual is recomputed from b - A x.  FMDDM_ENOTCONV when maxit is
 * reached (the best iterate is returned).  Synchronises the stream.
 *
 * With mode FMM and a reduced precision every restart cycle is a step of
 * iterative refinement: the residual r = rhs - A D it starts from is
 * computed with the FP64 FMM product A, the cycle's Arnoldi steps use the
 * reduced-precision product A' (basis, orthogonalisation, rotations and the
 * update of D stay FP64), and convergence is ||r|| <= tol ||rhs|| with the
 * FP64 product.  maxit bounds the reduced-precision products; ENOTCONV also
 * when a cycle fails to reduce ||r|| (A' too far from A for the system's
 * conditioning).  info->refinements counts the FP64 residuals. */
fmddm_status fmddm_solve(fmddm_ctx *ctx, fmddm_tree *t, int mode, const double *rhs,
                         double *D, fmddm_solve_info *info);

/* Stress intensity factors of eq. 2.6 from the DDs of tip element `elem`
 * (D: device, 2n), reading "a" as that element's half-length:
 * K = 0.806 E / (4 (1 - nu^2)) sqrt(pi / (2 a)) D.  Synchronises. */
fmddm_status fmddm_sif(fmddm_ctx *ctx, fmddm_tree *t, const double *D, int64_t elem,
                       double *KI, double *KII);

/* Measured device peaks (fmddm_measure_peaks). */
typedef struct {
    double fp64_vector_tflops;  /* FP64 FMA loop on the vector ALUs */
    double fp64_mfma_tflops;    /* FP64 16x16x4 MFMA loop */
    double copy_gbps;           /* device-to-device copy of 1 GiB, bytes read + written per second */
} fmddm_peaks;

/* Microbenchmarks of the current device, the measured roofline denominators
 * reported beside the vendor figures: register-resident FP64 FMA and MFMA
 * loops over 16 blocks per compute unit, and a 1 GiB stream copy.  Runs on
 * a stream of its own and synchronises it; allocates 2 GiB for the copy. */
fmddm_status fmddm_measure_peaks(fmddm_peaks *out);

/* One configuration tried by fmddm_autotune. */
typedef struct {
    int32_t leaf, p;
    double ms;                /* mean time of one FMM product (ms); -1 when not
                                 timed (error target missed) */
    double err;               /* ||y - y_exact|| / ||y_exact|| for uniform opening */
    int32_t m2l_tiles;        /* tile set the product was timed with */
} fmddm_tune_entry;

/* Choose the leaf size and the Chebyshev order for one geometry (host
 * endpoints, n elements).  The paper sets the order by hand and gives no
 * rule for the leaf size (Section 5); this measures both: for every leaf
 * size in leaves[0..nleaves) the orders ps[0..nps) are tried in ascending
 * order until the FMM product's relative error (2-norm) against the exact
 * product is at most target_err; that configuration's product is
 * timed (reps products on the device) and the fastest over the leaf sizes
 * is kept; then every M2L tile set (m2l_tiles) is timed on it and the
 * fastest kept (log entries for those carry err of the chosen leaf and p).  The test vector is a uniform opening (Dn = 1e-3, Ds = 0 on every
 * element): smooth, like the DDs of loaded fractures, it weighs the far
 * field as solutions do, where a random vector is dominated by the near
 * field (which the FMM evaluates exactly).  Every other field of *base
 * (material, M2L mode, precision,
 * solver settings) is used as given.  *best = *base with leaf and p set.
 * log[0..log_cap) receives each configuration tried (log may be NULL when
 * log_cap = 0), *nlog (may be NULL) their number.  FMDDM_ENOTCONV when no
 * configuration meets the target (*best is then the most accurate one).
 * Runs on a stream of its own on the current device and synchronises it;
 * allocates trees and operators for the duration of the call. */
fmddm_status fmddm_autotune(const fmddm_params *base, int64_t n, const double *x1,
                            const double *y1, const double *x2, const double *y2,
                            const int32_t *leaves, int32_t nleaves, const int32_t *ps,
                            int32_t nps, double target_err, int32_t reps, fmddm_params *best,
                            fmddm_tune_entry *log, int32_t log_cap, int32_t *nlog);

/* Phases of one FMM product, for fmddm_profile. */
typedef enum {                /* one entry per kernel of an FMM product */
    FMDDM_PH_PREP = 0,        /* D to tree order, source charges */
    FMDDM_PH_P2M = 1,         /* leaf weights (eq. 3.6) */
    FMDDM_PH_M2M = 2,         /* upward pass (eq. 3.7): partial weights per work item */
    FMDDM_PH_M2M_SUM = 3,     /* upward pass: partials summed per cell */
    FMDDM_PH_COMPRESS = 4,    /* weights projected on the M2L singular vectors (SVD mode) */
    FMDDM_PH_COMPRESS_SUM = 5,/* split-K partials of the projection summed (SVD mode) */
    FMDDM_PH_M2L = 6,         /* one operator product per interaction pair (eq. 3.8) */
    FMDDM_PH_M2L_SUM = 7,     /* pair results summed per target cell (eq. 3.8) */
    FMDDM_PH_DECOMPRESS = 8,  /* M2L fields back on the Chebyshev nodes (SVD mode) */
    FMDDM_PH_L2P = 9,         /* downward pass and L2P (eqs. 3.9-3.11, far part) */
    FMDDM_PH_P2P = 10,        /* direct neighbour interactions (eq. 3.11, near part) */
    FMDDM_PH_FINAL = 11,      /* far + near stress to tractions, caller order */
    FMDDM_PH_COUNT = 12
} fmddm_phase;

/* Record HIP events around the kernels whose bit (1 << fmddm_phase) is set
 * in `mask`, on the stream each runs on, for every following FMM product
 * (0 disables).  Adds two event records per timed kernel and product. */
fmddm_status fmddm_profile(fmddm_ctx *ctx, unsigned mask);

/* Elapsed milliseconds summed per phase (ms[FMDDM_PH_COUNT]) and the number
 * of timed launches (count[FMDDM_PH_COUNT], may be NULL) since the previous
 * read; resets the sums.  Synchronises the stream. */
fmddm_status fmddm_profile_read(fmddm_ctx *ctx, double *ms, int64_t *count);

/* ------------------------------------------------------------------------
 * Poroelastic time marching (Section 2, eqs. 2.1-2.5).
 *
 * Unknowns per element j: D[3j] = D_s, D[3j+1] = D_n (m, as above),
 * D[3j+2] = D_q, the fluid volume leaving the fracture per unit time and
 * unit element length (m^2/s).  Responses per element i: out[3i] shear
 * traction, out[3i+1] normal traction, out[3i+2] pore pressure change at
 * the midpoint (Pa).  The medium is fully coupled Biot poroelastic: the
 * context's E and nu are the drained constants, fmddm_poro_params adds the
 * undrained Poisson ratio, the Biot coefficient and the mobility
 * (permeability / viscosity).  Time is discretised in equal intervals dt
 * with constant DDs in each interval, collocated at interval ends: the
 * system of step h is
 *     K_0 D^h = b_h - sum_{k=1}^{h-1} K_{h-k} D^k,
 * K_0 = F(dt), K_m = F((m+1) dt) - F(m dt), F(t) the response at time t to
 * unit sources switched on at 0 and held.  With mode FMDDM_APPLY_DIRECT the
 * products evaluate every element integral exactly (cost n^2 per time
 * level); with FMDDM_APPLY_FMM the far field goes through the black-box
 * FMM of Section 3 with the time-dependent kernel (operators per tree
 * level and time level, built on first use and kept with the tree).
 * FMDDM_APPLY_DENSE is the history-only variant (the earlier method the
 * paper builds on, Section 2): the left-hand side K_0 as a stored dense
 * 3n x 3n matrix of exact element integrals (72 n^2 bytes, assembled on
 * first use; ENOMEM if it does not fit), the history coefficients K_m,
 * m >= 1, and the history sum through the FMM.
 * ------------------------------------------------------------------------ */
typedef struct {
    double nu_u;              /* undrained Poisson ratio, nu < nu_u < 0.5 */
    double alpha;             /* Biot coefficient, (0, 1] */
    double perm, visc;        /* permeability (m^2) and fluid viscosity (Pa s) */
    double dt;                /* time step (s) */
    double p0;                /* initial pore pressure (Pa), for fmddm_poro_rhs */
    int32_t mode;             /* FMDDM_APPLY_DIRECT: exact element integrals for every pair;
                                 FMDDM_APPLY_FMM: the same for neighbouring elements and
                                 Chebyshev multipoles (the context's p, 2..16) for well-separated
                                 cells, the time levels contracted in one M2L product;
                                 FMDDM_APPLY_DENSE: K_0 stored dense and exact, history by FMM */
    int64_t near_cache_bytes; /* FMDDM_APPLY_FMM only: device memory for the near-field cache.
                                 The exact element integrals of neighbouring elements depend only
                                 on the geometry, the medium and the time level, so each level's
                                 4 x 3 response blocks (96 bytes per near pair) are integrated
                                 once, on first use, and kept with the tree; later products at
                                 that level are block-sparse products.  Levels beyond the budget
                                 are integrated on the fly at every product.  When the budget
                                 holds two levels, the left-hand side F(dt) also gets its own
                                 blocks with the drained elastic part added (one more level's
                                 96 bytes per near pair), and is then one multipole pass.  0: a
                                 quarter of the free device memory at first use, at most 32 GiB;
                                 > 0: that many bytes; < 0: no cache. */
    int32_t m2l;              /* FMDDM_APPLY_FMM left-hand side (the product GMRES applies):
                                 FMDDM_M2L_DENSE (0): the (4p^2)^2 operator per (tree level,
                                 offset) of eq. 3.8; FMDDM_M2L_SVD (1): those operators
                                 compressed per cell size (bases of all 40 V-list offsets at
                                 that size from a truncated SVD at the context's m2l_tol),
                                 used when the stored near field holds the left-hand side.
                                 The compressed operators of a cell size are built once and
                                 kept in a cache that the contexts of one server share; a
                                 one-time cost that pays over many products. */
    int32_t exact_far_levels; /* FMDDM_APPLY_FMM history sums and lag products: 0 (default):
                                 where every V-list pair lies far outside the diffusion length
                                 at the last time level (z = r^2 / (4 c t) >= 50, checked per
                                 tree level from the cell size), the transient kernel is affine
                                 in t to double precision, and the far field takes two
                                 multipole terms (the first two time levels' operators) for any
                                 number of levels; 1: one term per time level always.  The near
                                 field is exact per level either way. */
} fmddm_poro_params;

/* Attaches the poroelastic medium to the context (validated: EINVAL). */
fmddm_status fmddm_poro_set(fmddm_ctx *ctx, const fmddm_poro_params *pp);

/* out = K_lag D (device, 3n each; out must not alias D): lag 0 is the
 * left-hand side F(dt) including the drained elastic part, lag >= 1 the
 * history coefficient F((lag+1) dt) - F(lag dt). */
fmddm_status fmddm_poro_apply(fmddm_ctx *ctx, fmddm_tree *t, int lag, const double *D, double *out);

/* rhs -= sum_{k=1}^{h-1} K_{h-k} D^k for step h >= 1 (h = 1: nothing).
 * Dhist (device) holds D^1, ..., D^{h-1}, 3n each, consecutively; rhs
 * (device, 3n) must not alias it.  The sum is evaluated once per time
 * level j dt (j = 1..h) on differences of the stored DDs. */
fmddm_status fmddm_add_history(fmddm_ctx *ctx, fmddm_tree *t, int h, const double *Dhist, double *rhs);

/* Right-hand side of one step without history (Section 4): the induced
 * tractions cancel the fluid pressure pf (device, n) and the far field (SH,
 * Sh compressive, along x and y); the induced pore pressure at the faces is
 * pf - p0.  rhs: device, 3n. */
fmddm_status fmddm_poro_rhs(fmddm_ctx *ctx, fmddm_tree *t, const double *pf, double SH, double Sh,
                            double *rhs);

/* Solves K_0 D = rhs by restarted GMRES (the context's restart, maxit,
 * tol); D (device, 3n) is the initial guess and receives the solution. */
fmddm_status fmddm_poro_solve(fmddm_ctx *ctx, fmddm_tree *t, const double *rhs, double *D,
                              fmddm_solve_info *info);

/* Device memory of the library on the current device.  Every device buffer
 * comes from a cache: a block released by a freed tree or context is kept
 * and handed out again instead of being returned to the runtime (hipFree
 * would wait for all work on the device).  in_use counts the bytes held by
 * live objects, cached the bytes kept for reuse; fmddm_trim_cache returns
 * the cached blocks to the runtime and reports how many bytes it freed.  An
 * allocation that fails empties the cache and is retried once. */
int64_t fmddm_memory_in_use(void);
int64_t fmddm_memory_cached(void);
int64_t fmddm_trim_cache(void);

/* ------------------------------------------------------------------------
 * Serving: many fracture solves of different sizes on one device.
 *
 * Each request is the problem of Section 4 for its own geometry: build the
 * tree, form the right-hand side, solve with GMRES whose products are FMM
 * products.  On an elastic server `steps` load steps ramp the fluid
 * pressure linearly from pf/steps to pf (far-field stress constant), each
 * solved to `tol` starting from the previous step's DDs.  On a server given
 * a poroelastic medium (fmddm_server_set_poro) a request is a time march of
 * `steps` steps of dt (Section 2, eqs. 2.3-2.5): constant loads pf, SH, Sh
 * from t = 0, step h solving F(dt) D^h = b - sum_{k<h} K_{h-k} D^k as
 * fmddm_poro_rhs, fmddm_add_history and fmddm_poro_solve do, with the
 * multipole form on the product and the history sum; the result is D^steps
 * (3 unknowns per element).
 *
 * Continuous batching: fmddm_server_step advances every admitted request by
 * one unit of work (one GMRES residual or Arnoldi step, enqueued on that
 * request's own streams, so the work of different requests overlaps on the
 * device) and admits at most one queued request when a slot is free and the
 * device-memory estimate of the queued request fits the budget next to the
 * admitted ones (first come, first served).  Requests never share device
 * buffers and every kernel is deterministic, so a result does not depend on
 * which other requests ran beside it.
 *
 * The server's parameters apply to every request.  With a reduced
 * precision, a solve's Arnoldi steps use the reduced-precision FMM product
 * and its residuals and stopping test the FP64 product (as fmddm_solve).
 * Requests of at most direct_below elements use the exact on-the-fly
 * product instead of the FMM (FP64).
 *
 * Threading: a server is driven from one host thread.  All host memory
 * passed in is copied; nothing is kept after the call returns.
 * ------------------------------------------------------------------------ */
typedef struct fmddm_server fmddm_server;

typedef struct {
    int64_t n;                /* elements */
    const double *x1, *y1, *x2, *y2;  /* host: element endpoints (n each) */
    const double *pf;         /* host: fluid pressure per element at the last step (Pa) */
    double SH, Sh;            /* far-field compressive stresses along x and y (Pa) */
    int32_t steps;            /* load steps, >= 1 */
    double tol;               /* GMRES relative residual per step, in (0, 1) */
} fmddm_request;

typedef enum {
    FMDDM_REQ_QUEUED = 0,
    FMDDM_REQ_RUNNING = 1,
    FMDDM_REQ_DONE = 2,
    FMDDM_REQ_FAILED = 3      /* `status` says why (e.g. FMDDM_ENOTCONV, FMDDM_ENOMEM) */
} fmddm_req_state;

typedef struct {
    int32_t state;            /* fmddm_req_state */
    int32_t status;           /* fmddm_status of a finished request */
    int32_t steps_done;
    int32_t iters;            /* GMRES products over all steps */
    double relres;            /* true relative residual of the last step */
    double t_submit, t_admit, t_done;  /* seconds on the server's clock */
    int64_t device_bytes;     /* device memory charged against the budget (the estimate) */
} fmddm_result;

/* Creates a server for problems with parameters `p` (material, tree and FMM
 * settings, GMRES restart and maxit; p->tol is ignored, each request has
 * its own).  At most `max_slots` requests are admitted at once (1..64);
 * `hbm_budget` bytes (0: 90 % of the device memory free at creation, counting
 * the blocks the library caches for reuse) bound
 * the sum of the admitted requests' estimated footprints.  The M2L operators
 * are built once here and shared by all requests. */
fmddm_status fmddm_server_create(const fmddm_params *p, int max_slots, int64_t hbm_budget,
                                 fmddm_server **out);
void fmddm_server_destroy(fmddm_server *s);
const char *fmddm_server_last_error(const fmddm_server *s);

/* Makes the server poroelastic (eqs. 2.1-2.5): the medium, dt and p0 of
 * fmddm_poro_set apply to every later request (mode must be
 * FMDDM_APPLY_FMM; near_cache_bytes 0 gives each request a quarter of the
 * budget divided by max_slots for its stored near blocks).  With m2l =
 * FMDDM_M2L_SVD each request's tree gets a root square of power-of-two
 * side centred on its midpoints' bounding box, so that requests of one
 * scale share cell sizes, and the compressed left-hand-side operators of a
 * cell size are built once and shared by all slots.  Only while no
 * request is queued or running (EINVAL otherwise); EINVAL / EUNSUPPORTED
 * as fmddm_poro_set. */
fmddm_status fmddm_server_set_poro(fmddm_server *s, const fmddm_poro_params *pp);

/* Device-memory estimate (bytes) the server charges a request of n
 * elements against the budget (poroelastic servers: a march of 10 steps;
 * a submitted request is charged for its own step count). */
int64_t fmddm_server_footprint(const fmddm_server *s, int64_t n);

/* Queues a request; *ticket identifies it.  Validates the request (EINVAL)
 * and copies its arrays. */
fmddm_status fmddm_server_submit(fmddm_server *s, const fmddm_request *r, int64_t *ticket);

/* One engine step (see above).  *active (may be NULL) receives the number
 * of admitted, unfinished requests and *queued the number waiting.  Does
 * not block on device work except while admitting a request (tree build
 * and its one-time set-up). */
fmddm_status fmddm_server_step(fmddm_server *s, int *active, int *queued);

/* State of a request.  Once it is DONE, D (host, may be NULL) receives its
 * DDs in the convention of fmddm_apply (2n doubles) or, on a poroelastic
 * server, of fmddm_poro_apply (3n doubles); the server keeps them until
 * fmddm_server_release. */
fmddm_status fmddm_server_poll(fmddm_server *s, int64_t ticket, fmddm_result *res, double *D);

/* Forgets a finished request. */
fmddm_status fmddm_server_release(fmddm_server *s, int64_t ticket);

#ifdef __cplusplus
}
#endif

#endif /* FMDDM_H */
