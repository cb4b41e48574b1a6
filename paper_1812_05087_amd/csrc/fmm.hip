// Black-box FMM product (Section 3.2) on gfx950.
//
// Expansion layout: every cell holds Mp doubles (3 p^2 used, the rest zero):
// index c * p^2 + l * p + m for component c and Chebyshev node (l, m) of the
// cell's square.  Multipole weights W carry the three charge components
// (b_x n_x, b_y n_y, b_x n_y + b_y n_x) integrated against the interpolants;
// M2L fields G carry (sxx, syy, sxy).
//
// Passes of one product:
//   prep      D (caller order) -> D and charges in tree order
//   p2m       leaf weights, eq. 3.6.  Each element's anterpolation weights
//             (its p-point Gauss-Legendre integral of the interpolants, exact
//             for a straight segment) depend on geometry only, so they are
//             built once per tree; a product streams them (HBM bound)
//   m2m       eq. 3.7, one level at a time, separable p x p transfers
//   m2l       eq. 3.8 as batched dense contractions on FP64 MFMA.  V-list
//             pairs are grouped by relative offset; each group is multiplied
//             by the unit-size operator of its offset and scaled by h^-2 (the
//             kernel is homogeneous of degree -2).  Optionally the operators
//             are compressed by a truncated SVD of all of them stacked
//             (the reduction of Fong & Darve's black-box FMM): weights are
//             projected on r singular vectors, multiplied by r x r operators,
//             and expanded back.  One product per pair is stored and the
//             pairs of a cell are summed in list order (no atomics).
//   l2p       eqs. 3.10-3.11 (far part) in one launch: the M2L fields of a
//             leaf and of all its ancestors evaluated at its midpoints (the
//             downward chain of interpolations composes to exactly this)
//   p2p       eq. 3.11, second term: exact element interactions over U, W
//             and the X lists of the leaf and its ancestors, in work items
//             of at most NEAR_CHUNK sources
//   final     far + near partials summed per point in a fixed order,
//             projected to (shear, normal) traction, caller order.
#include "elem.h"
#include "internal.h"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>

namespace fmddm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// XCD-aware block order: the hardware deals consecutive workgroups to the
// 8 XCDs round-robin, so block b runs on XCD b % 8.  Give XCD x the
// contiguous run of work items [start_x, start_x + count_x), where XCD x
// receives count_x = nb/8 (+1 for the first nb%8 XCDs) blocks: neighbouring
// leaves, which share sources, then share that XCD's L2.  A bijection on
// [0, nb).
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    int q = nb >> 3, rem = nb & 7, x = b & 7;
    return x * q + min(x, rem) + (b >> 3);
}

__global__ void k_prep(int n, const int *__restrict__ perm, const double *__restrict__ D,
                       const double *__restrict__ cb, const double *__restrict__ sb,
                       double *__restrict__ Ds, double *__restrict__ q)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int j = perm[i];
    double s = D[2 * j], nn = D[2 * j + 1];
    Ds[2 * i] = s;
    Ds[2 * i + 1] = nn;
    double q0, q1, q2;
    charge(cb[i], sb[i], s, nn, q0, q1, q2);
    q[3 * i] = q0;
    q[3 * i + 1] = q1;
    q[3 * i + 2] = q2;
}

// S_p(xbar_l, u) by the Chebyshev sum 1/p + 2/p sum_k T_k(xbar_l) T_k(u);
// tn_l[k] = T_k(xbar_l).  Valid (and stable) also outside [-1, 1].
__device__ __forceinline__ double cheb_S(int p, const double *tn_l, double u)
{
    double s = 0.0, t0 = 1.0, t1 = u;
    for (int k = 1; k < p; ++k) {
        s += tn_l[k] * t1;
        double t2 = 2.0 * u * t1 - t0;
        t0 = t1;
        t1 = t2;
    }
    return (1.0 + 2.0 * s) / p;
}

// All p interpolants at u in [-1, 1] by the barycentric formula for
// first-kind Chebyshev nodes (weights (-1)^l sin((2l+1) pi / 2p)).
template <int P>
__device__ __forceinline__ void bary(const double *xb, const double *bw, double u, double (&S)[P])
{
    double den = 0.0;
    int hit = -1;
#pragma unroll
    for (int k = 0; k < P; ++k) {
        double d = u - xb[k];
        if (d == 0.0) hit = k;
        double t = bw[k] * recip(d);
        S[k] = t;
        den += t;
    }
    double id = recip(den);
#pragma unroll
    for (int k = 0; k < P; ++k) S[k] = hit < 0 ? S[k] * id : (k == hit ? 1.0 : 0.0);
}

// ---------------------------------------------------- P2M (per tree)
// Anterpolation weights of every element: M_j[l][m] = integral over the
// element of S(xbar_l, x) S(xbar_m, y), by p-point Gauss-Legendre.
__global__ __launch_bounds__(256) void k_p2m_mats(int nleaf, const int *__restrict__ leaves,
                                                  const int *__restrict__ pbeg, const int *__restrict__ pend,
                                                  const double *__restrict__ ccx, const double *__restrict__ ccy,
                                                  const double *__restrict__ chw, const double *__restrict__ cx,
                                                  const double *__restrict__ cy, const double *__restrict__ cb,
                                                  const double *__restrict__ sb, const double *__restrict__ a,
                                                  const double *__restrict__ tnode, const double *__restrict__ glt,
                                                  const double *__restrict__ glw, int p, double *__restrict__ Pm)
{
    __shared__ double tn[MAXP * MAXP];
    __shared__ double Sx[MAXP * MAXP], Sy[MAXP * MAXP];  // [g][l]
    __shared__ double wg[MAXP];
    int c = leaves[blockIdx.x];
    int tid = threadIdx.x, p2 = p * p;
    for (int e = tid; e < p2; e += 256) tn[e] = tnode[e];
    double x0 = ccx[c], y0 = ccy[c], ih = 1.0 / chw[c];
    __syncthreads();
    for (int j = pbeg[c]; j < pend[c]; ++j) {
        double ex = cx[j], ey = cy[j], ec = cb[j], es = sb[j], ea = a[j];
        for (int t = tid; t < 2 * p2; t += 256) {
            int coord = t / p2, r = t - coord * p2;
            int g = r / p, l = r - g * p;
            double xi = ea * glt[g];
            double u = coord ? (ey + xi * es - y0) * ih : (ex + xi * ec - x0) * ih;
            double v = cheb_S(p, tn + l * p, u);
            if (coord) Sy[g * MAXP + l] = v;
            else Sx[g * MAXP + l] = v;
        }
        if (tid < p) wg[tid] = ea * glw[tid];
        __syncthreads();
        for (int e = tid; e < p2; e += 256) {
            int l = e / p, m = e - l * p;
            double s = 0.0;
            for (int g = 0; g < p; ++g) s += wg[g] * Sx[g * MAXP + l] * Sy[g * MAXP + m];
            Pm[(size_t)j * p2 + e] = s;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------- P2M (per product)
// eq. 3.6: leaf weights from the stored per-element anterpolation matrices
// (HBM bound: the matrices are streamed once).  For p^2 < 256 the block's
// threads split the leaf's elements into G = 256 / p^2 interleaved groups,
// so that G rows of the matrices are in flight at once; the group partials
// are added in group order.
__global__ __launch_bounds__(256) void k_p2m(int nleaf, const int *__restrict__ leaves,
                                             const int *__restrict__ pbeg, const int *__restrict__ pend,
                                             const double *__restrict__ Pm, const double *__restrict__ q,
                                             int p2, int Mp, double *__restrict__ W)
{
    __shared__ double red[3][256];
    int c = leaves[xcd_remap(blockIdx.x, nleaf)];
    int b = pbeg[c], e = pend[c];
    double *Wc = W + (size_t)c * Mp;
    if (p2 >= 128) {
        for (int t = threadIdx.x; t < p2; t += 256) {
            double w0 = 0.0, w1 = 0.0, w2 = 0.0;
#pragma unroll 4
            for (int j = b; j < e; ++j) {
                double m = Pm[(size_t)j * p2 + t];
                w0 += q[3 * j] * m;
                w1 += q[3 * j + 1] * m;
                w2 += q[3 * j + 2] * m;
            }
            Wc[t] = w0;
            Wc[p2 + t] = w1;
            Wc[2 * p2 + t] = w2;
        }
        return;
    }
    int G = 256 / p2, tid = threadIdx.x, g = tid / p2, t = tid - g * p2;
    double w0 = 0.0, w1 = 0.0, w2 = 0.0;
    if (g < G) {
#pragma unroll 4
        for (int j = b + g; j < e; j += G) {
            double m = Pm[(size_t)j * p2 + t];
            w0 += q[3 * j] * m;
            w1 += q[3 * j + 1] * m;
            w2 += q[3 * j + 2] * m;
        }
    }
    red[0][tid] = w0;
    red[1][tid] = w1;
    red[2][tid] = w2;
    __syncthreads();
    if (tid < p2) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int h = 0; h < G; ++h) {
            s0 += red[0][h * p2 + tid];
            s1 += red[1][h * p2 + tid];
            s2 += red[2][h * p2 + tid];
        }
        Wc[tid] = s0;
        Wc[p2 + tid] = s1;
        Wc[2 * p2 + tid] = s2;
    }
}

// ------------------------------------------------------------ M2M
// eq. 3.7: a parent's weights are its children's weights interpolated onto
// the parent's nodes and summed.  A child is exactly one quadrant of its
// parent, so the 1D transfer from a child on side s (0: low, 1: high) is the
// same p x p matrix at every level,
//   S_s[l][l'] = S_p(xbar_l, (xbar_l' + 2s - 1) / 2),
// and child d (x side d & 1, y side d >> 1, the order of Fig. 3) adds
// S_{d&1} W_d S_{d>>1}^T to each component.  Children of equal y side share
// their y transfer:
//   W_A = sum_sy (sum_sx S_sx W_{sx,sy}) S_sy^T,
// so a parent costs four x passes and two y passes, all on FP64 MFMA
// (16x16x4 blocks).  The transfer matrices stay in registers for the whole
// block; the children's weights go straight from memory into the x pass's
// B operands, its results through LDS into the y pass's A operands.
//
// A block works through a chain of parents in order, writing each parent's
// weights before the next starts (a barrier orders them), so a chain may
// climb: the subtrees below a cut level go one chain each in one launch,
// and every level above it is one launch of one-parent chains.  Each child
// transfer is done once.
constexpr int XT = 256;

// NC components per cell (3 stress charges; 4 with a fluid source).  Cell
// k's weights for term blockIdx.y are at W + k ldw + blockIdx.y tstride.
// MFMA operands: lane L holds A[L%16][L/16] and B[L/16][L%16]; accumulator
// register r of lane L holds D[4r + L/16][L%16].
// Chain b is the steps coff[b] .. coff[b+1] - 1 (step b alone when coff is
// null); step i is item[5 i .. 5 i + 4] = (parent, its four children or -1).
template <int P, int NC>
__global__ __launch_bounds__(XT) void k_m2m(int nchain, const int *__restrict__ coff, const int *__restrict__ item,
                                            const double *__restrict__ S, int ldw, int tstride,
                                            double *__restrict__ W)
{
    constexpr int P2 = P * P, R = NC * P, RS = P + 1;
    constexpr int MT = (P + 15) / 16, KS = (P + 3) / 4, NT = (R + 15) / 16;  // x pass (P x P).(P x R)
    constexpr int MY = (R + 15) / 16, NY = (P + 15) / 16, MYW = (MY + 3) / 4;  // y pass (R x P).(P x P)
    __shared__ double X[4][R * RS];  // x pass of child d: X_d[(c, l)][m], rows padded
    W += (size_t)blockIdx.y * tstride;
    const int b = xcd_remap(blockIdx.x, nchain);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    // x pass A operands: S_{wave & 1}[16 mt + li][4 ks + lk]
    double ax[MT][KS];
    {
        const double *Sx = S + (wave & 1) * P2;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int r = 16 * mt + li, k = 4 * ks + lk;
                ax[mt][ks] = (r < P && k < P) ? Sx[r * P + k] : 0.0;
            }
    }
    // y pass B operands: B[k][n] = S_sy[n][k] at n = 16 nt + li, k = 4 ks + lk
    double by[2][KS][NY];
#pragma unroll
    for (int sy = 0; sy < 2; ++sy)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int nt = 0; nt < NY; ++nt) {
                const int n = 16 * nt + li, k = 4 * ks + lk;
                by[sy][ks][nt] = (n < P && k < P) ? S[sy * P2 + n * P + k] : 0.0;
            }
    const int i0 = coff ? coff[b] : b, i1 = coff ? coff[b + 1] : b + 1;
    // child ch's weights as the x pass's B operands: bw[ks][nt] =
    // W_ch[l' = 4 ks + lk][(c, m) = 16 nt + li]
    double bw[KS][NT];
    auto load_child = [&](int ch) {
        const double *Wd = W + (size_t)ch * ldw;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int k = 4 * ks + lk, col = 16 * nt + li, c = col / P, m = col - c * P;
                bw[ks][nt] = (k < P && col < R) ? Wd[c * P2 + k * P + m] : 0.0;
            }
    };
    int ch = i0 < i1 ? item[5 * i0 + 1 + wave] : -1;
    if (ch >= 0) load_child(ch);
    for (int it = i0; it < i1; ++it) {
        const int A = item[5 * it];
        // x pass, wave d on child d: X_d = S_{d&1} . W_d with W_d as the
        // P x R matrix [l'][(c, m)]
        {
            double *Xd = X[wave];
            if (ch >= 0) {
                d4 acc[MT][NT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt)
                            acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax[mt][ks], bw[ks][nt], acc[mt][nt],
                                                                               0, 0, 0);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int l = 16 * mt + 4 * r + lk, col = 16 * nt + li, c = col / P, m = col - c * P;
                            if (l < P && col < R) Xd[(c * P + l) * RS + m] = acc[mt][nt][r];
                        }
            } else {
                for (int e = lane; e < R * RS; e += 64) Xd[e] = 0.0;
            }
        }
        // the next step's child is fetched while this step's y pass runs,
        // unless it is this step's parent (written below)
        const int chn = it + 1 < i1 ? item[5 * (it + 1) + 1 + wave] : -1;
        const bool early = chn >= 0 && chn != A;
        if (early) load_child(chn);
        __syncthreads();
        // y pass: W_A = sum_sy (X_{0,sy} + X_{1,sy}) . S_sy^T, wave w on row
        // tiles w, w + 4, ... of the R x P result
        {
            double *WA = W + (size_t)A * ldw;
#pragma unroll
            for (int i = 0; i < MYW; ++i) {
                const int mt = wave + 4 * i;
                if (mt < MY) {
                    d4 acc[NY];
#pragma unroll
                    for (int nt = 0; nt < NY; ++nt) acc[nt] = d4{0.0, 0.0, 0.0, 0.0};
                    const int row = 16 * mt + li;
#pragma unroll
                    for (int sy = 0; sy < 2; ++sy)
#pragma unroll
                        for (int ks = 0; ks < KS; ++ks) {
                            const int k = 4 * ks + lk;
                            const double a = (row < R && k < P)
                                                 ? X[2 * sy][row * RS + k] + X[2 * sy + 1][row * RS + k]
                                                 : 0.0;
#pragma unroll
                            for (int nt = 0; nt < NY; ++nt)
                                acc[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, by[sy][ks][nt], acc[nt], 0, 0, 0);
                        }
#pragma unroll
                    for (int nt = 0; nt < NY; ++nt)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int rr = 16 * mt + 4 * r + lk, n = 16 * nt + li;
                            if (rr < R && n < P) WA[rr * P + n] = acc[nt][r];
                        }
                }
            }
        }
        // the parent's weights are written before a later parent of the
        // chain reads them, and X is free again
        __syncthreads();
        if (chn >= 0 && !early) load_child(chn);
        ch = chn;
    }
}

// ------------------------------------------------- gathered MFMA GEMM
// For every pair k of a tile (all pairs of a tile share operator o):
//   Z[dst[k]] = scale[k] * Op_o . X[src[k]]
// Op_o = ops + o * op_stride, row-major (Mrows x Kd, leading dim lda);
// X rows have leading dim ldx, Z rows ldz.  Mrows = gridDim.y * BM, Kd a
// multiple of 16; gridDim.z > 1 splits K, slice z of the result going to
// Z + z * zsplit.  Block: 4 waves in 2 x 2, each (BM/2) x (BN/2) built from
// 16x16x4 FP64 MFMA blocks.  Operand layout of v_mfma_f64_16x16x4f64: lane L
// holds A[L%16][L/16] and B[L/16][L%16]; accumulator register r of lane L
// holds D[4r + L/16][L%16].
template <int BM, int BN, int GK>
__global__ __launch_bounds__(256) void k_ggemm(const double *__restrict__ ops, size_t op_stride, int lda,
                                               int Kd, const double *__restrict__ X, int ldx,
                                               const int *__restrict__ tile_op, const int *__restrict__ tile_beg,
                                               const int *__restrict__ tile_end, const int *__restrict__ pair_src,
                                               const int *__restrict__ pair_dst,
                                               const double *__restrict__ pair_scale, double *__restrict__ Z,
                                               int ldz, size_t zsplit)
{
    constexpr int WM = BM / 32, WN = BN / 32;
    constexpr int RA = (BM * GK + 255) / 256, RB = (BN * GK + 255) / 256;
    __shared__ double As[BM][GK + 1];
    __shared__ double Bs[GK][BN + 1];
    __shared__ int src[BN];
    int tile = xcd_remap(blockIdx.x, gridDim.x), mt = blockIdx.y;  // an XCD takes a run of tiles (few operators)
    int o = tile_op[tile], pb = tile_beg[tile], np = tile_end[tile] - pb;
    int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    int wm = wave >> 1, wn = wave & 1;
    // split-K: this block sums k in [kb, ke); partial results go to slice z
    int ksteps = Kd / GK, per = (ksteps + gridDim.z - 1) / gridDim.z;
    int kb = min(Kd, (int)blockIdx.z * per * GK), ke = min(Kd, kb + per * GK);
    Z += (size_t)blockIdx.z * zsplit;
    if (tid < BN) src[tid] = tid < np ? pair_src[pb + tid] : -1;
    const double *A = ops + (size_t)o * op_stride + (size_t)mt * BM * lda;
    d4 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    __syncthreads();
    // the next k-step's operands are fetched into registers while the
    // current one is multiplied
    double ra[RA], rb[RB];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int r = 0; r < RA; ++r) {
            int e = tid + r * 256;
            if (e < BM * GK) ra[r] = A[(size_t)(e / GK) * lda + k0 + e % GK];
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            int e = tid + r * 256;
            if (e < BN * GK) {
                int s = src[e / GK];
                rb[r] = s >= 0 ? X[(size_t)s * ldx + k0 + e % GK] : 0.0;
            }
        }
    };
    if (kb < ke) fetch(kb);
    for (int k0 = kb; k0 < ke; k0 += GK) {
#pragma unroll
        for (int r = 0; r < RA; ++r) {
            int e = tid + r * 256;
            if (e < BM * GK) As[e / GK][e % GK] = ra[r];
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            int e = tid + r * 256;
            if (e < BN * GK) Bs[e % GK][e / GK] = rb[r];
        }
        __syncthreads();
        if (k0 + GK < ke) fetch(k0 + GK);
#pragma unroll
        for (int kk = 0; kk < GK; kk += 4) {
            double av[WM], bv[WN];
#pragma unroll
            for (int i = 0; i < WM; ++i) av[i] = As[wm * (BM / 2) + i * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < WN; ++j) bv[j] = Bs[kk + (lane >> 4)][wn * (BN / 2) + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < WN; ++j) {
        int col = wn * (BN / 2) + j * 16 + (lane & 15);
        if (col >= np) continue;
        double sc = pair_scale ? pair_scale[pb + col] : 1.0;
        double *z = Z + (size_t)pair_dst[pb + col] * ldz + mt * BM;
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) z[wm * (BM / 2) + i * 16 + 4 * r + (lane >> 4)] = sc * acc[i][j][r];
    }
}

// out[i] = sum over the split-K slices of part[z * stride + i], in order.
template <typename T>
__global__ void k_reduce_split(int64_t count, int nsplit, size_t stride, const T *__restrict__ part,
                               T *__restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    T s = 0;
    for (int z = 0; z < nsplit; ++z) s += part[(size_t)z * stride + i];
    out[i] = s;
}

// out[c] = sum of the pair products of cell c, in V-list order, accumulated
// in the precision of the products.
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_sum_pairs(int nfar, const int *__restrict__ far_cells,
                                                   const int *__restrict__ voff, const TI *__restrict__ Z,
                                                   int ldz, int width, TO *__restrict__ out, int ldo)
{
    constexpr int U = 8;  // loads in flight per thread; the sum stays in list order
    int c = far_cells[xcd_remap(blockIdx.x, nfar)];
    int kb = voff[c], ke = voff[c + 1];
    for (int e = threadIdx.x; e < width; e += 256) {
        TI s = 0;
        for (int k0 = kb; k0 < ke; k0 += U) {
            TI v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = Z[(size_t)min(k0 + u, ke - 1) * ldz + e];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (k0 + u < ke) s += v[u];
        }
        out[(size_t)c * ldo + e] = (TO)s;
    }
}

// ------------------------------------------- reduced-precision M2L products
// The grouped product of k_ggemm with operands held in FP32 or BF16 and the
// sums accumulated in FP32.  Operands are converted to the compute type CT
// (float, or bf16 as uint16_t bits) as they are staged in LDS, where both
// sit with k contiguous: As[m][k], Bs[n][k].  In each 16-deep k-step lane L
// reads the four consecutive k = kk + 4 (L/16) + i of row L%16 of both: one
// v_mfma_f32_16x16x16bf16_1k, or four v_mfma_f32_16x16x4f32 of which the
// i-th sums k = kk + 4 (L/16) + i (the order of a sum's index is free as
// long as A and B agree).  Accumulator register r of lane L holds
// D[4 (L/16) + r][L%16] for both instructions.
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

// float -> bf16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint32_t bf16_bits(float x)
{
    uint32_t u = __float_as_uint(x);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ void ld4(const double *p, float v[4])
{
    double2 a = *(const double2 *)p, b = *(const double2 *)(p + 2);
    v[0] = (float)a.x; v[1] = (float)a.y; v[2] = (float)b.x; v[3] = (float)b.y;
}
__device__ __forceinline__ void ld4(const float *p, float v[4])
{
    float4 a = *(const float4 *)p;
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}
__device__ __forceinline__ void ld4(const uint16_t *p, float v[4])
{
    uint2 a = *(const uint2 *)p;
    v[0] = __uint_as_float(a.x << 16); v[1] = __uint_as_float(a.x & 0xffff0000u);
    v[2] = __uint_as_float(a.y << 16); v[3] = __uint_as_float(a.y & 0xffff0000u);
}
__device__ __forceinline__ void st4(float *p, const float v[4]) { *(float4 *)p = float4{v[0], v[1], v[2], v[3]}; }
__device__ __forceinline__ void st4(uint16_t *p, const float v[4])
{
    *(uint2 *)p = uint2{bf16_bits(v[0]) | (bf16_bits(v[1]) << 16), bf16_bits(v[2]) | (bf16_bits(v[3]) << 16)};
}

template <typename CT> struct LdsPad;           // row padding of the LDS tiles, in elements
template <> struct LdsPad<float> { static constexpr int v = 4; };
template <> struct LdsPad<uint16_t> { static constexpr int v = 8; };

template <int BM, int BN, int GK, typename CT, typename TA, typename TX, typename TZ>
__global__ __launch_bounds__(256) void k_lgemm(const TA *__restrict__ ops, size_t op_stride, int lda, int Kd,
                                               const TX *__restrict__ X, int ldx, const int *__restrict__ tile_op,
                                               const int *__restrict__ tile_beg, const int *__restrict__ tile_end,
                                               const int *__restrict__ pair_src, const int *__restrict__ pair_dst,
                                               const double *__restrict__ pair_scale, TZ *__restrict__ Z, int ldz,
                                               size_t zsplit)
{
    constexpr int WM = BM / 32, WN = BN / 32, KP = GK + LdsPad<CT>::v;
    constexpr int G4 = GK / 4;                       // 4-element groups per row and k-step
    constexpr int RA = (BM * G4 + 255) / 256, RB = (BN * G4 + 255) / 256;
    __shared__ __align__(16) CT As[BM][KP];
    __shared__ __align__(16) CT Bs[BN][KP];
    __shared__ int src[BN];
    int tile = xcd_remap(blockIdx.x, gridDim.x), mt = blockIdx.y;  // an XCD takes a run of tiles (few operators)
    int o = tile_op[tile], pb = tile_beg[tile], np = tile_end[tile] - pb;
    int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    int wm = wave >> 1, wn = wave & 1;
    int ksteps = Kd / GK, per = (ksteps + gridDim.z - 1) / gridDim.z;
    int kb = min(Kd, (int)blockIdx.z * per * GK), ke = min(Kd, kb + per * GK);
    Z += (size_t)blockIdx.z * zsplit;
    if (tid < BN) src[tid] = tid < np ? pair_src[pb + tid] : -1;
    const TA *A = ops + (size_t)o * op_stride + (size_t)mt * BM * lda;
    f4 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    __syncthreads();
    float ra[RA][4], rb[RB][4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int r = 0; r < RA; ++r) {
            int e = tid + r * 256;
            if (e < BM * G4) ld4(A + (size_t)(e / G4) * lda + k0 + 4 * (e % G4), ra[r]);
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            int e = tid + r * 256;
            if (e < BN * G4) {
                int s = src[e / G4];
                if (s >= 0) ld4(X + (size_t)s * ldx + k0 + 4 * (e % G4), rb[r]);
                else rb[r][0] = rb[r][1] = rb[r][2] = rb[r][3] = 0.f;
            }
        }
    };
    if (kb < ke) fetch(kb);
    for (int k0 = kb; k0 < ke; k0 += GK) {
#pragma unroll
        for (int r = 0; r < RA; ++r) {
            int e = tid + r * 256;
            if (e < BM * G4) st4(&As[e / G4][4 * (e % G4)], ra[r]);
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            int e = tid + r * 256;
            if (e < BN * G4) st4(&Bs[e / G4][4 * (e % G4)], rb[r]);
        }
        __syncthreads();
        if (k0 + GK < ke) fetch(k0 + GK);
#pragma unroll
        for (int kk = 0; kk < GK; kk += 16) {
            int kq = kk + 4 * (lane >> 4);
            if constexpr (sizeof(CT) == 4) {
                f4 av[WM], bv[WN];
#pragma unroll
                for (int i = 0; i < WM; ++i) av[i] = *(const f4 *)&As[wm * (BM / 2) + i * 16 + (lane & 15)][kq];
#pragma unroll
                for (int j = 0; j < WN; ++j) bv[j] = *(const f4 *)&Bs[wn * (BN / 2) + j * 16 + (lane & 15)][kq];
#pragma unroll
                for (int i = 0; i < WM; ++i)
#pragma unroll
                    for (int j = 0; j < WN; ++j)
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i][c], bv[j][c], acc[i][j], 0, 0, 0);
            } else {
                s4 av[WM], bv[WN];
#pragma unroll
                for (int i = 0; i < WM; ++i) av[i] = *(const s4 *)&As[wm * (BM / 2) + i * 16 + (lane & 15)][kq];
#pragma unroll
                for (int j = 0; j < WN; ++j) bv[j] = *(const s4 *)&Bs[wn * (BN / 2) + j * 16 + (lane & 15)][kq];
#pragma unroll
                for (int i = 0; i < WM; ++i)
#pragma unroll
                    for (int j = 0; j < WN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[i], bv[j], acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < WN; ++j) {
        int col = wn * (BN / 2) + j * 16 + (lane & 15);
        if (col >= np) continue;
        float sc = pair_scale ? (float)pair_scale[pb + col] : 1.0f;
        TZ *z = Z + (size_t)pair_dst[pb + col] * ldz + mt * BM;
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) z[wm * (BM / 2) + i * 16 + 4 * (lane >> 4) + r] = (TZ)(sc * acc[i][j][r]);
    }
}

// Operator copies for the reduced-precision products.
__global__ void k_to_f32(int64_t n, const double *__restrict__ a, float *__restrict__ b)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}
__global__ void k_to_bf16(int64_t n, const double *__restrict__ a, uint16_t *__restrict__ b)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (uint16_t)bf16_bits((float)a[i]);
}

// Unit-size M2L operators: target square centred at the origin, half-width
// 1; source square centred at (2 dx, 2 dy).  One thread per node pair.
__global__ void k_m2l_ops(int nop, const int *__restrict__ odx, const int *__restrict__ ody,
                          const double *__restrict__ xbar, int p, int Mp, double gc,
                          double *__restrict__ ops)
{
    int p2 = p * p;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t per = (int64_t)p2 * p2;
    if (t >= per * nop) return;
    int o = (int)(t / per);
    int r = (int)(t - (int64_t)o * per);
    int tn = r / p2, sn = r - tn * p2;
    double X = xbar[tn / p], Y = xbar[tn % p];
    double sx = 2.0 * odx[o] + xbar[sn / p], sy = 2.0 * ody[o] + xbar[sn % p];
    double K[9];
    point_kernel(X - sx, Y - sy, gc, K);
    double *op = ops + (size_t)o * Mp * Mp;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) op[(size_t)(a * p2 + tn) * Mp + b * p2 + sn] = K[a * 3 + b];
}

// All operators side by side, column-major M x (nop M):
// fat[(o M + k) M + i] = K_o[i][k].
// uniform random numbers in [-1, 1) from the splitmix64 finaliser of the
// index (the range finder's test matrices; deterministic)
__global__ void k_rf_rand(int64_t count, uint64_t seed, double *__restrict__ out)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(e + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    out[e] = (double)(z >> 11) * 0x1.0p-52 - 1.0;
}

// L = R^T from the QR factorisation of B^T (N x k, leading dimension N,
// R in its upper triangle): the LQ factor of B, k x k column-major
__global__ void k_rf_lower(int k, int64_t N, const double *__restrict__ qr, double *__restrict__ L)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= k * k) return;
    int j = e / k, i = e - j * k;
    L[e] = i >= j ? qr[(size_t)i * N + j] : 0.0;
}

__global__ void k_pack_fat(int nop, int M, int Mp, const double *__restrict__ ops, double *__restrict__ fat)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t tot = (int64_t)nop * M * M;
    if (t >= tot) return;
    int i = (int)(t % M);
    int64_t col = t / M;
    int o = (int)(col / M), k = (int)(col % M);
    fat[t] = ops[(size_t)o * Mp * Mp + (size_t)i * Mp + k];
}

// From the column-major left singular vectors U (M x M, leading dim M):
// Vt (rp x Mp, row i = vector i) and Ur (Mp x rp, column i = vector i);
// zero outside the first r vectors and the first M entries.
__global__ void k_bases(int M, int Mp, int r, int rp, const double *__restrict__ U, double *__restrict__ Vt,
                        double *__restrict__ Ur)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)rp * Mp) return;
    int i = (int)(t / Mp), k = (int)(t % Mp);
    double v = (i < r && k < M) ? U[(size_t)i * M + k] : 0.0;
    Vt[(size_t)i * Mp + k] = v;
    Ur[(size_t)k * rp + i] = v;
}

// ops[o][j][i] = scale * Ct[o rp + i][j]
__global__ void k_transpose_ops(int nop, int rp, double scale, const double *__restrict__ Ct,
                                double *__restrict__ ops)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nop * rp * rp) return;
    int o = (int)(t / ((int64_t)rp * rp));
    int r = (int)(t % ((int64_t)rp * rp));
    int j = r / rp, i = r % rp;
    ops[t] = scale * Ct[((size_t)o * rp + i) * rp + j];
}

// ------------------------------------------------------------ L2P
// Far-field stress at every midpoint, eqs. 3.9-3.11: the chain of
// parent-to-child interpolations of the downward pass followed by the
// interpolation at the point is the evaluation of each ancestor's M2L
// field (a polynomial on that ancestor's square) at the point, so every
// far cell's field is evaluated directly at the points below it.  Work
// items are (far cell, chunk of up to 32 of its points); an item loads the
// cell's field once, forms the barycentric interpolants Sx, Sy of its
// points, computes R[(c,l)][t] = sum_m G[c][l][m] Sy[t][m] on FP64 MFMA
// (rows (c,l) in 16-row tiles, one per wave; points in two 16-column
// tiles; m in k-steps of 4) and sigma_c(t) = sum_l Sx[t][l] R[(c,l)][t]
// (summed within each row tile in registers and by a fixed butterfly, then
// over the tiles in order), and writes it to the slot of the cell's level:
// far[((level - 2) n + point) NC + c].  The final pass sums a point's levels
// in order.
constexpr int LT = 256, LTM = 32;

// NC field components per cell (rows of G, stride ldg).
template <int P, int NC>
__global__ __launch_bounds__(LT) void k_l2p(int nitem, const int *__restrict__ it_cell,
                                            const int *__restrict__ it_p0, const int *__restrict__ pend,
                                            const int *__restrict__ level, const double *__restrict__ ccx,
                                            const double *__restrict__ ccy, const double *__restrict__ chw,
                                            const double *__restrict__ cx, const double *__restrict__ cy,
                                            const double *__restrict__ G, int ldg, const double *__restrict__ xbar,
                                            const double *__restrict__ bw, int n, double *__restrict__ far)
{
    constexpr int P2 = P * P, N3 = NC * P2;
    constexpr int RT = (NC * P + 15) / 16;  // 16-row tiles over (c, l)
    constexpr int KS = (P + 3) / 4;         // k-steps over m
    __shared__ double Gb[N3];
    __shared__ double Sx[LTM][P + 1], Sy[LTM][P + 1];
    __shared__ double part[RT][NC][LTM];  // per row tile: sum over its rows of each component
    __shared__ double s_xb[P], s_bw[P];
    int item = xcd_remap(blockIdx.x, nitem);
    int A = it_cell[item], t0 = it_p0[item];
    int ntp = min(LTM, pend[A] - t0);
    int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const double *GA = G + (size_t)A * ldg;
    for (int e = tid; e < N3; e += LT) Gb[e] = GA[e];
    if (tid < P) {
        s_xb[tid] = xbar[tid];
        s_bw[tid] = bw[tid];
    }
    __syncthreads();
    if (tid < 2 * LTM) {
        int t = tid >> 1, coord = tid & 1;
        double *dst = coord ? Sy[t] : Sx[t];
        if (t < ntp) {
            double ih = 1.0 / chw[A];
            double u = coord ? (cy[t0 + t] - ccy[A]) * ih : (cx[t0 + t] - ccx[A]) * ih;
            double S[P];
            bary<P>(s_xb, s_bw, u, S);
#pragma unroll
            for (int m = 0; m < P; ++m) dst[m] = S[m];
        } else {
#pragma unroll
            for (int m = 0; m < P; ++m) dst[m] = 0.0;
        }
    }
    __syncthreads();
    for (int mt = wave; mt < RT; mt += 4) {
        d4 r0 = {0.0, 0.0, 0.0, 0.0}, r1 = {0.0, 0.0, 0.0, 0.0};
        int row = 16 * mt + (lane & 15);
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            int m = 4 * s + (lane >> 4);
            double av = (row < NC * P && m < P) ? Gb[row * P + m] : 0.0;
            double b0 = m < P ? Sy[lane & 15][m] : 0.0;
            double b1 = m < P ? Sy[16 + (lane & 15)][m] : 0.0;
            r0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b0, r0, 0, 0, 0);
            r1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b1, r1, 0, 0, 0);
        }
        // sigma_c(t) over this tile's rows: each lane sums its four rows
        // (r ascending) per component, then the four row groups of a column
        // are combined by a fixed butterfly
        const int t = lane & 15;
        double a0[NC], a1[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) a0[c] = a1[c] = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int rw = 16 * mt + 4 * r + (lane >> 4);
            if (rw < NC * P) {
                const int c = rw / P, l = rw - c * P;
                const double x0 = r0[r] * Sx[t][l], x1 = r1[r] * Sx[t + 16][l];
#pragma unroll
                for (int cc = 0; cc < NC; ++cc)
                    if (cc == c) {
                        a0[cc] += x0;
                        a1[cc] += x1;
                    }
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            a0[c] += __shfl_xor(a0[c], 16);
            a1[c] += __shfl_xor(a1[c], 16);
            a0[c] += __shfl_xor(a0[c], 32);
            a1[c] += __shfl_xor(a1[c], 32);
        }
        if (lane < 16)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                part[mt][c][t] = a0[c];
                part[mt][c][t + 16] = a1[c];
            }
    }
    __syncthreads();
    if (tid < NC * LTM) {
        int t = tid & 31, comp = tid >> 5;
        if (t < ntp) {
            double sum = 0.0;
#pragma unroll
            for (int mt = 0; mt < RT; ++mt) sum += part[mt][comp][t];
            far[(((size_t)(level[A] - 2)) * n + t0 + t) * NC + comp] = sum;
        }
    }
}

// ------------------------------------------------------------ P2P
// Exact element interactions.  A work item is one leaf and a chunk of at
// most NEAR_CHUNK of its near sources (the sources of its U and W lists and
// of the X lists of the leaf and its ancestors, flattened per leaf), so a
// leaf with a large near list is spread over several blocks.  Sources are
// staged in LDS; `tpt` adjacent lanes per point combine in a fixed order;
// the item's partial stresses go to part_s.  RT = float is the
// reduced-precision variant: offsets formed in FP64, the element formulas
// and the per-point sums in FP32.
constexpr int NT = 128;

template <typename RT>
__global__ __launch_bounds__(NT) void k_p2p(
    int nitem, const int *__restrict__ it_leaf, const int *__restrict__ it_s0, const int *__restrict__ it_s1,
    const int *__restrict__ it_poff, const int *__restrict__ leaves, const int *__restrict__ pbeg,
    const int *__restrict__ pend, const int *__restrict__ nfoff, const int *__restrict__ nflat,
    const double *__restrict__ cx, const double *__restrict__ cy, const double *__restrict__ cb,
    const double *__restrict__ sb, const double *__restrict__ a, const double *__restrict__ Ds, double gc,
    double *__restrict__ part)
{
    __shared__ double s_cx[NEAR_CHUNK], s_cy[NEAR_CHUNK];
    __shared__ RT s_cb[NEAR_CHUNK], s_sb[NEAR_CHUNK], s_c2[NEAR_CHUNK], s_s2[NEAR_CHUNK], s_a[NEAR_CHUNK],
        s_ds[NEAR_CHUNK], s_dn[NEAR_CHUNK];
    __shared__ double s_red[3 * NT];
    int k = xcd_remap(blockIdx.x, nitem);
    int li = it_leaf[k], s0 = it_s0[k], s1 = it_s1[k];
    int c = leaves[li];
    int tid = threadIdx.x;
    int tb = pbeg[c], te = pend[c], nt = te - tb;
    // the leaf's near sources, flattened: position v is point nflat[nfoff[li] + v]
    const int *src = nflat + nfoff[li];
    for (int v = s0 + tid; v < s1; v += NT) {
        int j = src[v];
        int q = v - s0;
        double cc = cb[j], ss = sb[j];
        s_cx[q] = cx[j]; s_cy[q] = cy[j]; s_cb[q] = (RT)cc; s_sb[q] = (RT)ss;
        s_c2[q] = (RT)(cc * cc - ss * ss); s_s2[q] = (RT)(2.0 * cc * ss);
        s_a[q] = (RT)a[j]; s_ds[q] = (RT)Ds[2 * j]; s_dn[q] = (RT)Ds[2 * j + 1];
    }
    __syncthreads();
    const int cnt = s1 - s0;
    // tpt lanes per target point, tpt = NT / nt (at most 16): with leaves of
    // 33-63 points a power of two would idle up to half the lanes.  Lane
    // (g, sub) takes sources sub, sub + tpt, ...; the tpt partials of a
    // point are summed in LDS in lane order.
    const int tpt = nt >= NT ? 1 : min(16, NT / nt);
    const int tpg = NT / tpt, g = tid / tpt, sub = tid - g * tpt;
    double *pk = part + 3 * (size_t)it_poff[k];
    for (int t0 = tb; t0 < te; t0 += tpg) {
        const int i = t0 + g;
        const bool act = g < tpg && i < te;
        double X = act ? cx[i] : 0.0, Y = act ? cy[i] : 0.0;
        RT sxx = 0, syy = 0, sxy = 0;
        if (act) {
            if constexpr (sizeof(RT) == 8) {
                for (int q = sub; q < cnt; q += tpt)
                    elem_stress_unit(X, Y, s_cx[q], s_cy[q], s_cb[q], s_sb[q], s_c2[q], s_s2[q], s_a[q], s_ds[q],
                                     s_dn[q], sxx, syy, sxy);
                sxx *= -gc;
                syy *= -gc;
                sxy *= -gc;
            } else {
                float gf = (float)gc;
                for (int q = sub; q < cnt; q += tpt)
                    elem_stress_add32((float)(X - s_cx[q]), (float)(Y - s_cy[q]), s_cb[q], s_sb[q], s_a[q],
                                      s_ds[q], s_dn[q], gf, sxx, syy, sxy);
            }
        }
        if (tpt == 1) {
            if (act) {
                double *o = pk + 3 * (size_t)(i - tb);
                o[0] = sxx;
                o[1] = syy;
                o[2] = sxy;
            }
            continue;
        }
        s_red[tid] = sxx;
        s_red[NT + tid] = syy;
        s_red[2 * NT + tid] = sxy;
        __syncthreads();
        if (act && sub == 0) {
            double r0 = 0.0, r1 = 0.0, r2 = 0.0;
            for (int u = tid; u < tid + tpt; ++u) {
                r0 += s_red[u];
                r1 += s_red[NT + u];
                r2 += s_red[2 * NT + u];
            }
            double *o = pk + 3 * (size_t)(i - tb);
            o[0] = r0;
            o[1] = r1;
            o[2] = r2;
        }
        __syncthreads();
    }
}

// Total stress at each point = far field + the near-field partials of its
// leaf's work items (in item order); projected to (shear, normal) traction
// and written in caller order.
__global__ void k_final(int n, const int *__restrict__ tleaf, const int *__restrict__ leaves,
                        const int *__restrict__ pbeg, const int *__restrict__ level,
                        const int *__restrict__ lk_off, const int *__restrict__ it_poff,
                        const double *__restrict__ part, const double *__restrict__ far,
                        const double *__restrict__ cb, const double *__restrict__ sb, const int *__restrict__ perm,
                        double *__restrict__ out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int li = tleaf[i];
    int c = leaves[li];
    int t = i - pbeg[c];
    double sxx = 0.0, syy = 0.0, sxy = 0.0;
    if (far)  // the fields of the point's cells at levels 2 .. its leaf's, in level order
        for (int l = 2; l <= level[c]; ++l) {
            const double *f = far + ((size_t)(l - 2) * n + i) * 3;
            sxx += f[0];
            syy += f[1];
            sxy += f[2];
        }
    for (int k = lk_off[li]; k < lk_off[li + 1]; ++k) {
        const double *o = part + 3 * ((size_t)it_poff[k] + t);
        sxx += o[0];
        syy += o[1];
        sxy += o[2];
    }
    double ts, tn;
    traction(cb[i], sb[i], sxx, syy, sxy, ts, tn);
    int j = perm[i];
    out[2 * j] = ts;
    out[2 * j + 1] = tn;
}

// ------------------------------------------------------- host helpers



constexpr int TILE_N = 32;  // pairs per GEMM tile (the BN of the launches)
// M2L GEMM tile sets (fmddm_params.m2l_tiles): split-K factor of the
// projection onto the singular vectors, row-tile height of the pair
// products and of the expansion back onto the nodes
struct TileSet {
    int ksplit, bm_pair, bm_back;
};
constexpr TileSet TILESETS[4] = {{4, 64, 64}, {2, 32, 64}, {8, 64, 32}, {4, 32, 32}};
constexpr int KSPLIT_MAX = 8;

void upload(hipStream_t s, DBuf<int> &d, const std::vector<int> &h)
{
    d.alloc(h.size());
    if (!h.empty()) FM_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * 4, hipMemcpyHostToDevice, s));
}

void upload(hipStream_t s, DBuf<double> &d, const std::vector<double> &h)
{
    d.alloc(h.size());
    if (!h.empty()) FM_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * 8, hipMemcpyHostToDevice, s));
}

// Upward-pass schedule (eq. 3.7 bottom-up).  Every internal cell of level
// >= 2 is a parent.  The subtrees below a cut level Lc run as one chain
// each in one launch; each level above Lc is a launch of one-parent
// chains.  Lc minimises a latency model: a launch costs about T_LAUNCH, a
// parent on its block about T_PARENT (both microseconds, measured on
// MI355X at p = 20), so the deep launch costs its longest chain.
void m2m_schedule(hipStream_t s, fmddm_tree *t)
{
    constexpr double T_LAUNCH = 4.0, T_PARENT = 2.5;
    constexpr int WAVE_BLOCKS = 512;  // parents one launch runs side by side
    const int ncell = t->ncell, maxlev = t->nlevel - 1;
    t->m2m_launch.clear();
    std::vector<int> hch(4 * (size_t)std::max(ncell, 1));
    FM_HIP(hipMemcpyAsync(hch.data(), t->cchild.p, 4 * (size_t)ncell * sizeof(int), hipMemcpyDeviceToHost, s));
    FM_HIP(hipStreamSynchronize(s));
    std::vector<std::vector<int>> bylev(std::max(maxlev + 1, 3));
    for (int c = 0; c < ncell; ++c)
        if (!t->h_isleaf[c] && t->h_level[c] >= 2) bylev[t->h_level[c]].push_back(c);
    // internal cells of each parent's subtree (itself included)
    std::vector<int> sub(ncell, 0);
    for (int l = maxlev; l >= 2; --l)
        for (int c : bylev[l]) {
            sub[c] = 1;
            for (int d = 0; d < 4; ++d)
                if (hch[4 * c + d] >= 0) sub[c] += sub[hch[4 * c + d]];
        }
    int best = maxlev + 1;
    double best_cost = 1e300;
    for (int Lc = 2; Lc <= maxlev + 1; ++Lc) {
        double cost = 0.0;
        int longest = 0;
        if (Lc <= maxlev)
            for (int c : bylev[Lc]) longest = std::max(longest, sub[c]);
        if (longest) cost += T_LAUNCH + longest * T_PARENT;
        for (int l = 2; l < Lc && l <= maxlev; ++l)
            if (!bylev[l].empty())
                cost += T_LAUNCH + T_PARENT * (double)((bylev[l].size() + WAVE_BLOCKS - 1) / WAVE_BLOCKS);
        if (cost < best_cost) {
            best_cost = cost;
            best = Lc;
        }
    }
    std::vector<int> coff(1, 0), par;
    auto close_launch = [&](int first) {
        int nch = (int)coff.size() - 1 - first;
        if (nch <= 0) return;
        fmddm_tree::M2MLaunch L;
        L.first = first;
        L.nchain = nch;
        L.step0 = coff[first];
        L.single = coff[first + nch] - coff[first] == nch;
        t->m2m_launch.push_back(L);
    };
    // deep launch: each subtree rooted at level best, deepest parents first
    if (best <= maxlev) {
        int first = (int)coff.size() - 1;
        std::vector<int> cells, stack;
        for (int r : bylev[best]) {
            cells.clear();
            stack.assign(1, r);
            while (!stack.empty()) {
                int c = stack.back();
                stack.pop_back();
                cells.push_back(c);
                for (int d = 0; d < 4; ++d) {
                    int k = hch[4 * c + d];
                    if (k >= 0 && !t->h_isleaf[k]) stack.push_back(k);
                }
            }
            std::stable_sort(cells.begin(), cells.end(),
                             [&](int a, int b) { return t->h_level[a] > t->h_level[b]; });
            par.insert(par.end(), cells.begin(), cells.end());
            coff.push_back((int)par.size());
        }
        close_launch(first);
    }
    // one launch per level above it, deepest first
    for (int l = std::min(best, maxlev + 1) - 1; l >= 2; --l) {
        int first = (int)coff.size() - 1;
        for (int c : bylev[l]) {
            par.push_back(c);
            coff.push_back((int)par.size());
        }
        close_launch(first);
    }
    t->m2m_cut = best;
    // per launch: chain offsets from its first step (at m2m_coff + first)
    std::vector<int> item(5 * par.size());
    for (size_t i = 0; i < par.size(); ++i) {
        item[5 * i] = par[i];
        for (int d = 0; d < 4; ++d) item[5 * i + 1 + d] = hch[4 * (size_t)par[i] + d];
    }
    std::vector<int> loff;
    for (fmddm_tree::M2MLaunch &L : t->m2m_launch) {
        int at = (int)loff.size();
        for (int c = L.first; c <= L.first + L.nchain; ++c) loff.push_back(coff[c] - L.step0);
        L.first = at;
    }
    upload(s, t->m2m_coff, loff);
    upload(s, t->m2m_item, item);
    FM_HIP(hipStreamSynchronize(s));
}

template <int BM, int BN>
void launch_ggemm(hipStream_t s, int ntile, int Mrows, const double *ops, size_t op_stride, int lda, int Kd,
                  const double *X, int ldx, const int *top, const int *tbeg, const int *tend,
                  const int *psrc, const int *pdst, const double *pscale, double *Z, int ldz,
                  int nsplit = 1, size_t zsplit = 0)
{
    if (ntile == 0) return;
    if (Mrows % BM || Kd % 16) throw Error{FMDDM_EDEVICE, "GEMM shape not tiled"};
    // long K: 64-deep k-steps keep 16 MFMA per wave busy per fetched tile;
    // short K: 16-deep steps, smaller tiles in LDS and more blocks per CU
    if (Kd % 64 == 0 && Kd >= 512)
        hipLaunchKernelGGL((k_ggemm<BM, BN, 64>), dim3(ntile, Mrows / BM, nsplit), dim3(256), 0, s, ops, op_stride,
                           lda, Kd, X, ldx, top, tbeg, tend, psrc, pdst, pscale, Z, ldz, zsplit);
    else
        hipLaunchKernelGGL((k_ggemm<BM, BN, 16>), dim3(ntile, Mrows / BM, nsplit), dim3(256), 0, s, ops, op_stride,
                           lda, Kd, X, ldx, top, tbeg, tend, psrc, pdst, pscale, Z, ldz, zsplit);
    FM_CHECK_LAUNCH();
}

template <int BM, int BN, typename CT, typename TA, typename TX, typename TZ>
void launch_lgemm(hipStream_t s, int ntile, int Mrows, const TA *ops, size_t op_stride, int lda, int Kd,
                  const TX *X, int ldx, const int *top, const int *tbeg, const int *tend, const int *psrc,
                  const int *pdst, const double *pscale, TZ *Z, int ldz, int nsplit = 1, size_t zsplit = 0)
{
    if (ntile == 0) return;
    // 4-element vector loads need rows and k-steps on multiples of 4
    if (Mrows % BM || Kd % 16 || lda % 4 || ldx % 4 || op_stride % 4)
        throw Error{FMDDM_EDEVICE, "GEMM shape not tiled"};
    if (Kd % 64 == 0 && Kd >= 512)
        hipLaunchKernelGGL((k_lgemm<BM, BN, 64, CT, TA, TX, TZ>), dim3(ntile, Mrows / BM, nsplit), dim3(256), 0, s,
                           ops, op_stride, lda, Kd, X, ldx, top, tbeg, tend, psrc, pdst, pscale, Z, ldz, zsplit);
    else
        hipLaunchKernelGGL((k_lgemm<BM, BN, 16, CT, TA, TX, TZ>), dim3(ntile, Mrows / BM, nsplit), dim3(256), 0, s,
                           ops, op_stride, lda, Kd, X, ldx, top, tbeg, tend, psrc, pdst, pscale, Z, ldz, zsplit);
    FM_CHECK_LAUNCH();
}

// launch_ggemm / launch_lgemm with the row-tile height chosen at run time
template <class... A>
void ggemm_bm(int bm, hipStream_t s, A... a)
{
    if (bm == 32) launch_ggemm<32, 32>(s, a...);
    else launch_ggemm<64, 32>(s, a...);
}

template <typename CT, class... A>
void lgemm_bm(int bm, hipStream_t s, A... a)
{
    if (bm == 32) launch_lgemm<32, 32, CT>(s, a...);
    else launch_lgemm<64, 32, CT>(s, a...);
}

// The M2L products (projection, translation, expansion) at reduced
// precision: CT the MFMA operand type, TO the stored operators' type.
// Weights in: Wexp (FP64); fields out: Gexp (FP64); FP32 in between.
template <typename CT, typename TO>
void m2l_lowp(hipStream_t s, fmddm_tree *t, const M2LOps &M, const TO *Vt, const TO *ops, const TO *Ur,
              Profiler &P, const TileSet &ts)
{
    int Mp = M.Mp, rp = M.rp;
    hipEvent_t e0;
    if (M.mode == FMDDM_M2L_SVD) {
        P.begin(FMDDM_PH_COMPRESS, s, e0);
        launch_lgemm<32, 32, CT>(s, t->nftile, rp, Vt, 0, Mp, Mp, t->Wexp.p, Mp, t->ftile_op.p, t->ftile_beg.p,
                                 t->ftile_end.p, t->far_cells.p, t->far_cells.p, nullptr, t->ksplit32.p, rp,
                                 ts.ksplit, (size_t)t->ncell * rp);
        P.end(FMDDM_PH_COMPRESS, s, e0);
        P.begin(FMDDM_PH_COMPRESS_SUM, s, e0);
        {
            int64_t c0 = t->level_start[2], cnt = (int64_t)(t->ncell - c0) * rp;
            hipLaunchKernelGGL(k_reduce_split<float>, dim3(cdiv(cnt, 256)), dim3(256), 0, s, cnt, ts.ksplit,
                               (size_t)t->ncell * rp, t->ksplit32.p + c0 * rp, t->What32.p + c0 * rp);
            FM_CHECK_LAUNCH();
        }
        P.end(FMDDM_PH_COMPRESS_SUM, s, e0);
        P.begin(FMDDM_PH_M2L, s, e0);
        lgemm_bm<CT>(ts.bm_pair, s, t->ntile, rp, ops, (size_t)rp * rp, rp, rp, t->What32.p, rp, t->tile_op.p,
                                 t->tile_beg.p, t->tile_end.p, t->pair_src.p, t->pair_dst.p, t->pair_scale.p,
                                 t->Zm2l32.p, rp);
        P.end(FMDDM_PH_M2L, s, e0);
        P.begin(FMDDM_PH_M2L_SUM, s, e0);
        hipLaunchKernelGGL((k_sum_pairs<float, float>), dim3(t->nfar), dim3(256), 0, s, t->nfar, t->far_cells.p,
                           t->loff[1].p, t->Zm2l32.p, rp, rp, t->Ghat32.p, rp);
        FM_CHECK_LAUNCH();
        P.end(FMDDM_PH_M2L_SUM, s, e0);
        P.begin(FMDDM_PH_DECOMPRESS, s, e0);
        lgemm_bm<CT>(ts.bm_back, s, t->nftile, Mp, Ur, 0, rp, rp, t->Ghat32.p, rp, t->ftile_op.p,
                                 t->ftile_beg.p, t->ftile_end.p, t->far_cells.p, t->far_cells.p, nullptr,
                                 t->Gexp.p, Mp);
        P.end(FMDDM_PH_DECOMPRESS, s, e0);
    } else {
        P.begin(FMDDM_PH_M2L, s, e0);
        lgemm_bm<CT>(ts.bm_pair, s, t->ntile, Mp, ops, (size_t)Mp * Mp, Mp, Mp, t->Wexp.p, Mp, t->tile_op.p,
                                 t->tile_beg.p, t->tile_end.p, t->pair_src.p, t->pair_dst.p, t->pair_scale.p,
                                 t->Zm2l32.p, Mp);
        P.end(FMDDM_PH_M2L, s, e0);
        P.begin(FMDDM_PH_M2L_SUM, s, e0);
        hipLaunchKernelGGL((k_sum_pairs<float, double>), dim3(t->nfar), dim3(256), 0, s, t->nfar,
                           t->far_cells.p, t->loff[1].p, t->Zm2l32.p, Mp, Mp, t->Gexp.p, Mp);
        FM_CHECK_LAUNCH();
        P.end(FMDDM_PH_M2L_SUM, s, e0);
    }
}

}  // namespace

// Leading left singular vectors of A (m x N, column-major, N >= m) down to
// tol of the largest singular value, by a randomized range finder (Halko,
// Martinsson and Tropp, 2011): Y = A Om for k uniform random columns,
// Q = orth(Y) (Householder QR), B = Q^T A, B = L P (LQ, taken as the QR
// factorisation B^T = P^T L^T of the tall transpose), L = U_L S W^T
// (one-sided Jacobi SVD); then A ~ (Q U_L) S (P^T W)^T.  k starts at 192
// and doubles until the k-th singular value is a decade below tol (k = m:
// exact).
// U (m x m, leading dimension m) receives the vectors in its first k
// columns, sv the k singular values (descending); returns the number above
// tol (at least 1).  Runs on the handle's stream and waits for it.
int range_basis(void *hv, hipStream_t s, int m, int N, const double *A, double tol, double *U,
                std::vector<double> &sv)
{
    rocblas_handle h = (rocblas_handle)hv;
    const size_t mm = (size_t)m * m;
    DBuf<double> Om, Y, B, L, S, tau, UL, res;
    DBuf<int> info, sweeps;
    Om.alloc((size_t)N * std::min(m, 384));
    Y.alloc(mm);
    L.alloc(mm);
    UL.alloc(mm);
    S.alloc(m);
    tau.alloc(m);
    res.alloc(1);
    info.alloc(1);
    sweeps.alloc(1);
    const double one = 1.0, zero = 0.0;
    int k = std::min(m, 192);
    for (;;) {
        if ((size_t)N * k > Om.n) Om.alloc((size_t)N * k);
        if ((size_t)k * N > B.n) B.alloc((size_t)k * N);
        hipLaunchKernelGGL(k_rf_rand, dim3(cdiv((int64_t)N * k, 256)), dim3(256), 0, s, (int64_t)N * k,
                           (uint64_t)k, Om.p);
        FM_CHECK_LAUNCH();
        bool ok = rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, m, k, N, &one, A, m, Om.p, N,
                                &zero, Y.p, m) == rocblas_status_success;
        ok = ok && rocsolver_dgeqrf(h, m, k, Y.p, m, tau.p) == rocblas_status_success;
        ok = ok && rocsolver_dorgqr(h, m, k, k, Y.p, m, tau.p) == rocblas_status_success;
        // B = Q^T A (k x N) is wide; its LQ factor is R^T of the QR
        // factorisation of the tall B^T = A^T Q, which takes the blocked path
        ok = ok && rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, N, k, m, &one, A, m, Y.p,
                                 m, &zero, B.p, N) == rocblas_status_success;
        ok = ok && rocsolver_dgeqrf(h, N, k, B.p, N, tau.p) == rocblas_status_success;
        if (!ok) throw Error{FMDDM_EDEVICE, "range finder: rocBLAS / rocSOLVER call failed"};
        hipLaunchKernelGGL(k_rf_lower, dim3(cdiv((int64_t)k * k, 256)), dim3(256), 0, s, k, (int64_t)N, B.p, L.p);
        FM_CHECK_LAUNCH();
        if (rocsolver_dgesvdj(h, rocblas_svect_singular, rocblas_svect_none, k, k, L.p, k, 0.0, res.p, 100,
                              sweeps.p, S.p, UL.p, k, nullptr, 1, info.p) != rocblas_status_success)
            throw Error{FMDDM_EDEVICE, "range finder: rocsolver_dgesvdj failed"};
        int hinfo = 0;
        sv.assign(k, 0.0);
        FM_HIP(hipMemcpyAsync(&hinfo, info.p, 4, hipMemcpyDeviceToHost, s));
        FM_HIP(hipMemcpyAsync(sv.data(), S.p, (size_t)k * 8, hipMemcpyDeviceToHost, s));
        FM_HIP(hipStreamSynchronize(s));
        if (hinfo != 0) throw Error{FMDDM_EDEVICE, "range finder: the Jacobi SVD did not converge"};
        if (k < m && sv[k - 1] > 0.1 * tol * sv[0]) {  // a decade of margin below the cut
            k = std::min(m, 2 * k);
            continue;
        }
        if (rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, m, k, k, &one, Y.p, m, UL.p, k, &zero,
                          U, m) != rocblas_status_success)
            throw Error{FMDDM_EDEVICE, "range finder: rocblas_dgemm failed"};
        int r = 1;
        for (int i = 0; i < k; ++i)
            if (sv[0] > 0.0 && sv[i] > tol * sv[0]) r = i + 1;
        FM_HIP(hipStreamSynchronize(s));
        return r;
    }
}

// Reduced-precision copies of the operator set, made once (on first use,
// or up front where several threads share the set)
void lowp_ops(fmddm_ctx *ctx, int prec)
{
    M2LOps &M = *ctx->m2l;
    hipStream_t s = ctx->stream;
    auto conv32 = [&](const DBuf<double> &a, DBuf<float> &b) {
        b.alloc(a.n);
        hipLaunchKernelGGL(k_to_f32, dim3(cdiv(a.n, 256)), dim3(256), 0, s, (int64_t)a.n, a.p, b.p);
        FM_CHECK_LAUNCH();
    };
    auto conv16 = [&](const DBuf<double> &a, DBuf<uint16_t> &b) {
        b.alloc(a.n);
        hipLaunchKernelGGL(k_to_bf16, dim3(cdiv(a.n, 256)), dim3(256), 0, s, (int64_t)a.n, a.p, b.p);
        FM_CHECK_LAUNCH();
    };
    bool svd = M.mode == FMDDM_M2L_SVD;
    if (prec == FMDDM_PREC_FP32 && !M.have32) {
        conv32(M.ops, M.ops32);
        if (svd) {
            conv32(M.Vt, M.Vt32);
            conv32(M.Ur, M.Ur32);
        }
        FM_HIP(hipStreamSynchronize(s));
        M.have32 = true;
    }
    if (prec == FMDDM_PREC_BF16 && !M.have16) {
        conv16(M.ops, M.ops16);
        if (svd) {
            conv16(M.Vt, M.Vt16);
            conv16(M.Ur, M.Ur16);
        }
        FM_HIP(hipStreamSynchronize(s));
        M.have16 = true;
    }
}

namespace {

// the operator copies and the tree's FP32 intermediates (once per tree)
void setup_lowp(fmddm_ctx *ctx, fmddm_tree *t, int prec)
{
    lowp_ops(ctx, prec);
    M2LOps &M = *ctx->m2l;
    hipStream_t s = ctx->stream;
    bool svd = M.mode == FMDDM_M2L_SVD;
    if (!t->Zm2l32.p) {
        int w = svd ? M.rp : M.Mp;
        t->Zm2l32.alloc((size_t)std::max<int64_t>(t->nV, 1) * w);
        if (svd) {
            t->What32.alloc((size_t)t->ncell * M.rp);
            t->Ghat32.alloc((size_t)t->ncell * M.rp);
            t->ksplit32.alloc((size_t)KSPLIT_MAX * t->ncell * M.rp);
            t->What32.zero(s);
            t->Ghat32.zero(s);
        }
        FM_HIP(hipStreamSynchronize(s));
    }
}

template <int P, int NC = 3>
void launch_m2m(hipStream_t s, fmddm_ctx *ctx, fmddm_tree *t, int ldw, int nterm, int tstride, double *W)
{
    for (const fmddm_tree::M2MLaunch &L : t->m2m_launch) {
        hipLaunchKernelGGL((k_m2m<P, NC>), dim3(L.nchain, nterm), dim3(XT), 0, s, L.nchain,
                           L.single ? (const int *)nullptr : t->m2m_coff.p + L.first, t->m2m_item.p + 5 * L.step0,
                           ctx->cheb->m2mS.p, ldw, tstride, W);
        FM_CHECK_LAUNCH();
    }
}

template <int P, int NC = 3>
void launch_l2p(hipStream_t s, fmddm_ctx *ctx, fmddm_tree *t, const double *G, int ldg, double *far)
{
    if (t->nlpitem == 0) return;
    hipLaunchKernelGGL((k_l2p<P, NC>), dim3(t->nlpitem), dim3(LT), 0, s, t->nlpitem, t->lp_cell.p, t->lp_p0.p,
                       t->cpend.p, t->clevel.p, t->ccx.p, t->ccy.p, t->chw.p, t->scx.p, t->scy.p, G, ldg,
                       ctx->cheb->xbar.p, ctx->cheb->bw.p, (int)t->n, far);
    FM_CHECK_LAUNCH();
}

#define FM_DISPATCH_P(p, CALL)                                                          \
    switch (p) {                                                                        \
    case 1: CALL(1); break;   case 2: CALL(2); break;   case 3: CALL(3); break;        \
    case 4: CALL(4); break;   case 5: CALL(5); break;   case 6: CALL(6); break;        \
    case 7: CALL(7); break;   case 8: CALL(8); break;   case 9: CALL(9); break;        \
    case 10: CALL(10); break; case 11: CALL(11); break; case 12: CALL(12); break;      \
    case 13: CALL(13); break; case 14: CALL(14); break; case 15: CALL(15); break;      \
    case 16: CALL(16); break; case 17: CALL(17); break; case 18: CALL(18); break;      \
    case 19: CALL(19); break; case 20: CALL(20); break; case 21: CALL(21); break;      \
    case 22: CALL(22); break; case 23: CALL(23); break; case 24: CALL(24); break;      \
    case 25: CALL(25); break; case 26: CALL(26); break; case 27: CALL(27); break;      \
    case 28: CALL(28); break; case 29: CALL(29); break; case 30: CALL(30); break;      \
    case 31: CALL(31); break; case 32: CALL(32); break;                                \
    default: throw Error{FMDDM_EINVAL, "p out of range"};                               \
    }

// p of the four-component (poroelastic) passes
#define FM_DISPATCH_P16(p, CALL)                                                        \
    switch (p) {                                                                        \
    case 2: CALL(2); break;   case 3: CALL(3); break;   case 4: CALL(4); break;        \
    case 5: CALL(5); break;   case 6: CALL(6); break;   case 7: CALL(7); break;        \
    case 8: CALL(8); break;   case 9: CALL(9); break;   case 10: CALL(10); break;      \
    case 11: CALL(11); break; case 12: CALL(12); break; case 13: CALL(13); break;      \
    case 14: CALL(14); break; case 15: CALL(15); break; case 16: CALL(16); break;      \
    default: throw Error{FMDDM_EUNSUPPORTED, "four-component FMM needs 2 <= p <= 16"};  \
    }

}  // namespace

int offset_slot(int dx, int dy) { return (dx + 3) + 7 * (dy + 3); }

// Offsets (dx, dy) in [-3, 3]^2 outside [-1, 1]^2: the 40 relative
// positions of a V-list cell.
void v_offsets(std::vector<int> &dx, std::vector<int> &dy, std::vector<int> &slot2op)
{
    slot2op.assign(49, -1);
    for (int y = -3; y <= 3; ++y)
        for (int x = -3; x <= 3; ++x) {
            if (std::abs(x) <= 1 && std::abs(y) <= 1) continue;
            slot2op[offset_slot(x, y)] = (int)dx.size();
            dx.push_back(x);
            dy.push_back(y);
        }
}

// Gauss-Legendre nodes/weights on [-1, 1] (Newton on the Legendre
// recurrence).
void gauss_legendre(int n, std::vector<double> &t, std::vector<double> &w)
{
    t.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dpn = 1;
        for (int it = 0; it < 200; ++it) {
            double pm = 1.0, pc = x;
            for (int k = 2; k <= n; ++k) {
                double pk = ((2.0 * k - 1.0) * x * pc - (k - 1.0) * pm) / k;
                pm = pc;
                pc = pk;
            }
            if (n == 1) { pc = x; pm = 1.0; }
            dpn = n * (x * pc - pm) / (x * x - 1.0);
            double dx = pc / dpn;
            x -= dx;
            if (std::fabs(dx) < 1e-17) break;
        }
        double pm = 1.0, pc = x;
        for (int k = 2; k <= n; ++k) {
            double pk = ((2.0 * k - 1.0) * x * pc - (k - 1.0) * pm) / k;
            pm = pc;
            pc = pk;
        }
        if (n == 1) { pc = x; pm = 1.0; }
        dpn = n * (x * pc - pm) / (x * x - 1.0);
        t[i] = x;
        w[i] = 2.0 / ((1.0 - x * x) * dpn * dpn);
    }
}

// ------------------------------------------------------------ profiler
Profiler::~Profiler()
{
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    for (auto &v : rec)
        for (auto &pr : v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
}

hipEvent_t Profiler::take()
{
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e;
    FM_HIP(hipEventCreate(&e));
    return e;
}

void Profiler::begin(int ph, hipStream_t s, hipEvent_t &e0)
{
    e0 = nullptr;
    if (!(mask >> ph & 1u)) return;
    e0 = take();
    FM_HIP(hipEventRecord(e0, s));
}

void Profiler::end(int ph, hipStream_t s, hipEvent_t e0)
{
    if (!e0) return;
    hipEvent_t e1 = take();
    FM_HIP(hipEventRecord(e1, s));
    rec[ph].emplace_back(e0, e1);
}

void Profiler::read(hipStream_t s, double *ms, int64_t *count)
{
    FM_HIP(hipStreamSynchronize(s));
    for (int ph = 0; ph < FMDDM_PH_COUNT; ++ph) {
        double tot = 0.0;
        for (auto &pr : rec[ph]) {
            float t = 0.0f;
            FM_HIP(hipEventElapsedTime(&t, pr.first, pr.second));
            tot += t;
            pool.push_back(pr.first);
            pool.push_back(pr.second);
        }
        if (ms) ms[ph] = tot;
        if (count) count[ph] = (int64_t)rec[ph].size();
        rec[ph].clear();
    }
}

// ------------------------------------------------------------- set-up
// ------------------------------------------------ generic passes
// The passes of the product above for fields with four components per node
// (three eigenstrain charges and a fluid source), several terms at once:
// weights of cell k and term j at W + k ldw + j tstride.
void fmm_m2m4(fmddm_ctx *ctx, fmddm_tree *t, int nterm, int ldw, int tstride, double *W)
{
    if (t->m2m_launch.empty()) return;
    hipStream_t s = ctx->stream;
    int p = ctx->prm.p;
#define FM_M2M4(PP) launch_m2m<PP, 4>(s, ctx, t, ldw, nterm, tstride, W)
    FM_DISPATCH_P16(p, FM_M2M4)
#undef FM_M2M4
}

void fmm_l2p4(fmddm_ctx *ctx, fmddm_tree *t, const double *G, int ldg, double *far)
{
    hipStream_t s = ctx->stream;
#define FM_L2P4(PP) launch_l2p<PP, 4>(s, ctx, t, G, ldg, far)
    FM_DISPATCH_P16(ctx->prm.p, FM_L2P4)
#undef FM_L2P4
}

void fmm_pair_gemm(hipStream_t s, int ntile, int Mrows, const double *ops, size_t op_stride, int lda, int Kd,
                   const double *X, int ldx, const int *tile_op, const int *tile_beg, const int *tile_end,
                   const int *psrc, const int *pdst, double *Z, int ldz)
{
    launch_ggemm<64, 32>(s, ntile, Mrows, ops, op_stride, lda, Kd, X, ldx, tile_op, tile_beg, tile_end, psrc, pdst,
                         nullptr, Z, ldz);
}

// The same product with K split over nsplit slices (partials at part + z
// zsplit, leading dimension ldz) and the slices summed in order into
// Z[0 .. count): for few tiles over a long K.
void fmm_pair_gemm_split(hipStream_t s, int ntile, int Mrows, const double *ops, size_t op_stride, int lda, int Kd,
                         const double *X, int ldx, const int *tile_op, const int *tile_beg, const int *tile_end,
                         const int *psrc, const int *pdst, double *part, int ldz, int nsplit, size_t zsplit,
                         double *Z, int64_t count)
{
    if (ntile == 0) return;
    launch_ggemm<64, 32>(s, ntile, Mrows, ops, op_stride, lda, Kd, X, ldx, tile_op, tile_beg, tile_end, psrc, pdst,
                         nullptr, part, ldz, nsplit, zsplit);
    hipLaunchKernelGGL(k_reduce_split<double>, dim3(cdiv(count, 256)), dim3(256), 0, s, count, nsplit, zsplit, part,
                       Z);
    FM_CHECK_LAUNCH();
}

void fmm_sum_pairs(hipStream_t s, fmddm_tree *t, const double *Z, int ldz, int width, double *out, int ldo)
{
    if (t->nfar == 0) return;
    hipLaunchKernelGGL((k_sum_pairs<double, double>), dim3(t->nfar), dim3(256), 0, s, t->nfar, t->far_cells.p, t->loff[1].p, Z, ldz,
                       width, out, ldo);
    FM_CHECK_LAUNCH();
}

// The side stream and the fork/join events of a context (default priority).
void init_streams(fmddm_ctx *ctx)
{
    FM_HIP(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
    FM_HIP(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
    FM_HIP(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
    FM_HIP(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
}

void setup_cheb(fmddm_ctx *ctx)
{
    int p = ctx->prm.p;
    Cheb &C = *ctx->cheb;
    C.p = p;
    C.h_xbar.resize(p);
    C.h_bw.resize(p);
    C.h_tnode.resize(p * p);
    for (int l = 0; l < p; ++l) {
        double th = (2.0 * l + 1.0) * M_PI / (2.0 * p);
        C.h_xbar[l] = std::cos(th);
        C.h_bw[l] = (l & 1 ? -1.0 : 1.0) * std::sin(th);
        for (int k = 0; k < p; ++k) C.h_tnode[l * p + k] = std::cos(k * th);
    }
    gauss_legendre(p, C.h_glt, C.h_glw);
    // child-to-parent transfers of eq. 3.7: S_s[l][l'] = S_p(xbar_l, u) at
    // u = (xbar_l' + 2s - 1) / 2, by the Chebyshev sum 1/p + 2/p sum_k
    // T_k(xbar_l) T_k(u) with T_k(u) from the three-term recurrence
    C.h_m2mS.assign(2 * (size_t)p * p, 0.0);
    for (int sd = 0; sd < 2; ++sd)
        for (int l2 = 0; l2 < p; ++l2) {
            double u = 0.5 * (C.h_xbar[l2] + 2.0 * sd - 1.0);
            std::vector<double> T(p);
            T[0] = 1.0;
            if (p > 1) T[1] = u;
            for (int k = 2; k < p; ++k) T[k] = 2.0 * u * T[k - 1] - T[k - 2];
            for (int l = 0; l < p; ++l) {
                double acc = 0.0;
                for (int k = 1; k < p; ++k) acc += C.h_tnode[l * p + k] * T[k];
                C.h_m2mS[(size_t)sd * p * p + l * p + l2] = (1.0 + 2.0 * acc) / p;
            }
        }
    hipStream_t s = ctx->stream;
    upload(s, C.xbar, C.h_xbar);
    upload(s, C.bw, C.h_bw);
    upload(s, C.tnode, C.h_tnode);
    upload(s, C.gl_t, C.h_glt);
    upload(s, C.gl_w, C.h_glw);
    upload(s, C.m2mS, C.h_m2mS);
    FM_HIP(hipStreamSynchronize(s));
}

void build_m2l_ops(fmddm_ctx *ctx)
{
    M2LOps &M = *ctx->m2l;
    if (M.ready) return;
    int p = ctx->prm.p, p2 = p * p;
    M.mode = ctx->prm.m2l;
    M.M = 3 * p2;
    M.Mp = (M.M + 63) / 64 * 64;
    std::vector<int> dx, dy, slot;
    v_offsets(dx, dy, slot);
    int nop = (int)dx.size();
    hipStream_t s = ctx->stream;
    DBuf<int> ddx, ddy;
    upload(s, ddx, dx);
    upload(s, ddy, dy);
    int64_t tot = (int64_t)nop * p2 * p2;
    if (M.mode == FMDDM_M2L_DENSE) {
        M.r = M.M;
        M.rp = M.Mp;
        M.ops.alloc((size_t)nop * M.Mp * M.Mp);
        M.ops.zero(s);
        hipLaunchKernelGGL(k_m2l_ops, dim3(cdiv(tot, 256)), dim3(256), 0, s, nop, ddx.p, ddy.p,
                           ctx->cheb->xbar.p, p, M.Mp, ctx->gc, M.ops.p);
        FM_CHECK_LAUNCH();
        FM_HIP(hipStreamSynchronize(s));
        M.ready = 1;
        return;
    }
    // Compressed operators.  The point kernel is symmetric and even, so the
    // transpose of an offset's operator is the operator of the opposite
    // offset: the column space of all operators side by side is also their
    // row space, and one SVD gives both bases.
    DBuf<double> raw;
    raw.alloc((size_t)nop * M.Mp * M.Mp);
    raw.zero(s);
    hipLaunchKernelGGL(k_m2l_ops, dim3(cdiv(tot, 256)), dim3(256), 0, s, nop, ddx.p, ddy.p,
                       ctx->cheb->xbar.p, p, M.Mp, 1.0, raw.p);
    FM_CHECK_LAUNCH();
    int m = M.M, ncol = nop * M.M;
    DBuf<double> fat, U;
    fat.alloc((size_t)m * ncol);
    U.alloc((size_t)m * m);
    int64_t ftot = (int64_t)m * ncol;
    hipLaunchKernelGGL(k_pack_fat, dim3(cdiv(ftot, 256)), dim3(256), 0, s, nop, m, M.Mp, raw.p, fat.p);
    FM_CHECK_LAUNCH();
    rocblas_handle h;
    if (rocblas_create_handle(&h) != rocblas_status_success) throw Error{FMDDM_EDEVICE, "rocblas handle"};
    rocblas_set_stream(h, s);
    std::vector<double> hs;
    int r = 0;
    try {
        r = range_basis(h, s, m, ncol, fat.p, ctx->prm.m2l_tol, U.p, hs);
    } catch (...) {
        rocblas_destroy_handle(h);
        throw;
    }
    rocblas_destroy_handle(h);
    M.sv.assign(m, 0.0);
    for (size_t i = 0; i < hs.size(); ++i) M.sv[i] = hs[0] > 0 ? hs[i] / hs[0] : 0.0;
    r = std::max(r, 1);
    M.r = r;
    M.rp = (r + 63) / 64 * 64;
    int rp = M.rp, Mp = M.Mp;
    M.Vt.alloc((size_t)rp * Mp);
    M.Ur.alloc((size_t)Mp * rp);
    hipLaunchKernelGGL(k_bases, dim3(cdiv((int64_t)rp * Mp, 256)), dim3(256), 0, s, m, Mp, r, rp, U.p, M.Vt.p,
                       M.Ur.p);
    FM_CHECK_LAUNCH();
    // C_o = V^T K_o V: first T1[o rp + i] = K_o V[:, i], then
    // Ct[o rp + i] = V^T T1[o rp + i] (= column i of C_o)
    std::vector<int> top, tb, te, src, dst, zero;
    for (int o = 0; o < nop; ++o)
        for (int i0 = 0; i0 < rp; i0 += TILE_N) {
            top.push_back(o);
            zero.push_back(0);
            tb.push_back((int)src.size());
            for (int i = i0; i < std::min(rp, i0 + TILE_N); ++i) {
                src.push_back(i);
                dst.push_back(o * rp + i);
            }
            te.push_back((int)src.size());
        }
    DBuf<int> dtop, dtb, dte, dsrc, ddst, dzero;
    upload(s, dtop, top);
    upload(s, dtb, tb);
    upload(s, dte, te);
    upload(s, dsrc, src);
    upload(s, ddst, dst);
    upload(s, dzero, zero);
    DBuf<double> T1, Ct;
    T1.alloc((size_t)nop * rp * Mp);
    Ct.alloc((size_t)nop * rp * rp);
    launch_ggemm<64, 32>(s, (int)top.size(), Mp, raw.p, (size_t)Mp * Mp, Mp, Mp, M.Vt.p, Mp, dtop.p, dtb.p,
                         dte.p, dsrc.p, ddst.p, nullptr, T1.p, Mp);
    launch_ggemm<64, 32>(s, (int)top.size(), rp, M.Vt.p, 0, Mp, Mp, T1.p, Mp, dzero.p, dtb.p, dte.p, ddst.p,
                         ddst.p, nullptr, Ct.p, rp);
    M.ops.alloc((size_t)nop * rp * rp);
    hipLaunchKernelGGL(k_transpose_ops, dim3(cdiv((int64_t)nop * rp * rp, 256)), dim3(256), 0, s, nop, rp,
                       ctx->gc, Ct.p, M.ops.p);
    FM_CHECK_LAUNCH();
    FM_HIP(hipStreamSynchronize(s));
    M.ready = 1;
}

void setup_fmm(fmddm_ctx *ctx, fmddm_tree *t)
{
    if (t->Wexp.p) return;
    build_m2l_ops(ctx);
    hipStream_t s = ctx->stream;
    const M2LOps &M = *ctx->m2l;
    int Mp = M.Mp, rp = M.rp, ncell = t->ncell, p = ctx->prm.p;
    // M2L schedule: V pairs grouped by offset, tiles of TILE_N pairs
    std::vector<int> hv(t->nV), hix(ncell), hiy(ncell);
    std::vector<double> hhw(ncell);
    if (t->nV) FM_HIP(hipMemcpyAsync(hv.data(), t->lidx[1].p, t->nV * 4, hipMemcpyDeviceToHost, s));
    FM_HIP(hipMemcpyAsync(hix.data(), t->cix.p, ncell * 4, hipMemcpyDeviceToHost, s));
    FM_HIP(hipMemcpyAsync(hiy.data(), t->ciy.p, ncell * 4, hipMemcpyDeviceToHost, s));
    FM_HIP(hipMemcpyAsync(hhw.data(), t->chw.p, ncell * 8, hipMemcpyDeviceToHost, s));
    FM_HIP(hipStreamSynchronize(s));
    std::vector<int> dx, dy, slot;
    v_offsets(dx, dy, slot);
    int nop = (int)dx.size();
    std::vector<std::vector<int>> byop(nop);
    const std::vector<int> &vo = t->h_loff[1];
    std::vector<int> owner(t->nV);
    for (int c = 0; c < ncell; ++c)
        for (int k = vo[c]; k < vo[c + 1]; ++k) {
            int src = hv[k];
            owner[k] = c;
            int ox = (int)hix[src] - (int)hix[c], oy = (int)hiy[src] - (int)hiy[c];
            if (std::abs(ox) > 3 || std::abs(oy) > 3 || slot[offset_slot(ox, oy)] < 0)
                throw Error{FMDDM_EDEVICE, "V-list entry outside the offset stencil"};
            byop[slot[offset_slot(ox, oy)]].push_back(k);
        }
    std::vector<int> top, tbeg, tend, psrc, pdst;
    std::vector<double> pscale;
    for (int o = 0; o < nop; ++o) {
        const std::vector<int> &ks = byop[o];
        for (size_t b = 0; b < ks.size(); b += TILE_N) {
            top.push_back(o);
            tbeg.push_back((int)psrc.size());
            for (size_t i = b; i < std::min(ks.size(), b + TILE_N); ++i) {
                int k = ks[i];
                double h = hhw[owner[k]];
                psrc.push_back(hv[k]);
                pdst.push_back(k);
                pscale.push_back(1.0 / (h * h));
            }
            tend.push_back((int)psrc.size());
        }
    }
    t->ntile = (int)top.size();
    upload(s, t->tile_op, top);
    upload(s, t->tile_beg, tbeg);
    upload(s, t->tile_end, tend);
    upload(s, t->pair_src, psrc);
    upload(s, t->pair_dst, pdst);
    upload(s, t->pair_scale, pscale);
    // cells at level >= 2
    std::vector<int> far, fop, fb, fe;
    for (int c = 0; c < ncell; ++c)
        if (t->h_level[c] >= 2) far.push_back(c);
    for (size_t b = 0; b < far.size(); b += TILE_N) {
        fop.push_back(0);
        fb.push_back((int)b);
        fe.push_back((int)std::min(far.size(), b + TILE_N));
    }
    t->nfar = (int)far.size();
    t->nftile = (int)fop.size();
    upload(s, t->far_cells, far);
    upload(s, t->ftile_op, fop);
    upload(s, t->ftile_beg, fb);
    upload(s, t->ftile_end, fe);
    // per-element anterpolation weights
    t->p2m_mat.alloc((size_t)t->n * p * p);
    hipLaunchKernelGGL(k_p2m_mats, dim3(t->nleaf), dim3(256), 0, s, t->nleaf, t->dleaves.p, t->cpbeg.p,
                       t->cpend.p, t->ccx.p, t->ccy.p, t->chw.p, t->scx.p, t->scy.p, t->scb.p, t->ssb.p,
                       t->sa.p, ctx->cheb->tnode.p, ctx->cheb->gl_t.p, ctx->cheb->gl_w.p, p, t->p2m_mat.p);
    FM_CHECK_LAUNCH();
    t->Wexp.alloc((size_t)ncell * Mp);
    t->Gexp.alloc((size_t)ncell * Mp);
    t->Zm2l.alloc((size_t)std::max<int64_t>(t->nV, 1) * rp);
    t->Wexp.zero(s);
    t->Gexp.zero(s);
    m2m_schedule(s, t);
    if (M.mode == FMDDM_M2L_SVD) {
        t->What.alloc((size_t)ncell * rp);
        t->Ghat.alloc((size_t)ncell * rp);
        t->What.zero(s);
        t->Ghat.zero(s);
    }
    t->q.alloc(3 * (size_t)t->n);
    t->Dsort.alloc(2 * (size_t)t->n);
    // downward-pass items: every far cell's points in chunks of 32
    {
        std::vector<int> hb(ncell), he(ncell), lc, lp;
        FM_HIP(hipMemcpyAsync(hb.data(), t->cpbeg.p, ncell * 4, hipMemcpyDeviceToHost, s));
        FM_HIP(hipMemcpyAsync(he.data(), t->cpend.p, ncell * 4, hipMemcpyDeviceToHost, s));
        FM_HIP(hipStreamSynchronize(s));
        int maxlev = 0;
        for (int c = 0; c < ncell; ++c) {
            if (t->h_level[c] < 2) continue;
            maxlev = std::max(maxlev, t->h_level[c]);
            for (int q = hb[c]; q < he[c]; q += LTM) {
                lc.push_back(c);
                lp.push_back(q);
            }
        }
        t->nlpitem = (int)lc.size();
        t->nfarlev = maxlev >= 2 ? maxlev - 1 : 0;
        upload(s, t->lp_cell, lc);
        upload(s, t->lp_p0, lp);
    }
    t->far_s.alloc(3 * (size_t)std::max(t->nfarlev, 1) * t->n);
    t->part_s.alloc(3 * (size_t)t->npartial);
    if (M.mode == FMDDM_M2L_SVD) t->ksplit.alloc((size_t)KSPLIT_MAX * ncell * rp);
    FM_HIP(hipStreamSynchronize(s));
}

FmmBufs tree_bufs(fmddm_tree *t)
{
    return FmmBufs{t->Dsort.p, t->q.p, t->part_s.p, t->Wexp.p, t->ksplit.p, t->What.p,
                   t->Zm2l.p,  t->Ghat.p, t->Gexp.p, t->far_s.p};
}

int fmm_ksplit(const fmddm_ctx *ctx) { return TILESETS[ctx->prm.m2l_tiles].ksplit; }

void fmm_apply(fmddm_ctx *ctx, fmddm_tree *t, const double *D, double *out, int prec)
{
    setup_fmm(ctx, t);
    if (prec != FMDDM_PREC_FP64) setup_lowp(ctx, t, prec);
    fmm_apply_bufs(ctx, t, D, out, prec, tree_bufs(t));
}

void fmm_apply_bufs(fmddm_ctx *ctx, fmddm_tree *t, const double *D, double *out, int prec, const FmmBufs &B)
{
    // the reduced-precision M2L products keep their intermediates with the tree
    if (prec != FMDDM_PREC_FP64 && B.Wexp != t->Wexp.p)
        throw Error{FMDDM_EUNSUPPORTED, "reduced-precision products use the tree's buffers"};
    hipStream_t s = ctx->stream;
    const M2LOps &M = *ctx->m2l;
    int p = ctx->prm.p, Mp = M.Mp, rp = M.rp, n = (int)t->n;
    const Cheb &C = *ctx->cheb;
    Profiler &P = ctx->prof;
    const TileSet &ts = TILESETS[ctx->prm.m2l_tiles];
    hipEvent_t e0;
    P.begin(FMDDM_PH_PREP, s, e0);
    hipLaunchKernelGGL(k_prep, dim3(cdiv(n, 256)), dim3(256), 0, s, n, t->perm.p, D, t->scb.p, t->ssb.p,
                       B.Dsort, B.q);
    FM_CHECK_LAUNCH();
    P.end(FMDDM_PH_PREP, s, e0);
    // the near field depends only on the prepared sources: it runs on the
    // side stream while the far-field passes run here
    hipStream_t s2 = ctx->side;
    FM_HIP(hipEventRecord(ctx->ev_fork, s));
    FM_HIP(hipStreamWaitEvent(s2, ctx->ev_fork, 0));
    hipEvent_t e1;
    P.begin(FMDDM_PH_P2P, s2, e1);
    if (prec == FMDDM_PREC_FP64)
        hipLaunchKernelGGL(k_p2p<double>, dim3(t->nitem), dim3(NT), 0, s2, t->nitem, t->it_leaf.p, t->it_s0.p,
                           t->it_s1.p, t->it_poff.p, t->dleaves.p, t->cpbeg.p, t->cpend.p, t->nfoff.p, t->nflat.p,
                           t->scx.p, t->scy.p, t->scb.p, t->ssb.p, t->sa.p, B.Dsort, ctx->gc, B.part_s);
    else
        hipLaunchKernelGGL(k_p2p<float>, dim3(t->nitem), dim3(NT), 0, s2, t->nitem, t->it_leaf.p, t->it_s0.p,
                           t->it_s1.p, t->it_poff.p, t->dleaves.p, t->cpbeg.p, t->cpend.p, t->nfoff.p, t->nflat.p,
                           t->scx.p, t->scy.p, t->scb.p, t->ssb.p, t->sa.p, B.Dsort, ctx->gc, B.part_s);
    FM_CHECK_LAUNCH();
    P.end(FMDDM_PH_P2P, s2, e1);
    FM_HIP(hipEventRecord(ctx->ev_join, s2));
    bool far = t->nV > 0;
    if (far) {
        P.begin(FMDDM_PH_P2M, s, e0);
        hipLaunchKernelGGL(k_p2m, dim3(t->nleaf), dim3(256), 0, s, t->nleaf, t->dleaves.p, t->cpbeg.p,
                           t->cpend.p, t->p2m_mat.p, B.q, p * p, Mp, B.Wexp);
        FM_CHECK_LAUNCH();
        P.end(FMDDM_PH_P2M, s, e0);
        if (!t->m2m_launch.empty()) {
            P.begin(FMDDM_PH_M2M, s, e0);
#define FM_M2M(PP) launch_m2m<PP>(s, ctx, t, Mp, 1, 0, B.Wexp)
            FM_DISPATCH_P(p, FM_M2M)
#undef FM_M2M
            P.end(FMDDM_PH_M2M, s, e0);
        }
        if (prec == FMDDM_PREC_FP32) {
            m2l_lowp<float>(s, t, M, M.Vt32.p, M.ops32.p, M.Ur32.p, P, ts);
        } else if (prec == FMDDM_PREC_BF16) {
            m2l_lowp<uint16_t>(s, t, M, M.Vt16.p, M.ops16.p, M.Ur16.p, P, ts);
        } else if (M.mode == FMDDM_M2L_SVD) {
            // projection onto the singular vectors: K = 3p^2 is long and the
            // output small, so K is split over ts.ksplit blocks and summed after
            P.begin(FMDDM_PH_COMPRESS, s, e0);
            launch_ggemm<32, 32>(s, t->nftile, rp, M.Vt.p, 0, Mp, Mp, B.Wexp, Mp, t->ftile_op.p,
                                 t->ftile_beg.p, t->ftile_end.p, t->far_cells.p, t->far_cells.p, nullptr,
                                 B.ksplit, rp, ts.ksplit, (size_t)t->ncell * rp);
            P.end(FMDDM_PH_COMPRESS, s, e0);
            P.begin(FMDDM_PH_COMPRESS_SUM, s, e0);
            {
                int64_t c0 = t->level_start[2], cnt = (int64_t)(t->ncell - c0) * rp;
                hipLaunchKernelGGL(k_reduce_split<double>, dim3(cdiv(cnt, 256)), dim3(256), 0, s, cnt, ts.ksplit,
                                   (size_t)t->ncell * rp, B.ksplit + c0 * rp, B.What + c0 * rp);
                FM_CHECK_LAUNCH();
            }
            P.end(FMDDM_PH_COMPRESS_SUM, s, e0);
            P.begin(FMDDM_PH_M2L, s, e0);
            ggemm_bm(ts.bm_pair, s, t->ntile, rp, M.ops.p, (size_t)rp * rp, rp, rp, B.What, rp, t->tile_op.p,
                                 t->tile_beg.p, t->tile_end.p, t->pair_src.p, t->pair_dst.p, t->pair_scale.p,
                                 B.Zm2l, rp);
            P.end(FMDDM_PH_M2L, s, e0);
            P.begin(FMDDM_PH_M2L_SUM, s, e0);
            hipLaunchKernelGGL((k_sum_pairs<double, double>), dim3(t->nfar), dim3(256), 0, s, t->nfar, t->far_cells.p,
                               t->loff[1].p, B.Zm2l, rp, rp, B.Ghat, rp);
            FM_CHECK_LAUNCH();
            P.end(FMDDM_PH_M2L_SUM, s, e0);
            P.begin(FMDDM_PH_DECOMPRESS, s, e0);
            ggemm_bm(ts.bm_back, s, t->nftile, Mp, M.Ur.p, 0, rp, rp, B.Ghat, rp, t->ftile_op.p,
                                 t->ftile_beg.p, t->ftile_end.p, t->far_cells.p, t->far_cells.p, nullptr,
                                 B.Gexp, Mp);
            P.end(FMDDM_PH_DECOMPRESS, s, e0);
        } else {
            P.begin(FMDDM_PH_M2L, s, e0);
            ggemm_bm(ts.bm_pair, s, t->ntile, Mp, M.ops.p, (size_t)Mp * Mp, Mp, Mp, B.Wexp, Mp, t->tile_op.p,
                                 t->tile_beg.p, t->tile_end.p, t->pair_src.p, t->pair_dst.p, t->pair_scale.p,
                                 B.Zm2l, Mp);
            P.end(FMDDM_PH_M2L, s, e0);
            P.begin(FMDDM_PH_M2L_SUM, s, e0);
            hipLaunchKernelGGL((k_sum_pairs<double, double>), dim3(t->nfar), dim3(256), 0, s, t->nfar, t->far_cells.p,
                               t->loff[1].p, B.Zm2l, Mp, Mp, B.Gexp, Mp);
            FM_CHECK_LAUNCH();
            P.end(FMDDM_PH_M2L_SUM, s, e0);
        }
        P.begin(FMDDM_PH_L2P, s, e0);
#define FM_L2P(PP) launch_l2p<PP>(s, ctx, t, B.Gexp, Mp, B.far_s)
        FM_DISPATCH_P(p, FM_L2P)
#undef FM_L2P
        P.end(FMDDM_PH_L2P, s, e0);
    }
    FM_HIP(hipStreamWaitEvent(s, ctx->ev_join, 0));
    P.begin(FMDDM_PH_FINAL, s, e0);
    hipLaunchKernelGGL(k_final, dim3(cdiv(n, 256)), dim3(256), 0, s, n, t->tleaf.p, t->dleaves.p, t->cpbeg.p,
                       t->clevel.p, t->lk_off.p, t->it_poff.p, B.part_s,
                       far ? B.far_s : (const double *)nullptr,
                       t->scb.p, t->ssb.p, t->perm.p, out);
    FM_CHECK_LAUNCH();
    P.end(FMDDM_PH_FINAL, s, e0);
}

}  // namespace fmddm
