// Black-box FMM product (Section 3.2) on gfx950.
//
// Expansion layout: every cell holds Mp doubles (3 p^2 used, the rest zero):
// index c * p^2 + l * p + m for component c and Chebyshev node (l, m) of the
// cell's square.  Multipole weights W carry the three charge components
// (b_x n_x, b_y n_y, b_x n_y + b_y n_x) integrated against the interpolants;
// local fields F carry (sxx, syy, sxy).
//
// Passes of one product:
//   prep      D (caller order) -> D and charges in tree order
//   p2m       leaf weights, eq. 3.6; each element integrated along its
//             length with p-point Gauss-Legendre (exact: the interpolant on
//             a straight segment is a polynomial of degree 2(p-1))
//   m2m       eq. 3.7, one level at a time, separable p x p transfers
//   m2l       eq. 3.8 as a batched dense contraction on FP64 MFMA: V-list
//             pairs grouped by relative offset, each group multiplied by the
//             (unit-size) offset operator and scaled by h^-2 (the kernel is
//             homogeneous of degree -2); one product per pair is stored
//   down      eq. 3.10: sum of the pair products of the cell (fixed order,
//             no atomics) plus the parent's field interpolated (L2L)
//   l2p_p2p   eq. 3.11: local field at each midpoint plus direct element
//             interactions over U, W and the X lists of the leaf's
//             ancestors; projected to (shear, normal) traction and
//             scattered to caller order
#include "elem.h"
#include "internal.h"

#include <cmath>
#include <algorithm>

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

// S_p(xbar_l, u) for all l into out[l]; tnode[l*p + k] = T_k(xbar_l).
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

// ------------------------------------------------------------------ P2M
constexpr int P2M_T = 256;

__global__ __launch_bounds__(P2M_T) void k_p2m(int nleaf, const int *__restrict__ leaves,
                                               const int *__restrict__ pbeg, const int *__restrict__ pend,
                                               const double *__restrict__ ccx, const double *__restrict__ ccy,
                                               const double *__restrict__ chw, const double *__restrict__ cx,
                                               const double *__restrict__ cy, const double *__restrict__ cb,
                                               const double *__restrict__ sb, const double *__restrict__ a,
                                               const double *__restrict__ q, const double *__restrict__ tnode,
                                               const double *__restrict__ glt, const double *__restrict__ glw,
                                               int p, int Mp, double *__restrict__ W)
{
    __shared__ double tn[MAXP * MAXP];
    __shared__ double Sx[MAXP * MAXP], Sy[MAXP * MAXP];  // [g][l]
    __shared__ double wg[MAXP];
    int c = leaves[xcd_remap(blockIdx.x, nleaf)];
    int tid = threadIdx.x;
    int p2 = p * p;
    for (int e = tid; e < p2; e += P2M_T) tn[e] = tnode[e];
    double x0 = ccx[c], y0 = ccy[c], ih = 1.0 / chw[c];
    // thread owns node entries e = tid + k * P2M_T (< p^2), 3 components each
    constexpr int EPT = (MAXP * MAXP + P2M_T - 1) / P2M_T;
    double acc[3][EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) acc[0][k] = acc[1][k] = acc[2][k] = 0.0;
    __syncthreads();
    for (int j = pbeg[c]; j < pend[c]; ++j) {
        double ex = cx[j], ey = cy[j], ec = cb[j], es = sb[j], ea = a[j];
        // interpolant values at the p Gauss points of element j
        for (int t = tid; t < 2 * p2; t += P2M_T) {
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
        double q0 = q[3 * j], q1 = q[3 * j + 1], q2 = q[3 * j + 2];
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            int e = tid + k * P2M_T;
            if (e < p2) {
                int l = e / p, m = e - l * p;
                double s = 0.0;
                for (int g = 0; g < p; ++g) s += wg[g] * Sx[g * MAXP + l] * Sy[g * MAXP + m];
                acc[0][k] += q0 * s;
                acc[1][k] += q1 * s;
                acc[2][k] += q2 * s;
            }
        }
        __syncthreads();
    }
    double *Wc = W + (size_t)c * Mp;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        int e = tid + k * P2M_T;
        if (e < p2) {
            Wc[e] = acc[0][k];
            Wc[p2 + e] = acc[1][k];
            Wc[2 * p2 + e] = acc[2][k];
        }
    }
}

// ------------------------------------------------------------------ M2M / L2L
// T[side][l][l'] = S_p(xbar_l, side_sign/2 + xbar_l'/2), side 0 = lower/left.
constexpr int TT = 256;

__global__ __launch_bounds__(TT) void k_m2m(int c0, int nc, const int *__restrict__ leaf,
                                            const int *__restrict__ child, const double *__restrict__ Tm,
                                            int p, int Mp, double *__restrict__ W)
{
    __shared__ double T[2 * MAXP * MAXP];
    __shared__ double in[3 * MAXP * MAXP], tmp[3 * MAXP * MAXP];
    int c = c0 + xcd_remap(blockIdx.x, nc);
    if (leaf[c]) return;
    int tid = threadIdx.x, p2 = p * p, n3 = 3 * p2;
    for (int e = tid; e < 2 * p2; e += TT) T[e] = Tm[e];
    constexpr int EPT = (3 * MAXP * MAXP + TT - 1) / TT;
    double acc[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) acc[k] = 0.0;
    for (int d = 0; d < 4; ++d) {
        int k = child[4 * c + d];
        if (k < 0) continue;
        const double *Tx = T + (d & 1) * p2, *Ty = T + (d >> 1) * p2;
        __syncthreads();
        for (int e = tid; e < n3; e += TT) in[e] = W[(size_t)k * Mp + e];
        __syncthreads();
        // tmp[c][l][m'] = sum_l' Tx[l][l'] in[c][l'][m']
        for (int e = tid; e < n3; e += TT) {
            int cc = e / p2, r = e - cc * p2, l = r / p, m2 = r - l * p;
            double s = 0.0;
            for (int l2 = 0; l2 < p; ++l2) s += Tx[l * p + l2] * in[cc * p2 + l2 * p + m2];
            tmp[e] = s;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < EPT; ++kk) {
            int e = tid + kk * TT;
            if (e < n3) {
                int cc = e / p2, r = e - cc * p2, l = r / p, m = r - l * p;
                double s = 0.0;
                for (int m2 = 0; m2 < p; ++m2) s += Ty[m * p + m2] * tmp[cc * p2 + l * p + m2];
                acc[kk] += s;
            }
        }
    }
#pragma unroll
    for (int kk = 0; kk < EPT; ++kk) {
        int e = tid + kk * TT;
        if (e < n3) W[(size_t)c * Mp + e] = acc[kk];
    }
}

// Downward pass for the cells of one level: F = (sum of its M2L pair
// products) + L2L(parent field).
__global__ __launch_bounds__(TT) void k_down(int c0, int nc, const int *__restrict__ parent,
                                             const uint32_t *__restrict__ cix, const uint32_t *__restrict__ ciy,
                                             const int *__restrict__ voff, const double *__restrict__ Z,
                                             const double *__restrict__ Tm, int p, int Mp, int do_l2l,
                                             double *__restrict__ F)
{
    __shared__ double T[2 * MAXP * MAXP];
    __shared__ double in[3 * MAXP * MAXP], tmp[3 * MAXP * MAXP];
    int c = c0 + xcd_remap(blockIdx.x, nc);
    int tid = threadIdx.x, p2 = p * p, n3 = 3 * p2;
    constexpr int EPT = (3 * MAXP * MAXP + TT - 1) / TT;
    double acc[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) acc[k] = 0.0;
    // M2L pair products of this cell, summed in list order
    int kb = voff[c], ke = voff[c + 1];
    for (int k = kb; k < ke; ++k) {
        const double *z = Z + (size_t)k * Mp;
#pragma unroll
        for (int kk = 0; kk < EPT; ++kk) {
            int e = tid + kk * TT;
            if (e < n3) acc[kk] += z[e];
        }
    }
    if (do_l2l) {
        int P = parent[c];
        int sx = (int)(cix[c] & 1u), sy = (int)(ciy[c] & 1u);
        for (int e = tid; e < 2 * p2; e += TT) T[e] = Tm[e];
        for (int e = tid; e < n3; e += TT) in[e] = F[(size_t)P * Mp + e];
        __syncthreads();
        const double *Tx = T + sx * p2, *Ty = T + sy * p2;
        // tmp[c][l][m'] = sum_l' Tx[l'][l] in[c][l'][m']
        for (int e = tid; e < n3; e += TT) {
            int cc = e / p2, r = e - cc * p2, l = r / p, m2 = r - l * p;
            double s = 0.0;
            for (int l2 = 0; l2 < p; ++l2) s += Tx[l2 * p + l] * in[cc * p2 + l2 * p + m2];
            tmp[e] = s;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < EPT; ++kk) {
            int e = tid + kk * TT;
            if (e < n3) {
                int cc = e / p2, r = e - cc * p2, l = r / p, m = r - l * p;
                double s = 0.0;
                for (int m2 = 0; m2 < p; ++m2) s += Ty[m2 * p + m] * tmp[cc * p2 + l * p + m2];
                acc[kk] += s;
            }
        }
    }
#pragma unroll
    for (int kk = 0; kk < EPT; ++kk) {
        int e = tid + kk * TT;
        if (e < n3) F[(size_t)c * Mp + e] = acc[kk];
    }
}

// ------------------------------------------------------------------ M2L
// Z[pair] = scale[pair] * Op[o] . X[src[pair]] for the pairs of one tile
// (all of the same offset o).  64 x 64 output tile per 256-thread block,
// 4 waves of 32 x 32 built from 2 x 2 MFMA 16x16x4 (FP64) blocks.  Operand
// layout of v_mfma_f64_16x16x4f64: lane L holds A[L%16][L/16] and
// B[L/16][L%16]; accumulator register r of lane L holds D[4r + L/16][L%16].
constexpr int GM = 64, GN = 64, GK = 16;

__global__ __launch_bounds__(256) void k_m2l_gemm(const double *__restrict__ ops, int Mp,
                                                  const double *__restrict__ X,
                                                  const int *__restrict__ tile_op,
                                                  const int *__restrict__ tile_beg,
                                                  const int *__restrict__ tile_end,
                                                  const int *__restrict__ pair_k,
                                                  const int *__restrict__ pair_src,
                                                  const double *__restrict__ pair_scale,
                                                  double *__restrict__ Z)
{
    __shared__ double As[GM][GK + 1];
    __shared__ double Bs[GK][GN + 1];
    __shared__ int src[GN];
    int tile = blockIdx.x, mt = blockIdx.y;
    int o = tile_op[tile], pb = tile_beg[tile], np = tile_end[tile] - pb;
    int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    int wm = wave >> 1, wn = wave & 1;
    if (tid < GN) src[tid] = tid < np ? pair_src[pb + tid] : -1;
    const double *A = ops + (size_t)o * Mp * Mp + (size_t)mt * GM * Mp;
    d4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    __syncthreads();
    for (int k0 = 0; k0 < Mp; k0 += GK) {
#pragma unroll
        for (int r = 0; r < (GM * GK) / 256; ++r) {
            int e = tid + r * 256;
            int row = e / GK, col = e % GK;
            As[row][col] = A[(size_t)row * Mp + k0 + col];
        }
#pragma unroll
        for (int r = 0; r < (GN * GK) / 256; ++r) {
            int e = tid + r * 256;
            int j = e / GK, col = e % GK;
            int s = src[j];
            Bs[col][j] = s >= 0 ? X[(size_t)s * Mp + k0 + col] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; kk += 4) {
            double av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = As[wm * 32 + i * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < 2; ++j) bv[j] = Bs[kk + (lane >> 4)][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        int col = wn * 32 + j * 16 + (lane & 15);
        if (col >= np) continue;
        double sc = pair_scale[pb + col];
        double *z = Z + (size_t)pair_k[pb + col] * Mp + mt * GM;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) z[wm * 32 + i * 16 + 4 * r + (lane >> 4)] = sc * acc[i][j][r];
    }
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

// ------------------------------------------------------------ L2P + P2P
constexpr int PT = 256, TPT = 4, TGT = PT / TPT, STILE = 256, MAXNEAR = 512;

__global__ __launch_bounds__(PT) void k_l2p_p2p(
    int nleaf, const int *__restrict__ leaves, const int *__restrict__ pbeg, const int *__restrict__ pend,
    const int *__restrict__ noff, const int *__restrict__ nsrc, const double *__restrict__ ccx,
    const double *__restrict__ ccy, const double *__restrict__ chw, const double *__restrict__ cx,
    const double *__restrict__ cy, const double *__restrict__ cb, const double *__restrict__ sb,
    const double *__restrict__ a, const double *__restrict__ Ds, const int *__restrict__ perm,
    const double *__restrict__ F, const double *__restrict__ tnode, int p, int Mp, double gc,
    int use_far, double *__restrict__ out)
{
    __shared__ double tn[MAXP * MAXP];
    __shared__ double s_cx[STILE], s_cy[STILE], s_cb[STILE], s_sb[STILE], s_a[STILE], s_ds[STILE],
        s_dn[STILE];
    __shared__ int s_pre[MAXNEAR + 1], s_beg[MAXNEAR];
    int li = xcd_remap(blockIdx.x, nleaf);
    int c = leaves[li];
    int tid = threadIdx.x, sub = tid & (TPT - 1), tl = tid / TPT;
    int p2 = p * p;
    for (int e = tid; e < p2; e += PT) tn[e] = tnode[e];
    // flattened near-source ranges
    int nb = noff[li], ne = noff[li + 1], nn = ne - nb;
    if (tid == 0) {
        int s = 0;
        for (int k = 0; k < nn && k < MAXNEAR; ++k) {
            int sc = nsrc[nb + k];
            s_pre[k] = s;
            s_beg[k] = pbeg[sc];
            s += pend[sc] - pbeg[sc];
        }
        s_pre[nn < MAXNEAR ? nn : MAXNEAR] = s;
    }
    __syncthreads();
    int nchunks = (nn + MAXNEAR - 1) / MAXNEAR;
    double x0 = ccx[c], y0 = ccy[c], ih = 1.0 / chw[c];
    int tb = pbeg[c], te = pend[c];
    for (int t0 = tb; t0 < te; t0 += TGT) {
        int i = t0 + tl;
        bool act = i < te;
        double X = act ? cx[i] : 0.0, Y = act ? cy[i] : 0.0;
        double sxx = 0.0, syy = 0.0, sxy = 0.0;
        if (act && use_far) {
            // local expansion at the midpoint: this sub-lane takes rows l = sub (mod 4)
            double u = (X - x0) * ih, v = (Y - y0) * ih;
            double Sy[MAXP];
            for (int m = 0; m < p; ++m) Sy[m] = cheb_S(p, tn + m * p, v);
            const double *Fc = F + (size_t)c * Mp;
            for (int l = sub; l < p; l += TPT) {
                double sx = cheb_S(p, tn + l * p, u);
                double r0 = 0.0, r1 = 0.0, r2 = 0.0;
                for (int m = 0; m < p; ++m) {
                    r0 += Fc[l * p + m] * Sy[m];
                    r1 += Fc[p2 + l * p + m] * Sy[m];
                    r2 += Fc[2 * p2 + l * p + m] * Sy[m];
                }
                sxx += sx * r0;
                syy += sx * r1;
                sxy += sx * r2;
            }
        }
        // direct interactions, sources staged through LDS
        for (int ch = 0; ch < nchunks; ++ch) {
            int total;
            if (ch > 0) {
                __syncthreads();
                if (tid == 0) {
                    int s = 0, kb = ch * MAXNEAR;
                    int kn = min(nn - kb, MAXNEAR);
                    for (int k = 0; k < kn; ++k) {
                        int sc = nsrc[nb + kb + k];
                        s_pre[k] = s;
                        s_beg[k] = pbeg[sc];
                        s += pend[sc] - pbeg[sc];
                    }
                    s_pre[kn] = s;
                }
                __syncthreads();
            }
            int kn = min(nn - ch * MAXNEAR, MAXNEAR);
            total = s_pre[kn];
            for (int base = 0; base < total; base += STILE) {
                __syncthreads();
                int vpos = base + tid;
                if (tid < STILE && vpos < total) {
                    int lo = 0, hi = kn - 1;  // last k with s_pre[k] <= vpos
                    while (lo < hi) {
                        int mid = (lo + hi + 1) >> 1;
                        if (s_pre[mid] <= vpos) lo = mid;
                        else hi = mid - 1;
                    }
                    int j = s_beg[lo] + (vpos - s_pre[lo]);
                    s_cx[tid] = cx[j]; s_cy[tid] = cy[j]; s_cb[tid] = cb[j]; s_sb[tid] = sb[j];
                    s_a[tid] = a[j]; s_ds[tid] = Ds[2 * j]; s_dn[tid] = Ds[2 * j + 1];
                }
                __syncthreads();
                int cnt = min(STILE, total - base);
                if (act)
                    for (int k = sub; k < cnt; k += TPT)
                        elem_stress_add(X, Y, s_cx[k], s_cy[k], s_cb[k], s_sb[k], s_a[k], s_ds[k], s_dn[k],
                                        gc, sxx, syy, sxy);
            }
            if (ch + 1 < nchunks) __syncthreads();
        }
        // reduce the 4 sub-lanes (adjacent lanes), fixed order
        sxx += __shfl_xor(sxx, 1); syy += __shfl_xor(syy, 1); sxy += __shfl_xor(sxy, 1);
        sxx += __shfl_xor(sxx, 2); syy += __shfl_xor(syy, 2); sxy += __shfl_xor(sxy, 2);
        if (act && sub == 0) {
            double ts, tnn;
            traction(cb[i], sb[i], sxx, syy, sxy, ts, tnn);
            int o = perm[i];
            out[2 * o] = ts;
            out[2 * o + 1] = tnn;
        }
        if (nchunks > 1 && t0 + TGT < te) {
            // restore chunk 0 for the next target group
            __syncthreads();
            if (tid == 0) {
                int s = 0;
                for (int k = 0; k < nn && k < MAXNEAR; ++k) {
                    int sc = nsrc[nb + k];
                    s_pre[k] = s;
                    s_beg[k] = pbeg[sc];
                    s += pend[sc] - pbeg[sc];
                }
                s_pre[MAXNEAR] = s;
            }
            __syncthreads();
        }
    }
}

// Gauss-Legendre nodes/weights on [-1, 1] (Newton on the Legendre
// recurrence), host side.
void gauss_legendre(int n, std::vector<double> &t, std::vector<double> &w)
{
    t.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double pn = 0, dpn = 1;
        for (int it = 0; it < 200; ++it) {
            double pm = 1.0, pc = x;
            for (int k = 2; k <= n; ++k) {
                double pk = ((2.0 * k - 1.0) * x * pc - (k - 1.0) * pm) / k;
                pm = pc;
                pc = pk;
            }
            if (n == 1) { pc = x; pm = 1.0; }
            pn = pc;
            dpn = n * (x * pc - pm) / (x * x - 1.0);
            double dx = pn / dpn;
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

double host_cheb_S(int p, int l, double u)
{
    double th = (2.0 * l + 1.0) * M_PI / (2.0 * p);
    double s = 0.0, t0 = 1.0, t1 = u;
    for (int k = 1; k < p; ++k) {
        s += std::cos(k * th) * t1;
        double t2 = 2.0 * u * t1 - t0;
        t0 = t1;
        t1 = t2;
    }
    return (1.0 + 2.0 * s) / p;
}

}  // namespace

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

void setup_cheb(fmddm_ctx *ctx)
{
    int p = ctx->prm.p;
    Cheb &C = ctx->cheb;
    C.p = p;
    C.h_xbar.resize(p);
    C.h_tnode.resize(p * p);
    for (int l = 0; l < p; ++l) {
        double th = (2.0 * l + 1.0) * M_PI / (2.0 * p);
        C.h_xbar[l] = std::cos(th);
        for (int k = 0; k < p; ++k) C.h_tnode[l * p + k] = std::cos(k * th);
    }
    gauss_legendre(p, C.h_glt, C.h_glw);
    C.h_m2m.resize(2 * p * p);
    for (int side = 0; side < 2; ++side)
        for (int l = 0; l < p; ++l)
            for (int l2 = 0; l2 < p; ++l2)
                C.h_m2m[side * p * p + l * p + l2] =
                    host_cheb_S(p, l, (side ? 0.5 : -0.5) + 0.5 * C.h_xbar[l2]);
    hipStream_t s = ctx->stream;
    C.xbar.alloc(p); C.tnode.alloc(p * p); C.gl_t.alloc(p); C.gl_w.alloc(p); C.m2m.alloc(2 * p * p);
    FM_HIP(hipMemcpyAsync(C.xbar.p, C.h_xbar.data(), p * 8, hipMemcpyHostToDevice, s));
    FM_HIP(hipMemcpyAsync(C.tnode.p, C.h_tnode.data(), p * p * 8, hipMemcpyHostToDevice, s));
    FM_HIP(hipMemcpyAsync(C.gl_t.p, C.h_glt.data(), p * 8, hipMemcpyHostToDevice, s));
    FM_HIP(hipMemcpyAsync(C.gl_w.p, C.h_glw.data(), p * 8, hipMemcpyHostToDevice, s));
    FM_HIP(hipMemcpyAsync(C.m2m.p, C.h_m2m.data(), 2 * p * p * 8, hipMemcpyHostToDevice, s));
    FM_HIP(hipStreamSynchronize(s));
}

static int offset_slot(int dx, int dy) { return (dx + 3) + 7 * (dy + 3); }

// Offsets (dx, dy) in [-3, 3]^2 outside [-1, 1]^2: the 40 relative
// positions of a V-list cell.
static void v_offsets(std::vector<int> &dx, std::vector<int> &dy, std::vector<int> &slot2op)
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

static void build_m2l_ops(fmddm_ctx *ctx)
{
    M2LOps &M = ctx->m2l;
    if (M.ready) return;
    int p = ctx->prm.p, p2 = p * p;
    M.M = 3 * p2;
    M.Mp = (M.M + 63) / 64 * 64;
    M.rank = M.Mp;
    std::vector<int> dx, dy, slot;
    v_offsets(dx, dy, slot);
    int nop = (int)dx.size();
    hipStream_t s = ctx->stream;
    DBuf<int> ddx, ddy;
    ddx.alloc(nop);
    ddy.alloc(nop);
    FM_HIP(hipMemcpyAsync(ddx.p, dx.data(), nop * 4, hipMemcpyHostToDevice, s));
    FM_HIP(hipMemcpyAsync(ddy.p, dy.data(), nop * 4, hipMemcpyHostToDevice, s));
    M.ops.alloc((size_t)nop * M.Mp * M.Mp);
    M.ops.zero(s);
    int64_t tot = (int64_t)nop * p2 * p2;
    hipLaunchKernelGGL(k_m2l_ops, dim3(cdiv(tot, 256)), dim3(256), 0, s, nop, ddx.p, ddy.p,
                       ctx->cheb.xbar.p, p, M.Mp, ctx->gc, M.ops.p);
    FM_CHECK_LAUNCH();
    FM_HIP(hipStreamSynchronize(s));
    M.ready = 1;
}

void setup_fmm(fmddm_ctx *ctx, fmddm_tree *t)
{
    if (t->Wexp.p) return;
    build_m2l_ops(ctx);
    hipStream_t s = ctx->stream;
    int Mp = ctx->m2l.Mp, ncell = t->ncell;
    // M2L schedule: V pairs grouped by offset, tiles of GN pairs
    std::vector<int> hv(t->nV), hix(ncell), hiy(ncell);
    std::vector<double> hhw(ncell);
    FM_HIP(hipMemcpyAsync(hv.data(), t->lidx[1].p, t->nV * 4, hipMemcpyDeviceToHost, s));
    FM_HIP(hipMemcpyAsync(hix.data(), t->cix.p, ncell * 4, hipMemcpyDeviceToHost, s));
    FM_HIP(hipMemcpyAsync(hiy.data(), t->ciy.p, ncell * 4, hipMemcpyDeviceToHost, s));
    FM_HIP(hipMemcpyAsync(hhw.data(), t->chw.p, ncell * 8, hipMemcpyDeviceToHost, s));
    FM_HIP(hipStreamSynchronize(s));
    std::vector<int> dx, dy, slot;
    v_offsets(dx, dy, slot);
    int nop = (int)dx.size();
    std::vector<std::vector<int>> byop(nop);
    const std::vector<int> &vo = t->h_loff[1];
    for (int c = 0; c < ncell; ++c)
        for (int k = vo[c]; k < vo[c + 1]; ++k) {
            int src = hv[k];
            int ox = (int)hix[src] - (int)hix[c], oy = (int)hiy[src] - (int)hiy[c];
            if (std::abs(ox) > 3 || std::abs(oy) > 3 || slot[offset_slot(ox, oy)] < 0)
                throw Error{FMDDM_EDEVICE, "V-list entry outside the offset stencil"};
            byop[slot[offset_slot(ox, oy)]].push_back(k);
        }
    std::vector<int> top, tbeg, tend, pk, psrc;
    std::vector<double> pscale;
    for (int o = 0; o < nop; ++o) {
        const std::vector<int> &ks = byop[o];
        for (size_t b = 0; b < ks.size(); b += GN) {
            top.push_back(o);
            tbeg.push_back((int)pk.size());
            size_t e = std::min(ks.size(), b + GN);
            for (size_t i = b; i < e; ++i) {
                int k = ks[i];
                int c = (int)(std::upper_bound(vo.begin(), vo.end(), k) - vo.begin()) - 1;
                pk.push_back(k);
                psrc.push_back(hv[k]);
                pscale.push_back(1.0 / (hhw[c] * hhw[c]));
            }
            tend.push_back((int)pk.size());
        }
    }
    t->ntile = (int)top.size();
    t->tile_op.alloc(t->ntile); t->tile_beg.alloc(t->ntile); t->tile_end.alloc(t->ntile);
    t->pair_k.alloc(pk.size()); t->pair_src.alloc(pk.size()); t->pair_scale.alloc(pk.size());
    if (t->ntile) {
        FM_HIP(hipMemcpyAsync(t->tile_op.p, top.data(), top.size() * 4, hipMemcpyHostToDevice, s));
        FM_HIP(hipMemcpyAsync(t->tile_beg.p, tbeg.data(), tbeg.size() * 4, hipMemcpyHostToDevice, s));
        FM_HIP(hipMemcpyAsync(t->tile_end.p, tend.data(), tend.size() * 4, hipMemcpyHostToDevice, s));
        FM_HIP(hipMemcpyAsync(t->pair_k.p, pk.data(), pk.size() * 4, hipMemcpyHostToDevice, s));
        FM_HIP(hipMemcpyAsync(t->pair_src.p, psrc.data(), psrc.size() * 4, hipMemcpyHostToDevice, s));
        FM_HIP(hipMemcpyAsync(t->pair_scale.p, pscale.data(), pscale.size() * 8, hipMemcpyHostToDevice, s));
    }
    t->Wexp.alloc((size_t)ncell * Mp);
    t->Fexp.alloc((size_t)ncell * Mp);
    t->Zm2l.alloc((size_t)std::max<int64_t>(t->nV, 1) * Mp);
    t->Wexp.zero(s);
    t->Fexp.zero(s);
    t->q.alloc(3 * (size_t)t->n);
    t->Dsort.alloc(2 * (size_t)t->n);  // D in tree order
    FM_HIP(hipStreamSynchronize(s));
}

void fmm_apply(fmddm_ctx *ctx, fmddm_tree *t, const double *D, double *out)
{
    setup_fmm(ctx, t);
    hipStream_t s = ctx->stream;
    int p = ctx->prm.p, Mp = ctx->m2l.Mp, n = (int)t->n;
    const Cheb &C = ctx->cheb;
    Profiler &P = ctx->prof;
    hipEvent_t e0;
    P.begin(FMDDM_PH_PREP, s, e0);
    hipLaunchKernelGGL(k_prep, dim3(cdiv(n, 256)), dim3(256), 0, s, n, t->perm.p, D, t->scb.p,
                       t->ssb.p, t->Dsort.p, t->q.p);
    FM_CHECK_LAUNCH();
    P.end(FMDDM_PH_PREP, s, e0);
    bool far = t->nV > 0;
    if (far) {
        P.begin(FMDDM_PH_P2M, s, e0);
        hipLaunchKernelGGL(k_p2m, dim3(t->nleaf), dim3(P2M_T), 0, s, t->nleaf, t->dleaves.p, t->cpbeg.p,
                           t->cpend.p, t->ccx.p, t->ccy.p, t->chw.p, t->scx.p, t->scy.p, t->scb.p,
                           t->ssb.p, t->sa.p, t->q.p, C.tnode.p, C.gl_t.p, C.gl_w.p, p, Mp, t->Wexp.p);
        FM_CHECK_LAUNCH();
        P.end(FMDDM_PH_P2M, s, e0);
        P.begin(FMDDM_PH_M2M, s, e0);
        for (int l = t->nlevel - 2; l >= 0; --l) {
            int c0 = t->level_start[l], nc = t->level_start[l + 1] - c0;
            hipLaunchKernelGGL(k_m2m, dim3(nc), dim3(TT), 0, s, c0, nc, t->cleaf.p, t->cchild.p,
                               C.m2m.p, p, Mp, t->Wexp.p);
            FM_CHECK_LAUNCH();
        }
        P.end(FMDDM_PH_M2M, s, e0);
        P.begin(FMDDM_PH_M2L, s, e0);
        if (t->ntile) {
            hipLaunchKernelGGL(k_m2l_gemm, dim3(t->ntile, Mp / GM), dim3(256), 0, s, ctx->m2l.ops.p, Mp,
                               t->Wexp.p, t->tile_op.p, t->tile_beg.p, t->tile_end.p, t->pair_k.p,
                               t->pair_src.p, t->pair_scale.p, t->Zm2l.p);
            FM_CHECK_LAUNCH();
        }
        P.end(FMDDM_PH_M2L, s, e0);
        P.begin(FMDDM_PH_DOWN, s, e0);
        for (int l = 1; l < t->nlevel; ++l) {
            int c0 = t->level_start[l], nc = t->level_start[l + 1] - c0;
            hipLaunchKernelGGL(k_down, dim3(nc), dim3(TT), 0, s, c0, nc, t->cparent.p, t->cix.p, t->ciy.p,
                               t->loff[1].p, t->Zm2l.p, C.m2m.p, p, Mp, l >= 2 ? 1 : 0, t->Fexp.p);
            FM_CHECK_LAUNCH();
        }
        P.end(FMDDM_PH_DOWN, s, e0);
    }
    P.begin(FMDDM_PH_NEAR, s, e0);
    hipLaunchKernelGGL(k_l2p_p2p, dim3(t->nleaf), dim3(PT), 0, s, t->nleaf, t->dleaves.p, t->cpbeg.p,
                       t->cpend.p, t->noff.p, t->nsrc.p, t->ccx.p, t->ccy.p, t->chw.p, t->scx.p, t->scy.p,
                       t->scb.p, t->ssb.p, t->sa.p, t->Dsort.p, t->perm.p, t->Fexp.p, C.tnode.p, p, Mp,
                       ctx->gc, far ? 1 : 0, out);
    FM_CHECK_LAUNCH();
    P.end(FMDDM_PH_NEAR, s, e0);
}

}  // namespace fmddm
