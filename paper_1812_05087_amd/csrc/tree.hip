// Quad-tree over element midpoints and the U/V/W/X interaction lists
// (Section 3.1), built on the device.
//
//   geometry   endpoints -> midpoint, tangent, half-length (caller order)
//   root box   bounding square of the midpoints (or the user's square)
//   keys       coordinates quantised to a 2^31 grid, bits interleaved with x
//              in the even positions (so child order is BL, BR, TL, TR: left
//              to right, then bottom to top, as in the paper's Fig. 3d)
//   sort       stable LSD radix sort of (key, element index), 4-bit digits
//   split      level by level: a cell splits into its non-empty children
//              when it holds more than `leaf` points, is below the level
//              cap, and its children stay at least kappa x the largest
//              element half-length it holds wide
//   lists      one thread per cell, neighbour lookups by binary search in
//              the per-level Morton-sorted cell table
#include "internal.h"

#include <algorithm>
#include <cmath>

// Every floating-point decision of the tree (grid coordinates, half-lengths
// in the split test, cell centres) uses separately rounded operations.
// hipcc contracts a * b + c into an FMA by default, and __dmul_rn /
// __dadd_rn are plain operators, so this file is built with
// -ffp-contract=off (the build script's per-file flags).

namespace fmddm {
namespace {

constexpr int RS_T = 256, RS_I = 8, RS_CHUNK = RS_T * RS_I;

__global__ void k_elem_geom(int n, const double *__restrict__ x1, const double *__restrict__ y1,
                            const double *__restrict__ x2, const double *__restrict__ y2,
                            double *cx, double *cy, double *cb, double *sb, double *a, int *bad)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double dx = x2[i] - x1[i], dy = y2[i] - y1[i];
    // separately rounded products, sum and (correctly rounded) square root:
    // the half-length decides splits (child side >= kappa * largest
    // half-length)
    double len = __dsqrt_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)));
    cx[i] = 0.5 * (x1[i] + x2[i]);
    cy[i] = 0.5 * (y1[i] + y2[i]);
    bool ok = isfinite(x1[i]) && isfinite(y1[i]) && isfinite(x2[i]) && isfinite(y2[i]) && len > 0.0;
    cb[i] = ok ? dx / len : 1.0;
    sb[i] = ok ? dy / len : 0.0;
    a[i] = ok ? 0.5 * len : 0.0;
    if (!ok) atomicOr(bad, 1);
}

// Single-block min/max of the midpoints (order-independent, hence exact).
__global__ __launch_bounds__(1024) void k_bbox(int n, const double *cx, const double *cy, double *out)
{
    __shared__ double s[4][1024];
    double mnx = INFINITY, mxx = -INFINITY, mny = INFINITY, mxy = -INFINITY;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        mnx = fmin(mnx, cx[i]); mxx = fmax(mxx, cx[i]);
        mny = fmin(mny, cy[i]); mxy = fmax(mxy, cy[i]);
    }
    s[0][threadIdx.x] = mnx; s[1][threadIdx.x] = mxx;
    s[2][threadIdx.x] = mny; s[3][threadIdx.x] = mxy;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + w]);
            s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + w]);
            s[2][threadIdx.x] = fmin(s[2][threadIdx.x], s[2][threadIdx.x + w]);
            s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[0] = s[0][0]; out[1] = s[1][0]; out[2] = s[2][0]; out[3] = s[3][0]; }
}

__device__ __forceinline__ uint64_t spread32(uint64_t v)
{
    v &= 0xffffffffull;
    v = (v | (v << 16)) & 0x0000ffff0000ffffull;
    v = (v | (v << 8)) & 0x00ff00ff00ff00ffull;
    v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0full;
    v = (v | (v << 2)) & 0x3333333333333333ull;
    v = (v | (v << 1)) & 0x5555555555555555ull;
    return v;
}

// Grid coordinate: floor((x - x0) * scale) clamped to [0, 2^31 - 1], with
// the subtraction and the product each rounded separately.
__device__ __forceinline__ uint64_t quantise(double x, double x0, double scale)
{
    double t = __dmul_rn(__dsub_rn(x, x0), scale);
    if (!(t > 0.0)) return 0;
    if (t >= 2147483647.0) return 2147483647ull;
    return (uint64_t)t;
}

__global__ void k_keys(int n, const double *cx, const double *cy, double x0, double y0, double scale,
                       int use_box, double L, uint64_t *key, int *idx, int *bad)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x = cx[i], y = cy[i];
    if (use_box && !(x >= x0 && x <= x0 + L && y >= y0 && y <= y0 + L)) atomicOr(bad, 2);
    uint64_t qx = quantise(x, x0, scale), qy = quantise(y, y0, scale);
    key[i] = spread32(qx) | (spread32(qy) << 1);
    idx[i] = i;
}

// ---------------------------------------------------------- radix sort
__global__ __launch_bounds__(RS_T) void k_rs_hist(const uint64_t *key, int n, int shift, int *hist)
{
    __shared__ int cnt[16];
    if (threadIdx.x < 16) cnt[threadIdx.x] = 0;
    __syncthreads();
    int base = blockIdx.x * RS_CHUNK;
    for (int i = threadIdx.x; i < RS_CHUNK; i += RS_T) {
        int g = base + i;
        if (g < n) atomicAdd(&cnt[(int)((key[g] >> shift) & 15ull)], 1);
    }
    __syncthreads();
    if (threadIdx.x < 16) hist[threadIdx.x * gridDim.x + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive block scan of one int per thread (blockDim <= 1024).
__device__ int block_exscan(int v, int *tmp, int *total)
{
    int t = threadIdx.x;
    tmp[t] = v;
    __syncthreads();
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {
        int add = t >= off ? tmp[t - off] : 0;
        __syncthreads();
        tmp[t] += add;
        __syncthreads();
    }
    int incl = tmp[t];
    int tot = tmp[blockDim.x - 1];
    __syncthreads();
    if (total) *total = tot;
    return incl - v;
}

// Single-block exclusive scan of m ints in place (any m).
__global__ __launch_bounds__(1024) void k_scan_small(int *a, int m, int *total)
{
    __shared__ int tmp[1024];
    int per = (m + blockDim.x - 1) / blockDim.x;
    int b = threadIdx.x * per, e = min(m, b + per);
    int s = 0;
    for (int i = b; i < e; ++i) s += a[i];
    int tot;
    int pre = block_exscan(s, tmp, &tot);
    for (int i = b; i < e; ++i) {
        int v = a[i];
        a[i] = pre;
        pre += v;
    }
    if (threadIdx.x == 0 && total) *total = tot;
}

__global__ __launch_bounds__(RS_T) void k_rs_scatter(const uint64_t *kin, const int *vin, uint64_t *kout,
                                                     int *vout, int n, int shift, const int *offs)
{
    __shared__ int sc[16 * RS_T];
    __shared__ int tmp[RS_T];
    int t = threadIdx.x;
    int base = blockIdx.x * RS_CHUNK + t * RS_I;
    uint64_t k[RS_I];
    int v[RS_I], d[RS_I];
    int c[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) c[e] = 0;
#pragma unroll
    for (int i = 0; i < RS_I; ++i) {
        int g = base + i;
        if (g < n) {
            k[i] = kin[g];
            v[i] = vin[g];
            d[i] = (int)((k[i] >> shift) & 15ull);
#pragma unroll
            for (int e = 0; e < 16; ++e) c[e] += (d[i] == e);
        } else {
            d[i] = -1;
        }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) sc[e * RS_T + t] = c[e];
    __syncthreads();
    // exclusive scan over sc in (digit, thread) order; thread t owns 16
    // consecutive entries
    int loc[16];
    int s = 0;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        loc[e] = s;
        s += sc[16 * t + e];
    }
    int pre = block_exscan(s, tmp, nullptr);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 16; ++e) sc[16 * t + e] = loc[e] + pre;
    __syncthreads();
    int run[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) run[e] = sc[e * RS_T + t] - sc[e * RS_T];
#pragma unroll
    for (int i = 0; i < RS_I; ++i) {
        if (d[i] < 0) continue;
        int r = 0, off = 0;
#pragma unroll
        for (int e = 0; e < 16; ++e)
            if (d[i] == e) { r = run[e]++; off = offs[e * gridDim.x + blockIdx.x]; }
        kout[off + r] = k[i];
        vout[off + r] = v[i];
    }
}

__global__ void k_gather_sorted(int n, const int *perm, const double *cx, const double *cy,
                                const double *cb, const double *sb, const double *a, double *scx,
                                double *scy, double *scb, double *ssb, double *sa)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int j = perm[i];
    scx[i] = cx[j]; scy[i] = cy[j]; scb[i] = cb[j]; ssb[i] = sb[j]; sa[i] = a[j];
}

// ------------------------------------------------------------ splitting
__global__ __launch_bounds__(256) void k_split_count(int c0, const int *pbeg, const int *pend,
                                                     const double *sa, const uint64_t *key, int level,
                                                     int leaf, int cap, double child_side,
                                                     double kappa, int *nchild, int *bounds)
{
    __shared__ double red[256];
    int c = c0 + blockIdx.x;
    int b = pbeg[c], e = pend[c];
    double m = 0.0;
    for (int k = b + threadIdx.x; k < e; k += 256) m = fmax(m, sa[k]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    double amax = red[0];
    bool split = (e - b > leaf) && (level < cap) && (child_side >= kappa * amax);
    int *bd = bounds + 5 * blockIdx.x;
    if (!split) {
        nchild[blockIdx.x] = 0;
        return;
    }
    int sh = 62 - 2 * (level + 1);
    bd[0] = b;
    bd[4] = e;
    for (int d = 1; d < 4; ++d) {
        int lo = b, hi = e;  // first index with digit >= d
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if ((int)((key[mid] >> sh) & 3ull) < d) lo = mid + 1;
            else hi = mid;
        }
        bd[d] = lo;
    }
    int cnt = 0;
    for (int d = 0; d < 4; ++d) cnt += bd[d + 1] > bd[d];
    nchild[blockIdx.x] = cnt;
}

__global__ void k_split_write(int c0, int nc, int cnext, const int *nchild_ex, const int *nchild_cnt,
                              const int *bounds, int level, double x0, double y0, double L,
                              int *clevel, uint32_t *cix, uint32_t *ciy, int *cparent, int *cchild,
                              int *cpbeg, int *cpend, int *cleaf, uint64_t *cmk, double *ccx,
                              double *ccy, double *chw)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc) return;
    int c = c0 + i;
    if (nchild_cnt[i] == 0) return;
    cleaf[c] = 0;
    const int *bd = bounds + 5 * i;
    int idx = cnext + nchild_ex[i];
    double side = ldexp(L, -(level + 1));
    for (int d = 0; d < 4; ++d) {
        if (bd[d + 1] <= bd[d]) {
            cchild[4 * c + d] = -1;
            continue;
        }
        uint32_t ix = 2u * cix[c] + (uint32_t)(d & 1);
        uint32_t iy = 2u * ciy[c] + (uint32_t)(d >> 1);
        cchild[4 * c + d] = idx;
        clevel[idx] = level + 1;
        cix[idx] = ix;
        ciy[idx] = iy;
        cparent[idx] = c;
        cpbeg[idx] = bd[d];
        cpend[idx] = bd[d + 1];
        cleaf[idx] = 1;
        for (int k = 0; k < 4; ++k) cchild[4 * idx + k] = -1;
        cmk[idx] = spread32(ix) | (spread32(iy) << 1);
        ccx[idx] = __dadd_rn(x0, __dmul_rn((double)ix + 0.5, side));
        ccy[idx] = __dadd_rn(y0, __dmul_rn((double)iy + 0.5, side));
        chw[idx] = 0.5 * side;
        ++idx;
    }
}

// ---------------------------------------------------------------- lists
struct CellView {
    const int *level, *parent, *child, *leaf, *lstart;
    const uint32_t *ix, *iy;
    const uint64_t *mk;
    int nlevel;
};

__device__ int find_cell(const CellView &v, int l, int64_t ix, int64_t iy)
{
    if (l < 0 || l >= v.nlevel) return -1;
    int64_t lim = (int64_t)1 << l;
    if (ix < 0 || iy < 0 || ix >= lim || iy >= lim) return -1;
    uint64_t m = spread32((uint64_t)ix) | (spread32((uint64_t)iy) << 1);
    int lo = v.lstart[l], hi = v.lstart[l + 1];
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (v.mk[mid] < m) lo = mid + 1;
        else hi = mid;
    }
    return (lo < v.lstart[l + 1] && v.mk[lo] == m) ? lo : -1;
}

__device__ bool adjacent(const CellView &v, int c, int d)
{
    int lc = v.level[c], ld = v.level[d];
    int lm = lc > ld ? lc : ld;
    uint64_t cx0 = (uint64_t)v.ix[c] << (lm - lc), cx1 = ((uint64_t)v.ix[c] + 1) << (lm - lc);
    uint64_t cy0 = (uint64_t)v.iy[c] << (lm - lc), cy1 = ((uint64_t)v.iy[c] + 1) << (lm - lc);
    uint64_t dx0 = (uint64_t)v.ix[d] << (lm - ld), dx1 = ((uint64_t)v.ix[d] + 1) << (lm - ld);
    uint64_t dy0 = (uint64_t)v.iy[d] << (lm - ld), dy1 = ((uint64_t)v.iy[d] + 1) << (lm - ld);
    return cx0 <= dx1 && dx0 <= cx1 && cy0 <= dy1 && dy0 <= cy1;
}

// Emits into a list: counts in pass 0, writes in pass 1.
struct Emit {
    int *out;
    int n = 0;
    __device__ void put(int c)
    {
        if (out) out[n] = c;
        ++n;
    }
};

__device__ void sort_seg(int *a, int n)
{
    for (int i = 1; i < n; ++i) {
        int v = a[i], j = i - 1;
        while (j >= 0 && a[j] > v) { a[j + 1] = a[j]; --j; }
        a[j + 1] = v;
    }
}

constexpr int DFS_MAX = 256;

// which: 0 U, 1 V, 2 W, 3 X.  pass 0 writes counts[c]; pass 1 fills at off[c].
__global__ void k_lists(CellView v, int ncell, int which, int pass, int *counts, const int *off,
                        int *idx, int *bad)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    Emit em;
    em.out = pass ? idx + off[c] : nullptr;
    int l = v.level[c];
    int64_t ix = v.ix[c], iy = v.iy[c];
    if (which == 1) {  // V
        if (c != 0) {
            int P = v.parent[c];
            int64_t px = v.ix[P], py = v.iy[P];
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int C = find_cell(v, l - 1, px + dx, py + dy);
                    if (C < 0) continue;
                    for (int d = 0; d < 4; ++d) {
                        int A = v.child[4 * C + d];
                        if (A >= 0 && !adjacent(v, A, c)) em.put(A);
                    }
                }
        }
    } else if (which == 0 || which == 2) {  // U or W (leaves only)
        if (v.leaf[c]) {
            int stack[DFS_MAX];
            int sp = 0;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int C = find_cell(v, l, ix + dx, iy + dy);
                    if (C < 0) continue;
                    if (v.leaf[C]) {
                        if (which == 0) em.put(C);
                        continue;
                    }
                    // finer cells under a same-level neighbour
                    stack[sp++] = C;
                    while (sp > 0) {
                        int Q = stack[--sp];
                        for (int d = 0; d < 4; ++d) {
                            int A = v.child[4 * Q + d];
                            if (A < 0) continue;
                            if (!adjacent(v, A, c)) {
                                if (which == 2) em.put(A);
                            } else if (v.leaf[A]) {
                                if (which == 0) em.put(A);
                            } else if (sp < DFS_MAX) {
                                stack[sp++] = A;
                            } else {
                                atomicOr(bad, 4);
                            }
                        }
                    }
                }
            if (which == 0) {
                // coarser leaves adjacent to c: neighbours of its ancestors
                for (int la = 0; la < l; ++la) {
                    int64_t ax = ix >> (l - la), ay = iy >> (l - la);
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            if (dx == 0 && dy == 0) continue;
                            int C = find_cell(v, la, ax + dx, ay + dy);
                            if (C >= 0 && v.leaf[C] && adjacent(v, C, c)) em.put(C);
                        }
                }
            }
        }
    } else {  // X: leaves B, coarser than c, adjacent to parent(c), not to c
        if (c != 0) {
            int P = v.parent[c];
            for (int la = 0; la < l; ++la) {
                int64_t ax = ix >> (l - la), ay = iy >> (l - la);
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        if (dx == 0 && dy == 0) continue;
                        int C = find_cell(v, la, ax + dx, ay + dy);
                        if (C >= 0 && v.leaf[C] && adjacent(v, P, C) && !adjacent(v, c, C)) em.put(C);
                    }
            }
        }
    }
    if (pass == 0) counts[c] = em.n;
    else sort_seg(idx + off[c], em.n);
}

// Near-field sources of each leaf: U, then W, then X of the leaf and of
// each ancestor up to the root.
__global__ void k_near(int nleaf, const int *leaves, const int *parent, const int *const *loff,
                       const int *const *lidx, int pass, int *counts, const int *off, int *out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nleaf) return;
    int c = leaves[i];
    int n = 0;
    int *o = pass ? out + off[i] : nullptr;
    for (int w = 0; w <= 2; w += 2)
        for (int k = loff[w][c]; k < loff[w][c + 1]; ++k) {
            if (o) o[n] = lidx[w][k];
            ++n;
        }
    for (int a = c; a >= 0; a = parent[a])
        for (int k = loff[3][a]; k < loff[3][a + 1]; ++k) {
            if (o) o[n] = lidx[3][k];
            ++n;
        }
    if (!pass) counts[i] = n;
}

void exscan_small(int *d, int m, int *d_total, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, s, d, m, d_total);
    FM_CHECK_LAUNCH();
}

}  // namespace

void build_tree(fmddm_ctx *ctx, fmddm_tree *t, int64_t n64, const double *x1, const double *y1,
                const double *x2, const double *y2, int on_device)
{
    hipStream_t s = ctx->stream;
    const fmddm_params &P = ctx->prm;
    if (n64 <= 0 || n64 > (int64_t)1 << 30) throw Error{FMDDM_EINVAL, "n out of range"};
    int n = (int)n64;
    t->n = n;
    DBuf<double> ex1, ey1, ex2, ey2;
    const double *px1 = x1, *py1 = y1, *px2 = x2, *py2 = y2;
    if (!on_device) {
        ex1.alloc(n); ey1.alloc(n); ex2.alloc(n); ey2.alloc(n);
        FM_HIP(hipMemcpyAsync(ex1.p, x1, n * 8, hipMemcpyHostToDevice, s));
        FM_HIP(hipMemcpyAsync(ey1.p, y1, n * 8, hipMemcpyHostToDevice, s));
        FM_HIP(hipMemcpyAsync(ex2.p, x2, n * 8, hipMemcpyHostToDevice, s));
        FM_HIP(hipMemcpyAsync(ey2.p, y2, n * 8, hipMemcpyHostToDevice, s));
        px1 = ex1.p; py1 = ey1.p; px2 = ex2.p; py2 = ey2.p;
    }
    t->ocx.alloc(n); t->ocy.alloc(n); t->ocb.alloc(n); t->osb.alloc(n); t->oa.alloc(n);
    DBuf<int> flag;
    flag.alloc(4);
    flag.zero(s);
    hipLaunchKernelGGL(k_elem_geom, dim3(cdiv(n, 256)), dim3(256), 0, s, n, px1, py1, px2, py2,
                       t->ocx.p, t->ocy.p, t->ocb.p, t->osb.p, t->oa.p, flag.p);
    FM_CHECK_LAUNCH();

    // root square
    if (P.use_root_box) {
        t->x0 = P.root_x0; t->y0 = P.root_y0; t->L = P.root_L;
    } else {
        DBuf<double> bb;
        bb.alloc(4);
        hipLaunchKernelGGL(k_bbox, dim3(1), dim3(1024), 0, s, n, t->ocx.p, t->ocy.p, bb.p);
        FM_CHECK_LAUNCH();
        double h[4];
        FM_HIP(hipMemcpyAsync(h, bb.p, sizeof(h), hipMemcpyDeviceToHost, s));
        FM_HIP(hipStreamSynchronize(s));
        t->x0 = h[0];
        t->y0 = h[2];
        double dx = h[1] - h[0], dy = h[3] - h[2];
        t->L = dx > dy ? dx : dy;
        if (t->L == 0.0) t->L = 1.0;
    }
    if (!(t->L > 0.0) || !std::isfinite(t->L)) throw Error{FMDDM_EGEOM, "degenerate root box"};
    double scale = 2147483648.0 / t->L;

    // keys and sort
    DBuf<uint64_t> k0, k1;
    DBuf<int> v0, v1;
    k0.alloc(n); k1.alloc(n); v0.alloc(n); v1.alloc(n);
    hipLaunchKernelGGL(k_keys, dim3(cdiv(n, 256)), dim3(256), 0, s, n, t->ocx.p, t->ocy.p, t->x0,
                       t->y0, scale, P.use_root_box, t->L, k0.p, v0.p, flag.p);
    FM_CHECK_LAUNCH();
    int nb = cdiv(n, RS_CHUNK);
    DBuf<int> hist;
    hist.alloc(16 * nb);
    for (int shift = 0; shift < 64; shift += 4) {
        hipLaunchKernelGGL(k_rs_hist, dim3(nb), dim3(RS_T), 0, s, k0.p, n, shift, hist.p);
        FM_CHECK_LAUNCH();
        exscan_small(hist.p, 16 * nb, nullptr, s);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(RS_T), 0, s, k0.p, v0.p, k1.p, v1.p, n,
                           shift, hist.p);
        FM_CHECK_LAUNCH();
        std::swap(k0.p, k1.p);
        std::swap(v0.p, v1.p);
    }
    int hflag = 0;
    FM_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    FM_HIP(hipStreamSynchronize(s));
    if (hflag & 1) throw Error{FMDDM_EGEOM, "zero-length or non-finite element"};
    if (hflag & 2) throw Error{FMDDM_EGEOM, "element midpoint outside the root box"};
    t->key.alloc(n);
    t->perm.alloc(n);
    FM_HIP(hipMemcpyAsync(t->key.p, k0.p, n * 8, hipMemcpyDeviceToDevice, s));
    FM_HIP(hipMemcpyAsync(t->perm.p, v0.p, n * 4, hipMemcpyDeviceToDevice, s));
    t->scx.alloc(n); t->scy.alloc(n); t->scb.alloc(n); t->ssb.alloc(n); t->sa.alloc(n);
    hipLaunchKernelGGL(k_gather_sorted, dim3(cdiv(n, 256)), dim3(256), 0, s, n, t->perm.p, t->ocx.p,
                       t->ocy.p, t->ocb.p, t->osb.p, t->oa.p, t->scx.p, t->scy.p, t->scb.p, t->ssb.p,
                       t->sa.p);
    FM_CHECK_LAUNCH();

    // cell capacity: at level l at most min(4^l, 4 * split cells of the
    // level above), split cells hold > leaf points each
    int cap = P.max_level;
    int64_t maxsplit = n / (P.leaf + 1) + 1;
    int64_t capc = 1;
    for (int l = 1; l <= cap; ++l) {
        int64_t lim = l < 31 ? ((int64_t)1 << (2 * l)) : INT64_MAX;
        capc += std::min<int64_t>(lim, 4 * maxsplit);
    }
    if (capc > (int64_t)1 << 30) throw Error{FMDDM_EINVAL, "tree too large"};
    t->clevel.alloc(capc); t->cix.alloc(capc); t->ciy.alloc(capc); t->cparent.alloc(capc);
    t->cchild.alloc(4 * capc); t->cpbeg.alloc(capc); t->cpend.alloc(capc); t->cleaf.alloc(capc);
    t->cmk.alloc(capc); t->ccx.alloc(capc); t->ccy.alloc(capc); t->chw.alloc(capc);
    {
        int zi = 0, m1 = -1, one = 1, npts = n;
        uint32_t zu = 0;
        uint64_t zk = 0;
        int ch[4] = {-1, -1, -1, -1};
        double cx0 = t->x0 + 0.5 * t->L, cy0 = t->y0 + 0.5 * t->L, hw = 0.5 * t->L;
        FM_HIP(hipMemcpyAsync(t->clevel.p, &zi, 4, hipMemcpyHostToDevice, s));
        FM_HIP(hipMemcpyAsync(t->cix.p, &zu, 4, hipMemcpyHostToDevice, s));
        FM_HIP(hipMemcpyAsync(t->ciy.p, &zu, 4, hipMemcpyHostToDevice, s));
        FM_HIP(hipMemcpyAsync(t->cparent.p, &m1, 4, hipMemcpyHostToDevice, s));
        FM_HIP(hipMemcpyAsync(t->cchild.p, ch, 16, hipMemcpyHostToDevice, s));
        FM_HIP(hipMemcpyAsync(t->cpbeg.p, &zi, 4, hipMemcpyHostToDevice, s));
        FM_HIP(hipMemcpyAsync(t->cpend.p, &npts, 4, hipMemcpyHostToDevice, s));
        FM_HIP(hipMemcpyAsync(t->cleaf.p, &one, 4, hipMemcpyHostToDevice, s));
        FM_HIP(hipMemcpyAsync(t->cmk.p, &zk, 8, hipMemcpyHostToDevice, s));
        FM_HIP(hipMemcpyAsync(t->ccx.p, &cx0, 8, hipMemcpyHostToDevice, s));
        FM_HIP(hipMemcpyAsync(t->ccy.p, &cy0, 8, hipMemcpyHostToDevice, s));
        FM_HIP(hipMemcpyAsync(t->chw.p, &hw, 8, hipMemcpyHostToDevice, s));
        FM_HIP(hipStreamSynchronize(s));  // host values above go out of scope
    }
    t->level_start.assign(1, 0);
    int c0 = 0, nc = 1, level = 0;
    DBuf<int> nch, nchx, bounds, tot;
    tot.alloc(1);
    while (nc > 0) {
        t->level_start.push_back(c0 + nc);
        nch.alloc(nc); nchx.alloc(nc); bounds.alloc(5 * nc);
        double child_side = ldexp(t->L, -(level + 1));
        hipLaunchKernelGGL(k_split_count, dim3(nc), dim3(256), 0, s, c0, t->cpbeg.p, t->cpend.p,
                           t->sa.p, t->key.p, level, P.leaf, cap, child_side, P.kappa, nch.p,
                           bounds.p);
        FM_CHECK_LAUNCH();
        FM_HIP(hipMemcpyAsync(nchx.p, nch.p, nc * 4, hipMemcpyDeviceToDevice, s));
        exscan_small(nchx.p, nc, tot.p, s);
        int total = 0;
        FM_HIP(hipMemcpyAsync(&total, tot.p, 4, hipMemcpyDeviceToHost, s));
        FM_HIP(hipStreamSynchronize(s));
        if (total == 0) break;
        if ((int64_t)c0 + nc + total > capc) throw Error{FMDDM_EDEVICE, "cell capacity exceeded"};
        hipLaunchKernelGGL(k_split_write, dim3(cdiv(nc, 128)), dim3(128), 0, s, c0, nc, c0 + nc,
                           nchx.p, nch.p, bounds.p, level, t->x0, t->y0, t->L, t->clevel.p, t->cix.p,
                           t->ciy.p, t->cparent.p, t->cchild.p, t->cpbeg.p, t->cpend.p, t->cleaf.p,
                           t->cmk.p, t->ccx.p, t->ccy.p, t->chw.p);
        FM_CHECK_LAUNCH();
        c0 += nc;
        nc = total;
        ++level;
    }
    t->ncell = t->level_start.back();
    t->nlevel = (int)t->level_start.size() - 1;

    // lists
    DBuf<int> lstart;
    lstart.alloc(t->nlevel + 1);
    FM_HIP(hipMemcpyAsync(lstart.p, t->level_start.data(), (t->nlevel + 1) * 4,
                          hipMemcpyHostToDevice, s));
    CellView v{t->clevel.p, t->cparent.p, t->cchild.p, t->cleaf.p, lstart.p,
               t->cix.p, t->ciy.p, t->cmk.p, t->nlevel};
    int ncell = t->ncell;
    DBuf<int> cnt;
    cnt.alloc(ncell + 1);
    for (int w = 0; w < 4; ++w) {
        t->loff[w].alloc(ncell + 1);
        t->loff[w].zero(s);
        hipLaunchKernelGGL(k_lists, dim3(cdiv(ncell, 128)), dim3(128), 0, s, v, ncell, w, 0,
                           t->loff[w].p, (const int *)nullptr, (int *)nullptr, flag.p);
        FM_CHECK_LAUNCH();
        exscan_small(t->loff[w].p, ncell + 1, nullptr, s);
        t->h_loff[w].resize(ncell + 1);
        FM_HIP(hipMemcpyAsync(t->h_loff[w].data(), t->loff[w].p, (ncell + 1) * 4,
                              hipMemcpyDeviceToHost, s));
        FM_HIP(hipStreamSynchronize(s));
        t->lidx[w].alloc(t->h_loff[w][ncell]);
        hipLaunchKernelGGL(k_lists, dim3(cdiv(ncell, 128)), dim3(128), 0, s, v, ncell, w, 1,
                           (int *)nullptr, (const int *)t->loff[w].p, t->lidx[w].p, flag.p);
        FM_CHECK_LAUNCH();
    }
    FM_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    t->h_isleaf.resize(ncell);
    t->h_level.resize(ncell);
    FM_HIP(hipMemcpyAsync(t->h_isleaf.data(), t->cleaf.p, ncell * 4, hipMemcpyDeviceToHost, s));
    FM_HIP(hipMemcpyAsync(t->h_level.data(), t->clevel.p, ncell * 4, hipMemcpyDeviceToHost, s));
    FM_HIP(hipStreamSynchronize(s));
    if (hflag & 4) throw Error{FMDDM_EDEVICE, "list traversal stack overflow"};
    t->nV = t->h_loff[1][ncell];

    // near-field source lists per leaf
    t->leaves.clear();
    for (int c = 0; c < ncell; ++c)
        if (t->h_isleaf[c]) t->leaves.push_back(c);
    t->nleaf = (int)t->leaves.size();
    t->dleaves.alloc(t->nleaf);
    FM_HIP(hipMemcpyAsync(t->dleaves.p, t->leaves.data(), t->nleaf * 4, hipMemcpyHostToDevice, s));
    DBuf<const int *> ploff, plidx;
    ploff.alloc(4);
    plidx.alloc(4);
    const int *hoff[4], *hidx[4];
    for (int w = 0; w < 4; ++w) { hoff[w] = t->loff[w].p; hidx[w] = t->lidx[w].p; }
    FM_HIP(hipMemcpyAsync(ploff.p, hoff, sizeof(hoff), hipMemcpyHostToDevice, s));
    FM_HIP(hipMemcpyAsync(plidx.p, hidx, sizeof(hidx), hipMemcpyHostToDevice, s));
    t->noff.alloc(t->nleaf + 1);
    t->noff.zero(s);
    hipLaunchKernelGGL(k_near, dim3(cdiv(t->nleaf, 128)), dim3(128), 0, s, t->nleaf, t->dleaves.p,
                       t->cparent.p, ploff.p, plidx.p, 0, t->noff.p, (const int *)nullptr,
                       (int *)nullptr);
    FM_CHECK_LAUNCH();
    exscan_small(t->noff.p, t->nleaf + 1, nullptr, s);
    std::vector<int> hnoff(t->nleaf + 1);
    FM_HIP(hipMemcpyAsync(hnoff.data(), t->noff.p, (t->nleaf + 1) * 4, hipMemcpyDeviceToHost, s));
    FM_HIP(hipStreamSynchronize(s));
    t->nsrc.alloc(hnoff[t->nleaf]);
    hipLaunchKernelGGL(k_near, dim3(cdiv(t->nleaf, 128)), dim3(128), 0, s, t->nleaf, t->dleaves.p,
                       t->cparent.p, ploff.p, plidx.p, 1, (int *)nullptr, (const int *)t->noff.p,
                       t->nsrc.p);
    FM_CHECK_LAUNCH();
    // flattened near-source ranges and ancestor lists per leaf (schedule
    // for the near-field kernel), and the count of direct pairs
    {
        std::vector<int> hn(hnoff[t->nleaf]), hb(ncell), he(ncell), hp(ncell);
        if (!hn.empty())
            FM_HIP(hipMemcpyAsync(hn.data(), t->nsrc.p, hn.size() * 4, hipMemcpyDeviceToHost, s));
        FM_HIP(hipMemcpyAsync(hb.data(), t->cpbeg.p, ncell * 4, hipMemcpyDeviceToHost, s));
        FM_HIP(hipMemcpyAsync(he.data(), t->cpend.p, ncell * 4, hipMemcpyDeviceToHost, s));
        FM_HIP(hipMemcpyAsync(hp.data(), t->cparent.p, ncell * 4, hipMemcpyDeviceToHost, s));
        FM_HIP(hipStreamSynchronize(s));
        std::vector<int> nbeg(hn.size()), npre(hn.size()), ntot(t->nleaf), aoff(t->nleaf + 1, 0), aidx;
        int64_t pairs = 0;
        for (int i = 0; i < t->nleaf; ++i) {
            int c = t->leaves[i];
            int acc = 0;
            for (int k = hnoff[i]; k < hnoff[i + 1]; ++k) {
                nbeg[k] = hb[hn[k]];
                npre[k] = acc;
                acc += he[hn[k]] - hb[hn[k]];
            }
            ntot[i] = acc;
            pairs += (int64_t)acc * (he[c] - hb[c]);
            for (int A = c; A >= 0; A = hp[A])
                if (t->h_level[A] >= 2) aidx.push_back(A);
            aoff[i + 1] = (int)aidx.size();
            t->l2p_pairs += (int64_t)(aoff[i + 1] - aoff[i]) * (he[c] - hb[c]);
        }
        t->near_pairs = pairs;
        // upward pass (eq. 3.7): one transfer per cell whose parent has an
        // expansion (level >= 2)
        for (int c = 0; c < ncell; ++c)
            if (hp[c] >= 0 && t->h_level[hp[c]] >= 2) ++t->m2m_pairs;
        auto up = [&](DBuf<int> &d, const std::vector<int> &h) {
            d.alloc(h.size());
            if (!h.empty()) FM_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * 4, hipMemcpyHostToDevice, s));
        };
        up(t->nbeg, nbeg);
        up(t->npre, npre);
        up(t->ntot, ntot);
        // the same near sources as one flat list of points per leaf (the
        // elastic near-field kernel indexes it directly)
        {
            std::vector<int> nfoff(t->nleaf + 1, 0), nflat;
            for (int i = 0; i < t->nleaf; ++i) nfoff[i + 1] = nfoff[i] + ntot[i];
            nflat.reserve(nfoff[t->nleaf]);
            for (int i = 0; i < t->nleaf; ++i)
                for (int k = hnoff[i]; k < hnoff[i + 1]; ++k)
                    for (int j = hb[hn[k]]; j < he[hn[k]]; ++j) nflat.push_back(j);
            up(t->nfoff, nfoff);
            up(t->nflat, nflat);
        }
        up(t->aoff, aoff);
        up(t->aidx, aidx);
        // near-field work items and the leaf of every point
        std::vector<int> it_leaf, it_s0, it_s1, it_poff, lk_off(t->nleaf + 1, 0), tleaf(n, -1);
        std::vector<int64_t> it_coff;  // pairs (target, source) before each item
        int64_t poff = 0, coff = 0;
        for (int i = 0; i < t->nleaf; ++i) {
            int c = t->leaves[i];
            int nt = he[c] - hb[c];
            for (int k = hb[c]; k < he[c]; ++k) tleaf[k] = i;
            int s0 = 0;
            do {
                int s1 = std::min(ntot[i], s0 + NEAR_CHUNK);
                it_leaf.push_back(i);
                it_s0.push_back(s0);
                it_s1.push_back(s1);
                it_poff.push_back((int)poff);
                it_coff.push_back(coff);
                poff += nt;
                coff += (int64_t)nt * (s1 - s0);
                s0 = s1;
            } while (s0 < ntot[i]);
            lk_off[i + 1] = (int)it_leaf.size();
        }
        if (poff > (int64_t)1 << 30) throw Error{FMDDM_EINVAL, "near-field partials too large"};
        if (coff != t->near_pairs) throw Error{FMDDM_EDEVICE, "near-field schedule does not cover the near pairs"};
        t->nitem = (int)it_leaf.size();
        t->npartial = poff;
        up(t->it_leaf, it_leaf);
        up(t->it_s0, it_s0);
        up(t->it_s1, it_s1);
        up(t->it_poff, it_poff);
        t->it_coff.alloc(it_coff.size());
        if (!it_coff.empty())
            FM_HIP(hipMemcpyAsync(t->it_coff.p, it_coff.data(), it_coff.size() * 8, hipMemcpyHostToDevice, s));
        up(t->lk_off, lk_off);
        up(t->tleaf, tleaf);
        FM_HIP(hipStreamSynchronize(s));
    }
}

}  // namespace fmddm
