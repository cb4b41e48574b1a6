// Poroelastic influence and the history term (Section 2, eqs. 2.1-2.5),
// evaluated exactly on the device.
//
// Unknowns per element: shear and normal displacement discontinuity and
// fluid source (D_s, D_n, D_q); responses per element: shear and normal
// traction and pore pressure at the midpoint.  The continuous-impulse
// fundamental solutions (a source switched on at t = 0 and held) of a
// fully coupled Biot medium in plane strain are, for a point eigenstrain
// with charges q and a point fluid source of volume rate q_f:
//   sigma = drained elastic field of q
//         + 2G (grad grad phi - I lap phi),   lap phi = eta p,
//   p     = (alpha kd / S)(a cos 2t + b sin 2t) P(2,z) / r^2
//           - (alpha / S) V e^-z / (4 pi c t) + q_f E1(z) / (4 pi kappa),
// with z = r^2 / (4 c t), a = 2G (q0 - q1), b = 2G q2, kd = (1 - 2nu) /
// (4 pi G (1 - nu)), V = -(q0 + q1)(1 - 2nu) / (2 (1 - nu)), P(2,z) =
// 1 - e^-z (1 + z), eta = alpha (1 - 2nu) / (2G (1 - nu)), S = 1/M + alpha
// eta, c = kappa / S.  phi is known in closed form: for the cos 2t / sin 2t
// part phi = (alpha kd eta / S)(a F(r)(x^2 - y^2) + b F(r) 2xy) with
// F = -h(z) / (4 r^2), h = 1 - (1 - e^-z) / z; the point term and the fluid
// source give radial phi with phi'/r = K (1 - e^-z) / r^2 and
// phi'/r = (q_f eta t / (2 pi S))(z E1 + 1 - e^-z) / r^2.  The paper cites
// these solutions without stating them; they are derived from the field
// equations and reduce to the undrained (nu_u) and drained (nu) elastic
// fields at t -> 0+ and t -> infinity.
//
// Constant temporal elements: the response at t_h to an interval (t_{k-1},
// t_k] is F(t_h - t_{k-1}) - F(t_h - t_k); the left-hand side is F(dt) and
// the history coefficient of lag m is K_m = F((m+1) dt) - F(m dt).  The
// history sum is rearranged so that every F(j dt) is evaluated once, on
// differences of the stored DDs (the drained parts cancel).
//
// Element integrals: the transient part is integrated along the element by
// composite Gauss-Legendre, split at the foot of the perpendicular from the
// receiver and graded there (s = s0 +- L u^3, absorbing the logarithmic
// singularity of the fluid source), with panels sized by the diffusion
// length; a receiver far from the element (8 x the larger of its length and
// the diffusion length) takes one 8-point rule over the whole element.  The
// drained part is the closed-form constant element.
#include "elem.h"
#include "gj.h"
#include "internal.h"

#include <rocblas/rocblas.h>

#include <algorithm>
#include <atomic>
#include <mutex>

#include <cmath>

namespace fmddm {
namespace {

struct PoroK {
    double G, nu, alpha, kappa, S, c, eta, gc;
    // derived (host): vfac = (1-2nu)/(2(1-nu)), ap = alpha kd / S with
    // kd = (1-2nu)/(4 pi G (1-nu)), pv = alpha / (4 pi S), cphi = alpha kd eta / S,
    // kdf = -alpha eta / (2 pi S), i4pk = 1 / (4 pi kappa), fe = eta / (2 pi S)
    double vfac, ap, pv, cphi, kdf, i4pk, fe;
};

// E1(z), z > 0.  Below 2: -gamma - ln z + Ein(z), with the series
// Ein(z) = sum (-1)^(k+1) z^k / (k k!) nested as z (1 - z/4 (1 - 2z/9
// (1 - 3z/16 (...)))) to depth 30; above: the continued fraction
// e^-z / (z + 1 - 1/(z + 3 - 4/(z + 5 - ...))) evaluated backwards from
// depth 2 + 90/z (its truncation error falls like exp(-4 sqrt(depth z)),
// below 1e-16 there); zero where e^-z underflows.
// Series coefficients, computed on the host and uploaded with the
// quadrature rules so that the series below are division-free:
// c_e1w[k] = k / (k+1)^2, c_hc[k] = (-1)^(k+1) / (k+1)!, c_p2c[k] =
// (-1)^k (k-1) / k!.
// ROLL keeps the series loops rolled: a coefficient load per term, but far
// fewer registers than the unrolled form, which holds every coefficient;
// the kernel that builds the stored near blocks uses it to run more waves.
// Both forms do the same operations in the same order.
__constant__ double c_e1w[31], c_hc[23], c_p2c[18];

template <bool ROLL = false>
__device__ double e1(double z)
{
    if (z <= 2.0) {
        double v = 1.0;
        if constexpr (ROLL) {
#pragma unroll 1
            for (int k = 30; k >= 1; --k) v = 1.0 - z * c_e1w[k] * v;
        } else {
            for (int k = 30; k >= 1; --k) v = 1.0 - z * c_e1w[k] * v;
        }
        return -0.57721566490153286061 - log(z) + z * v;
    }
    if (z > 745.0) return 0.0;
    // the reciprocal refined to full precision (within two ulp of the
    // division) in the fraction's steps
    int depth = min(64, 2 + (int)(90.0 / z));
    double f = 0.0;
    for (int k = depth; k >= 1; --k) f = (double)k * k * recip(z + 2.0 * k + 1.0 - f);
    return exp(-z) * recip(z + 1.0 - f);
}

// h(z) = 1 - (1 - e^-z)/z with h', h'' (series below 0.5).
template <bool ROLL = false>
__device__ void hfun(double z, double &h, double &h1, double &h2)
{
    if (z < 0.5) {
        // h = sum_{k>=1} c_k z^k, c_k = (-1)^(k+1) / (k+1)!, by Horner
        // from k = 22 down (the first omitted term is below 1e-26)
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        auto term = [&](int k) {
            double ck = c_hc[k];
            a0 = a0 * z + ck;
            a1 = a1 * z + ck * k;
            if (k >= 2) a2 = a2 * z + ck * k * (k - 1);
        };
        if constexpr (ROLL) {
#pragma unroll 1
            for (int k = 22; k >= 1; --k) term(k);
        } else {
            for (int k = 22; k >= 1; --k) term(k);
        }
        h = a0 * z;
        h1 = a1;
        h2 = a2;
        return;
    }
    double em = exp(-z), om = -expm1(-z);
    double iz = recip(z);
    h = 1.0 - om * iz;
    h1 = om * iz * iz - em * iz;
    h2 = -2.0 * om * iz * iz * iz + 2.0 * em * iz * iz + em * iz;
}

template <bool ROLL = false>
__device__ double p2fun(double z)
{
    if (z < 0.1) {
        // sum_{k=2}^{17} (-1)^k (k-1) z^k / k!, by Horner
        double s = 0.0;
        if constexpr (ROLL) {
#pragma unroll 1
            for (int k = 17; k >= 2; --k) s = s * z + c_p2c[k];
        } else {
            for (int k = 17; k >= 2; --k) s = s * z + c_p2c[k];
        }
        return s * z * z;
    }
    return 1.0 - exp(-z) * (1.0 + z);
}

// (xx, yy, xy) second derivatives of a radial phi from phi'/r and phi''
__device__ __forceinline__ void rad2(double x, double y, double ir2, double f1, double f2, double &dxx,
                                     double &dyy, double &dxy)
{
    dxx += (f2 * x * x + f1 * y * y) * ir2;
    dyy += (f2 * y * y + f1 * x * x) * ir2;
    dxy += (f2 - f1) * x * y * ir2;
}

// Parts of the transient point response at offset (x, y) and time t that
// do not depend on the source strengths: the charges enter only through
// a = 2G (q0 - q1), b = 2G q2 and V, and the fluid source through q_f.
struct TPoint {
    double ir2, ict, z, ez, om, gxy, g2, P2;
    // second derivatives of phi_c = F (x^2 - y^2) and phi_s = F 2xy
    double cxx, cyy, cxy, sxx, syy, sxy;
};

template <bool ROLL = false>
__device__ __forceinline__ void tpoint(const PoroK &K, double x, double y, double t, TPoint &T)
{
    double r2 = x * x + y * y, ir2 = recip(r2), r = sqrt(r2), ir = recip(r);
    double ict = recip(K.c * t);  // 1 / (c t)
    double z = 0.25 * r2 * ict;
    T.ir2 = ir2;
    T.ict = ict;
    T.z = z;
    T.ez = exp(-z);
    T.om = -expm1(-z);
    T.gxy = x * x - y * y;
    T.g2 = 2.0 * x * y;
    T.P2 = p2fun<ROLL>(z);
    double h, h1, h2;
    hfun<ROLL>(z, h, h1, h2);
    double F = -0.25 * h * ir2;
    double F1 = (h - z * h1) * 0.5 * ir2 * ir;                // F'(r)
    double F2 = (-2.0 * z * z * h2 - 3.0 * h + 3.0 * z * h1) * 0.5 * ir2 * ir2;  // F''(r)
    // second derivatives of F(r): F_xx etc. (F1/r plays phi'/r)
    double fxx = 0.0, fyy = 0.0, fxy = 0.0;
    rad2(x, y, ir2, F1 * ir, F2, fxx, fyy, fxy);
    double Fx = F1 * x * ir, Fy = F1 * y * ir;
    double gxy = T.gxy, g2 = T.g2;
    T.cxx = fxx * gxy + 4.0 * Fx * x + 2.0 * F;
    T.cyy = fyy * gxy - 4.0 * Fy * y - 2.0 * F;
    T.cxy = fxy * gxy - 2.0 * Fx * y + 2.0 * Fy * x;
    T.sxx = fxx * g2 + 4.0 * Fx * y;
    T.syy = fyy * g2 + 4.0 * Fy * x;
    T.sxy = fxy * g2 + 2.0 * Fx * x + 2.0 * Fy * y + 2.0 * F;
}

// Transient response (sxx, syy, sxy, p) at offset (x, y) and time t.
__device__ void transient(const PoroK &K, double x, double y, double t, const double q[3], double qf,
                          double o[4])
{
    TPoint T;
    tpoint(K, x, y, t, T);
    double ir2 = T.ir2, z = T.z, ez = T.ez, om = T.om;
    double a = 2.0 * K.G * (q[0] - q[1]), b = 2.0 * K.G * q[2];
    double V = -(q[0] + q[1]) * K.vfac;
    double p = K.ap * (a * T.gxy + b * T.g2) * ir2 * ir2 * T.P2 - K.pv * V * ez * T.ict;
    double Cphi = K.cphi;
    double pxx = Cphi * (a * T.cxx + b * T.sxx), pyy = Cphi * (a * T.cyy + b * T.syy),
           pxy = Cphi * (a * T.cxy + b * T.sxy);
    double Kd = K.kdf * V;
    rad2(x, y, ir2, Kd * om * ir2, Kd * (2.0 * z * ez - om) * ir2, pxx, pyy, pxy);
    if (qf != 0.0) {
        double E = e1(z);
        p += qf * E * K.i4pk;
        double Kf = qf * K.fe * t;
        double A = z * E + om;
        rad2(x, y, ir2, Kf * A * ir2, Kf * (2.0 * z * E - A) * ir2, pxx, pyy, pxy);
    }
    o[0] = -2.0 * K.G * pyy;
    o[1] = -2.0 * K.G * pxx;
    o[2] = 2.0 * K.G * pxy;
    o[3] = p;
}

// The same response to each source strength alone, added times w into R:
// R[4 s + k] is response k (sxx, syy, sxy, p) to unit s (a, b, V, q_f).
__device__ __forceinline__ void transient_basis(const PoroK &K, double x, double y, double t, double w,
                                                double R[16])
{
    TPoint T;
    tpoint<true>(K, x, y, t, T);
    double ir2 = T.ir2, z = T.z, ez = T.ez, om = T.om;
    double m2g = -2.0 * K.G * w, p2g = 2.0 * K.G * w;
    double pc = K.ap * ir2 * ir2 * T.P2 * w, Cw = K.cphi;
    R[0] += m2g * Cw * T.cyy;
    R[1] += m2g * Cw * T.cxx;
    R[2] += p2g * Cw * T.cxy;
    R[3] += pc * T.gxy;
    R[4] += m2g * Cw * T.syy;
    R[5] += m2g * Cw * T.sxx;
    R[6] += p2g * Cw * T.sxy;
    R[7] += pc * T.g2;
    double dxx = 0.0, dyy = 0.0, dxy = 0.0;
    rad2(x, y, ir2, K.kdf * om * ir2, K.kdf * (2.0 * z * ez - om) * ir2, dxx, dyy, dxy);
    R[8] += m2g * dyy;
    R[9] += m2g * dxx;
    R[10] += p2g * dxy;
    R[11] -= w * K.pv * ez * T.ict;
    double E = e1<true>(z), A = z * E + om, ft = K.fe * t;
    dxx = dyy = dxy = 0.0;
    rad2(x, y, ir2, ft * A * ir2, ft * (2.0 * z * E - A) * ir2, dxx, dyy, dxy);
    R[12] += m2g * dyy;
    R[13] += m2g * dxx;
    R[14] += p2g * dxy;
    R[15] += w * E * K.i4pk;
}

constexpr int QN = 12;  // Gauss-Legendre points per panel
__constant__ double c_gl_t[QN], c_gl_w[QN], c_gl8_t[8], c_gl8_w[8];

// Quadrature of a function along the element (cx, cy, cb, sb, a) seen from
// the receiver (X, Y) at time t: f(x, y, w) for every point, with (x, y)
// the receiver's offset from the point and w the weight per unit length.
// Where the receiver lies for the element's quadrature: xl its coordinate
// along the element, ell the diffusion length; far: beyond 8 x the larger
// of the element's length and ell (one 8-point rule), else the composite
// graded rule on both sides of the foot xl.
struct QuadGeom {
    double xl, ell;
    bool far;
};

__device__ __forceinline__ QuadGeom quad_geom(const PoroK &K, double X, double Y, double cx, double cy, double cb,
                                              double sb, double a, double t)
{
    double dx = X - cx, dy = Y - cy;
    double xl = dx * cb + dy * sb, yl = dy * cb - dx * sb;
    double ell = sqrt(4.0 * K.c * t);
    double far = 8.0 * fmax(2.0 * a, ell);
    double ox = fabs(xl) - a;
    double d2 = yl * yl + (ox > 0.0 ? ox * ox : 0.0);
    return QuadGeom{xl, ell, d2 >= far * far};
}

// panels of the composite rule on side `side` (0: from the foot towards
// -a, 1: towards +a) of the length L it covers
__device__ __forceinline__ int quad_panels(double L, double ell)
{
    return L <= 0.0 ? 0 : min(4 + (int)ceil(2.0 * L / ell), 400);
}

template <class Fn>
__device__ __forceinline__ void elem_quad(const PoroK &K, double X, double Y, double cx, double cy, double cb,
                                          double sb, double a, double t, Fn &&f)
{
    const QuadGeom Q = quad_geom(K, X, Y, cx, cy, cb, sb, a, t);
    const double xl = Q.xl, ell = Q.ell;
    if (Q.far) {
        for (int g = 0; g < 8; ++g) {
            double s = a * c_gl8_t[g];
            f(X - (cx + s * cb), Y - (cy + s * sb), a * c_gl8_w[g]);
        }
        return;
    }
    double s0 = fmin(a, fmax(-a, xl));
    for (int side = 0; side < 2; ++side) {
        double L = side ? a - s0 : s0 + a;
        const int np = quad_panels(L, ell);
        if (np == 0) continue;
        double du = 1.0 / np;
        for (int pn = 0; pn < np; ++pn) {
            for (int g = 0; g < QN; ++g) {
                double u = (pn + 0.5 + 0.5 * c_gl_t[g]) * du;
                double w = 0.5 * du * c_gl_w[g] * 3.0 * L * u * u;
                double s = side ? s0 + L * u * u * u : s0 - L * u * u * u;
                f(X - (cx + s * cb), Y - (cy + s * sb), w);
            }
        }
    }
}

// Element integral of the transient response at time t, added into o:
// element (cx, cy, cb, sb, a) with charges q per unit length and fluid
// source qf, receiver (X, Y).
__device__ void elem_transient(const PoroK &K, double X, double Y, double cx, double cy, double cb, double sb,
                               double a, const double q[3], double qf, double t, double o[4])
{
    elem_quad(K, X, Y, cx, cy, cb, sb, a, t, [&](double x, double y, double w) {
        double r[4];
        transient(K, x, y, t, q, qf, r);
        for (int k = 0; k < 4; ++k) o[k] += w * r[k];
    });
}

__device__ void block_of_unit_responses(const PoroK &K, double cb, double sb, const double R[16], double B[12]);

// The element's 4 x 3 response block at time t: B[3 k + c] is response k
// (sxx, syy, sxy, p) at (X, Y) to unit D_s (c = 0), D_n (1) or D_q (2) on
// the element.  The strengths (a, b, V) of a unit DD are constant along the
// element, so the four unit-strength responses are integrated once and
// combined at the end.
__device__ void elem_block(const PoroK &K, double X, double Y, double cx, double cy, double cb, double sb,
                           double a, double t, double B[12])
{
    double R[16];
    for (int k = 0; k < 16; ++k) R[k] = 0.0;
    elem_quad(K, X, Y, cx, cy, cb, sb, a, t,
              [&](double x, double y, double w) { transient_basis(K, x, y, t, w, R); });
    block_of_unit_responses(K, cb, sb, R, B);
}

// B (4 x 3, per unit D_s, D_n, D_q) from the integrated unit-strength
// responses R (per unit a, b, V, q_f) of an element with direction (cb, sb)
__device__ void block_of_unit_responses(const PoroK &K, double cb, double sb, const double R[16], double B[12])
{
    double sa[2], sbb[2], sv[2];
    for (int c = 0; c < 2; ++c) {
        double q[3];
        charge(cb, sb, c == 0 ? 1.0 : 0.0, c == 1 ? 1.0 : 0.0, q[0], q[1], q[2]);
        sa[c] = 2.0 * K.G * (q[0] - q[1]);
        sbb[c] = 2.0 * K.G * q[2];
        sv[c] = -(q[0] + q[1]) * K.vfac;
    }
    for (int k = 0; k < 4; ++k) {
        B[3 * k] = sa[0] * R[k] + sbb[0] * R[4 + k] + sv[0] * R[8 + k];
        B[3 * k + 1] = sa[1] * R[k] + sbb[1] * R[4 + k] + sv[1] * R[8 + k];
        B[3 * k + 2] = R[12 + k];
    }
}

constexpr int PT = 64;   // receivers per block (one per lane)
constexpr int PS = 64;   // sources per chunk

// part[chunk][3 i + r] = sum over the chunk's sources j and the terms k of
// T(times[k]) applied to E[k][3 j ..], plus the drained elastic part of
// term `drained_term` (if >= 0); r = shear traction, normal traction,
// pressure at receiver i.
__global__ __launch_bounds__(PT) void k_poro_pairs(int n, const double *__restrict__ cx,
                                                   const double *__restrict__ cy, const double *__restrict__ cb,
                                                   const double *__restrict__ sb, const double *__restrict__ ha,
                                                   int nterm, const double *__restrict__ times,
                                                   const double *__restrict__ E, int drained_term, PoroK K,
                                                   double *__restrict__ part)
{
    int i = blockIdx.x * PT + threadIdx.x;
    int chunk = blockIdx.y;
    int j0 = chunk * PS, j1 = min(n, j0 + PS);
    bool live = i < n;
    double X = live ? cx[i] : 0.0, Y = live ? cy[i] : 0.0;
    double o[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = j0; j < j1 && live; ++j) {
        double ecx = cx[j], ecy = cy[j], ecb = cb[j], esb = sb[j], ea = ha[j];
        for (int k = 0; k < nterm; ++k) {
            const double *Ej = E + (size_t)k * 3 * n + 3 * j;
            double Ds = Ej[0], Dn = Ej[1], Dq = Ej[2];
            if (Ds == 0.0 && Dn == 0.0 && Dq == 0.0) continue;
            double q[3];
            charge(ecb, esb, Ds, Dn, q[0], q[1], q[2]);
            elem_transient(K, X, Y, ecx, ecy, ecb, esb, ea, q, Dq, times[k], o);
            if (k == drained_term) elem_stress_add(X, Y, ecx, ecy, ecb, esb, ea, Ds, Dn, K.gc, o[0], o[1], o[2]);
        }
    }
    if (!live) return;
    double ts, tn;
    traction(cb[i], sb[i], o[0], o[1], o[2], ts, tn);
    double *pp = part + (size_t)chunk * 3 * n + 3 * i;
    pp[0] = ts;
    pp[1] = tn;
    pp[2] = o[3];
}

// The left-hand side F(dt) as a dense matrix (history-only variant): row
// 3i + r (shear traction, normal traction, pressure at element i), column
// 3j + c (unit D_s, D_n, D_q on element j), caller order, row-major.  One
// thread per (i, j): the element's transient block by the near-field
// quadrature plus the drained elastic part in closed form.
__global__ __launch_bounds__(256) void k_pdense(int n, const double *__restrict__ cx, const double *__restrict__ cy,
                                                const double *__restrict__ cb, const double *__restrict__ sb,
                                                const double *__restrict__ ha, double dt, PoroK K,
                                                double *__restrict__ A)
{
    const int i = blockIdx.x, j = blockIdx.y * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double X = cx[i], Y = cy[i];
    double B[12];
    elem_block(K, X, Y, cx[j], cy[j], cb[j], sb[j], ha[j], dt, B);
    for (int c = 0; c < 2; ++c) {
        double sxx = 0.0, syy = 0.0, sxy = 0.0;
        elem_stress_add(X, Y, cx[j], cy[j], cb[j], sb[j], ha[j], c == 0 ? 1.0 : 0.0, c == 1 ? 1.0 : 0.0, K.gc, sxx,
                        syy, sxy);
        B[c] += sxx;
        B[3 + c] += syy;
        B[6 + c] += sxy;
    }
    const size_t ld = 3 * (size_t)n;
    double *row = A + 3 * (size_t)i * ld + 3 * (size_t)j;
    for (int c = 0; c < 3; ++c) {
        double ts, tn;
        traction(cb[i], sb[i], B[c], B[3 + c], B[6 + c], ts, tn);
        row[c] = ts;
        row[ld + c] = tn;
        row[2 * ld + c] = B[9 + c];
    }
}

// Block-Jacobi blocks of the left-hand side F(dt): one workgroup per group
// of m <= PPB elements (tree order), A[3i + r][3j + c] = response r (shear
// traction, normal traction, pressure) at element i to a unit unknown c
// (D_s, D_n, D_q) on element j, by the same element integrals as the
// product; inverted in LDS, written column-major at inv + off[b].
constexpr int PPB = GJN / 3;

__global__ __launch_bounds__(256) void k_ppc_build(int nblk, const int *__restrict__ beg,
                                                   const int *__restrict__ cnt, const int64_t *__restrict__ off,
                                                   const double *__restrict__ cx, const double *__restrict__ cy,
                                                   const double *__restrict__ cb, const double *__restrict__ sb,
                                                   const double *__restrict__ ha, double dt, PoroK K,
                                                   double *__restrict__ inv, int *__restrict__ bad)
{
    __shared__ double A[GJN][GJN + 1];
    __shared__ double colk[GJN];
    __shared__ int piv[GJN];
    __shared__ double e_cx[PPB], e_cy[PPB], e_cb[PPB], e_sb[PPB], e_a[PPB];
    int b = blockIdx.x, tid = threadIdx.x;
    int s0 = beg[b], m = cnt[b], nb = 3 * m;
    if (tid < m) {
        e_cx[tid] = cx[s0 + tid]; e_cy[tid] = cy[s0 + tid]; e_cb[tid] = cb[s0 + tid];
        e_sb[tid] = sb[s0 + tid]; e_a[tid] = ha[s0 + tid];
    }
    __syncthreads();
    for (int e = tid; e < 3 * m * m; e += 256) {
        int c = e / (m * m), ij = e - c * m * m, i = ij / m, j = ij - i * m;
        double Ds = c == 0 ? 1.0 : 0.0, Dn = c == 1 ? 1.0 : 0.0, Dq = c == 2 ? 1.0 : 0.0;
        double q[3], o[4] = {0.0, 0.0, 0.0, 0.0};
        charge(e_cb[j], e_sb[j], Ds, Dn, q[0], q[1], q[2]);
        elem_transient(K, e_cx[i], e_cy[i], e_cx[j], e_cy[j], e_cb[j], e_sb[j], e_a[j], q, Dq, dt, o);
        elem_stress_add(e_cx[i], e_cy[i], e_cx[j], e_cy[j], e_cb[j], e_sb[j], e_a[j], Ds, Dn, K.gc, o[0], o[1],
                        o[2]);
        double ts, tn;
        traction(e_cb[i], e_sb[i], o[0], o[1], o[2], ts, tn);
        A[3 * i][3 * j + c] = ts;
        A[3 * i + 1][3 * j + c] = tn;
        A[3 * i + 2][3 * j + c] = o[3];
    }
    __syncthreads();
    gj_invert(A, nb, colk, piv, bad);
    double *o = inv + off[b];
    for (int e = tid; e < nb * nb; e += 256) {
        int c = e / nb, r = e % nb;
        o[e] = A[r][c];
    }
}

// The same blocks taken from the left-hand side's stored near blocks (blk:
// 12 entries per near pair, the drained part included, in the layout of
// k_pnear_build) instead of integrating them again: a group lies in one
// leaf, whose near sources include the leaf itself, so the pair (i, j) is
// source pos_j of leaf li, in the item whose chunk holds pos_j.  A pair not
// found there is integrated as in k_ppc_build.
__global__ __launch_bounds__(256) void k_ppc_gather(
    int nblk, const int *__restrict__ beg, const int *__restrict__ cnt, const int64_t *__restrict__ off,
    const int *__restrict__ tleaf, const int *__restrict__ leaves, const int *__restrict__ pbeg,
    const int *__restrict__ pend, const int *__restrict__ lk_off, const int *__restrict__ it_s0,
    const int *__restrict__ it_s1, const int64_t *__restrict__ it_coff, const int *__restrict__ nfoff,
    const int *__restrict__ nflat, const double *__restrict__ blk, const double *__restrict__ cx,
    const double *__restrict__ cy, const double *__restrict__ cb, const double *__restrict__ sb,
    const double *__restrict__ ha, double dt, PoroK K, double *__restrict__ inv, int *__restrict__ bad)
{
    __shared__ double A[GJN][GJN + 1];
    __shared__ double colk[GJN];
    __shared__ int piv[GJN];
    __shared__ int s_item[PPB], s_v[PPB];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int s0 = beg[b], m = cnt[b], nb = 3 * m;
    const int li = tleaf[s0], c = leaves[li], tb = pbeg[c], nt = pend[c] - tb;
    if (tid < m) {
        // source s0 + tid in the leaf's near list, and its item and slot
        const int j = s0 + tid, f0 = nfoff[li], len = nfoff[li + 1] - f0;
        int pos = -1;
        for (int u = 0; u < len && pos < 0; ++u)
            if (nflat[f0 + u] == j) pos = u;
        int item = -1, v = 0;
        if (pos >= 0)
            for (int k = lk_off[li]; k < lk_off[li + 1]; ++k)
                if (it_s0[k] <= pos && pos < it_s1[k]) {
                    item = k;
                    v = pos - it_s0[k];
                    break;
                }
        s_item[tid] = item;
        s_v[tid] = v;
    }
    __syncthreads();
    for (int e = tid; e < m * m; e += 256) {
        const int i = e / m, j = e - i * m, ti = s0 + i, tj = s0 + j;
        double B[12];
        const int item = s_item[j];
        if (item >= 0 && tleaf[ti] == li) {
            const double *q = blk + 12 * it_coff[item] + (int64_t)12 * s_v[j] * nt + (ti - tb);
#pragma unroll
            for (int r = 0; r < 12; ++r) B[r] = q[(int64_t)r * nt];
        } else {
            elem_block(K, cx[ti], cy[ti], cx[tj], cy[tj], cb[tj], sb[tj], ha[tj], dt, B);
            for (int cc = 0; cc < 2; ++cc) {
                double sxx = 0.0, syy = 0.0, sxy = 0.0;
                elem_stress_add(cx[ti], cy[ti], cx[tj], cy[tj], cb[tj], sb[tj], ha[tj], cc == 0 ? 1.0 : 0.0,
                                cc == 1 ? 1.0 : 0.0, K.gc, sxx, syy, sxy);
                B[cc] += sxx;
                B[3 + cc] += syy;
                B[6 + cc] += sxy;
            }
        }
        for (int cc = 0; cc < 3; ++cc) {
            double ts, tn;
            traction(cb[ti], sb[ti], B[cc], B[3 + cc], B[6 + cc], ts, tn);
            A[3 * i][3 * j + cc] = ts;
            A[3 * i + 1][3 * j + cc] = tn;
            A[3 * i + 2][3 * j + cc] = B[9 + cc];
        }
    }
    __syncthreads();
    gj_invert(A, nb, colk, piv, bad);
    double *o = inv + off[b];
    for (int e = tid; e < nb * nb; e += 256) {
        int cc = e / nb, r = e % nb;
        o[e] = A[r][cc];
    }
}

__global__ void k_scale_copy(int m, double a, const double *__restrict__ x, double *__restrict__ y)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) y[e] = a * x[e];
}

// y = 0 (a buffer from the cache may hold any bit pattern, NaN included,
// which a product with zero would keep)
__global__ void k_zero(int64_t m, double *__restrict__ y)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) y[e] = 0.0;
}

// out[e] (mode 0: =, mode 1: -=) sum of the chunk partials, in chunk order.
__global__ void k_poro_reduce(int m3, int nchunk, const double *__restrict__ part, int mode,
                              double *__restrict__ out)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m3) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[(size_t)c * m3 + e];
    out[e] = mode ? out[e] - s : s;
}

// History terms: E[0] = -D^{h-1} at t = dt, E[j-1] = D^{h-j+1} - D^{h-j} at
// t = j dt (2 <= j <= h-1), E[h-1] = D^1 at t = h dt.  Dh holds D^1..D^{h-1}.
__global__ void k_hist_terms(int m3, int h, const double *__restrict__ Dh, double *__restrict__ E)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y + 1;  // 1..h
    if (e >= m3) return;
    double v;
    if (j == 1) v = -Dh[(size_t)(h - 2) * m3 + e];
    else if (j == h) v = Dh[e];
    else v = Dh[(size_t)(h - j) * m3 + e] - Dh[(size_t)(h - j - 1) * m3 + e];
    E[(size_t)(j - 1) * m3 + e] = v;
}

__global__ void k_poro_rhs(int n, const double *__restrict__ cb, const double *__restrict__ sb,
                           const double *__restrict__ pf, double p0, double SH, double Sh,
                           double *__restrict__ rhs)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double ts, tn;
    traction(cb[i], sb[i], -SH, -Sh, 0.0, ts, tn);
    rhs[3 * i] = -ts;
    rhs[3 * i + 1] = -pf[i] - tn;
    rhs[3 * i + 2] = pf[i] - p0;
}

// ------------------------------------------------ multipole form (FMM)
// Far field of well-separated cells by the black-box FMM of Section 3 with
// the transient kernel: four charges per node (q0, q1, q2, q_f) and four
// responses (sxx, syy, sxy, p).  The kernel is not homogeneous, so the M2L
// operators are formed per (tree level, offset) and per time level; the
// operators of all time levels of a (level, offset) are stored side by
// side, so one product contracts over the time levels and the interaction
// list together (the weights of a cell for all time levels are contiguous).

// operator entry block: target node tn, source node sn, time level j of
// combo c; rows (component_out, tn), columns (j, component_in, sn)
__global__ void k_pops(int ncombo, const int *__restrict__ clvl, const int *__restrict__ cox,
                       const int *__restrict__ coy, double rootL, const double *__restrict__ xbar, int p, int H,
                       double dt, int Mq, PoroK K, int drained, double *__restrict__ ops)
{
    int p2 = p * p;
    int64_t per = (int64_t)p2 * p2 * H;
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= per * ncombo) return;
    int c = (int)(g / per);
    int64_t r = g - (int64_t)c * per;
    int j = (int)(r / ((int64_t)p2 * p2));
    int rr = (int)(r - (int64_t)j * p2 * p2);
    int tn = rr / p2, sn = rr - tn * p2;
    double hw = rootL / (double)(2LL << clvl[c]);  // half-width of a cell of that level
    double X = hw * xbar[tn / p], Y = hw * xbar[tn % p];
    double sx = hw * (2.0 * cox[c] + xbar[sn / p]), sy = hw * (2.0 * coy[c] + xbar[sn % p]);
    double t = (j + 1) * dt;
    const size_t ld = (size_t)H * Mq;
    double *op = ops + (size_t)c * Mq * ld;
    double Kd[9];  // drained elastic point kernel (left-hand-side operators only)
    if (drained) point_kernel(X - sx, Y - sy, K.gc, Kd);
    for (int ci = 0; ci < 4; ++ci) {
        double q[3] = {ci == 0 ? 1.0 : 0.0, ci == 1 ? 1.0 : 0.0, ci == 2 ? 1.0 : 0.0};
        double o[4];
        transient(K, X - sx, Y - sy, t, q, ci == 3 ? 1.0 : 0.0, o);
        if (drained && ci < 3)
            for (int co = 0; co < 3; ++co) o[co] += Kd[co * 3 + ci];
        for (int co = 0; co < 4; ++co) op[(size_t)(co * p2 + tn) * ld + (size_t)j * Mq + ci * p2 + sn] = o[co];
    }
}

// Compressed left-hand-side M2L.  For the combinations o of one tree level
// (operators K_o, m x m with m = 4 p^2, stored row-major with leading
// dimension Mq), side 0 packs [K_o1 | K_o2 | ...] and side 1 [K_o1^T |
// K_o2^T | ...], m x (n m) column-major: the left singular vectors of the
// first span the operators' column space, of the second their row space.
__global__ void k_pc_pack(int nc, const int *__restrict__ combos, int m, int Mq, int side,
                          const double *__restrict__ ops, double *__restrict__ fat)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)m * nc * m) return;
    int col = (int)(e / m), i = (int)(e - (int64_t)col * m);
    int o = col / m, j = col - o * m;
    const double *K = ops + (size_t)combos[o] * Mq * Mq;
    fat[e] = side == 0 ? K[(size_t)i * Mq + j] : K[(size_t)j * Mq + i];
}

// Bases of level slot k from the left singular vectors (column-major m x m)
// of its column space (Uc) and row space (Ur), rank[k] columns kept:
// Vt (rq x Mq) and UT (rq x Mq) hold the vectors as rows, U (Mq x rq) the
// column-space vectors as columns; the padding is zero.
__global__ void k_pc_bases(int nlev, int m, int Mq, int rq, const int *__restrict__ rank,
                           const double *__restrict__ Uc, const double *__restrict__ Ur, double *__restrict__ Vt,
                           double *__restrict__ UT, double *__restrict__ U)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nlev * rq * Mq) return;
    int k = (int)(e / ((int64_t)rq * Mq));
    int r = (int)(e - (int64_t)k * rq * Mq);
    int a = r / Mq, i = r - a * Mq;
    bool in = a < rank[k] && i < m;
    const size_t mm = (size_t)m * m;
    double vr = in ? Ur[k * mm + (size_t)a * m + i] : 0.0;
    double vc = in ? Uc[k * mm + (size_t)a * m + i] : 0.0;
    Vt[e] = vr;
    UT[e] = vc;
    U[((size_t)k * Mq + i) * rq + a] = vc;
}

// C_o[b][a] = Ct[o rq + a][b] (row-major rq x rq per combination)
__global__ void k_pc_transpose(int nc, int rq, const double *__restrict__ Ct, double *__restrict__ C)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nc * rq * rq) return;
    int o = (int)(e / ((int64_t)rq * rq));
    int r = (int)(e - (int64_t)o * rq * rq);
    int b = r / rq, a = r - b * rq;
    C[e] = Ct[((size_t)o * rq + a) * rq + b];
}

// charges per element (tree order) and term: Q[(j n + i) 4 + c], and the
// DDs in tree order D3[(j n + i) 3 + c]
__global__ void k_pprep(int n, int H, const int *__restrict__ perm, const double *__restrict__ E,
                        const double *__restrict__ cb, const double *__restrict__ sb, double *__restrict__ Q,
                        double *__restrict__ D3)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    if (i >= n) return;
    const double *e = E + (size_t)j * 3 * n + 3 * (size_t)perm[i];
    double q0, q1, q2;
    charge(cb[i], sb[i], e[0], e[1], q0, q1, q2);
    double *qq = Q + ((size_t)j * n + i) * 4;
    qq[0] = q0;
    qq[1] = q1;
    qq[2] = q2;
    qq[3] = e[2];
    double *d = D3 + ((size_t)j * n + i) * 3;
    d[0] = e[0];
    d[1] = e[1];
    d[2] = e[2];
}

// The far field of a history sum in two terms.  Where every V-list pair is
// far outside the diffusion length (z = r^2 / (4 c t) >= 50 at the last
// time level), the transient kernel is affine in t to double precision:
// h(z) = 1 - 1/z, P(2, z) = 1 and z E1(z) + 1 - e^-z = 1 up to e^-z terms,
// so F(t) = A + t B.  Then sum_j F(j dt) E_j = F(dt) sum_j (2 - j) E_j
// + F(2 dt) sum_j (j - 1) E_j: two multipole terms with the operators of
// the first two time levels, whatever the number of levels.  Q2 gets the
// two combined charges [(m n + i) 4 + c], D3 the DDs of every level (the
// near field stays exact per level).
__global__ void k_pprep_affine(int n, int H, const int *__restrict__ perm, const double *__restrict__ E,
                               const double *__restrict__ cb, const double *__restrict__ sb,
                               double *__restrict__ Q2, double *__restrict__ D3)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a[4] = {0.0, 0.0, 0.0, 0.0}, b[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = 0; j < H; ++j) {  // time level j + 1
        const double *e = E + (size_t)j * 3 * n + 3 * (size_t)perm[i];
        double q0, q1, q2;
        charge(cb[i], sb[i], e[0], e[1], q0, q1, q2);
        const double wa = (double)(1 - j), wb = (double)j;
        a[0] += wa * q0;
        a[1] += wa * q1;
        a[2] += wa * q2;
        a[3] += wa * e[2];
        b[0] += wb * q0;
        b[1] += wb * q1;
        b[2] += wb * q2;
        b[3] += wb * e[2];
        double *d = D3 + ((size_t)j * n + i) * 3;
        d[0] = e[0];
        d[1] = e[1];
        d[2] = e[2];
    }
    for (int c = 0; c < 4; ++c) {
        Q2[(size_t)i * 4 + c] = a[c];
        Q2[((size_t)n + i) * 4 + c] = b[c];
    }
}

// leaf weights per term (eq. 3.6): W[(leaf H + j) Mq + c p^2 + t]
__global__ __launch_bounds__(256) void k_pp2m(int nleaf, const int *__restrict__ leaves,
                                              const int *__restrict__ pbeg, const int *__restrict__ pend,
                                              const double *__restrict__ Pm, const double *__restrict__ Q, int n,
                                              int p2, int H, int Mq, double *__restrict__ W)
{
    int c = leaves[blockIdx.x];
    int j = blockIdx.y;
    int b = pbeg[c], e = pend[c];
    const double *Qj = Q + (size_t)j * n * 4;
    double *Wc = W + ((size_t)c * H + j) * Mq;
    for (int t = threadIdx.x; t < p2; t += 256) {
        double w0 = 0.0, w1 = 0.0, w2 = 0.0, w3 = 0.0;
        for (int i = b; i < e; ++i) {
            double m = Pm[(size_t)i * p2 + t];
            w0 += Qj[4 * i] * m;
            w1 += Qj[4 * i + 1] * m;
            w2 += Qj[4 * i + 2] * m;
            w3 += Qj[4 * i + 3] * m;
        }
        Wc[t] = w0;
        Wc[p2 + t] = w1;
        Wc[2 * p2 + t] = w2;
        Wc[3 * p2 + t] = w3;
    }
}

// Near field per work item (a leaf and a chunk of its near sources, as in
// the elastic product): exact transient element integrals for every term;
// partial (sxx, syy, sxy, p) per target point of the item.
constexpr int PN = 128;
__global__ __launch_bounds__(PN) void k_pp2p(int nitem, const int *__restrict__ it_leaf,
                                             const int *__restrict__ it_s0, const int *__restrict__ it_s1,
                                             const int *__restrict__ it_poff, const int *__restrict__ leaves,
                                             const int *__restrict__ pbeg, const int *__restrict__ pend,
                                             const int *__restrict__ noff, const int *__restrict__ nbeg,
                                             const int *__restrict__ npre, const double *__restrict__ cx,
                                             const double *__restrict__ cy, const double *__restrict__ cb,
                                             const double *__restrict__ sb, const double *__restrict__ a, int n,
                                             int j0, int H, double dt, const double *__restrict__ D3, PoroK K,
                                             int acc, double *__restrict__ part)
{
    int k = blockIdx.x;
    int li = it_leaf[k], s0 = it_s0[k], s1 = it_s1[k];
    int c = leaves[li];
    int tb = pbeg[c], te = pend[c], nt = te - tb;
    int nb = noff[li], nn = noff[li + 1] - nb;
    // tpt adjacent lanes per target point take every tpt-th source and
    // combine by a fixed butterfly
    int tpt = 1;
    while (tpt < 16 && tpt * 2 * nt <= PN) tpt *= 2;
    int tpg = PN / tpt, sub = threadIdx.x & (tpt - 1);
    double *pk = part + 4 * (size_t)it_poff[k];
    for (int t0 = tb; t0 < te; t0 += tpg) {
        int i = t0 + (int)threadIdx.x / tpt;
        bool act = i < te;
        double X = act ? cx[i] : 0.0, Y = act ? cy[i] : 0.0;
        double o[4] = {0.0, 0.0, 0.0, 0.0};
        if (act) {
            int lo = 0;
            for (int v = s0 + sub; v < s1; v += tpt) {
                while (lo + 1 < nn && npre[nb + lo + 1] <= v) ++lo;  // v ascends
                int jsrc = nbeg[nb + lo] + (v - npre[nb + lo]);
                double ecx = cx[jsrc], ecy = cy[jsrc], ecb = cb[jsrc], esb = sb[jsrc], ea = a[jsrc];
                for (int j = j0; j < H; ++j) {
                    const double *d = D3 + ((size_t)j * n + jsrc) * 3;
                    if (d[0] == 0.0 && d[1] == 0.0 && d[2] == 0.0) continue;
                    double q[3];
                    charge(ecb, esb, d[0], d[1], q[0], q[1], q[2]);
                    elem_transient(K, X, Y, ecx, ecy, ecb, esb, ea, q, d[2], (j + 1) * dt, o);
                }
            }
        }
        for (int w = 1; w < tpt; w <<= 1)
            for (int cc = 0; cc < 4; ++cc) o[cc] += __shfl_xor(o[cc], w);
        if (act && sub == 0) {
            double *pp = pk + 4 * (size_t)(i - tb);
            for (int cc = 0; cc < 4; ++cc) pp[cc] = acc ? pp[cc] + o[cc] : o[cc];
        }
    }
}

// Near pair g: item k (it_coff[k] <= g < it_coff[k+1]), target i of the
// item's leaf (points tb .. tb + nt - 1), source v of the item's chunk,
// the source's point jsrc.
struct NearPair {
    int k, tb, nt, i, v, jsrc;
};

__device__ __forceinline__ NearPair near_pair(int64_t g, int nitem, const int64_t *__restrict__ it_coff,
                                              const int *__restrict__ it_leaf, const int *__restrict__ it_s0,
                                              const int *__restrict__ leaves, const int *__restrict__ pbeg,
                                              const int *__restrict__ pend, const int *__restrict__ nfoff,
                                              const int *__restrict__ nflat)
{
    int lo = 0, hi = nitem - 1;  // last item with it_coff <= g
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (it_coff[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    NearPair P;
    P.k = lo;
    const int li = it_leaf[lo], c = leaves[li];
    P.tb = pbeg[c];
    P.nt = pend[c] - P.tb;
    const int64_t e = g - it_coff[lo];
    P.v = (int)(e / P.nt);
    P.i = (int)(e - (int64_t)P.v * P.nt);
    P.jsrc = nflat[nfoff[li] + it_s0[lo] + P.v];
    return P;
}

// the block B of pair P (plus the drained elastic response in closed form)
// into its place: 12 it_coff[k] + (12 v + q) nt + i for entry q
__device__ __forceinline__ void store_block(const PoroK &K, const NearPair &P, const int64_t *__restrict__ it_coff,
                                            const double *__restrict__ cx, const double *__restrict__ cy,
                                            const double *__restrict__ cb, const double *__restrict__ sb,
                                            const double *__restrict__ a, int drained, double B[12],
                                            double *__restrict__ blk)
{
    const int tgt = P.tb + P.i, j = P.jsrc;
    if (drained)
        for (int c = 0; c < 2; ++c) {
            double sxx = 0.0, syy = 0.0, sxy = 0.0;
            elem_stress_add(cx[tgt], cy[tgt], cx[j], cy[j], cb[j], sb[j], a[j], c == 0 ? 1.0 : 0.0,
                            c == 1 ? 1.0 : 0.0, K.gc, sxx, syy, sxy);
            B[c] += sxx;
            B[3 + c] += syy;
            B[6 + c] += sxy;
        }
    double *o = blk + 12 * it_coff[P.k] + (int64_t)12 * P.v * P.nt + P.i;
    for (int q = 0; q < 12; ++q) o[(int64_t)q * P.nt] = B[q];
}

// Near-field blocks of time level (t = (j+1) dt) for every near pair, one
// thread per pair: pair g lies in item k with it_coff[k] <= g <
// it_coff[k+1]; within the item, pair e = v nt + i (source v of the chunk,
// target i of the leaf) stores its 12 entries at 12 it_coff[k] + (12 v + c)
// nt + i, so that consecutive targets are adjacent for every entry c.
// With near_list, pairs whose receiver is within the composite rule's
// reach (up to 800 points against 8) are listed there instead, for
// k_pnear_build_close: one of them in a lane would hold its whole wave.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_pnear_build(
    int64_t npair, int nitem, const int64_t *__restrict__ it_coff, const int *__restrict__ it_leaf,
    const int *__restrict__ it_s0, const int *__restrict__ leaves, const int *__restrict__ pbeg,
    const int *__restrict__ pend, const int *__restrict__ nfoff, const int *__restrict__ nflat,
    const double *__restrict__ cx, const double *__restrict__ cy, const double *__restrict__ cb,
    const double *__restrict__ sb, const double *__restrict__ a, double t, PoroK K, int drained,
    double *__restrict__ blk, int64_t *__restrict__ near_list, unsigned long long *__restrict__ near_count)
{
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= npair) return;
    const NearPair P = near_pair(g, nitem, it_coff, it_leaf, it_s0, leaves, pbeg, pend, nfoff, nflat);
    const int tgt = P.tb + P.i, j = P.jsrc;
    if (near_list && !quad_geom(K, cx[tgt], cy[tgt], cx[j], cy[j], cb[j], sb[j], a[j], t).far) {
        near_list[atomicAdd(near_count, 1ull)] = g;
        return;
    }
    double B[12];
    elem_block(K, cx[tgt], cy[tgt], cx[j], cy[j], cb[j], sb[j], a[j], t, B);
    store_block(K, P, it_coff, cx, cy, cb, sb, a, drained, B, blk);
}

// The listed close pairs, one wave each (a fixed grid of waves takes the
// list in turn): the 64 lanes split the composite rule's points, and the
// 16 unit-strength responses are summed across the wave by a fixed
// butterfly, so a pair's block does not depend on the list's order.
__global__ __launch_bounds__(256) void k_pnear_build_close(
    const int64_t *__restrict__ near_list, const unsigned long long *__restrict__ near_count, int nitem,
    const int64_t *__restrict__ it_coff, const int *__restrict__ it_leaf, const int *__restrict__ it_s0,
    const int *__restrict__ leaves, const int *__restrict__ pbeg, const int *__restrict__ pend,
    const int *__restrict__ nfoff, const int *__restrict__ nflat, const double *__restrict__ cx,
    const double *__restrict__ cy, const double *__restrict__ cb, const double *__restrict__ sb,
    const double *__restrict__ ha, double t, PoroK K, int drained, double *__restrict__ blk)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t cnt = (int64_t)*near_count;
    for (int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w < cnt; w += nw) {
        const NearPair P = near_pair(near_list[w], nitem, it_coff, it_leaf, it_s0, leaves, pbeg, pend, nfoff, nflat);
        const int tgt = P.tb + P.i, j = P.jsrc;
        const double X = cx[tgt], Y = cy[tgt], ecx = cx[j], ecy = cy[j], ecb = cb[j], esb = sb[j], a = ha[j];
        const QuadGeom Q = quad_geom(K, X, Y, ecx, ecy, ecb, esb, a, t);
        const double s0 = fmin(a, fmax(-a, Q.xl));
        const double L0 = s0 + a, L1 = a - s0;
        const int np0 = quad_panels(L0, Q.ell), np1 = quad_panels(L1, Q.ell);
        const int n0 = QN * np0, total = n0 + QN * np1;
        double R[16];
        for (int q = 0; q < 16; ++q) R[q] = 0.0;
        for (int idx = lane; idx < total; idx += 64) {
            const int side = idx >= n0;
            const int loc = side ? idx - n0 : idx, pn = loc / QN, gq = loc - pn * QN;
            const double L = side ? L1 : L0, du = 1.0 / (side ? np1 : np0);
            const double u = (pn + 0.5 + 0.5 * c_gl_t[gq]) * du;
            const double wq = 0.5 * du * c_gl_w[gq] * 3.0 * L * u * u;
            const double sq = side ? s0 + L * u * u * u : s0 - L * u * u * u;
            transient_basis(K, X - (ecx + sq * ecb), Y - (ecy + sq * esb), t, wq, R);
        }
        for (int m = 32; m >= 1; m >>= 1)
            for (int q = 0; q < 16; ++q) R[q] += __shfl_xor(R[q], m);
        if (lane == 0) {
            double B[12];
            block_of_unit_responses(K, ecb, esb, R, B);
            store_block(K, P, it_coff, cx, cy, cb, sb, ha, drained, B, blk);
        }
    }
}

// Near field from the stored blocks of time levels j0 .. j1-1 (lv[j] the
// level's blocks): partial (sxx, syy, sxy, p) per target point of every
// item, in the layout of k_pp2p, which adds the levels beyond the store.
// A stream of 96 bytes per pair and level: 256 lanes per item, tpt =
// 256 / (leaf points) lanes per point (all lanes busy for any leaf size,
// two sources' coefficients in flight per lane), sources from the
// flattened per-leaf list; a point's tpt partials (one per source slice)
// are summed in LDS in slice order.
constexpr int PNB = 256;
__global__ __launch_bounds__(PNB) void k_pnear(int nitem, const int *__restrict__ it_leaf,
                                               const int *__restrict__ it_s0, const int *__restrict__ it_s1,
                                               const int *__restrict__ it_poff, const int64_t *__restrict__ it_coff,
                                               const int *__restrict__ leaves, const int *__restrict__ pbeg,
                                               const int *__restrict__ pend, const int *__restrict__ nfoff,
                                               const int *__restrict__ nflat, int n, int j0, int j1,
                                               const double *const *__restrict__ lv, const double *__restrict__ D3,
                                               double *__restrict__ part)
{
    __shared__ double s_red[4 * PNB];
    const int k = blockIdx.x, tid = threadIdx.x;
    const int li = it_leaf[k], s0 = it_s0[k], ns = it_s1[k] - s0;
    const int c = leaves[li];
    const int nt = pend[c] - pbeg[c];
    const int *src = nflat + nfoff[li] + s0;
    // lane tid takes target g = tid % tpg and source slice sub = tid / tpg,
    // so the lanes of one slice read consecutive targets' entries
    const int tpt = nt >= PNB ? 1 : min(16, PNB / nt);
    const int tpg = PNB / tpt, g = tid % tpg, sub = tid / tpg;
    const int64_t base = 12 * it_coff[k];
    double *pk = part + 4 * (size_t)it_poff[k];
    for (int t0 = 0; t0 < nt; t0 += tpg) {
        const int i = t0 + g;
        const bool act = sub < tpt && i < nt;
        double o[4] = {0.0, 0.0, 0.0, 0.0};
        if (act) {
#pragma unroll 2
            for (int v = sub; v < ns; v += tpt) {
                const int jsrc = src[v];
                const int64_t off = base + (int64_t)12 * v * nt + i;
                for (int j = j0; j < j1; ++j) {
                    const double *d = D3 + ((size_t)j * n + jsrc) * 3;
                    const double d0 = d[0], d1 = d[1], d2 = d[2];
                    const double *bq = lv[j] + off;
#pragma unroll
                    for (int cc = 0; cc < 4; ++cc)
                        o[cc] += bq[(3 * cc) * nt] * d0 + bq[(3 * cc + 1) * nt] * d1 + bq[(3 * cc + 2) * nt] * d2;
                }
            }
        }
        if (tpt == 1) {
            if (act)
                for (int cc = 0; cc < 4; ++cc) pk[4 * (size_t)i + cc] = o[cc];
            continue;
        }
        for (int cc = 0; cc < 4; ++cc) s_red[cc * PNB + tid] = o[cc];
        __syncthreads();
        if (act && sub == 0)
            for (int cc = 0; cc < 4; ++cc) {
                double r = 0.0;
                for (int u = 0; u < tpt; ++u) r += s_red[cc * PNB + u * tpg + g];
                pk[4 * (size_t)i + cc] = r;
            }
        __syncthreads();
    }
}

// far + near (in item order) -> (shear, normal traction, pressure), caller
// order; mode 0: =, 1: -=; o2 (if given): drained elastic tractions added
__global__ void k_pfinal(int n, const int *__restrict__ tleaf, const int *__restrict__ leaves,
                         const int *__restrict__ pbeg, const int *__restrict__ level,
                         const int *__restrict__ lk_off, const int *__restrict__ it_poff,
                         const double *__restrict__ part, const double *__restrict__ far,
                         const double *__restrict__ cb, const double *__restrict__ sb,
                         const int *__restrict__ perm, const double *__restrict__ o2, int mode,
                         double *__restrict__ out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int li = tleaf[i];
    int cl = leaves[li];
    int t = i - pbeg[cl];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    if (far)  // the point's cells at levels 2 .. its leaf's, in level order
        for (int l = 2; l <= level[cl]; ++l)
            for (int c = 0; c < 4; ++c) s[c] += far[((size_t)(l - 2) * n + i) * 4 + c];
    for (int k = lk_off[li]; k < lk_off[li + 1]; ++k) {
        const double *o = part + 4 * ((size_t)it_poff[k] + t);
        for (int c = 0; c < 4; ++c) s[c] += o[c];
    }
    double ts, tn;
    traction(cb[i], sb[i], s[0], s[1], s[2], ts, tn);
    int j = perm[i];
    if (o2) {
        ts += o2[2 * j];
        tn += o2[2 * j + 1];
    }
    double *y = out + 3 * (size_t)j;
    if (mode) {
        y[0] -= ts;
        y[1] -= tn;
        y[2] -= s[3];
    } else {
        y[0] = ts;
        y[1] = tn;
        y[2] = s[3];
    }
}

__global__ void k_take2(int n, const double *__restrict__ E, double *__restrict__ D2)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    D2[2 * i] = E[3 * i];
    D2[2 * i + 1] = E[3 * i + 1];
}

// quadrature rules and series coefficients in constant memory, uploaded
// once per device (serving set-ups may ask from several host threads)
std::atomic<bool> g_gl_ready[64];
std::mutex g_gl_mu;

void upload_rules(int device)
{
    if (device >= 0 && device < 64 && g_gl_ready[device].load(std::memory_order_acquire)) return;
    std::lock_guard<std::mutex> lock(g_gl_mu);
    if (device >= 0 && device < 64 && g_gl_ready[device].load(std::memory_order_acquire)) return;
    std::vector<double> t, w, t8, w8;
    gauss_legendre(QN, t, w);
    gauss_legendre(8, t8, w8);
    FM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_gl_t), t.data(), QN * 8));
    FM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_gl_w), w.data(), QN * 8));
    FM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_gl8_t), t8.data(), 64));
    FM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_gl8_w), w8.data(), 64));
    double e1w[31] = {0.0}, hc[23] = {0.0}, p2c[18] = {0.0};
    for (int k = 1; k <= 30; ++k) e1w[k] = k / ((k + 1.0) * (k + 1.0));
    double fact = 1.0;  // (k+1)!
    for (int k = 1; k <= 22; ++k) {
        fact *= (k + 1);
        hc[k] = ((k & 1) ? 1.0 : -1.0) / fact;
    }
    fact = 1.0;  // k!
    for (int k = 1; k <= 17; ++k) {
        fact *= k;
        if (k >= 2) p2c[k] = ((k & 1) ? -1.0 : 1.0) * (k - 1) / fact;
    }
    FM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_e1w), e1w, sizeof(e1w)));
    FM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_hc), hc, sizeof(hc)));
    FM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_p2c), p2c, sizeof(p2c)));
    if (device >= 0 && device < 64) g_gl_ready[device].store(true, std::memory_order_release);
}

PoroK poro_constants(const fmddm_ctx *ctx)
{
    const fmddm_params &p = ctx->prm;
    const fmddm_poro_params &q = ctx->poro;
    double G = p.E / (2.0 * (1.0 + p.nu));
    double M = 2.0 * G * (q.nu_u - p.nu) / (q.alpha * q.alpha * (1.0 - 2.0 * q.nu_u) * (1.0 - 2.0 * p.nu));
    double eta = q.alpha * (1.0 - 2.0 * p.nu) / (2.0 * G * (1.0 - p.nu));
    double S = 1.0 / M + q.alpha * eta;
    double kap = q.perm / q.visc;
    PoroK K{G, p.nu, q.alpha, kap, S, kap / S, eta, ctx->gc};
    double kd = (1.0 - 2.0 * p.nu) / (4.0 * M_PI * G * (1.0 - p.nu));
    K.vfac = (1.0 - 2.0 * p.nu) / (2.0 * (1.0 - p.nu));
    K.ap = q.alpha * kd / S;
    K.pv = q.alpha / (4.0 * M_PI * S);
    K.cphi = q.alpha * kd * eta / S;
    K.kdf = -q.alpha * eta / (2.0 * M_PI * S);
    K.i4pk = 1.0 / (4.0 * M_PI * kap);
    K.fe = eta / (2.0 * M_PI * S);
    return K;
}

// sum over terms, into out (mode 0) or subtracted from out (mode 1)
void poro_sum(fmddm_ctx *ctx, fmddm_tree *t, int nterm, const std::vector<double> &times, const double *E,
              int drained_term, int mode, double *out)
{
    if (!ctx->poro_set) throw Error{FMDDM_EINVAL, "poroelastic parameters not set (fmddm_poro_set)"};
    hipStream_t s = ctx->stream;
    upload_rules(ctx->device);
    const int n = (int)t->n, m3 = 3 * n;
    const int nchunk = cdiv(n, PS);
    if (t->poro_part.n < (size_t)nchunk * m3) t->poro_part.alloc((size_t)nchunk * m3);
    if (t->poro_times.n < (size_t)nterm) t->poro_times.alloc(nterm);
    FM_HIP(hipMemcpyAsync(t->poro_times.p, times.data(), nterm * 8, hipMemcpyHostToDevice, s));
    PoroK K = poro_constants(ctx);
    hipLaunchKernelGGL(k_poro_pairs, dim3(cdiv(n, PT), nchunk), dim3(PT), 0, s, n, t->ocx.p, t->ocy.p, t->ocb.p,
                       t->osb.p, t->oa.p, nterm, t->poro_times.p, E, drained_term, K, t->poro_part.p);
    FM_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_poro_reduce, dim3(cdiv(m3, 256)), dim3(256), 0, s, m3, nchunk, t->poro_part.p, mode, out);
    FM_CHECK_LAUNCH();
}

// Everything a transient kernel value depends on besides the geometry.
void medium_key(const fmddm_ctx *ctx, double k[8])
{
    const fmddm_poro_params &q = ctx->poro;
    k[0] = q.nu_u;
    k[1] = q.alpha;
    k[2] = q.perm;
    k[3] = q.visc;
    k[4] = q.dt;
    k[5] = ctx->prm.E;
    k[6] = ctx->prm.nu;
    k[7] = (double)q.near_cache_bytes;
}

bool same_key(const double a[8], const double b[8], int nk)
{
    for (int k = 0; k < nk; ++k)
        if (a[k] != b[k]) return false;
    return true;
}

// One time level's near blocks (at time t, with the drained part when
// drained): far pairs one per thread, close pairs one per wave.
void build_near_blocks(fmddm_ctx *ctx, fmddm_tree *t, double time, const PoroK &K, int drained, double *out)
{
    if (t->near_pairs == 0) return;
    hipStream_t s = ctx->stream;
    if (t->pn_close.n < (size_t)t->near_pairs) t->pn_close.alloc((size_t)t->near_pairs);
    if (t->pn_ccount.n < 1) t->pn_ccount.alloc(1);
    t->pn_ccount.zero(s);
    hipLaunchKernelGGL(k_pnear_build, dim3(cdiv(t->near_pairs, 256)), dim3(256), 0, s, t->near_pairs, t->nitem,
                       t->it_coff.p, t->it_leaf.p, t->it_s0.p, t->dleaves.p, t->cpbeg.p, t->cpend.p, t->nfoff.p,
                       t->nflat.p, t->scx.p, t->scy.p, t->scb.p, t->ssb.p, t->sa.p, time, K, drained, out,
                       t->pn_close.p, t->pn_ccount.p);
    FM_CHECK_LAUNCH();
    const int nblk = (int)std::min<int64_t>(cdiv(t->near_pairs, 4), 2048);
    hipLaunchKernelGGL(k_pnear_build_close, dim3(nblk), dim3(256), 0, s, t->pn_close.p, t->pn_ccount.p, t->nitem,
                       t->it_coff.p, t->it_leaf.p, t->it_s0.p, t->dleaves.p, t->cpbeg.p, t->cpend.p, t->nfoff.p,
                       t->nflat.p, t->scx.p, t->scy.p, t->scb.p, t->ssb.p, t->sa.p, time, K, drained, out);
    FM_CHECK_LAUNCH();
}

constexpr int PN_MAXLEV = 4096;  // stored near-field levels at most

// Makes the near-field blocks of time levels 0 .. min(H, budget) - 1
// resident, integrating the missing ones, and returns how many are.
int near_levels(fmddm_ctx *ctx, fmddm_tree *t, int H)
{
    double key[8];
    medium_key(ctx, key);
    const int64_t per = 96 * std::max<int64_t>(t->near_pairs, 1);
    if (t->pn_cap < 0 || !same_key(key, t->pn_key, 8)) {
        for (auto &l : t->pn_lvl) t->bytes -= (int64_t)l->bytes();
        t->pn_lvl.clear();
        t->pn_hptr.clear();
        if (t->pn_lhs_ok) t->bytes -= (int64_t)t->pn_lhs.bytes();
        t->pn_lhs_ok = 0;
        ++t->poro_gen;
        int64_t budget = ctx->poro.near_cache_bytes;
        if (budget == 0) {
            size_t fr = 0, tot = 0;
            FM_HIP(hipMemGetInfo(&fr, &tot));
            budget = std::min<int64_t>((int64_t)(fr / 4), (int64_t)32 << 30);
        }
        t->pn_cap = budget > 0 ? (int)std::min<int64_t>(budget / per, PN_MAXLEV) : 0;
        t->pn_hptr.reserve(PN_MAXLEV);
        if (t->pn_cap > 0 && t->pn_ptr.n < (size_t)PN_MAXLEV) t->pn_ptr.alloc(PN_MAXLEV);
        for (int k = 0; k < 8; ++k) t->pn_key[k] = key[k];
    }
    const int want = std::min(H, t->pn_cap);
    if ((int)t->pn_lvl.size() >= want) return want;
    hipStream_t s = ctx->stream;
    const PoroK K = poro_constants(ctx);
    // a level counts as stored only once it is allocated, built and its
    // address is in the device table, so an error leaves the levels before
    // it intact and no half-built one behind
    for (int j = (int)t->pn_lvl.size(); j < want; ++j) {
        std::unique_ptr<DBuf<double>> b(new DBuf<double>());
        b->alloc((size_t)12 * std::max<int64_t>(t->near_pairs, 1));
        if (t->near_pairs > 0) {
            build_near_blocks(ctx, t, (j + 1) * ctx->poro.dt, K, 0, b->p);
        }
        t->pn_hptr.resize(j);
        t->pn_hptr.push_back(b->p);
        FM_HIP(hipMemcpyAsync(t->pn_ptr.p + j, t->pn_hptr.data() + j, sizeof(double *), hipMemcpyHostToDevice, s));
        FM_HIP(hipStreamSynchronize(s));
        t->bytes += (int64_t)b->bytes();
        t->pn_lvl.push_back(std::move(b));
    }
    return want;
}

// The left-hand side's near blocks (first level plus the drained elastic
// part), built on first use when the budget holds two levels; returns
// whether they are resident.
bool near_lhs(fmddm_ctx *ctx, fmddm_tree *t)
{
    near_levels(ctx, t, 0);  // refreshes the key and the budget
    if (t->pn_lhs_ok) return true;
    if (t->pn_cap < 2) return false;
    hipStream_t s = ctx->stream;
    t->pn_lhs.alloc((size_t)12 * std::max<int64_t>(t->near_pairs, 1));
    if (t->near_pairs > 0) {
        build_near_blocks(ctx, t, ctx->poro.dt, poro_constants(ctx), 1, t->pn_lhs.p);
    }
    if (t->pn_lhs_ptr.n < 1) t->pn_lhs_ptr.alloc(1);
    t->pn_lhs_host = t->pn_lhs.p;
    FM_HIP(hipMemcpyAsync(t->pn_lhs_ptr.p, &t->pn_lhs_host, sizeof(double *), hipMemcpyHostToDevice, s));
    FM_HIP(hipStreamSynchronize(s));
    t->bytes += (int64_t)t->pn_lhs.bytes();
    t->pn_lhs_ok = 1;
    ++t->poro_gen;
    return true;
}

// Schedule and operators of the multipole form for H time levels.
void poro_fmm_setup(fmddm_ctx *ctx, fmddm_tree *t, int H)
{
    setup_fmm(ctx, t);
    hipStream_t s = ctx->stream;
    const int p = ctx->prm.p, p2 = p * p, Mq = (4 * p2 + 63) / 64 * 64;
    const fmddm_poro_params &pp = ctx->poro;
    double key[8];
    medium_key(ctx, key);
    bool same = t->pf_ready && t->pf_p == p && same_key(key, t->pf_key, 7);
    if (!same) {
        const int ncell = t->ncell;
        std::vector<int> hv(t->nV), hix(ncell), hiy(ncell);
        if (t->nV) FM_HIP(hipMemcpyAsync(hv.data(), t->lidx[1].p, t->nV * 4, hipMemcpyDeviceToHost, s));
        FM_HIP(hipMemcpyAsync(hix.data(), t->cix.p, ncell * 4, hipMemcpyDeviceToHost, s));
        FM_HIP(hipMemcpyAsync(hiy.data(), t->ciy.p, ncell * 4, hipMemcpyDeviceToHost, s));
        FM_HIP(hipStreamSynchronize(s));
        const std::vector<int> &vo = t->h_loff[1];
        std::vector<int> key2combo(64 * 49, -1), clvl, cox, coy;
        std::vector<std::vector<int>> bycombo;
        for (int c = 0; c < ncell; ++c)
            for (int k = vo[c]; k < vo[c + 1]; ++k) {
                int src = hv[k];
                int ox = (int)hix[src] - (int)hix[c], oy = (int)hiy[src] - (int)hiy[c];
                int key = t->h_level[c] * 49 + offset_slot(ox, oy);
                if (key2combo[key] < 0) {
                    key2combo[key] = (int)clvl.size();
                    clvl.push_back(t->h_level[c]);
                    cox.push_back(ox);
                    coy.push_back(oy);
                    bycombo.emplace_back();
                }
                bycombo[key2combo[key]].push_back(k);
            }
        std::vector<int> top, tbeg, tend, psrc, pdst;
        for (size_t cmb = 0; cmb < bycombo.size(); ++cmb)
            for (size_t b = 0; b < bycombo[cmb].size(); b += 32) {
                top.push_back((int)cmb);
                tbeg.push_back((int)psrc.size());
                for (size_t i = b; i < std::min(bycombo[cmb].size(), b + 32); ++i) {
                    int k = bycombo[cmb][i];
                    psrc.push_back(hv[k]);
                    pdst.push_back(k);
                }
                tend.push_back((int)psrc.size());
            }
        auto up = [&](DBuf<int> &d, const std::vector<int> &h) {
            d.alloc(std::max<size_t>(h.size(), 1));
            if (!h.empty()) FM_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * 4, hipMemcpyHostToDevice, s));
        };
        up(t->pf_tile_op, top);
        up(t->pf_tile_beg, tbeg);
        up(t->pf_tile_end, tend);
        up(t->pf_psrc, psrc);
        up(t->pf_pdst, pdst);
        up(t->pf_combo_lvl, clvl);
        up(t->pf_combo_ox, cox);
        up(t->pf_combo_oy, coy);
        t->pf_ncombo = (int)clvl.size();
        t->pf_ntile = (int)top.size();
        t->pf_h_combo_lvl = clvl;
        t->pf_h_combo_ox = cox;
        t->pf_h_combo_oy = coy;
        t->pf_p = p;
        t->pf_Mq = Mq;
        t->pf_dt = pp.dt;
        for (int k = 0; k < 8; ++k) t->pf_key[k] = key[k];
        t->pf_H = 0;
        t->pf_ops0_ok = 0;
        t->pc_ok = 0;
        t->pf_G.alloc((size_t)ncell * Mq);
        t->pf_G.zero(s);
        t->pf_Z.alloc((size_t)std::max<int64_t>(t->nV, 1) * Mq);
        t->pf_far.alloc(4 * (size_t)std::max(t->nfarlev, 1) * t->n);
        t->pf_near.alloc(4 * (size_t)std::max<int64_t>(t->npartial, 1));
        t->pf_D2.alloc(2 * (size_t)t->n);
        t->pf_o2.alloc(2 * (size_t)t->n);
        t->pf_ready = 1;
        ++t->poro_gen;
        FM_HIP(hipStreamSynchronize(s));
    }
    if (t->pf_H < H) {
        int Hn = std::max(H, 2 * t->pf_H);
        if (t->pf_ncombo > 0) {
            size_t tot = (size_t)t->pf_ncombo * Mq * Hn * Mq;
            t->pf_ops.alloc(tot);
            t->pf_ops.zero(s);
            int64_t work = (int64_t)p2 * p2 * Hn * t->pf_ncombo;
            hipLaunchKernelGGL(k_pops, dim3(cdiv(work, 256)), dim3(256), 0, s, t->pf_ncombo, t->pf_combo_lvl.p,
                               t->pf_combo_ox.p, t->pf_combo_oy.p, t->L, ctx->cheb->xbar.p, p, Hn, pp.dt, Mq,
                               poro_constants(ctx), 0, t->pf_ops.p);
            FM_CHECK_LAUNCH();
        }
        t->pf_W.alloc((size_t)t->ncell * Hn * Mq);
        t->pf_W.zero(s);
        ++t->poro_gen;
        t->pf_Q.alloc((size_t)Hn * t->n * 4);
        t->pf_D3.alloc((size_t)Hn * t->n * 3);
        t->pf_H = Hn;
        FM_HIP(hipStreamSynchronize(s));
    }
}

// The left-hand side's M2L operators (first level plus the drained elastic
// point kernel), built once per operator set.
void lhs_ops(fmddm_ctx *ctx, fmddm_tree *t)
{
    if (t->pf_ops0_ok) return;
    if (t->pf_ncombo > 0) {
        hipStream_t s = ctx->stream;
        const int p = ctx->prm.p, p2 = p * p, Mq = t->pf_Mq;
        t->pf_ops0.alloc((size_t)t->pf_ncombo * Mq * Mq);
        t->pf_ops0.zero(s);
        int64_t work = (int64_t)p2 * p2 * t->pf_ncombo;
        hipLaunchKernelGGL(k_pops, dim3(cdiv(work, 256)), dim3(256), 0, s, t->pf_ncombo, t->pf_combo_lvl.p,
                           t->pf_combo_ox.p, t->pf_combo_oy.p, t->L, ctx->cheb->xbar.p, p, 1, ctx->poro.dt, Mq,
                           poro_constants(ctx), 1, t->pf_ops0.p);
        FM_CHECK_LAUNCH();
        FM_HIP(hipStreamSynchronize(s));
    }
    t->pf_ops0_ok = 1;
    ++t->poro_gen;
}

// The left-hand side's M2L operators compressed for one cell half-width hw
// (the kernel is not homogeneous, so unlike the elastic operators each
// cell size has its own bases): the operators K_o of all 40 V-list offsets
// at that size (k_pops), the leading left singular vectors of [K_o ...]
// (column space, U) and of [K_o^T ...] (row space, V) from the randomized
// range finder (range_basis), cut where the singular values fall below
// m2l_tol of the largest; then K_o ~ U C_o V^T with C_o = U^T K_o V.  The
// ranks are far below m = 4p^2 (~90 of 400 at p = 10, of 1024 at p = 16).
// Kept in the context's cache, which a server's slots share: every tree
// with cells of that size takes them from there.
std::shared_ptr<PoroLhsBasis> level_basis(fmddm_ctx *ctx, double hw)
{
    const fmddm_poro_params &q = ctx->poro;
    const double tol = ctx->prm.m2l_tol;
    const int p = ctx->prm.p, p2 = p * p, m = 4 * p2, Mq = (m + 63) / 64 * 64;
    const std::vector<double> key = {hw, q.nu_u, q.alpha, q.perm, q.visc, q.dt, ctx->prm.E, ctx->prm.nu,
                                     (double)p, tol};
    if (ctx->pcache) {
        std::lock_guard<std::mutex> g(ctx->pcache->mu);
        auto it = ctx->pcache->lev.find(key);
        if (it != ctx->pcache->lev.end()) return it->second;
    }
    auto E = std::make_shared<PoroLhsBasis>();
    hipStream_t s = ctx->stream;
    std::vector<int> dx, dy, slot;
    v_offsets(dx, dy, slot);
    const int nop = (int)dx.size();
    std::vector<int> zero(nop, 0), all(nop);
    for (int o = 0; o < nop; ++o) all[o] = o;
    auto up = [&](DBuf<int> &d, const std::vector<int> &v) {
        d.alloc(std::max<size_t>(v.size(), 1));
        if (!v.empty()) FM_HIP(hipMemcpyAsync(d.p, v.data(), v.size() * 4, hipMemcpyHostToDevice, s));
    };
    DBuf<int> dlvl, dox, doy, dall;
    up(dlvl, zero);
    up(dox, dx);
    up(doy, dy);
    up(dall, all);
    // the operators at this size: level 0 of a root of side 2 hw
    DBuf<double> ops;
    ops.alloc((size_t)nop * Mq * Mq);
    ops.zero(s);
    hipLaunchKernelGGL(k_pops, dim3(cdiv((int64_t)p2 * p2 * nop, 256)), dim3(256), 0, s, nop, dlvl.p, dox.p, doy.p,
                       2.0 * hw, ctx->cheb->xbar.p, p, 1, q.dt, Mq, poro_constants(ctx), 1, ops.p);
    FM_CHECK_LAUNCH();
    if (!ctx->blas) {
        rocblas_handle h;
        if (rocblas_create_handle(&h) != rocblas_status_success) throw Error{FMDDM_EDEVICE, "rocblas handle"};
        ctx->blas = h;
    }
    rocblas_handle h = (rocblas_handle)ctx->blas;
    rocblas_set_stream(h, s);
    const size_t mm = (size_t)m * m;
    DBuf<double> fat, Uc, Ur;
    fat.alloc(mm * nop);
    Uc.alloc(mm);
    Ur.alloc(mm);
    std::vector<double> sv;
    int r = 1;
    for (int side = 0; side < 2; ++side) {
        hipLaunchKernelGGL(k_pc_pack, dim3(cdiv((int64_t)m * nop * m, 256)), dim3(256), 0, s, nop, dall.p, m, Mq, side,
                           ops.p, fat.p);
        FM_CHECK_LAUNCH();
        r = std::max(r, range_basis(h, s, m, nop * m, fat.p, tol, side == 0 ? Uc.p : Ur.p, sv));
    }
    E->r = r;
    E->rq = (r + 63) / 64 * 64;
    E->ok = 4 * r <= 3 * m && E->rq < Mq;
    if (E->ok) {
        const int rq = E->rq;
        DBuf<int> drank;
        std::vector<int> hr(1, r);
        up(drank, hr);
        DBuf<double> UT;
        E->Vt.alloc((size_t)rq * Mq);
        E->U.alloc((size_t)Mq * rq);
        UT.alloc((size_t)rq * Mq);
        hipLaunchKernelGGL(k_pc_bases, dim3(cdiv((int64_t)rq * Mq, 256)), dim3(256), 0, s, 1, m, Mq, rq, drank.p,
                           Uc.p, Ur.p, E->Vt.p, UT.p, E->U.p);
        FM_CHECK_LAUNCH();
        // C_o = U^T K_o V: T1[o rq + a] = K_o v_a, then Ct[o rq + a] = U^T T1[o rq + a]
        std::vector<int> top, tb, te, src, z0;
        for (int o = 0; o < nop; ++o)
            for (int a0 = 0; a0 < rq; a0 += 32) {
                top.push_back(o);
                z0.push_back(0);
                tb.push_back((int)src.size());
                for (int a = a0; a < std::min(rq, a0 + 32); ++a) src.push_back(o * rq + a);
                te.push_back((int)src.size());
            }
        std::vector<int> vrow(src.size());
        for (size_t i = 0; i < src.size(); ++i) vrow[i] = src[i] % rq;
        DBuf<int> dtop, dtb, dte, dsrc, dvrow, dz0;
        up(dtop, top);
        up(dtb, tb);
        up(dte, te);
        up(dsrc, src);
        up(dvrow, vrow);
        up(dz0, z0);
        DBuf<double> T1, Ct;
        T1.alloc((size_t)nop * rq * Mq);
        Ct.alloc((size_t)nop * rq * rq);
        fmm_pair_gemm(s, (int)top.size(), Mq, ops.p, (size_t)Mq * Mq, Mq, Mq, E->Vt.p, Mq, dtop.p, dtb.p, dte.p,
                      dvrow.p, dsrc.p, T1.p, Mq);
        fmm_pair_gemm(s, (int)top.size(), rq, UT.p, 0, Mq, Mq, T1.p, Mq, dz0.p, dtb.p, dte.p, dsrc.p, dsrc.p, Ct.p,
                      rq);
        E->C.alloc((size_t)nop * rq * rq);
        hipLaunchKernelGGL(k_pc_transpose, dim3(cdiv((int64_t)nop * rq * rq, 256)), dim3(256), 0, s, nop, rq, Ct.p,
                           E->C.p);
        FM_CHECK_LAUNCH();
    }
    FM_HIP(hipStreamSynchronize(s));  // complete before other streams may read it
    if (ctx->pcache) {
        std::lock_guard<std::mutex> g(ctx->pcache->mu);
        auto it = ctx->pcache->lev.find(key);
        if (it != ctx->pcache->lev.end()) return it->second;  // another thread was first
        if (ctx->pcache->lev.size() >= 64) ctx->pcache->lev.clear();  // trees keep what they hold
        ctx->pcache->lev[key] = E;
    }
    return E;
}

// The tree's compressed left-hand side: per level slot the bases of its
// cell size (level_basis), padded to the tree's largest rank rq, and per
// (level, offset) combination its C_o; then the schedules of a product:
// projection of every V-list source cell, the rq x rq translations per
// pair, and expansion of every cell with a V list, in tiles of at most 32
// cells of one level.  Left uncompressed (pc_ok = -1) when a level's rank
// would exceed 3/4 of 4p^2.
void lhs_compress(fmddm_ctx *ctx, fmddm_tree *t)
{
    const double tol = ctx->prm.m2l_tol;
    if (t->pc_ok != 0 && t->pc_tol == tol) return;
    t->pc_ok = -1;
    t->pc_tol = tol;
    const int nc = t->pf_ncombo;
    if (nc == 0) return;
    hipStream_t s = ctx->stream;
    const int Mq = t->pf_Mq;
    std::vector<int> levs(t->pf_h_combo_lvl);
    std::sort(levs.begin(), levs.end());
    levs.erase(std::unique(levs.begin(), levs.end()), levs.end());
    const int nlev = (int)levs.size();
    std::vector<int> slot_of(64, -1);
    std::vector<std::shared_ptr<PoroLhsBasis>> lb(nlev);
    int rq = 64;
    std::vector<int> rank(nlev);
    for (int k = 0; k < nlev; ++k) {
        slot_of[levs[k]] = k;
        lb[k] = level_basis(ctx, t->L / (double)(2LL << levs[k]));
        if (!lb[k]->ok) return;  // not worth it: the dense operators stay
        rq = std::max(rq, lb[k]->rq);
        rank[k] = lb[k]->r;
    }
    t->pc_rank = rank;
    t->pc_rq = rq;
    t->pc_nlev = nlev;
    t->pc_Vt.alloc((size_t)nlev * rq * Mq);
    t->pc_U.alloc((size_t)nlev * Mq * rq);
    t->pc_C.alloc((size_t)nc * rq * rq);
    t->pc_Vt.zero(s);
    t->pc_U.zero(s);
    t->pc_C.zero(s);
    for (int k = 0; k < nlev; ++k) {
        const int rk = lb[k]->rq;
        FM_HIP(hipMemcpyAsync(t->pc_Vt.p + (size_t)k * rq * Mq, lb[k]->Vt.p, (size_t)rk * Mq * 8,
                              hipMemcpyDeviceToDevice, s));
        FM_HIP(hipMemcpy2DAsync(t->pc_U.p + (size_t)k * Mq * rq, (size_t)rq * 8, lb[k]->U.p, (size_t)rk * 8,
                                (size_t)rk * 8, Mq, hipMemcpyDeviceToDevice, s));
    }
    std::vector<int> dx, dy, vslot;
    v_offsets(dx, dy, vslot);
    for (int o = 0; o < nc; ++o) {
        const PoroLhsBasis &B = *lb[slot_of[t->pf_h_combo_lvl[o]]];
        const int rk = B.rq, vo = vslot[offset_slot(t->pf_h_combo_ox[o], t->pf_h_combo_oy[o])];
        if (vo < 0) throw Error{FMDDM_EDEVICE, "V-list offset outside the 40 of the operator set"};
        FM_HIP(hipMemcpy2DAsync(t->pc_C.p + (size_t)o * rq * rq, (size_t)rq * 8, B.C.p + (size_t)vo * rk * rk,
                                (size_t)rk * 8, (size_t)rk * 8, rk, hipMemcpyDeviceToDevice, s));
    }
    auto up = [&](DBuf<int> &d, const std::vector<int> &v) {
        d.alloc(std::max<size_t>(v.size(), 1));
        if (!v.empty()) FM_HIP(hipMemcpyAsync(d.p, v.data(), v.size() * 4, hipMemcpyHostToDevice, s));
    };
    // schedules: projection of every V-list source cell, expansion of every
    // cell with a V list, in tiles of at most 32 cells of one level
    const int ncell = t->ncell;
    const std::vector<int> &vo = t->h_loff[1];
    std::vector<int> hv(t->nV);
    if (t->nV) FM_HIP(hipMemcpyAsync(hv.data(), t->lidx[1].p, t->nV * 4, hipMemcpyDeviceToHost, s));
    FM_HIP(hipStreamSynchronize(s));
    std::vector<char> is_src(ncell, 0);
    for (int v : hv) is_src[v] = 1;
    auto tiles = [&](bool proj, std::vector<int> &op, std::vector<int> &b, std::vector<int> &e,
                     std::vector<int> &cell) {
        for (int k = 0; k < nlev; ++k) {
            std::vector<int> cs;
            for (int c = 0; c < ncell; ++c)
                if (t->h_level[c] == levs[k] && (proj ? is_src[c] != 0 : vo[c + 1] > vo[c])) cs.push_back(c);
            for (size_t i0 = 0; i0 < cs.size(); i0 += 32) {
                op.push_back(k);
                b.push_back((int)cell.size());
                for (size_t i = i0; i < std::min(cs.size(), i0 + 32); ++i) cell.push_back(cs[i]);
                e.push_back((int)cell.size());
            }
        }
    };
    std::vector<int> pop, pb, pe, pcell, eop, eb, ee, ecell;
    tiles(true, pop, pb, pe, pcell);
    tiles(false, eop, eb, ee, ecell);
    up(t->pc_ptile_op, pop);
    up(t->pc_ptile_beg, pb);
    up(t->pc_ptile_end, pe);
    up(t->pc_pcell, pcell);
    up(t->pc_etile_op, eop);
    up(t->pc_etile_beg, eb);
    up(t->pc_etile_end, ee);
    up(t->pc_ecell, ecell);
    t->pc_nptile = (int)pop.size();
    t->pc_netile = (int)eop.size();
    t->pc_What.alloc((size_t)ncell * rq);
    t->pc_Z.alloc((size_t)std::max<int64_t>(t->nV, 1) * rq);
    t->pc_Ghat.alloc((size_t)ncell * rq);
    // the projection has one tile per 32 source cells and rq / 64 row
    // tiles, too few blocks for a long K (4p^2): K is split so that about
    // 512 blocks run, and the slices are summed in order; slices of cells
    // that are never projected stay zero
    {
        const int base = std::max(1, t->pc_nptile * (rq / 64));
        t->pc_ksplit = std::min(8, std::max(1, (512 + base - 1) / base));
        if (t->pc_ksplit > 1) {
            t->pc_Wsplit.alloc((size_t)t->pc_ksplit * ncell * rq);
            t->pc_Wsplit.zero(s);
        }
    }
    FM_HIP(hipStreamSynchronize(s));
    t->bytes += (int64_t)(t->pc_Vt.bytes() + t->pc_U.bytes() + t->pc_C.bytes() + t->pc_What.bytes() +
                          t->pc_Z.bytes() + t->pc_Ghat.bytes() + (t->pc_ksplit > 1 ? t->pc_Wsplit.bytes() : 0));
    t->pc_ok = 1;
    ++t->poro_gen;
}

// Whether the far field of an H-level history sum may take the two-term
// form (k_pprep_affine): the nodes of V-list cells at level l (half-width
// hw) are at least 2 hw apart, so z >= hw^2 / (c H dt) for every pair.
constexpr double FAR_AFFINE_Z = 50.0;  // e^-50 z^2 < 1e-18

bool far_affine(const fmddm_ctx *ctx, const fmddm_tree *t, int H)
{
    const PoroK K = poro_constants(ctx);
    const double ct = K.c * H * ctx->poro.dt;
    for (int l : t->pf_h_combo_lvl) {
        const double hw = t->L / (double)(2LL << l);
        if (hw * hw < FAR_AFFINE_Z * ct) return false;
    }
    return true;
}

// out (mode 0: =, 1: -=) the sum over time levels j = 1..H of F_transient(j dt)
// applied to E[j-1] (3n each, caller order), plus, if drained, the drained
// elastic part of E[0]; multipole form.  E[j-1] is zero for j <= jlo (the
// near field skips those levels).
void poro_fmm_sum(fmddm_ctx *ctx, fmddm_tree *t, int H, const double *E, bool drained, int mode, double *out,
                  int jlo = 0)
{
    upload_rules(ctx->device);
    bool affine = false;  // the far field in two terms (history sums only)
    if (!drained && H > 2 && ctx->poro.exact_far_levels == 0) {
        poro_fmm_setup(ctx, t, 2);
        affine = far_affine(ctx, t, H);
    }
    if (!affine) poro_fmm_setup(ctx, t, H);
    const int Hf = affine ? 2 : H;  // multipole terms
    hipStream_t s = ctx->stream;
    const int n = (int)t->n, p = ctx->prm.p, p2 = p * p, Mq = t->pf_Mq;
    PoroK K = poro_constants(ctx);
    // the left-hand side F(dt) in one pass: operators and near blocks that
    // include the drained elastic part (when the near budget holds them)
    const bool fused = H == 1 && drained && jlo == 0 && near_lhs(ctx, t);
    if (fused && ctx->poro.m2l == FMDDM_M2L_SVD) lhs_compress(ctx, t);
    const bool comp = fused && ctx->poro.m2l == FMDDM_M2L_SVD && t->pc_ok == 1;
    if (fused && !comp) lhs_ops(ctx, t);
    double *D3 = t->pf_D3.p;  // DDs per time level, tree order (near field)
    if (affine) {
        if (t->pf_D3a.n < (size_t)H * n * 3) t->pf_D3a.alloc((size_t)H * n * 3);
        D3 = t->pf_D3a.p;
        hipLaunchKernelGGL(k_pprep_affine, dim3(cdiv(n, 256)), dim3(256), 0, s, n, H, t->perm.p, E, t->scb.p,
                           t->ssb.p, t->pf_Q.p, D3);
    } else {
        hipLaunchKernelGGL(k_pprep, dim3(cdiv(n, 256), H), dim3(256), 0, s, n, H, t->perm.p, E, t->scb.p,
                           t->ssb.p, t->pf_Q.p, D3);
    }
    FM_CHECK_LAUNCH();
    bool far = t->nV > 0 && t->pf_ntile > 0;
    if (far) {
        hipLaunchKernelGGL(k_pp2m, dim3(t->nleaf, Hf), dim3(256), 0, s, t->nleaf, t->dleaves.p, t->cpbeg.p,
                           t->cpend.p, t->p2m_mat.p, t->pf_Q.p, n, p2, Hf, Mq, t->pf_W.p);
        FM_CHECK_LAUNCH();
        fmm_m2m4(ctx, t, Hf, Hf * Mq, Mq, t->pf_W.p);
        if (comp) {
            const int rq = t->pc_rq;
            if (t->pc_ksplit > 1)
                fmm_pair_gemm_split(s, t->pc_nptile, rq, t->pc_Vt.p, (size_t)rq * Mq, Mq, Mq, t->pf_W.p, Mq,
                                    t->pc_ptile_op.p, t->pc_ptile_beg.p, t->pc_ptile_end.p, t->pc_pcell.p,
                                    t->pc_pcell.p, t->pc_Wsplit.p, rq, t->pc_ksplit, (size_t)t->ncell * rq,
                                    t->pc_What.p, (int64_t)t->ncell * rq);
            else
                fmm_pair_gemm(s, t->pc_nptile, rq, t->pc_Vt.p, (size_t)rq * Mq, Mq, Mq, t->pf_W.p, Mq,
                              t->pc_ptile_op.p, t->pc_ptile_beg.p, t->pc_ptile_end.p, t->pc_pcell.p, t->pc_pcell.p,
                              t->pc_What.p, rq);
            fmm_pair_gemm(s, t->pf_ntile, rq, t->pc_C.p, (size_t)rq * rq, rq, rq, t->pc_What.p, rq, t->pf_tile_op.p,
                          t->pf_tile_beg.p, t->pf_tile_end.p, t->pf_psrc.p, t->pf_pdst.p, t->pc_Z.p, rq);
            fmm_sum_pairs(s, t, t->pc_Z.p, rq, rq, t->pc_Ghat.p, rq);
            fmm_pair_gemm(s, t->pc_netile, Mq, t->pc_U.p, (size_t)Mq * rq, rq, rq, t->pc_Ghat.p, rq,
                          t->pc_etile_op.p, t->pc_etile_beg.p, t->pc_etile_end.p, t->pc_ecell.p, t->pc_ecell.p,
                          t->pf_G.p, Mq);
        } else {
            if (fused)
                fmm_pair_gemm(s, t->pf_ntile, Mq, t->pf_ops0.p, (size_t)Mq * Mq, Mq, Mq, t->pf_W.p, Mq,
                              t->pf_tile_op.p, t->pf_tile_beg.p, t->pf_tile_end.p, t->pf_psrc.p, t->pf_pdst.p,
                              t->pf_Z.p, Mq);
            else
                fmm_pair_gemm(s, t->pf_ntile, Mq, t->pf_ops.p, (size_t)Mq * t->pf_H * Mq, t->pf_H * Mq, Hf * Mq,
                              t->pf_W.p, Hf * Mq, t->pf_tile_op.p, t->pf_tile_beg.p, t->pf_tile_end.p, t->pf_psrc.p,
                              t->pf_pdst.p, t->pf_Z.p, Mq);
            fmm_sum_pairs(s, t, t->pf_Z.p, Mq, Mq, t->pf_G.p, Mq);
        }
        fmm_l2p4(ctx, t, t->pf_G.p, Mq, t->pf_far.p);
    }
    if (fused) {
        hipLaunchKernelGGL(k_pnear, dim3(t->nitem), dim3(PNB), 0, s, t->nitem, t->it_leaf.p, t->it_s0.p,
                           t->it_s1.p, t->it_poff.p, t->it_coff.p, t->dleaves.p, t->cpbeg.p, t->cpend.p, t->nfoff.p,
                           t->nflat.p, n, 0, 1, (const double *const *)t->pn_lhs_ptr.p, D3, t->pf_near.p);
        FM_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_pfinal, dim3(cdiv(n, 256)), dim3(256), 0, s, n, t->tleaf.p, t->dleaves.p, t->cpbeg.p,
                           t->clevel.p, t->lk_off.p, t->it_poff.p, t->pf_near.p,
                           far ? t->pf_far.p : (const double *)nullptr, t->scb.p, t->ssb.p, t->perm.p,
                           (const double *)nullptr, mode, out);
        FM_CHECK_LAUNCH();
        return;
    }
    // near field: stored levels jlo .. Hc-1 as block-sparse products, the
    // rest integrated here
    const int Hc = near_levels(ctx, t, H);
    const bool stored = Hc > jlo;
    if (stored) {
        hipLaunchKernelGGL(k_pnear, dim3(t->nitem), dim3(PNB), 0, s, t->nitem, t->it_leaf.p, t->it_s0.p,
                           t->it_s1.p, t->it_poff.p, t->it_coff.p, t->dleaves.p, t->cpbeg.p, t->cpend.p, t->nfoff.p,
                           t->nflat.p, n, jlo, Hc, (const double *const *)t->pn_ptr.p, D3, t->pf_near.p);
        FM_CHECK_LAUNCH();
    }
    if (Hc < H || !stored) {
        hipLaunchKernelGGL(k_pp2p, dim3(t->nitem), dim3(PN), 0, s, t->nitem, t->it_leaf.p, t->it_s0.p, t->it_s1.p,
                           t->it_poff.p, t->dleaves.p, t->cpbeg.p, t->cpend.p, t->noff.p, t->nbeg.p, t->npre.p,
                           t->scx.p, t->scy.p, t->scb.p, t->ssb.p, t->sa.p, n, std::max(jlo, Hc), H,
                           ctx->poro.dt, D3, K, stored ? 1 : 0, t->pf_near.p);
        FM_CHECK_LAUNCH();
    }
    const double *o2 = nullptr;
    if (drained) {
        hipLaunchKernelGGL(k_take2, dim3(cdiv(n, 256)), dim3(256), 0, s, n, E, t->pf_D2.p);
        FM_CHECK_LAUNCH();
        fmm_apply(ctx, t, t->pf_D2.p, t->pf_o2.p);
        o2 = t->pf_o2.p;
    }
    hipLaunchKernelGGL(k_pfinal, dim3(cdiv(n, 256)), dim3(256), 0, s, n, t->tleaf.p, t->dleaves.p, t->cpbeg.p,
                       t->clevel.p, t->lk_off.p, t->it_poff.p, t->pf_near.p,
                       far ? t->pf_far.p : (const double *)nullptr,
                       t->scb.p, t->ssb.p, t->perm.p, o2, mode, out);
    FM_CHECK_LAUNCH();
}

}  // namespace

// out = F(dt) D with the stored dense left-hand side (assembled on first
// use, and again when the medium or dt changes).
void poro_dense_apply(fmddm_ctx *ctx, fmddm_tree *t, const double *D, double *out)
{
    const int n = (int)t->n;
    const size_t m = 3 * (size_t)n;
    double key[8];
    medium_key(ctx, key);
    hipStream_t s = ctx->stream;
    if (!t->pdense_ok || !same_key(key, t->pdense_key, 8)) {
        if (!t->pdense.p || t->pdense.n < m * m) {
            size_t freeb = 0, totalb = 0;
            FM_HIP(hipMemGetInfo(&freeb, &totalb));
            if (m * m * 8 + ((size_t)1 << 30) > freeb + dev_bytes(true))
                throw Error{FMDDM_ENOMEM, "dense poroelastic left-hand side does not fit"};
            t->pdense.alloc(m * m);
            t->bytes += (int64_t)(m * m * 8);
        }
        upload_rules(ctx->device);
        hipLaunchKernelGGL(k_pdense, dim3(n, cdiv(n, 256)), dim3(256), 0, s, n, t->ocx.p, t->ocy.p, t->ocb.p,
                           t->osb.p, t->oa.p, ctx->poro.dt, poro_constants(ctx), t->pdense.p);
        FM_CHECK_LAUNCH();
        for (int k = 0; k < 8; ++k) t->pdense_key[k] = key[k];
        t->pdense_ok = 1;
        ++t->poro_gen;
    }
    dense_gemv(s, (int)m, t->pdense.p, D, out);
}

void poro_apply(fmddm_ctx *ctx, fmddm_tree *t, int lag, const double *D, double *out)
{
    if (!ctx->poro_set) throw Error{FMDDM_EINVAL, "poroelastic parameters not set (fmddm_poro_set)"};
    const double dt = ctx->poro.dt;
    const int n = (int)t->n, m3 = 3 * n;
    const bool fmm = ctx->poro.mode != FMDDM_APPLY_DIRECT;  // DENSE: multipole history coefficients
    hipStream_t s = ctx->stream;
    if (lag == 0) {
        if (ctx->poro.mode == FMDDM_APPLY_DENSE) poro_dense_apply(ctx, t, D, out);
        else if (fmm) poro_fmm_sum(ctx, t, 1, D, true, 0, out);
        else poro_sum(ctx, t, 1, {dt}, D, 0, 0, out);
        return;
    }
    if (fmm) {
        // time levels 1..lag+1 with E[lag-1] = -D, E[lag] = D, the rest zero
        const int H = lag + 1;
        if (t->poro_E.n < (size_t)H * m3) t->poro_E.alloc((size_t)H * m3);
        hipLaunchKernelGGL(k_zero, dim3(cdiv((int64_t)H * m3, 256)), dim3(256), 0, s, (int64_t)H * m3,
                           t->poro_E.p);
        hipLaunchKernelGGL(k_scale_copy, dim3(cdiv(m3, 256)), dim3(256), 0, s, m3, -1.0, D,
                           t->poro_E.p + (size_t)(lag - 1) * m3);
        hipLaunchKernelGGL(k_scale_copy, dim3(cdiv(m3, 256)), dim3(256), 0, s, m3, 1.0, D,
                           t->poro_E.p + (size_t)lag * m3);
        FM_CHECK_LAUNCH();
        poro_fmm_sum(ctx, t, H, t->poro_E.p, false, 0, out, lag - 1);
        return;
    }
    // terms (t1, D) and (t0, -D): the drained parts cancel
    if (t->poro_E.n < (size_t)2 * m3) t->poro_E.alloc((size_t)2 * m3);
    hipLaunchKernelGGL(k_scale_copy, dim3(cdiv(m3, 256)), dim3(256), 0, s, m3, 1.0, D, t->poro_E.p);
    hipLaunchKernelGGL(k_scale_copy, dim3(cdiv(m3, 256)), dim3(256), 0, s, m3, -1.0, D, t->poro_E.p + m3);
    FM_CHECK_LAUNCH();
    poro_sum(ctx, t, 2, {(lag + 1) * dt, lag * dt}, t->poro_E.p, -1, 0, out);
}

void poro_history(fmddm_ctx *ctx, fmddm_tree *t, int h, const double *Dh, double *rhs)
{
    if (h < 2) return;
    if (!ctx->poro_set) throw Error{FMDDM_EINVAL, "poroelastic parameters not set (fmddm_poro_set)"};
    const double dt = ctx->poro.dt;
    const int n = (int)t->n, m3 = 3 * n;
    if (t->poro_E.n < (size_t)h * m3) t->poro_E.alloc((size_t)h * m3);
    hipStream_t s = ctx->stream;
    hipLaunchKernelGGL(k_hist_terms, dim3(cdiv(m3, 256), h), dim3(256), 0, s, m3, h, Dh, t->poro_E.p);
    FM_CHECK_LAUNCH();
    if (ctx->poro.mode != FMDDM_APPLY_DIRECT) {  // FMM, or the history-only variant
        poro_fmm_sum(ctx, t, h, t->poro_E.p, false, 1, rhs);
        return;
    }
    std::vector<double> times(h);
    for (int j = 1; j <= h; ++j) times[j - 1] = j * dt;
    poro_sum(ctx, t, h, times, t->poro_E.p, -1, 1, rhs);
}

// Everything a march of H steps builds on first use, built now: the
// multipole schedule and operators for H time levels, the left-hand side's
// operators and near blocks, and the history's near blocks for the levels
// the budget holds.  A serving loop calls this at admission so that the
// steps themselves enqueue work without waiting on the device.
void poro_prepare(fmddm_ctx *ctx, fmddm_tree *t, int H)
{
    if (!ctx->poro_set) throw Error{FMDDM_EINVAL, "poroelastic parameters not set (fmddm_poro_set)"};
    upload_rules(ctx->device);
    if (ctx->poro.mode != FMDDM_APPLY_FMM) return;
    // operators of the first two time levels, all H where the far field
    // of the history sums cannot take the two-term form
    poro_fmm_setup(ctx, t, std::min(std::max(H, 1), 2));
    if (H > 2 && !(ctx->poro.exact_far_levels == 0 && far_affine(ctx, t, H))) poro_fmm_setup(ctx, t, H);
    if (near_lhs(ctx, t)) {
        if (ctx->poro.m2l == FMDDM_M2L_SVD) lhs_compress(ctx, t);
        if (t->pc_ok != 1) lhs_ops(ctx, t);
    }
    if (H > 1) near_levels(ctx, t, H);
}

// Block-Jacobi preconditioner of the poroelastic left-hand side, rebuilt
// when the medium or the time step changes.
void pc_setup_poro(fmddm_ctx *ctx, fmddm_tree *t)
{
    if (!ctx->poro_set) throw Error{FMDDM_EINVAL, "poroelastic parameters not set (fmddm_poro_set)"};
    PcBlocks &B = t->ppc;
    const fmddm_poro_params &q = ctx->poro;
    const double key[6] = {q.nu_u, q.alpha, q.perm, q.visc, q.dt, ctx->prm.E + 1e-3 * ctx->prm.nu};
    bool same = B.nblk > 0;
    for (int k = 0; k < 6; ++k) same = same && B.key[k] == key[k];
    if (same) return;
    hipStream_t s = ctx->stream;
    upload_rules(ctx->device);
    pc_groups(ctx, t, PPB, 3, B);
    DBuf<int> bad;
    bad.alloc(1);
    bad.zero(s);
    if (t->near_pairs > 0 && near_lhs(ctx, t))
        hipLaunchKernelGGL(k_ppc_gather, dim3(B.nblk), dim3(256), 0, s, B.nblk, B.beg.p, B.cnt.p, B.off.p,
                           t->tleaf.p, t->dleaves.p, t->cpbeg.p, t->cpend.p, t->lk_off.p, t->it_s0.p, t->it_s1.p,
                           t->it_coff.p, t->nfoff.p, t->nflat.p, t->pn_lhs.p, t->scx.p, t->scy.p, t->scb.p,
                           t->ssb.p, t->sa.p, q.dt, poro_constants(ctx), B.inv.p, bad.p);
    else
        hipLaunchKernelGGL(k_ppc_build, dim3(B.nblk), dim3(256), 0, s, B.nblk, B.beg.p, B.cnt.p, B.off.p, t->scx.p,
                           t->scy.p, t->scb.p, t->ssb.p, t->sa.p, q.dt, poro_constants(ctx), B.inv.p, bad.p);
    FM_CHECK_LAUNCH();
    int hbad = 0;
    FM_HIP(hipMemcpyAsync(&hbad, bad.p, 4, hipMemcpyDeviceToHost, s));
    FM_HIP(hipStreamSynchronize(s));
    if (hbad) {
        B.nblk = 0;
        throw Error{FMDDM_EGEOM, "singular poroelastic preconditioner block"};
    }
    for (int k = 0; k < 6; ++k) B.key[k] = key[k];
    ++t->poro_gen;
}

void poro_rhs(fmddm_ctx *ctx, fmddm_tree *t, const double *pf, double SH, double Sh, double *rhs)
{
    int n = (int)t->n;
    hipLaunchKernelGGL(k_poro_rhs, dim3(cdiv(n, 256)), dim3(256), 0, ctx->stream, n, t->ocb.p, t->osb.p, pf,
                       ctx->poro.p0, SH, Sh, rhs);
    FM_CHECK_LAUNCH();
}

}  // namespace fmddm
