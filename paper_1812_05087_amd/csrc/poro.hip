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
#include "internal.h"

#include <cmath>

namespace fmddm {
namespace {

struct PoroK {
    double G, nu, alpha, kappa, S, c, eta, gc;
};

// E1(z), z > 0.  Below 2: -gamma - ln z + Ein(z), with the series
// Ein(z) = sum (-1)^(k+1) z^k / (k k!) nested as z (1 - z/4 (1 - 2z/9
// (1 - 3z/16 (...)))) to depth 30; above: the continued fraction
// e^-z / (z + 1 - 1/(z + 3 - 4/(z + 5 - ...))) evaluated backwards from
// depth 64.
__device__ double e1(double z)
{
    if (z <= 2.0) {
        double v = 1.0;
        for (int k = 30; k >= 1; --k) v = 1.0 - z * k / ((k + 1.0) * (k + 1.0)) * v;
        return -0.57721566490153286061 - log(z) + z * v;
    }
    double f = 0.0;
    for (int k = 64; k >= 1; --k) f = (double)k * k / (z + 2.0 * k + 1.0 - f);
    return exp(-z) / (z + 1.0 - f);
}

// h(z) = 1 - (1 - e^-z)/z with h', h'' (series below 0.5).
__device__ void hfun(double z, double &h, double &h1, double &h2)
{
    if (z < 0.5) {
        // h = sum_{k>=1} c_k z^k, c_k = (-1)^(k+1) / (k+1)!, by Horner
        // from k = 22 down (the first omitted term is below 1e-26)
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        double f = 1.0;
        for (int j = 2; j <= 23; ++j) f *= j;  // 23!
        for (int k = 22; k >= 1; --k) {
            double ck = ((k & 1) ? 1.0 : -1.0) / f;
            f /= (k + 1);
            a0 = a0 * z + ck;
            a1 = a1 * z + ck * k;
            if (k >= 2) a2 = a2 * z + ck * k * (k - 1);
        }
        h = a0 * z;
        h1 = a1;
        h2 = a2;
        return;
    }
    double em = exp(-z), om = -expm1(-z);
    double iz = 1.0 / z;
    h = 1.0 - om * iz;
    h1 = om * iz * iz - em * iz;
    h2 = -2.0 * om * iz * iz * iz + 2.0 * em * iz * iz + em * iz;
}

__device__ double p2fun(double z)
{
    if (z < 0.1) {
        // sum_{k>=2} (-1)^k (k-1) z^k / k!
        double s = 0.0, f = 2.0, zk = z * z;
        for (int k = 2; k < 18; ++k) {
            if (k > 2) {
                f *= k;
                zk *= z;
            }
            s += ((k & 1) ? -1.0 : 1.0) * (k - 1) * zk / f;
        }
        return s;
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

// Transient response (sxx, syy, sxy, p) at offset (x, y) and time t.
__device__ void transient(const PoroK &K, double x, double y, double t, const double q[3], double qf,
                          double o[4])
{
    double r2 = x * x + y * y, ir2 = 1.0 / r2, r = sqrt(r2);
    double z = r2 / (4.0 * K.c * t);
    double ez = exp(-z), om = -expm1(-z);
    double kd = (1.0 - 2.0 * K.nu) / (4.0 * M_PI * K.G * (1.0 - K.nu));
    double a = 2.0 * K.G * (q[0] - q[1]), b = 2.0 * K.G * q[2];
    double V = -(q[0] + q[1]) * (1.0 - 2.0 * K.nu) / (2.0 * (1.0 - K.nu));
    double gxy = x * x - y * y, g2 = 2.0 * x * y;
    double p = (K.alpha * kd / K.S) * (a * gxy + b * g2) * ir2 * ir2 * p2fun(z)
               - (K.alpha / K.S) * V * ez / (4.0 * M_PI * K.c * t);
    double h, h1, h2;
    hfun(z, h, h1, h2);
    double F = -0.25 * h * ir2;
    double F1 = (h - z * h1) * 0.5 * ir2 / r;                 // F'(r)
    double F2 = (-2.0 * z * z * h2 - 3.0 * h + 3.0 * z * h1) * 0.5 * ir2 * ir2;  // F''(r)
    // second derivatives of F(r): F_xx etc. (F1/r plays phi'/r)
    double fxx = 0.0, fyy = 0.0, fxy = 0.0;
    rad2(x, y, ir2, F1 / r, F2, fxx, fyy, fxy);
    double Fx = F1 * x / r, Fy = F1 * y / r;
    double Cphi = K.alpha * kd * K.eta / K.S;
    // phi_c = F (x^2 - y^2), phi_s = F 2xy
    double cxx = fxx * gxy + 4.0 * Fx * x + 2.0 * F;
    double cyy = fyy * gxy - 4.0 * Fy * y - 2.0 * F;
    double cxy = fxy * gxy - 2.0 * Fx * y + 2.0 * Fy * x;
    double sxx = fxx * g2 + 4.0 * Fx * y;
    double syy = fyy * g2 + 4.0 * Fy * x;
    double sxy = fxy * g2 + 2.0 * Fx * x + 2.0 * Fy * y + 2.0 * F;
    double pxx = Cphi * (a * cxx + b * sxx), pyy = Cphi * (a * cyy + b * syy), pxy = Cphi * (a * cxy + b * sxy);
    double Kd = -K.alpha * K.eta * V / (2.0 * M_PI * K.S);
    rad2(x, y, ir2, Kd * om * ir2, Kd * (2.0 * z * ez - om) * ir2, pxx, pyy, pxy);
    if (qf != 0.0) {
        double E = e1(z);
        p += qf * E / (4.0 * M_PI * K.kappa);
        double Kf = qf * K.eta * t / (2.0 * M_PI * K.S);
        double A = z * E + om;
        rad2(x, y, ir2, Kf * A * ir2, Kf * (2.0 * z * E - A) * ir2, pxx, pyy, pxy);
    }
    o[0] = -2.0 * K.G * pyy;
    o[1] = -2.0 * K.G * pxx;
    o[2] = 2.0 * K.G * pxy;
    o[3] = p;
}

constexpr int QN = 12;  // Gauss-Legendre points per panel
__constant__ double c_gl_t[QN], c_gl_w[QN], c_gl8_t[8], c_gl8_w[8];

// Element integral of the transient response at time t, added (times w0)
// into o: element (cx, cy, cb, sb, a) with charges q per unit length and
// fluid source qf, receiver (X, Y).
__device__ void elem_transient(const PoroK &K, double X, double Y, double cx, double cy, double cb, double sb,
                               double a, const double q[3], double qf, double t, double w0, double o[4])
{
    double dx = X - cx, dy = Y - cy;
    double xl = dx * cb + dy * sb, yl = dy * cb - dx * sb;
    double ell = sqrt(4.0 * K.c * t);
    double far = 8.0 * fmax(2.0 * a, ell);
    double ox = fabs(xl) - a;
    double d2 = yl * yl + (ox > 0.0 ? ox * ox : 0.0);
    double r[4];
    if (d2 >= far * far) {
        for (int g = 0; g < 8; ++g) {
            double s = a * c_gl8_t[g];
            transient(K, X - (cx + s * cb), Y - (cy + s * sb), t, q, qf, r);
            double w = w0 * a * c_gl8_w[g];
            for (int k = 0; k < 4; ++k) o[k] += w * r[k];
        }
        return;
    }
    double s0 = fmin(a, fmax(-a, xl));
    for (int side = 0; side < 2; ++side) {
        double L = side ? a - s0 : s0 + a;
        if (L <= 0.0) continue;
        int np = 4 + (int)ceil(2.0 * L / ell);
        np = min(np, 400);
        double du = 1.0 / np;
        for (int pn = 0; pn < np; ++pn) {
            for (int g = 0; g < QN; ++g) {
                double u = (pn + 0.5 + 0.5 * c_gl_t[g]) * du;
                double w = w0 * 0.5 * du * c_gl_w[g] * 3.0 * L * u * u;
                double s = side ? s0 + L * u * u * u : s0 - L * u * u * u;
                transient(K, X - (cx + s * cb), Y - (cy + s * sb), t, q, qf, r);
                for (int k = 0; k < 4; ++k) o[k] += w * r[k];
            }
        }
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
            elem_transient(K, X, Y, ecx, ecy, ecb, esb, ea, q, Dq, times[k], 1.0, o);
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

__global__ void k_scale_copy(int m, double a, const double *__restrict__ x, double *__restrict__ y)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) y[e] = a * x[e];
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

bool g_gl_ready[64] = {false};

void upload_rules(int device)
{
    if (device >= 0 && device < 64 && g_gl_ready[device]) return;
    std::vector<double> t, w, t8, w8;
    gauss_legendre(QN, t, w);
    gauss_legendre(8, t8, w8);
    FM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_gl_t), t.data(), QN * 8));
    FM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_gl_w), w.data(), QN * 8));
    FM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_gl8_t), t8.data(), 64));
    FM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_gl8_w), w8.data(), 64));
    if (device >= 0 && device < 64) g_gl_ready[device] = true;
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
    return PoroK{G, p.nu, q.alpha, kap, S, kap / S, eta, ctx->gc};
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

}  // namespace

void poro_apply(fmddm_ctx *ctx, fmddm_tree *t, int lag, const double *D, double *out)
{
    const double dt = ctx->poro.dt;
    const int n = (int)t->n, m3 = 3 * n;
    if (lag == 0) {
        poro_sum(ctx, t, 1, {dt}, D, 0, 0, out);
        return;
    }
    // terms (t1, D) and (t0, -D): the drained parts cancel
    if (t->poro_E.n < (size_t)2 * m3) t->poro_E.alloc((size_t)2 * m3);
    hipStream_t s = ctx->stream;
    hipLaunchKernelGGL(k_scale_copy, dim3(cdiv(m3, 256)), dim3(256), 0, s, m3, 1.0, D, t->poro_E.p);
    hipLaunchKernelGGL(k_scale_copy, dim3(cdiv(m3, 256)), dim3(256), 0, s, m3, -1.0, D, t->poro_E.p + m3);
    FM_CHECK_LAUNCH();
    poro_sum(ctx, t, 2, {(lag + 1) * dt, lag * dt}, t->poro_E.p, -1, 0, out);
}

void poro_history(fmddm_ctx *ctx, fmddm_tree *t, int h, const double *Dh, double *rhs)
{
    if (h < 2) return;
    const double dt = ctx->poro.dt;
    const int n = (int)t->n, m3 = 3 * n;
    if (t->poro_E.n < (size_t)h * m3) t->poro_E.alloc((size_t)h * m3);
    hipStream_t s = ctx->stream;
    hipLaunchKernelGGL(k_hist_terms, dim3(cdiv(m3, 256), h), dim3(256), 0, s, m3, h, Dh, t->poro_E.p);
    FM_CHECK_LAUNCH();
    std::vector<double> times(h);
    for (int j = 1; j <= h; ++j) times[j - 1] = j * dt;
    poro_sum(ctx, t, h, times, t->poro_E.p, -1, 1, rhs);
}

void poro_rhs(fmddm_ctx *ctx, fmddm_tree *t, const double *pf, double SH, double Sh, double *rhs)
{
    int n = (int)t->n;
    hipLaunchKernelGGL(k_poro_rhs, dim3(cdiv(n, 256)), dim3(256), 0, ctx->stream, n, t->ocb.p, t->osb.p, pf,
                       ctx->poro.p0, SH, Sh, rhs);
    FM_CHECK_LAUNCH();
}

}  // namespace fmddm
