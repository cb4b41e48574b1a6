// Constant displacement-discontinuity element (plane strain), device side.
//
// Stress at a receiver from a straight element of half-length a carrying a
// uniform shear (Ds, along the element) and normal (Dn) displacement
// discontinuity, opening-positive, tension-positive stress.  This is the
// influence coefficient A_ij of eqs. 2.3-2.5 for the elastic (drained or
// undrained) part; the paper cites rather than states it, and the classical
// closed form of the constant element is used: with the element on the
// local x-axis over [-a, a], r1^2 = (x-a)^2 + y^2, r2^2 = (x+a)^2 + y^2 and
// f the element integral of -C ln r, C = 1/(4 pi (1 - nu)),
//   sxx = -2G [Ds (2 f_xy + y f_xyy) + Dn (f_yy + y f_yyy)]
//   syy = -2G [Ds (-y f_xyy)        + Dn (f_yy - y f_yyy)]
//   sxy = -2G [Ds (f_yy + y f_yyy)  + Dn (-y f_xyy)]
// (the minus signs convert the classical D = u(-) - u(+) convention to the
// opening-positive one).  Only rational functions of the local coordinates
// appear.
#pragma once

#include <hip/hip_runtime.h>

namespace fmddm {

// 1/x to full double precision: the hardware reciprocal estimate refined by
// two Newton steps (each doubles the correct bits).  Cheaper than the
// correctly rounded division sequence; within an ulp or two of it.
__device__ __forceinline__ double recip(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// Adds the global-frame stress (sxx, syy, sxy) at (X, Y) from the element
// (cx, cy, cb = cos beta, sb = sin beta, a) with DDs (Ds, Dn).
// gc = 2 G C = G / (2 pi (1 - nu)).
__device__ __forceinline__ void elem_stress_add(double X, double Y, double cx, double cy,
                                                double cb, double sb, double a, double Ds,
                                                double Dn, double gc, double &sxx, double &syy,
                                                double &sxy)
{
    double dx = X - cx, dy = Y - cy;
    double x = dx * cb + dy * sb;
    double y = dy * cb - dx * sb;
    double xm = x - a, xp = x + a, y2 = y * y;
    double i1 = recip(xm * xm + y2);
    double i2 = recip(xp * xp + y2);
    double fxy = y * (i1 - i2);
    double fyy = xp * i2 - xm * i1;
    double j1 = i1 * i1, j2 = i2 * i2;
    double fxyy = (xm * xm - y2) * j1 - (xp * xp - y2) * j2;
    double fyyy = 2.0 * y * (xm * j1 - xp * j2);
    double yfxyy = y * fxyy, yfyyy = y * fyyy;
    double lxx = -gc * (Ds * (2.0 * fxy + yfxyy) + Dn * (fyy + yfyyy));
    double lyy = -gc * (Dn * (fyy - yfyyy) - Ds * yfxyy);
    double lxy = -gc * (Ds * (fyy + yfyyy) - Dn * yfxyy);
    // rotate back: sigma = R l R^T, R = [[cb, -sb], [sb, cb]]
    double c2 = cb * cb, s2 = sb * sb, cs = cb * sb;
    sxx += c2 * lxx - 2.0 * cs * lxy + s2 * lyy;
    syy += s2 * lxx + 2.0 * cs * lxy + c2 * lyy;
    sxy += cs * (lxx - lyy) + (c2 - s2) * lxy;
}

// elem_stress_add without the factor -gc (the caller scales the sum once),
// with one reciprocal for both end-point distances (r = 1/(d1 d2) to full
// precision, 1/d1 = d2 r, 1/d2 = d1 r, within two ulp), and the rotation to
// the global frame in double-angle form.  With c2 = cos 2 beta and s2 =
// sin 2 beta of the source (computed once per source by the caller):
//   sxx = m + d c2 - lxy s2,  syy = m - d c2 + lxy s2,  sxy = d s2 + lxy c2,
// m = (lxx + lyy) / 2 = Ds f_xy + Dn f_yy,
// d = (lxx - lyy) / 2 = Ds (f_xy + y f_xyy) + Dn y f_yyy,
// the local-frame stresses l of elem_stress_add.  For the inner loops of
// the near field and the exact product.
__device__ __forceinline__ void elem_stress_unit(double X, double Y, double cx, double cy, double cb, double sb,
                                                 double c2, double s2, double a, double Ds, double Dn, double &sxx,
                                                 double &syy, double &sxy)
{
    double dx = X - cx, dy = Y - cy;
    double x = dx * cb + dy * sb;
    double y = dy * cb - dx * sb;
    double xm = x - a, xp = x + a, y2 = y * y;
    double d1 = xm * xm + y2, d2 = xp * xp + y2;
    double r = recip(d1 * d2);
    double i1 = d2 * r, i2 = d1 * r;
    double fxy = y * (i1 - i2);
    double fyy = xp * i2 - xm * i1;
    double j1 = i1 * i1, j2 = i2 * i2;
    double fxyy = (xm * xm - y2) * j1 - (xp * xp - y2) * j2;
    double yfyyy = 2.0 * y2 * (xm * j1 - xp * j2);
    double yfxyy = y * fxyy;
    double m = Ds * fxy + Dn * fyy;
    double d = Ds * (fxy + yfxyy) + Dn * yfyyy;
    double lxy = Ds * (fyy + yfyyy) - Dn * yfxyy;
    double w = d * c2 - lxy * s2;
    sxx += m + w;
    syy += m - w;
    sxy += d * s2 + lxy * c2;
}

// The same element stress in FP32 arithmetic, for the reduced-precision
// product.  The receiver-element offset (dx, dy) comes in already formed in
// FP64 (coordinates of a 100 m domain would lose the element scale if
// rounded to FP32 first); the local frame, the rational functions and the
// rotation are FP32, with the hardware reciprocal (1 ulp).
__device__ __forceinline__ void elem_stress_add32(float dx, float dy, float cb, float sb, float a, float Ds,
                                                  float Dn, float gc, float &sxx, float &syy, float &sxy)
{
    float x = dx * cb + dy * sb;
    float y = dy * cb - dx * sb;
    float xm = x - a, xp = x + a, y2 = y * y;
    float i1 = __builtin_amdgcn_rcpf(xm * xm + y2);
    float i2 = __builtin_amdgcn_rcpf(xp * xp + y2);
    float fxy = y * (i1 - i2);
    float fyy = xp * i2 - xm * i1;
    float j1 = i1 * i1, j2 = i2 * i2;
    float fxyy = (xm * xm - y2) * j1 - (xp * xp - y2) * j2;
    float fyyy = 2.0f * y * (xm * j1 - xp * j2);
    float yfxyy = y * fxyy, yfyyy = y * fyyy;
    float lxx = -gc * (Ds * (2.0f * fxy + yfxyy) + Dn * (fyy + yfyyy));
    float lyy = -gc * (Dn * (fyy - yfyyy) - Ds * yfxyy);
    float lxy = -gc * (Ds * (fyy + yfyyy) - Dn * yfxyy);
    float c2 = cb * cb, s2 = sb * sb, cs = cb * sb;
    sxx += c2 * lxx - 2.0f * cs * lxy + s2 * lyy;
    syy += s2 * lxx + 2.0f * cs * lxy + c2 * lyy;
    sxy += cs * (lxx - lyy) + (c2 - s2) * lxy;
}

// Shear and normal traction on a receiver with tangent (cb, sb).
__device__ __forceinline__ void traction(double cb, double sb, double sxx, double syy, double sxy,
                                         double &ts, double &tn)
{
    double tx = sxy * cb - sxx * sb;
    double ty = syy * cb - sxy * sb;
    ts = cb * tx + sb * ty;
    tn = cb * ty - sb * tx;
}

// Source charge per unit length: q = (b_x n_x, b_y n_y, b_x n_y + b_y n_x),
// b = Ds s + Dn n, n = (-sb, cb).  The far field of an element is the
// integral along it of the point kernel applied to q.
__device__ __forceinline__ void charge(double cb, double sb, double Ds, double Dn, double &q0,
                                       double &q1, double &q2)
{
    double bx = Ds * cb - Dn * sb, by = Ds * sb + Dn * cb;
    q0 = -bx * sb;
    q1 = by * cb;
    q2 = bx * cb - by * sb;
}

// Point kernel K (3 x 3, row = stress component, column = charge
// component) at offset (x, y), per unit element length: the element
// formulas with the element integral of -C ln r replaced by -C ln r.
// Homogeneous of degree -2.
__device__ __forceinline__ void point_kernel(double x, double y, double gc, double K[9])
{
    double x2 = x * x, y2 = y * y, r2 = x2 + y2;
    double k = -gc / (r2 * r2 * r2);
    double A = -x2 * x2 + 6.0 * x2 * y2 - y2 * y2;
    double B = 3.0 * y2 * y2 - 6.0 * x2 * y2 - x2 * x2;
    double Cc = 3.0 * x2 * x2 - 6.0 * x2 * y2 - y2 * y2;
    double P = 6.0 * x2 * x * y - 2.0 * x * y2 * y;
    double Q = 6.0 * x * y2 * y - 2.0 * x2 * x * y;
    K[0] = k * Cc; K[1] = k * A; K[2] = k * P;
    K[3] = k * A;  K[4] = k * B; K[5] = k * Q;
    K[6] = k * P;  K[7] = k * Q; K[8] = k * A;
}

}  // namespace fmddm
