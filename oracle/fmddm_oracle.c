/*
 * fmddm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU oracle for the fast-multipole displacement
 * discontinuity method (Rezaei, Siddiqui, Bornia, Soliman 2019,
 * arXiv:1812.05087).  Only the test-suite, the smoke check and the CPU
 * baseline of the benchmark call it; the product library never links it and
 * shares no source, header, table or helper with it.
 *
 * Conventions used throughout (the paper does not state them):
 *   - plane strain, isotropic, shear modulus G, Poisson ratio nu;
 *   - stresses are tension-positive;
 *   - a displacement discontinuity is D = u(+) - u(-), where the + face is the
 *     side the element normal n points into, so D_n > 0 is opening;
 *   - element j: midpoint (cx,cy), unit tangent s = (cb,sb) = (cos b, sin b),
 *     unit normal n = (-sb, cb), half-length a;
 *   - the traction at a receiver is t = sigma.n; shear traction s.t,
 *     normal traction n.t;
 *   - vectors are element-major: D[2j] = D_s, D[2j+1] = D_n and
 *     out[2i] = shear traction, out[2i+1] = normal traction.
 *
 * Contents, each following the passage named:
 *   - constant-element influence (the coefficients A_ij of eqs. 2.3-2.5,
 *     whose formulas the paper only cites): the classical constant
 *     displacement-discontinuity element of Crouch & Starfield, written out;
 *   - dense assembly, dense and on-the-fly ("direct") matvec (Section 2);
 *   - restarted GMRES with modified Gram-Schmidt, Gaussian elimination
 *     (Section 4: the linear system of one time step);
 *   - stress intensity factors from tip-element DDs (eq. 2.6);
 *   - quad-tree (Section 3.1): level-0 square, 4-way split of any cell with
 *     more than a prescribed number of points, child order left-to-right then
 *     bottom-to-top, empty children not created;
 *   - neighbour / interaction lists (Section 3.1), extended to an adaptive
 *     tree with the usual U, V, W, X lists;
 *   - black-box FMM with Chebyshev interpolation (Section 3.2): weights at
 *     the leaves (eq. 3.6), M2M (eq. 3.7), M2L (eq. 3.8), L2L (eq. 3.10),
 *     L2P plus direct neighbour interactions (eq. 3.11).
 *
 * Nothing here is blocked, fused or reordered for speed; OpenMP is used only
 * to spread independent rows over host cores.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Constant displacement-discontinuity element (plane strain).               */
/* ------------------------------------------------------------------------ */

/* Stress (sxx, syy, sxy) at local point (x, y) induced by an element lying
 * on the local x-axis over [-a, a] carrying shear DD Ds (along x) and normal
 * DD Dn (along y), opening-positive.  The classical formulas are written for
 * the opposite sign convention (D = u(-) - u(+)); the two DDs are negated
 * first.  f below is the integral over the element of -C ln r,
 * C = 1/(4 pi (1-nu)); only its second and third derivatives enter. */
void ora_elem_stress_local(double x, double y, double a, double G, double nu,
                           double Ds, double Dn, double out[3])
{
    const double C = 1.0 / (4.0 * M_PI * (1.0 - nu));
    double xm = x - a, xp = x + a;
    double r1 = xm * xm + y * y;
    double r2 = xp * xp + y * y;
    double fxy = C * (y / r1 - y / r2);
    double fxx = C * (xm / r1 - xp / r2);
    double fyy = -fxx;
    double fxyy = C * ((xm * xm - y * y) / (r1 * r1) - (xp * xp - y * y) / (r2 * r2));
    double fyyy = 2.0 * C * y * (xm / (r1 * r1) - xp / (r2 * r2));
    double Dx = -Ds, Dy = -Dn;
    out[0] = 2.0 * G * (Dx * (2.0 * fxy + y * fxyy) + Dy * (fyy + y * fyyy));
    out[1] = 2.0 * G * (Dx * (-y * fxyy) + Dy * (fyy - y * fyyy));
    out[2] = 2.0 * G * (Dx * (fyy + y * fyyy) + Dy * (-y * fxyy));
}

/* Global stress at (X, Y) from element (cx, cy, cb, sb, a). */
void ora_elem_stress(double X, double Y, double cx, double cy, double cb,
                     double sb, double a, double G, double nu, double Ds,
                     double Dn, double sg[3])
{
    double dx = X - cx, dy = Y - cy;
    double x = dx * cb + dy * sb;
    double y = -dx * sb + dy * cb;
    double sl[3];
    ora_elem_stress_local(x, y, a, G, nu, Ds, Dn, sl);
    /* sigma = R sl R^T with R = [s | n] = [[cb, -sb], [sb, cb]] */
    sg[0] = cb * cb * sl[0] - 2.0 * cb * sb * sl[2] + sb * sb * sl[1];
    sg[1] = sb * sb * sl[0] + 2.0 * cb * sb * sl[2] + cb * cb * sl[1];
    sg[2] = cb * sb * (sl[0] - sl[1]) + (cb * cb - sb * sb) * sl[2];
}

/* Shear and normal traction on a receiver with tangent (cbi, sbi). */
void ora_traction(double cbi, double sbi, const double sg[3], double *ts,
                  double *tn)
{
    double tx = -sbi * sg[0] + cbi * sg[2];
    double ty = -sbi * sg[2] + cbi * sg[1];
    *ts = cbi * tx + sbi * ty;
    *tn = -sbi * tx + cbi * ty;
}

/* Point kernel: stress per unit element length at offset (x, y) from a
 * source point, as a 3x3 map K[out*3+in] from the source "charge"
 * q = (b_x n_x, b_y n_y, b_x n_y + b_y n_x), b = Ds s + Dn n, to
 * (sxx, syy, sxy).  Obtained from the element formulas by replacing the
 * element integral of -C ln r with -C ln r itself (so the element stress is
 * the integral of this kernel along the element); the e_xx column follows
 * from the e_yy column by reflection about the line y = x. */
void ora_point_kernel(double x, double y, double G, double nu, double K[9])
{
    const double C = 1.0 / (4.0 * M_PI * (1.0 - nu));
    double x2 = x * x, y2 = y * y;
    double r2 = x2 + y2;
    double k = -2.0 * G * C / (r2 * r2 * r2);
    double A = -x2 * x2 + 6.0 * x2 * y2 - y2 * y2;
    double B = 3.0 * y2 * y2 - 6.0 * x2 * y2 - x2 * x2;
    double Cc = 3.0 * x2 * x2 - 6.0 * x2 * y2 - y2 * y2;
    double P = 6.0 * x2 * x * y - 2.0 * x * y2 * y;
    double Q = -2.0 * x2 * x * y + 6.0 * x * y2 * y;
    K[0] = k * Cc; K[1] = k * A; K[2] = k * P;
    K[3] = k * A;  K[4] = k * B; K[5] = k * Q;
    K[6] = k * P;  K[7] = k * Q; K[8] = k * A;
}

/* Source charge of an element per unit length. */
void ora_charge(double cb, double sb, double Ds, double Dn, double q[3])
{
    double bx = Ds * cb - Dn * sb, by = Ds * sb + Dn * cb;
    double nx = -sb, ny = cb;
    q[0] = bx * nx;
    q[1] = by * ny;
    q[2] = bx * ny + by * nx;
}

/* A polynomial test kernel of degree <= 3 in each offset coordinate.  With
 * it every far-field step of the Chebyshev FMM is exact once p >= 4, so the
 * FMM must equal the dense product up to rounding. */
static void poly_kernel(double x, double y, double K[9])
{
    double px[4] = {1.0, x, x * x, x * x * x};
    double py[4] = {1.0, y, y * y, y * y * y};
    for (int c = 0; c < 9; ++c) {
        double s = 0.0;
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                /* fixed, arbitrary coefficients in [-1, 1] */
                double coef = sin(1.0 + 3.0 * c + 1.7 * i + 0.9 * j + 0.37 * i * j);
                s += coef * px[i] * py[j];
            }
        K[c] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre nodes on [-1, 1] by Newton iteration on P_n.               */
/* ------------------------------------------------------------------------ */
void ora_gauss_legendre(int n, double *t, double *w)
{
    for (int i = 0; i < n; ++i) {
        double x = cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = x; p0 = 1.0; }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = x; p0 = 1.0; }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
        }
        t[i] = x;
        w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

/* ------------------------------------------------------------------------ */
/* Chebyshev interpolation (Section 3.2.1).                                  */
/*   nodes: roots of T_p, xbar_l = cos((2l-1) pi / (2p)), l = 1..p           */
/*   S_p(xbar_l, x) = 1/p + (2/p) sum_{k=1}^{p-1} T_k(xbar_l) T_k(x)          */
/* ------------------------------------------------------------------------ */
void ora_cheb_nodes(int p, double *xb)
{
    for (int l = 0; l < p; ++l) xb[l] = cos((2.0 * l + 1.0) * M_PI / (2.0 * p));
}

double ora_cheb_S(int p, int l, double x)
{
    double node_angle = (2.0 * l + 1.0) * M_PI / (2.0 * p);
    double s = 1.0 / p;
    double t0 = 1.0, t1 = x;
    for (int k = 1; k < p; ++k) {
        s += (2.0 / p) * cos(k * node_angle) * t1;
        double t2 = 2.0 * x * t1 - t0;
        t0 = t1;
        t1 = t2;
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Dense influence matrix, direct matvec.                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    const double *cx, *cy, *cb, *sb, *a;
    double G, nu;
} geom_t;

/* Traction (ts, tn) at receiver i from element j carrying (Ds, Dn). */
static void pair_traction(const geom_t *g, int64_t i, int64_t j, double Ds,
                          double Dn, double *ts, double *tn)
{
    double sg[3];
    ora_elem_stress(g->cx[i], g->cy[i], g->cx[j], g->cy[j], g->cb[j], g->sb[j],
                    g->a[j], g->G, g->nu, Ds, Dn, sg);
    ora_traction(g->cb[i], g->sb[i], sg, ts, tn);
}

/* A is (2n x 2n) row-major: A[(2i+r)*2n + 2j+c]. */
void ora_dense_matrix(int64_t n, const double *cx, const double *cy,
                      const double *cb, const double *sb, const double *a,
                      double G, double nu, double *A)
{
    geom_t g = {n, cx, cy, cb, sb, a, G, nu};
    int64_t ld = 2 * n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double ts, tn;
            pair_traction(&g, i, j, 1.0, 0.0, &ts, &tn);
            A[(2 * i) * ld + 2 * j] = ts;
            A[(2 * i + 1) * ld + 2 * j] = tn;
            pair_traction(&g, i, j, 0.0, 1.0, &ts, &tn);
            A[(2 * i) * ld + 2 * j + 1] = ts;
            A[(2 * i + 1) * ld + 2 * j + 1] = tn;
        }
    }
}

void ora_dense_matvec(int64_t m, const double *A, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < m; ++j) s += A[i * m + j] * x[j];
        y[i] = s;
    }
}

/* Rows [r0, r1) of the on-the-fly product: out[2i], out[2i+1] for i in range */
void ora_direct_matvec_rows(int64_t n, const double *cx, const double *cy,
                            const double *cb, const double *sb, const double *a,
                            double G, double nu, const double *D, double *out,
                            int64_t r0, int64_t r1)
{
    geom_t g = {n, cx, cy, cb, sb, a, G, nu};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = r0; i < r1; ++i) {
        double s = 0.0, t = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double sg[3];
            ora_elem_stress(g.cx[i], g.cy[i], g.cx[j], g.cy[j], g.cb[j], g.sb[j],
                            g.a[j], G, nu, D[2 * j], D[2 * j + 1], sg);
            double ts, tn;
            ora_traction(g.cb[i], g.sb[i], sg, &ts, &tn);
            s += ts;
            t += tn;
        }
        out[2 * i] = s;
        out[2 * i + 1] = t;
    }
}

void ora_direct_matvec(int64_t n, const double *cx, const double *cy,
                       const double *cb, const double *sb, const double *a,
                       double G, double nu, const double *D, double *out)
{
    ora_direct_matvec_rows(n, cx, cy, cb, sb, a, G, nu, D, out, 0, n);
}

/* Selected rows of the on-the-fly product: out[2k], out[2k+1] for
 * receiver idx[k], k < nidx (for sampled checks at full size). */
void ora_direct_matvec_idx(int64_t n, const double *cx, const double *cy,
                           const double *cb, const double *sb, const double *a,
                           double G, double nu, const double *D, int64_t nidx,
                           const int64_t *idx, double *out)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < nidx; ++k) {
        int64_t i = idx[k];
        double s = 0.0, t = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double sg[3];
            ora_elem_stress(cx[i], cy[i], cx[j], cy[j], cb[j], sb[j], a[j], G, nu,
                            D[2 * j], D[2 * j + 1], sg);
            double ts, tn;
            ora_traction(cb[i], sb[i], sg, &ts, &tn);
            s += ts;
            t += tn;
        }
        out[2 * k] = s;
        out[2 * k + 1] = t;
    }
}

/* Dense matrix of the polynomial test kernel: element integrals by
 * 8-point Gauss-Legendre (exact for the degree-3 kernel). */
void ora_dense_matrix_poly(int64_t n, const double *cx, const double *cy,
                           const double *cb, const double *sb, const double *a,
                           double *A)
{
    double t[8], w[8];
    ora_gauss_legendre(8, t, w);
    int64_t ld = 2 * n;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            for (int c = 0; c < 2; ++c) {
                double q[3];
                ora_charge(cb[j], sb[j], c == 0 ? 1.0 : 0.0, c == 1 ? 1.0 : 0.0, q);
                double sg[3] = {0, 0, 0};
                for (int gq = 0; gq < 8; ++gq) {
                    double xi = a[j] * t[gq];
                    double K[9];
                    poly_kernel(cx[i] - (cx[j] + xi * cb[j]), cy[i] - (cy[j] + xi * sb[j]), K);
                    for (int r = 0; r < 3; ++r)
                        for (int s = 0; s < 3; ++s) sg[r] += a[j] * w[gq] * K[r * 3 + s] * q[s];
                }
                double ts, tn;
                ora_traction(cb[i], sb[i], sg, &ts, &tn);
                A[(2 * i) * ld + 2 * j + c] = ts;
                A[(2 * i + 1) * ld + 2 * j + c] = tn;
            }
}

/* ------------------------------------------------------------------------ */
/* Dense linear algebra: Gaussian elimination, restarted GMRES (MGS).        */
/* ------------------------------------------------------------------------ */
int ora_lu_solve(int64_t m, const double *A_in, const double *b, double *x)
{
    double *A = (double *)malloc(sizeof(double) * m * m);
    double *r = (double *)malloc(sizeof(double) * m);
    if (!A || !r) { free(A); free(r); return -2; }
    memcpy(A, A_in, sizeof(double) * m * m);
    memcpy(r, b, sizeof(double) * m);
    for (int64_t k = 0; k < m; ++k) {
        int64_t piv = k;
        for (int64_t i = k + 1; i < m; ++i)
            if (fabs(A[i * m + k]) > fabs(A[piv * m + k])) piv = i;
        if (A[piv * m + k] == 0.0) { free(A); free(r); return -1; }
        if (piv != k) {
            for (int64_t j = 0; j < m; ++j) {
                double tmp = A[k * m + j];
                A[k * m + j] = A[piv * m + j];
                A[piv * m + j] = tmp;
            }
            double tmp = r[k]; r[k] = r[piv]; r[piv] = tmp;
        }
        for (int64_t i = k + 1; i < m; ++i) {
            double f = A[i * m + k] / A[k * m + k];
            for (int64_t j = k; j < m; ++j) A[i * m + j] -= f * A[k * m + j];
            r[i] -= f * r[k];
        }
    }
    for (int64_t i = m - 1; i >= 0; --i) {
        double s = r[i];
        for (int64_t j = i + 1; j < m; ++j) s -= A[i * m + j] * x[j];
        x[i] = s / A[i * m + i];
    }
    free(A);
    free(r);
    return 0;
}

typedef void (*matvec_fn)(void *ctx, const double *x, double *y);

static double dot(int64_t m, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < m; ++i) s += a[i] * b[i];
    return s;
}

/* Right-restarted GMRES(restart), modified Gram-Schmidt, Givens rotations.
 * Stops when ||b - A x|| <= tol ||b|| (checked on the true residual at each
 * restart) or after maxit matvecs.  x holds the initial guess on entry.
 * Returns 0 when converged, 1 otherwise. */
static int gmres(int64_t m, matvec_fn mv, void *ctx, const double *b, double *x,
                 int restart, double tol, int maxit, int *iters, double *relres)
{
    double *V = (double *)calloc((size_t)(restart + 1) * m, sizeof(double));
    double *H = (double *)calloc((size_t)(restart + 1) * restart, sizeof(double));
    double *cs = (double *)calloc(restart, sizeof(double));
    double *sn = (double *)calloc(restart, sizeof(double));
    double *gv = (double *)calloc(restart + 1, sizeof(double));
    double *yv = (double *)calloc(restart, sizeof(double));
    double *w = (double *)calloc(m, sizeof(double));
    int it = 0, conv = 0;
    double bnorm = sqrt(dot(m, b, b));
    double rel = 0.0;
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < m; ++i) x[i] = 0.0;
        conv = 1;
        goto done;
    }
    for (;;) {
        mv(ctx, x, w);
        for (int64_t i = 0; i < m; ++i) w[i] = b[i] - w[i];
        double beta = sqrt(dot(m, w, w));
        rel = beta / bnorm;
        if (rel <= tol) { conv = 1; break; }
        if (it >= maxit) break;
        for (int64_t i = 0; i < m; ++i) V[i] = w[i] / beta;
        for (int k = 0; k <= restart; ++k) gv[k] = 0.0;
        gv[0] = beta;
        int k = 0;
        for (int j = 0; j < restart && it < maxit; ++j) {
            double *vj = V + (size_t)j * m, *vn = V + (size_t)(j + 1) * m;
            mv(ctx, vj, w);
            ++it;
            for (int i = 0; i <= j; ++i) {
                double h = dot(m, w, V + (size_t)i * m);
                H[i * restart + j] = h;
                for (int64_t t = 0; t < m; ++t) w[t] -= h * V[(size_t)i * m + t];
            }
            double hn = sqrt(dot(m, w, w));
            H[(j + 1) * restart + j] = hn;
            if (hn != 0.0)
                for (int64_t t = 0; t < m; ++t) vn[t] = w[t] / hn;
            for (int i = 0; i < j; ++i) {
                double h0 = H[i * restart + j], h1 = H[(i + 1) * restart + j];
                H[i * restart + j] = cs[i] * h0 + sn[i] * h1;
                H[(i + 1) * restart + j] = -sn[i] * h0 + cs[i] * h1;
            }
            double h0 = H[j * restart + j], h1 = H[(j + 1) * restart + j];
            double den = sqrt(h0 * h0 + h1 * h1);
            cs[j] = den == 0.0 ? 1.0 : h0 / den;
            sn[j] = den == 0.0 ? 0.0 : h1 / den;
            H[j * restart + j] = den;
            H[(j + 1) * restart + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            k = j + 1;
            if (fabs(gv[j + 1]) <= tol * bnorm || hn == 0.0) break;
        }
        for (int i = k - 1; i >= 0; --i) {
            double s = gv[i];
            for (int jj = i + 1; jj < k; ++jj) s -= H[i * restart + jj] * yv[jj];
            yv[i] = s / H[i * restart + i];
        }
        for (int i = 0; i < k; ++i)
            for (int64_t t = 0; t < m; ++t) x[t] += yv[i] * V[(size_t)i * m + t];
    }
done:
    *iters = it;
    *relres = rel;
    free(V); free(H); free(cs); free(sn); free(gv); free(yv); free(w);
    return conv ? 0 : 1;
}

typedef struct { int64_t m; const double *A; } dense_ctx;
static void dense_mv(void *c, const double *x, double *y)
{
    dense_ctx *d = (dense_ctx *)c;
    ora_dense_matvec(d->m, d->A, x, y);
}

int ora_gmres_dense(int64_t m, const double *A, const double *b, double *x,
                    int restart, double tol, int maxit, int *iters, double *relres)
{
    dense_ctx d = {m, A};
    return gmres(m, dense_mv, &d, b, x, restart, tol, maxit, iters, relres);
}

typedef struct { geom_t g; } direct_ctx;
static void direct_mv(void *c, const double *x, double *y)
{
    direct_ctx *d = (direct_ctx *)c;
    ora_direct_matvec(d->g.n, d->g.cx, d->g.cy, d->g.cb, d->g.sb, d->g.a, d->g.G,
                      d->g.nu, x, y);
}

int ora_gmres_direct(int64_t n, const double *cx, const double *cy,
                     const double *cb, const double *sb, const double *a,
                     double G, double nu, const double *b, double *x,
                     int restart, double tol, int maxit, int *iters, double *relres)
{
    direct_ctx d = {{n, cx, cy, cb, sb, a, G, nu}};
    return gmres(2 * n, direct_mv, &d, b, x, restart, tol, maxit, iters, relres);
}

/* ------------------------------------------------------------------------ */
/* Right-hand side of one elastic step (Section 4): the far field           */
/* (compression-positive SH along x, Sh along y) resolved on each element    */
/* and the fluid pressure on the faces.  The induced tractions must cancel   */
/* the far field and balance the pressure: t_induced = -p n - sigma_inf n.   */
/* ------------------------------------------------------------------------ */
void ora_rhs(int64_t n, const double *cb, const double *sb, const double *pf,
             double SH, double Sh, double *rhs)
{
    for (int64_t i = 0; i < n; ++i) {
        double sg[3] = {-SH, -Sh, 0.0};
        double ts, tn;
        ora_traction(cb[i], sb[i], sg, &ts, &tn);
        rhs[2 * i] = -ts;
        rhs[2 * i + 1] = -pf[i] - tn;
    }
}

/* Stress intensity factors from the tip-element DDs, eq. 2.6; a is read as
 * the tip element's half-length. */
void ora_sif(double E, double nu, double a, double Ds, double Dn, double *KI,
             double *KII)
{
    double f = 0.806 * E / (4.0 * (1.0 - nu * nu)) * sqrt(M_PI / (2.0 * a));
    *KI = f * Dn;
    *KII = f * Ds;
}

/* ------------------------------------------------------------------------ */
/* Quad-tree (Section 3.1).                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    double x0, y0, L;
    int leaf, cap;
    double kappa;
    int64_t *perm;       /* sorted position -> element index */
    uint64_t *key;       /* Morton key, sorted order */
    int64_t ncell, capcell;
    int32_t *level, *parent, *child, *isleaf;
    uint32_t *ix, *iy;
    int64_t *pbeg, *pend;
    /* lists, CSR over cells */
    int64_t *off[4];
    int32_t *lst[4];
} ora_tree;

enum { LIST_U = 0, LIST_V = 1, LIST_W = 2, LIST_X = 3 };

static uint64_t spread_bits(uint64_t v)
{
    uint64_t r = 0;
    for (int b = 0; b < 32; ++b) r |= ((v >> b) & 1ull) << (2 * b);
    return r;
}

static const uint64_t QMAX = 2147483647ull; /* 2^31 - 1 */

static uint64_t quantise(double x, double x0, double scale)
{
    double t = (x - x0) * scale;
    if (!(t > 0.0)) return 0;
    if (t >= 2147483647.0) return QMAX;
    return (uint64_t)t;
}

typedef struct { uint64_t key; int64_t idx; } kv_t;
static int kv_cmp(const void *a, const void *b)
{
    const kv_t *x = (const kv_t *)a, *y = (const kv_t *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}

static void tree_push(ora_tree *t, int32_t lvl, uint32_t ix, uint32_t iy,
                      int32_t par, int64_t b, int64_t e)
{
    if (t->ncell == t->capcell) {
        t->capcell = t->capcell ? 2 * t->capcell : 64;
        t->level = (int32_t *)realloc(t->level, sizeof(int32_t) * t->capcell);
        t->parent = (int32_t *)realloc(t->parent, sizeof(int32_t) * t->capcell);
        t->child = (int32_t *)realloc(t->child, sizeof(int32_t) * 4 * t->capcell);
        t->isleaf = (int32_t *)realloc(t->isleaf, sizeof(int32_t) * t->capcell);
        t->ix = (uint32_t *)realloc(t->ix, sizeof(uint32_t) * t->capcell);
        t->iy = (uint32_t *)realloc(t->iy, sizeof(uint32_t) * t->capcell);
        t->pbeg = (int64_t *)realloc(t->pbeg, sizeof(int64_t) * t->capcell);
        t->pend = (int64_t *)realloc(t->pend, sizeof(int64_t) * t->capcell);
    }
    int64_t c = t->ncell++;
    t->level[c] = lvl;
    t->ix[c] = ix;
    t->iy[c] = iy;
    t->parent[c] = par;
    for (int k = 0; k < 4; ++k) t->child[4 * c + k] = -1;
    t->isleaf[c] = 1;
    t->pbeg[c] = b;
    t->pend[c] = e;
}

/* Build the tree over element midpoints (xm, ym) with half-lengths a.
 * Root square: (bx0, by0, bL) when use_box, else x0 = min x, y0 = min y,
 * L = max extent (1 when all points coincide).  A cell splits when it holds
 * more than `leaf` points, its level is below `cap`, and its children would
 * still be at least kappa element half-lengths wide for every element it
 * holds (so an element never reaches far outside the cell it is filed in).
 * Returns NULL when a point lies outside a user box. */
ora_tree *ora_tree_build(int64_t n, const double *xm, const double *ym,
                         const double *a, int leaf, int cap, double kappa,
                         int use_box, double bx0, double by0, double bL)
{
    if (n <= 0 || leaf < 1 || cap < 0 || cap > 30) return NULL;
    ora_tree *t = (ora_tree *)calloc(1, sizeof(ora_tree));
    t->n = n;
    t->leaf = leaf;
    t->cap = cap;
    t->kappa = kappa;
    if (use_box) {
        t->x0 = bx0; t->y0 = by0; t->L = bL;
        for (int64_t i = 0; i < n; ++i)
            if (!(xm[i] >= bx0 && xm[i] <= bx0 + bL && ym[i] >= by0 && ym[i] <= by0 + bL)) {
                free(t);
                return NULL;
            }
    } else {
        double xmin = xm[0], xmax = xm[0], ymin = ym[0], ymax = ym[0];
        for (int64_t i = 1; i < n; ++i) {
            if (xm[i] < xmin) xmin = xm[i];
            if (xm[i] > xmax) xmax = xm[i];
            if (ym[i] < ymin) ymin = ym[i];
            if (ym[i] > ymax) ymax = ym[i];
        }
        t->x0 = xmin;
        t->y0 = ymin;
        double dx = xmax - xmin, dy = ymax - ymin;
        t->L = dx > dy ? dx : dy;
        if (t->L == 0.0) t->L = 1.0;
    }
    double scale = 2147483648.0 / t->L;
    kv_t *kv = (kv_t *)malloc(sizeof(kv_t) * n);
    for (int64_t i = 0; i < n; ++i) {
        uint64_t qx = quantise(xm[i], t->x0, scale);
        uint64_t qy = quantise(ym[i], t->y0, scale);
        kv[i].key = spread_bits(qx) | (spread_bits(qy) << 1);
        kv[i].idx = i;
    }
    qsort(kv, n, sizeof(kv_t), kv_cmp);
    t->perm = (int64_t *)malloc(sizeof(int64_t) * n);
    t->key = (uint64_t *)malloc(sizeof(uint64_t) * n);
    for (int64_t i = 0; i < n; ++i) {
        t->perm[i] = kv[i].idx;
        t->key[i] = kv[i].key;
    }
    free(kv);

    tree_push(t, 0, 0, 0, -1, 0, n);
    for (int64_t c = 0; c < t->ncell; ++c) {
        int lvl = t->level[c];
        int64_t b = t->pbeg[c], e = t->pend[c];
        double amax = 0.0;
        for (int64_t k = b; k < e; ++k)
            if (a[t->perm[k]] > amax) amax = a[t->perm[k]];
        double child_side = ldexp(t->L, -(lvl + 1));
        if (!(e - b > leaf && lvl < cap && child_side >= kappa * amax)) continue;
        t->isleaf[c] = 0;
        int sh = 62 - 2 * (lvl + 1);
        int64_t k = b;
        for (int d = 0; d < 4; ++d) {
            int64_t s = k;
            while (k < e && (int)((t->key[k] >> sh) & 3ull) == d) ++k;
            if (k > s) {
                uint32_t cix = 2 * t->ix[c] + (uint32_t)(d & 1);
                uint32_t ciy = 2 * t->iy[c] + (uint32_t)(d >> 1);
                t->child[4 * c + d] = (int32_t)t->ncell;
                tree_push(t, lvl + 1, cix, ciy, (int32_t)c, s, k);
            }
        }
    }
    return t;
}

int64_t ora_tree_ncell(const ora_tree *t) { return t->ncell; }

void ora_tree_export(const ora_tree *t, int64_t *perm, uint64_t *key,
                     int32_t *level, uint32_t *ix, uint32_t *iy, int32_t *parent,
                     int32_t *child, int64_t *pbeg, int64_t *pend,
                     int32_t *isleaf, double *root)
{
    memcpy(perm, t->perm, sizeof(int64_t) * t->n);
    memcpy(key, t->key, sizeof(uint64_t) * t->n);
    memcpy(level, t->level, sizeof(int32_t) * t->ncell);
    memcpy(ix, t->ix, sizeof(uint32_t) * t->ncell);
    memcpy(iy, t->iy, sizeof(uint32_t) * t->ncell);
    memcpy(parent, t->parent, sizeof(int32_t) * t->ncell);
    memcpy(child, t->child, sizeof(int32_t) * 4 * t->ncell);
    memcpy(pbeg, t->pbeg, sizeof(int64_t) * t->ncell);
    memcpy(pend, t->pend, sizeof(int64_t) * t->ncell);
    memcpy(isleaf, t->isleaf, sizeof(int32_t) * t->ncell);
    root[0] = t->x0;
    root[1] = t->y0;
    root[2] = t->L;
}

void ora_tree_free(ora_tree *t)
{
    if (!t) return;
    free(t->perm); free(t->key); free(t->level); free(t->parent); free(t->child);
    free(t->isleaf); free(t->ix); free(t->iy); free(t->pbeg); free(t->pend);
    for (int k = 0; k < 4; ++k) { free(t->off[k]); free(t->lst[k]); }
    free(t);
}

/* Closed squares of cells c and d share at least one point. */
static int adjacent(const ora_tree *t, int64_t c, int64_t d)
{
    int lc = t->level[c], ld = t->level[d];
    int lm = lc > ld ? lc : ld;
    uint64_t cx0 = (uint64_t)t->ix[c] << (lm - lc), cx1 = ((uint64_t)t->ix[c] + 1) << (lm - lc);
    uint64_t cy0 = (uint64_t)t->iy[c] << (lm - lc), cy1 = ((uint64_t)t->iy[c] + 1) << (lm - lc);
    uint64_t dx0 = (uint64_t)t->ix[d] << (lm - ld), dx1 = ((uint64_t)t->ix[d] + 1) << (lm - ld);
    uint64_t dy0 = (uint64_t)t->iy[d] << (lm - ld), dy1 = ((uint64_t)t->iy[d] + 1) << (lm - ld);
    return cx0 <= dx1 && dx0 <= cx1 && cy0 <= dy1 && dy0 <= cy1;
}

/* Membership tests, straight from the list definitions:
 *   U(B), B leaf:  leaves adjacent to B (B included);
 *   V(B):          cells at B's level, not adjacent to B, whose parent is
 *                  adjacent to B's parent (children of the parent's
 *                  neighbours that are well separated from B);
 *   W(B), B leaf:  cells A finer than B, not adjacent to B, whose parent is
 *                  adjacent to B;
 *   X(A):          leaves B with A in W(B). */
static int in_list(const ora_tree *t, int which, int64_t b, int64_t a)
{
    switch (which) {
    case LIST_U:
        return t->isleaf[b] && t->isleaf[a] && adjacent(t, a, b);
    case LIST_V:
        return b != 0 && t->level[a] == t->level[b] && !adjacent(t, a, b) &&
               adjacent(t, t->parent[a], t->parent[b]);
    case LIST_W:
        return t->isleaf[b] && t->level[a] > t->level[b] && !adjacent(t, a, b) &&
               adjacent(t, t->parent[a], b);
    case LIST_X:
        return t->isleaf[a] && t->level[b] > t->level[a] && !adjacent(t, b, a) &&
               adjacent(t, t->parent[b], a);
    }
    return 0;
}

/* Brute force over all cell pairs; lists come out sorted by cell index,
 * i.e. by (level, Morton key). */
void ora_lists_build(ora_tree *t)
{
    int64_t nc = t->ncell;
    for (int w = 0; w < 4; ++w) {
        free(t->off[w]);
        free(t->lst[w]);
        t->off[w] = (int64_t *)calloc(nc + 1, sizeof(int64_t));
        for (int64_t b = 0; b < nc; ++b) {
            int64_t cnt = 0;
            for (int64_t a = 0; a < nc; ++a) cnt += in_list(t, w, b, a);
            t->off[w][b + 1] = t->off[w][b] + cnt;
        }
        t->lst[w] = (int32_t *)malloc(sizeof(int32_t) * (t->off[w][nc] + 1));
        for (int64_t b = 0; b < nc; ++b) {
            int64_t k = t->off[w][b];
            for (int64_t a = 0; a < nc; ++a)
                if (in_list(t, w, b, a)) t->lst[w][k++] = (int32_t)a;
        }
    }
}

int64_t ora_list_size(const ora_tree *t, int which) { return t->off[which][t->ncell]; }

void ora_list_export(const ora_tree *t, int which, int64_t *off, int32_t *idx)
{
    memcpy(off, t->off[which], sizeof(int64_t) * (t->ncell + 1));
    memcpy(idx, t->lst[which], sizeof(int32_t) * t->off[which][t->ncell]);
}

/* ------------------------------------------------------------------------ */
/* Black-box FMM (Section 3.2) on the tree and lists above.                  */
/* kernel: 0 = elastic element kernel (far field: point kernel integrated    */
/* along each source element), 1 = polynomial test kernel.                   */
/* ------------------------------------------------------------------------ */
static void cell_geom(const ora_tree *t, int64_t c, double *ccx, double *ccy, double *h)
{
    double side = ldexp(t->L, -t->level[c]);
    *ccx = t->x0 + (t->ix[c] + 0.5) * side;
    *ccy = t->y0 + (t->iy[c] + 0.5) * side;
    *h = 0.5 * side;
}

/* Global stress at a receiver from one element, for either kernel. */
static void near_stress(int kernel, double X, double Y, int64_t j, const geom_t *g,
                        const double *D, const double *gt, const double *gw, int ng,
                        double sg[3])
{
    if (kernel == 0) {
        ora_elem_stress(X, Y, g->cx[j], g->cy[j], g->cb[j], g->sb[j], g->a[j],
                        g->G, g->nu, D[2 * j], D[2 * j + 1], sg);
        return;
    }
    double q[3];
    ora_charge(g->cb[j], g->sb[j], D[2 * j], D[2 * j + 1], q);
    sg[0] = sg[1] = sg[2] = 0.0;
    for (int k = 0; k < ng; ++k) {
        double xi = g->a[j] * gt[k];
        double K[9];
        poly_kernel(X - (g->cx[j] + xi * g->cb[j]), Y - (g->cy[j] + xi * g->sb[j]), K);
        for (int r = 0; r < 3; ++r)
            for (int s = 0; s < 3; ++s) sg[r] += g->a[j] * gw[k] * K[r * 3 + s] * q[s];
    }
}

int ora_fmm_apply(const ora_tree *t, const double *cx, const double *cy,
                  const double *cb, const double *sb, const double *a, double G,
                  double nu, int p, int kernel, const double *D, double *out)
{
    if (p < 1 || p > 64) return -1;
    geom_t g = {t->n, cx, cy, cb, sb, a, G, nu};
    int64_t nc = t->ncell, p2 = (int64_t)p * p;
    double *W = (double *)calloc((size_t)nc * 3 * p2, sizeof(double));
    double *F = (double *)calloc((size_t)nc * 3 * p2, sizeof(double));
    double *xb = (double *)malloc(sizeof(double) * p);
    double *gt = (double *)malloc(sizeof(double) * p);
    double *gw = (double *)malloc(sizeof(double) * p);
    double *Sx = (double *)malloc(sizeof(double) * p);
    double *Sy = (double *)malloc(sizeof(double) * p);
    double nt[8], nw[8];
    ora_cheb_nodes(p, xb);
    ora_gauss_legendre(p, gt, gw);
    ora_gauss_legendre(8, nt, nw);
    int maxlvl = 0;
    for (int64_t c = 0; c < nc; ++c)
        if (t->level[c] > maxlvl) maxlvl = t->level[c];

    /* Upward pass, leaves (eq. 3.6): weights at the Chebyshev nodes of the
     * leaf, each source element integrated along its length with p-point
     * Gauss-Legendre, exact since S_p restricted to a segment is a
     * polynomial of degree 2(p-1). */
    for (int64_t c = 0; c < nc; ++c) {
        if (!t->isleaf[c]) continue;
        double ccx, ccy, h;
        cell_geom(t, c, &ccx, &ccy, &h);
        for (int64_t k = t->pbeg[c]; k < t->pend[c]; ++k) {
            int64_t j = t->perm[k];
            double q[3];
            ora_charge(cb[j], sb[j], D[2 * j], D[2 * j + 1], q);
            for (int gq = 0; gq < p; ++gq) {
                double xi = a[j] * gt[gq], wq = a[j] * gw[gq];
                double u = (cx[j] + xi * cb[j] - ccx) / h;
                double v = (cy[j] + xi * sb[j] - ccy) / h;
                for (int l = 0; l < p; ++l) Sx[l] = ora_cheb_S(p, l, u);
                for (int m = 0; m < p; ++m) Sy[m] = ora_cheb_S(p, m, v);
                for (int comp = 0; comp < 3; ++comp)
                    for (int l = 0; l < p; ++l)
                        for (int m = 0; m < p; ++m)
                            W[(c * 3 + comp) * p2 + l * p + m] += wq * q[comp] * Sx[l] * Sy[m];
            }
        }
    }
    /* Upward pass, M2M (eq. 3.7), finest level first. */
    for (int lvl = maxlvl - 1; lvl >= 0; --lvl)
        for (int64_t c = 0; c < nc; ++c) {
            if (t->level[c] != lvl || t->isleaf[c]) continue;
            double ccx, ccy, h;
            cell_geom(t, c, &ccx, &ccy, &h);
            for (int d = 0; d < 4; ++d) {
                int64_t k = t->child[4 * c + d];
                if (k < 0) continue;
                double kx, ky, kh;
                cell_geom(t, k, &kx, &ky, &kh);
                for (int comp = 0; comp < 3; ++comp)
                    for (int l = 0; l < p; ++l)
                        for (int m = 0; m < p; ++m) {
                            double s = 0.0;
                            for (int l2 = 0; l2 < p; ++l2)
                                for (int m2 = 0; m2 < p; ++m2) {
                                    double u = (kx + kh * xb[l2] - ccx) / h;
                                    double v = (ky + kh * xb[m2] - ccy) / h;
                                    s += W[(k * 3 + comp) * p2 + l2 * p + m2] *
                                         ora_cheb_S(p, l, u) * ora_cheb_S(p, m, v);
                                }
                            W[(c * 3 + comp) * p2 + l * p + m] += s;
                        }
            }
        }
    /* Downward pass, M2L (eq. 3.8): kernel evaluated between target and
     * source Chebyshev nodes, summed over the interaction (V) list. */
    for (int64_t c = 0; c < nc; ++c) {
        double ccx, ccy, h;
        cell_geom(t, c, &ccx, &ccy, &h);
        for (int64_t e = t->off[LIST_V][c]; e < t->off[LIST_V][c + 1]; ++e) {
            int64_t s = t->lst[LIST_V][e];
            double sx, sy, sh;
            cell_geom(t, s, &sx, &sy, &sh);
            for (int l = 0; l < p; ++l)
                for (int m = 0; m < p; ++m) {
                    double X = ccx + h * xb[l], Y = ccy + h * xb[m];
                    double acc[3] = {0, 0, 0};
                    for (int l2 = 0; l2 < p; ++l2)
                        for (int m2 = 0; m2 < p; ++m2) {
                            double K[9];
                            double dx = X - (sx + sh * xb[l2]), dy = Y - (sy + sh * xb[m2]);
                            if (kernel == 0) ora_point_kernel(dx, dy, G, nu, K);
                            else poly_kernel(dx, dy, K);
                            for (int r = 0; r < 3; ++r)
                                for (int q = 0; q < 3; ++q)
                                    acc[r] += K[r * 3 + q] * W[(s * 3 + q) * p2 + l2 * p + m2];
                        }
                    for (int r = 0; r < 3; ++r) F[(c * 3 + r) * p2 + l * p + m] += acc[r];
                }
        }
    }
    /* Downward pass, L2L (eq. 3.10), coarsest level first: each child adds
     * its parent's local field interpolated at the child's nodes. */
    for (int lvl = 1; lvl <= maxlvl; ++lvl)
        for (int64_t c = 0; c < nc; ++c) {
            if (t->level[c] != lvl) continue;
            int64_t par = t->parent[c];
            double ccx, ccy, h, px, py, ph;
            cell_geom(t, c, &ccx, &ccy, &h);
            cell_geom(t, par, &px, &py, &ph);
            for (int comp = 0; comp < 3; ++comp)
                for (int l = 0; l < p; ++l)
                    for (int m = 0; m < p; ++m) {
                        double u = (ccx + h * xb[l] - px) / ph;
                        double v = (ccy + h * xb[m] - py) / ph;
                        double s = 0.0;
                        for (int l2 = 0; l2 < p; ++l2)
                            for (int m2 = 0; m2 < p; ++m2)
                                s += F[(par * 3 + comp) * p2 + l2 * p + m2] *
                                     ora_cheb_S(p, l2, u) * ora_cheb_S(p, m2, v);
                        F[(c * 3 + comp) * p2 + l * p + m] += s;
                    }
        }
    /* L2P plus direct interactions with neighbours (eq. 3.11).  On the
     * adaptive tree the directly evaluated sources of a leaf T are its U and
     * W lists and the X lists of T and its ancestors. */
    for (int64_t c = 0; c < nc; ++c) {
        if (!t->isleaf[c]) continue;
        double ccx, ccy, h;
        cell_geom(t, c, &ccx, &ccy, &h);
        for (int64_t k = t->pbeg[c]; k < t->pend[c]; ++k) {
            int64_t i = t->perm[k];
            double u = (cx[i] - ccx) / h, v = (cy[i] - ccy) / h;
            for (int l = 0; l < p; ++l) Sx[l] = ora_cheb_S(p, l, u);
            for (int m = 0; m < p; ++m) Sy[m] = ora_cheb_S(p, m, v);
            double sg[3] = {0, 0, 0};
            for (int comp = 0; comp < 3; ++comp)
                for (int l = 0; l < p; ++l)
                    for (int m = 0; m < p; ++m)
                        sg[comp] += F[(c * 3 + comp) * p2 + l * p + m] * Sx[l] * Sy[m];
            double sn[3];
            /* U and W: all points of the listed cells */
            for (int w = LIST_U; w <= LIST_W; w += 2)
                for (int64_t e = t->off[w][c]; e < t->off[w][c + 1]; ++e) {
                    int64_t s = t->lst[w][e];
                    for (int64_t kk = t->pbeg[s]; kk < t->pend[s]; ++kk) {
                        near_stress(kernel, cx[i], cy[i], t->perm[kk], &g, D, nt, nw, 8, sn);
                        sg[0] += sn[0]; sg[1] += sn[1]; sg[2] += sn[2];
                    }
                }
            for (int64_t anc = c; anc >= 0; anc = t->parent[anc])
                for (int64_t e = t->off[LIST_X][anc]; e < t->off[LIST_X][anc + 1]; ++e) {
                    int64_t s = t->lst[LIST_X][e];
                    for (int64_t kk = t->pbeg[s]; kk < t->pend[s]; ++kk) {
                        near_stress(kernel, cx[i], cy[i], t->perm[kk], &g, D, nt, nw, 8, sn);
                        sg[0] += sn[0]; sg[1] += sn[1]; sg[2] += sn[2];
                    }
                }
            double ts, tn;
            ora_traction(cb[i], sb[i], sg, &ts, &tn);
            out[2 * i] = ts;
            out[2 * i + 1] = tn;
        }
    }
    free(W); free(F); free(xb); free(gt); free(gw); free(Sx); free(Sy);
    return 0;
}


/* ------------------------------------------------------------------------ */
/* Poroelastic influence (fully coupled Biot theory, plane strain),          */
/* Section 2, eqs. 2.1-2.5.                                                  */
/* ------------------------------------------------------------------------ */
/* The paper writes the boundary integral equations with fundamental
 * solutions of instantaneous impulses and cites, without stating, their
 * continuous-impulse forms and the constant-element coefficients.  They are
 * derived here for an infinite plane, sources switched on at t = 0 and then
 * held (Heaviside in time).
 *
 * Field equations: total stress sigma = 2G eps + lambda tr(eps) I - alpha p I,
 * equilibrium div sigma = 0, fluid content zeta = alpha tr(eps_m) + p / M
 * with eps_m the strain of the porous matrix, and dzeta/dt = kappa lap p + g
 * (kappa = permeability / viscosity, g the fluid source).
 *
 * Solution: u = u_d + grad phi, where u_d is the drained elastic field of the
 * source and lap phi = eta p, eta = alpha (1 - 2 nu) / (2 G (1 - nu)).  Then
 * grad phi carries the stress 2G (grad grad phi - I lap phi), which is
 * divergence-free, and the pressure obeys S dp/dt - kappa lap p =
 * g - alpha d(tr eps_md)/dt with S = 1/M + alpha eta, so p diffuses with
 * c = kappa / S.
 *
 * Displacement discontinuity (point eigenstrain with charges q = (b_x n_x,
 * b_y n_y, b_x n_y + b_y n_x)): the matrix volumetric strain of the drained
 * field is a regular cos 2t / sin 2t part with coefficients a = 2G (q0 - q1),
 * b = 2G q2, times -(1 - 2 nu) / (4 pi G (1 - nu)) / r^2, plus a point term
 * V delta(x), V = -(q0 + q1)(1 - 2 nu) / (2 (1 - nu)) (the drained dilatation
 * at the source minus the eigenstrain itself, which is fracture volume, not
 * matrix strain).  Held from t = 0 it sets p(0+) = -(alpha/S) tr(eps_md),
 * which then diffuses: smoothing r^-2 {cos, sin} 2t by the heat kernel
 * multiplies it by P(2,z) = 1 - e^-z (1 + z), z = r^2 / (4 c t), and the
 * point term becomes the heat kernel e^-z / (4 pi c t).  phi follows from
 * lap phi = eta p in closed form.
 *
 * Fluid source of unit volume rate: p = E1(z) / (4 pi kappa), phi radial
 * with phi'/r = (eta t / (2 pi S)) (z E1(z) + 1 - e^-z) / r^2.
 *
 * Limits (the pins of the tests): t -> 0+ gives the undrained elastic field
 * (nu_u) with p = -B (1 + nu_u)(sxx + syy) / 3; t -> infinity the drained one
 * (nu) with p -> 0 for the displacement discontinuity.
 *
 * Everything below returns the transient part only, i.e. the response minus
 * the drained elastic field of the displacement discontinuity (which the
 * elastic element formulas above give in closed form).  Constants array
 * P: [0] G [1] nu [2] nu_u [3] alpha [4] kappa [5] M [6] S [7] c [8] eta [9] B. */

void ora_poro_consts(double E, double nu, double nuu, double alpha, double perm,
                     double visc, double P[10])
{
    double G = E / (2.0 * (1.0 + nu));
    double M = 2.0 * G * (nuu - nu) / (alpha * alpha * (1.0 - 2.0 * nuu) * (1.0 - 2.0 * nu));
    double eta = alpha * (1.0 - 2.0 * nu) / (2.0 * G * (1.0 - nu));
    double S = 1.0 / M + alpha * eta;
    double kap = perm / visc;
    P[0] = G; P[1] = nu; P[2] = nuu; P[3] = alpha; P[4] = kap; P[5] = M;
    P[6] = S; P[7] = kap / S; P[8] = eta;
    P[9] = 3.0 * (nuu - nu) / (alpha * (1.0 - 2.0 * nu) * (1.0 + nuu));
}

/* Exponential integral E1(z), z > 0: the power series of Abramowitz &
 * Stegun 5.1.11 for z <= 1.5, the continued fraction 5.1.22 (even part,
 * modified Lentz evaluation) above. */
double ora_E1(double z)
{
    if (z <= 1.5) {
        double s = 0.0, term = 1.0;
        for (int k = 1; k < 60; ++k) {
            term *= -z / k;               /* (-z)^k / k! */
            s += term / k;
            if (fabs(term / k) < 1e-18 * fabs(s)) break;
        }
        return -0.57721566490153286061 - log(z) - s;
    }
    /* E1 = e^-z / (z + 1 - 1/(z + 3 - 4/(z + 5 - 9/(...)))) */
    const double tiny = 1e-300;
    double f = z + 1.0, C = f, D = 0.0;
    for (int k = 1; k < 500; ++k) {
        double an = -(double)k * k, bn = z + 2.0 * k + 1.0;
        D = bn + an * D;
        if (fabs(D) < tiny) D = tiny;
        C = bn + an / C;
        if (fabs(C) < tiny) C = tiny;
        D = 1.0 / D;
        double del = C * D;
        f *= del;
        if (fabs(del - 1.0) < 1e-16) break;
    }
    return exp(-z) / f;
}

/* h(z) = 1 - (1 - e^-z)/z and its first two derivatives (series for small z). */
static void poro_h(double z, double *h, double *h1, double *h2)
{
    if (z < 0.5) {
        /* h = sum_{k>=1} (-1)^(k+1) z^k / (k+1)! */
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, fact = 1.0; /* fact = (k+1)! */
        for (int k = 1; k < 30; ++k) {
            fact *= (k + 1);
            double sg = (k & 1) ? 1.0 : -1.0;
            s0 += sg * pow(z, k) / fact;
            s1 += sg * k * pow(z, k - 1) / fact;
            if (k >= 2) s2 += sg * k * (k - 1) * pow(z, k - 2) / fact;
        }
        *h = s0; *h1 = s1; *h2 = s2;
        return;
    }
    double em = exp(-z), om = -expm1(-z); /* 1 - e^-z */
    *h = 1.0 - om / z;
    *h1 = om / (z * z) - em / z;
    *h2 = -2.0 * om / (z * z * z) + 2.0 * em / (z * z) + em / z;
}

/* P(2, z) = 1 - e^-z (1 + z). */
static double poro_P2(double z)
{
    if (z < 0.1) {
        double s = 0.0, fact = 1.0;
        for (int k = 2; k < 20; ++k) {
            fact = 1.0;
            for (int j = 2; j <= k; ++j) fact *= j;
            s += ((k & 1) ? -1.0 : 1.0) * (k - 1) * pow(z, k) / fact;
        }
        return s;
    }
    return 1.0 - exp(-z) * (1.0 + z);
}

/* Second derivatives (xx, yy, xy) of a radial function with derivatives
 * f1 = phi'(r)/r and f2 = phi''(r). */
static void radial_d2(double x, double y, double f1, double f2, double d[3])
{
    double r2 = x * x + y * y;
    d[0] = f2 * x * x / r2 + f1 * y * y / r2;
    d[1] = f2 * y * y / r2 + f1 * x * x / r2;
    d[2] = (f2 - f1) * x * y / r2;
}

/* Transient response (sxx, syy, sxy, p) at offset (x, y), time t > 0, of a
 * point displacement discontinuity with charges q (held from t = 0) and of a
 * point fluid source of volume rate qf (held from t = 0). */
void ora_poro_point_transient(const double *P, double x, double y, double t,
                              const double q[3], double qf, double out[4])
{
    const double G = P[0], nu = P[1], alpha = P[3], kap = P[4], S = P[6], c = P[7],
                 eta = P[8];
    double r2 = x * x + y * y, r = sqrt(r2);
    double z = r2 / (4.0 * c * t);
    double ez = exp(-z), om = -expm1(-z);
    double kd = (1.0 - 2.0 * nu) / (4.0 * M_PI * G * (1.0 - nu));
    double a = 2.0 * G * (q[0] - q[1]), b = 2.0 * G * q[2];
    double V = -(q[0] + q[1]) * (1.0 - 2.0 * nu) / (2.0 * (1.0 - nu));
    double cos2 = (x * x - y * y) / r2, sin2 = 2.0 * x * y / r2;
    /* pressure */
    double p = (alpha * kd / S) * (a * cos2 + b * sin2) * poro_P2(z) / r2
               - (alpha / S) * V * ez / (4.0 * M_PI * c * t);
    /* regular part: phi = Cphi (a F(r)(x^2 - y^2) + b F(r) 2xy),
     * F = -h(z) / (4 r^2) */
    double h, h1, h2;
    poro_h(z, &h, &h1, &h2);
    double F = -h / (4.0 * r2);
    double F1 = (h - z * h1) / (2.0 * r2 * r);
    double F2 = (-2.0 * z * z * h2 - 3.0 * h + 3.0 * z * h1) / (2.0 * r2 * r2);
    double Fd[3];
    radial_d2(x, y, F1 / r, F2, Fd);
    double Fx = F1 * x / r, Fy = F1 * y / r;
    /* g = x^2 - y^2 */
    double cxx = Fd[0] * (x * x - y * y) + 2.0 * Fx * 2.0 * x + F * 2.0;
    double cyy = Fd[1] * (x * x - y * y) + 2.0 * Fy * (-2.0 * y) - F * 2.0;
    double cxy = Fd[2] * (x * x - y * y) + Fx * (-2.0 * y) + Fy * (2.0 * x);
    /* g = 2xy */
    double sxx = Fd[0] * 2.0 * x * y + 2.0 * Fx * 2.0 * y;
    double syy = Fd[1] * 2.0 * x * y + 2.0 * Fy * 2.0 * x;
    double sxy = Fd[2] * 2.0 * x * y + Fx * 2.0 * x + Fy * 2.0 * y + F * 2.0;
    double Cphi = alpha * kd * eta / S;
    double pxx = Cphi * (a * cxx + b * sxx);
    double pyy = Cphi * (a * cyy + b * syy);
    double pxy = Cphi * (a * cxy + b * sxy);
    /* point term: radial phi, phi'/r = Kd (1 - e^-z) / r^2 */
    double Kd = -alpha * eta * V / (2.0 * M_PI * S);
    double d[3];
    radial_d2(x, y, Kd * om / r2, Kd * (2.0 * z * ez - om) / r2, d);
    pxx += d[0]; pyy += d[1]; pxy += d[2];
    /* fluid source */
    if (qf != 0.0) {
        double e1 = ora_E1(z);
        p += qf * e1 / (4.0 * M_PI * kap);
        double Kf = qf * eta * t / (2.0 * M_PI * S);
        double A = z * e1 + om;
        radial_d2(x, y, Kf * A / r2, Kf * (2.0 * z * e1 - A) / r2, d);
        pxx += d[0]; pyy += d[1]; pxy += d[2];
    }
    out[0] = -2.0 * G * pyy;
    out[1] = -2.0 * G * pxx;
    out[2] = 2.0 * G * pxy;
    out[3] = p;
}

/* Full response of a point DD (drained elastic point kernel + transient). */
void ora_poro_point(const double *P, double x, double y, double t,
                    const double q[3], double qf, double out[4])
{
    double K[9];
    ora_point_kernel(x, y, P[0], P[1], K);
    ora_poro_point_transient(P, x, y, t, q, qf, out);
    for (int r = 0; r < 3; ++r) out[r] += K[3 * r] * q[0] + K[3 * r + 1] * q[1] + K[3 * r + 2] * q[2];
}

/* Element integral of the transient response difference T(t1) - T(t0)
 * (t0 = 0: T(t1) alone) of element j (midpoint, cos/sin of its direction,
 * half-length a) carrying per-unit-length DDs (Ds, Dn) and fluid source Dq,
 * at the global point (X, Y).  The element is split at the foot of the
 * perpendicular from the receiver; on each side s = s0 +- L u^3 with
 * composite Gauss-Legendre in u (the substitution smooths the logarithmic
 * singularity of the fluid source and clusters nodes near the receiver);
 * panels are sized by the diffusion length sqrt(4 c t0).  nq = points per
 * panel, np_min = minimum panels (refinement studies double either). */
void ora_poro_elem_transient(const double *P, double X, double Y, double cx,
                             double cy, double cb, double sb, double a,
                             double Ds, double Dn, double Dq, double t1,
                             double t0, int nq, int np_min, double out[4])
{
    double q[3];
    ora_charge(cb, sb, Ds, Dn, q);
    double dx = X - cx, dy = Y - cy;
    double xl = dx * cb + dy * sb;
    double s0 = xl < -a ? -a : (xl > a ? a : xl);
    double tmin = t0 > 0.0 ? t0 : t1;
    double ell = sqrt(4.0 * P[7] * tmin);
    double gt[64], gw[64];
    ora_gauss_legendre(nq, gt, gw);
    for (int k = 0; k < 4; ++k) out[k] = 0.0;
    for (int side = 0; side < 2; ++side) {
        double L = side ? a - s0 : s0 + a;
        if (L <= 0.0) continue;
        int np = np_min + (int)ceil(2.0 * L / ell);
        if (np > 400) np = 400;
        for (int pn = 0; pn < np; ++pn) {
            double u0 = (double)pn / np, u1 = (double)(pn + 1) / np;
            for (int g = 0; g < nq; ++g) {
                double u = 0.5 * (u0 + u1) + 0.5 * (u1 - u0) * gt[g];
                double w = 0.5 * (u1 - u0) * gw[g] * 3.0 * L * u * u;
                double s = side ? s0 + L * u * u * u : s0 - L * u * u * u;
                double sx = cx + s * cb, sy = cy + s * sb;
                double r1[4], r0[4] = {0, 0, 0, 0};
                ora_poro_point_transient(P, X - sx, Y - sy, t1, q, Dq, r1);
                if (t0 > 0.0) ora_poro_point_transient(P, X - sx, Y - sy, t0, q, Dq, r0);
                for (int k = 0; k < 4; ++k) out[k] += w * (r1[k] - r0[k]);
            }
        }
    }
}

/* Time-marching operator of the constant spatial / constant temporal
 * elements (eqs. 2.3-2.5): the response at every midpoint (shear and normal
 * traction, pore pressure) to unit (Ds, Dn, Dq) on every element held over
 * one interval, evaluated m intervals after the interval ends:
 *   m = 0:  F(dt)                       (left-hand side; includes the
 *                                        drained elastic part)
 *   m >= 1: F((m+1) dt) - F(m dt)       (history coefficients)
 * Returned as the dense 3n x 3n matrix, row 3i + r (r: shear, normal,
 * pressure), column 3j + c (c: Ds, Dn, Dq). */
void ora_poro_matrix(int64_t n, const double *cx, const double *cy,
                     const double *cb, const double *sb, const double *a,
                     const double *P, double dt, int m, int nq, int np_min,
                     double *A)
{
    double t1 = (m + 1) * dt, t0 = m * dt;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            for (int col = 0; col < 3; ++col) {
                double Ds = col == 0, Dn = col == 1, Dq = col == 2;
                double o[4];
                ora_poro_elem_transient(P, cx[i], cy[i], cx[j], cy[j], cb[j], sb[j],
                                        a[j], Ds, Dn, Dq, t1, t0, nq, np_min, o);
                if (m == 0 && col < 2) {
                    double sg[3];
                    ora_elem_stress(cx[i], cy[i], cx[j], cy[j], cb[j], sb[j], a[j],
                                    P[0], P[1], Ds, Dn, sg);
                    o[0] += sg[0]; o[1] += sg[1]; o[2] += sg[2];
                }
                double ts, tn;
                ora_traction(cb[i], sb[i], o, &ts, &tn);
                A[(3 * i + 0) * 3 * n + 3 * j + col] = ts;
                A[(3 * i + 1) * 3 * n + 3 * j + col] = tn;
                A[(3 * i + 2) * 3 * n + 3 * j + col] = o[3];
            }
        }
    }
}

/* Rows of the same matrix for the receivers rows[0..nrow): R[(3 k + r) 3n +
 * 3 j + col] = A[(3 rows[k] + r) 3n + 3 j + col]. */
void ora_poro_matrix_rows(int64_t n, const double *cx, const double *cy,
                          const double *cb, const double *sb, const double *a,
                          const double *P, double dt, int m, int nq, int np_min,
                          int64_t nrow, const int64_t *rows, double *R)
{
    double t1 = (m + 1) * dt, t0 = m * dt;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t kj = 0; kj < nrow * n; ++kj) {
        int64_t k = kj / n, j = kj % n, i = rows[k];
        for (int col = 0; col < 3; ++col) {
            double Ds = col == 0, Dn = col == 1, Dq = col == 2;
            double o[4];
            ora_poro_elem_transient(P, cx[i], cy[i], cx[j], cy[j], cb[j], sb[j],
                                    a[j], Ds, Dn, Dq, t1, t0, nq, np_min, o);
            if (m == 0 && col < 2) {
                double sg[3];
                ora_elem_stress(cx[i], cy[i], cx[j], cy[j], cb[j], sb[j], a[j],
                                P[0], P[1], Ds, Dn, sg);
                o[0] += sg[0]; o[1] += sg[1]; o[2] += sg[2];
            }
            double ts, tn;
            ora_traction(cb[i], sb[i], o, &ts, &tn);
            R[(3 * k + 0) * 3 * n + 3 * j + col] = ts;
            R[(3 * k + 1) * 3 * n + 3 * j + col] = tn;
            R[(3 * k + 2) * 3 * n + 3 * j + col] = o[3];
        }
    }
}

/* Threads the OpenMP loops above use (reporting only). */
#ifdef _OPENMP
#include <omp.h>
int ora_num_threads(void) { return omp_get_max_threads(); }
/* Threads of the parallel loops from here on (n <= 0: one per processor);
 * timing only, no arithmetic depends on it. */
void ora_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : omp_get_num_procs()); }
#else
int ora_num_threads(void) { return 1; }
#endif
