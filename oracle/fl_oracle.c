/*
 * fl_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 (long-double accumulated) CPU reference for the
 * finite-difference discretisation of the integral fractional Laplacian of
 * Duo & Zhang, "Accurate numerical methods for two and three dimensional
 * integral fractional Laplacian with applications" (arXiv:1804.02718).
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header, table or
 * constant generator with the GPU library.
 *
 * What is computed (splitting parameter gamma in (alpha, 2], gamma = 2 the
 * paper's default):
 *   - J_d(p) = int_{[0,1]^{d-1}} (1+|s|^2)^{-p/2} ds, the angular factor of
 *     a radial power integrated over a cube corner (pyramid split of the
 *     cube along its diagonal planes).
 *   - element integrals E_e = int_{I_e} |xi|^{-q} dxi, q = d + alpha - gamma,
 *     over the elements I_e of Sec. 2 (2D) and Sec. 4 (3D), and over the
 *     intervals of the d = 1 case of the general-d scheme (Sec. 4, the
 *     theorems for any d >= 1), where every integral has a closed form.  The origin
 *     element is the closed form d h^{d-q} J_d(q)/(d-q) (in 2D this is the
 *     polar identity the paper uses in the proof of Theorem 1); every other
 *     element by tensor Gauss-Legendre quadrature, whose order is fixed by a
 *     plain table of the element's distance from the origin.
 *   - coefficients a_v of the scheme (Sec. 2, formulas for a_mn and a_00;
 *     Sec. 4, formulas for a_mns and a_000), with the origin-element
 *     corrections of the limit rules for gamma = 2 (none for gamma < 2).
 *   - the scheme itself as an explicit O(M^2) sum (Sec. 2 scheme for the
 *     2D operator, Sec. 4 scheme for the 3D operator), in long double.
 *
 * Parity of this file with the paper is pinned by tests (closed forms,
 * alpha -> 2 limits, high-precision quadrature, brute force on tiny grids).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------ */
/* Gauss-Legendre rule on [-1,1]: roots of P_n by Newton's method.      */
/* ------------------------------------------------------------------ */
static void gl_rule(int n, long double *x, long double *w)
{
    for (int i = 0; i < (n + 1) / 2; ++i) {
        long double z = cosl((long double)M_PI * (i + 0.75L) / (n + 0.5L));
        long double dp = 1.0L;
        for (int it = 0; it < 200; ++it) {
            long double p0 = 1.0L, p1 = z;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2.0L * k - 1.0L) * z * p1 - (k - 1.0L) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p0 = 1.0L; p1 = z; }
            dp = n * (z * p1 - p0) / (z * z - 1.0L);
            long double dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        {
            long double p0 = 1.0L, p1 = z;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2.0L * k - 1.0L) * z * p1 - (k - 1.0L) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0L);
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = 2.0L / ((1.0L - z * z) * dp * dp);
        w[n - 1 - i] = w[i];
    }
}

/* Exported so tests can check the rule against numpy's. */
void orc_gl_rule(int n, double *x, double *w)
{
    long double xl[128], wl[128];
    if (n < 1 || n > 128) return;
    gl_rule(n, xl, wl);
    for (int i = 0; i < n; ++i) { x[i] = (double)xl[i]; w[i] = (double)wl[i]; }
}

/* ------------------------------------------------------------------ */
/* J_d(p) = int_{[0,1]^{d-1}} (1+|s|^2)^{-p/2} ds, 40-point GL per axis.  */
/* ------------------------------------------------------------------ */
double orc_J(int d, double p)
{
    enum { NJ = 40 };
    long double x[NJ], w[NJ];
    gl_rule(NJ, x, w);
    long double acc = 0.0L;
    if (d == 1) return 1.0;
    if (d == 2) {
        for (int i = 0; i < NJ; ++i) {
            long double s = 0.5L * (x[i] + 1.0L);
            acc += 0.5L * w[i] * powl(1.0L + s * s, -0.5L * p);
        }
    } else {
        for (int i = 0; i < NJ; ++i)
            for (int j = 0; j < NJ; ++j) {
                long double s = 0.5L * (x[i] + 1.0L), t = 0.5L * (x[j] + 1.0L);
                acc += 0.25L * w[i] * w[j] * powl(1.0L + s * s + t * t, -0.5L * p);
            }
    }
    return (double)acc;
}

/* ------------------------------------------------------------------ */
/* Element integrals                                                    */
/* ------------------------------------------------------------------ */

/* Quadrature order for an element whose largest index is m (unit h): the
 * integrand's nearest singularity (the origin) lies about 4m half-widths from
 * the element, so n points give a relative error near (4m)^{-2n}. */
static int elem_order(int m)
{
    if (m <= 3) return 24;
    if (m <= 15) return 16;
    if (m <= 63) return 10;
    if (m <= 127) return 6;
    return 4;
}

/* int over [e1,e1+1]x[e2,e2+1](x[e3,e3+1]) of |xi|^{-q}, unit spacing. */
static long double elem_unit(int d, double q, const int *e)
{
    long double x[32], w[32];
    int m = 0;
    for (int i = 0; i < d; ++i) if (e[i] > m) m = e[i];
    int n = elem_order(m);
    gl_rule(n, x, w);
    long double acc = 0.0L;
    double hq = -0.5 * q;
    /* integrand in FP64 (pow), sums in long double */
    if (d == 2) {
        for (int i = 0; i < n; ++i) {
            double a = (double)(e[0] + 0.5L * (x[i] + 1.0L));
            for (int j = 0; j < n; ++j) {
                double b = (double)(e[1] + 0.5L * (x[j] + 1.0L));
                acc += w[i] * w[j] * (long double)pow(a * a + b * b, hq);
            }
        }
        return 0.25L * acc;
    }
    for (int i = 0; i < n; ++i) {
        double a = (double)(e[0] + 0.5L * (x[i] + 1.0L));
        for (int j = 0; j < n; ++j) {
            double b = (double)(e[1] + 0.5L * (x[j] + 1.0L));
            for (int k = 0; k < n; ++k) {
                double c = (double)(e[2] + 0.5L * (x[k] + 1.0L));
                acc += w[i] * w[j] * w[k] * (long double)pow(a * a + b * b + c * c, hq);
            }
        }
    }
    return 0.125L * acc;
}

/* int_e^{e+1} x^{-q} dx for e >= 1, as e^{1-q} expm1((1-q) log1p(1/e)) / (1-q)
 * (no cancellation between the two endpoint powers). */
static long double interval_unit(double q, int e)
{
    long double p = 1.0L - (long double)q;
    long double le = logl((long double)e);
    return expl(p * le) * expm1l(p * log1pl(1.0L / (long double)e)) / p;
}

/* Origin element, closed form: d h^{d-q} J_d(q) / (d-q). */
double orc_E0(int d, double q, double h)
{
    return d * pow(h, d - q) * orc_J(d, q) / (d - q);
}

/* Tail integral over R^d_+ minus (0,L)^d of |xi|^{-(d+alpha)}:
 * d L^{-alpha} J_d(d+alpha) / alpha (pyramid split, Sec. 2 and Sec. 4). */
double orc_D2(int d, double alpha, double L)
{
    return d * pow(L, -alpha) * orc_J(d, d + alpha) / alpha;
}

/* E[e] for e in [0,N-1]^d, x-index fastest.  q = d + alpha - gamma. */
int orc_elements_g(int d, double alpha, double gamma, double h, int N, double *E)
{
    if (d < 1 || d > 3) return 1;
    double q = d + alpha - gamma;
    long double scale = powl((long double)h, (long double)(d - q));
    int64_t total = 1;
    for (int i = 0; i < d; ++i) total *= N;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t idx = 0; idx < total; ++idx) {
        int e[3] = {0, 0, 0};
        int64_t t = idx;
        for (int i = 0; i < d; ++i) { e[i] = (int)(t % N); t /= N; }
        if (idx == 0)
            E[idx] = orc_E0(d, q, h);
        else if (d == 1)
            E[idx] = (double)(scale * interval_unit(q, e[0]));
        else
            E[idx] = (double)(scale * elem_unit(d, q, e));
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Coefficients a_v, v in [0,N]^d (x-index fastest); a[0] holds a_0.   */
/* Sec. 2: a_mn = 2^sigma/(4|xi_mn|^2) (int_{T_mn} w + cbar int_{I_00} w) */
/*   with cbar = +1 on (1,0),(0,1), -1 on (1,1).                         */
/* Sec. 4: a_mns = 2^sigma/(8|xi|^2) (int_{T_mns} w - cbar int_{I_000} w) */
/*   with cbar = -5/3 on axis unit vectors, +1 on (1,1,0)-type, and +1 on */
/*   (1,1,1) (the limit rule subtracts every corner with m+n+s>1).       */
/* a_0 = -sum_{v != 0} W'_v/|xi_v|^2 - 2^d D2, identical to the a_00 and */
/* a_000 formulas.                                                      */
/* ------------------------------------------------------------------ */
int orc_elements(int d, double alpha, double h, int N, double *E)
{
    return orc_elements_g(d, alpha, 2.0, h, N, E);
}

/* Sec. 2 with general gamma: a_mn = 2^sigma/(4|xi_mn|^gamma) (int_{T_mn} w    */
/* + cbar floor(gamma/2) int_{I_00} w), w = |xi|^{gamma-(2+alpha)}; the same */
/* in 3D with 8 and the 3D cbar.  floor(gamma/2) is 1 only for gamma = 2.    */
int orc_coeffs_g(int d, double alpha, double gamma, double h, int N, double *a, double *E_out)
{
    if (d < 1 || d > 3) return 1;
    if (!(alpha > 0.0 && alpha < 2.0) || N < 2 || !(h > 0.0)) return 2;
    if (!(gamma > alpha && gamma <= 2.0)) return 2;
    int64_t ne = 1, nv = 1;
    for (int i = 0; i < d; ++i) { ne *= N; nv *= (N + 1); }
    double *E = E_out ? E_out : (double *)malloc(sizeof(double) * ne);
    if (!E) return 3;
    orc_elements_g(d, alpha, gamma, h, N, E);
    double q = d + alpha - gamma;
    int fl_g = gamma == 2.0 ? 1 : 0;  /* floor(gamma/2) on (alpha, 2] */
    double E0 = E[0];
    int V = N + 1;
    long double twod = (long double)(1 << d);

#pragma omp parallel for schedule(static)
    for (int64_t idx = 1; idx < nv; ++idx) {
        int v[3] = {0, 0, 0};
        int64_t t = idx;
        for (int i = 0; i < d; ++i) { v[i] = (int)(t % V); t /= V; }
        /* W_v: sum of E_e over elements having xi_v as a vertex, inside D1 */
        long double W = 0.0L;
        int lo[3], hi[3];
        for (int i = 0; i < 3; ++i) { lo[i] = 0; hi[i] = 0; }
        for (int i = 0; i < d; ++i) {
            lo[i] = v[i] - 1 < 0 ? 0 : v[i] - 1;
            hi[i] = v[i] > N - 1 ? N - 1 : v[i];
        }
        if (d == 1) {
            for (int e0 = lo[0]; e0 <= hi[0]; ++e0) W += E[e0];
        } else if (d == 2) {
            for (int e1 = lo[1]; e1 <= hi[1]; ++e1)
                for (int e0 = lo[0]; e0 <= hi[0]; ++e0)
                    W += E[e0 + (int64_t)N * e1];
        } else {
            for (int e2 = lo[2]; e2 <= hi[2]; ++e2)
                for (int e1 = lo[1]; e1 <= hi[1]; ++e1)
                    for (int e0 = lo[0]; e0 <= hi[0]; ++e0)
                        W += E[e0 + (int64_t)N * (e1 + (int64_t)N * e2)];
        }
        int nz = 0, ones = 0, maxv = 0;
        for (int i = 0; i < d; ++i) {
            if (v[i] == 0) ++nz;
            if (v[i] == 1) ++ones;
            if (v[i] > maxv) maxv = v[i];
        }
        /* origin-element correction of the gamma = 2 limit rule (1D: the limit of
         * psi_2 at the origin is u'', taken as psi_2 at xi = h, so the origin's
         * share moves to vertex 1 as in the 2D axis rule) */
        if (maxv == 1 && fl_g) {
            int nonzero = d - nz;
            if (d <= 2)
                W += (nonzero == 1) ? (long double)E0 : -(long double)E0;
            else
                W += (nonzero == 1) ? (5.0L / 3.0L) * E0 : -(long double)E0;
        }
        long double r2 = 0.0L;
        for (int i = 0; i < d; ++i) r2 += (long double)v[i] * v[i];
        r2 *= (long double)h * h;
        long double rg = fl_g ? r2 : powl(r2, 0.5L * (long double)gamma);  /* |xi_v|^gamma */
        long double pw = (long double)(1 << nz);
        a[idx] = (double)(pw * W / (twod * rg));
    }
    /* a_0: sum of 2^d a_v / 2^sigma(v) over v != 0, compensated by long double */
    long double s = 0.0L;
    for (int64_t idx = 1; idx < nv; ++idx) {
        int64_t t = idx;
        int nz = 0;
        for (int i = 0; i < d; ++i) { if (t % V == 0) ++nz; t /= V; }
        s += twod * (long double)a[idx] / (long double)(1 << nz);
    }
    double L = N * h;
    a[0] = (double)(-s - twod * (long double)orc_D2(d, alpha, L));
    (void)q;
    if (!E_out) free(E);
    return 0;
}

int orc_coeffs(int d, double alpha, double h, int N, double *a, double *E_out)
{
    return orc_coeffs_g(d, alpha, 2.0, h, N, a, E_out);
}

/* c_{d,alpha} = 2^{alpha-1} alpha Gamma((d+alpha)/2) / (pi^{d/2} Gamma(1-alpha/2)) (Sec. 1) */
double orc_const(int d, double alpha)
{
    return pow(2.0, alpha - 1.0) * alpha * tgamma(0.5 * (d + alpha)) /
           (pow(M_PI, 0.5 * d) * tgamma(1.0 - 0.5 * alpha));
}

/* ------------------------------------------------------------------ */
/* The scheme as an explicit sum: (A u)_i = -c sum_j a_{|i-j|} u_j,     */
/* i, j over the interior nodes [1,N-1]^d (x fastest).                  */
/* rows: list of flat interior indices to evaluate (nrows of them);    */
/* rows == NULL evaluates every row.  absmode != 0 returns             */
/* c sum_j |a_{|i-j|}| |u_j| instead (the size of the sum's terms).     */
/* ------------------------------------------------------------------ */
/* The scheme on a box of nk[k] interior nodes per axis (x first), nk[k] <= N-1:
 * (A u)_i = -c sum_j a_{|i-j|} u_j over the box (Sec. 2 scheme, whose sums run
 * to N_x - 1 and N_y - 1; Sec. 4 likewise).  a is the (N+1)^d table of the
 * square (0, L)^d, L = N h, the longest side. */
int orc_apply_rows_box(int d, int N, const int *nk, double c, const double *a, const double *u,
                       const int64_t *rows, int64_t nrows, double *y, int absmode)
{
    if (d < 1 || d > 3) return 1;
    int V = N + 1;
    int n0 = nk[0], n1 = d >= 2 ? nk[1] : 1, n2 = d == 3 ? nk[2] : 1;
    for (int k = 0; k < d; ++k)
        if (nk[k] < 1 || nk[k] > N - 1) return 2;
    int64_t M = (int64_t)n0 * n1 * n2;
    int64_t R = rows ? nrows : M;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < R; ++r) {
        int64_t i = rows ? rows[r] : r;
        int i0 = (int)(i % n0), i1 = (int)((i / n0) % n1), i2 = (int)(i / ((int64_t)n0 * n1));
        long double acc = 0.0L;
        for (int j2 = 0; j2 < n2; ++j2) {
            int m2 = abs(i2 - j2);
            for (int j1 = 0; j1 < n1; ++j1) {
                int m1 = abs(i1 - j1);
                const double *arow = a + (int64_t)V * (m1 + (int64_t)V * m2);
                const double *urow = u + (int64_t)n0 * (j1 + (int64_t)n1 * j2);
                for (int j0 = 0; j0 < n0; ++j0) {
                    int m0 = abs(i0 - j0);
                    if (absmode) acc += fabsl((long double)arow[m0] * urow[j0]);
                    else acc += (long double)arow[m0] * urow[j0];
                }
            }
        }
        y[r] = absmode ? (double)(fabs(c) * acc) : (double)(-(long double)c * acc);
    }
    return 0;
}

int orc_apply_rows(int d, int N, double c, const double *a, const double *u,
                   const int64_t *rows, int64_t nrows, double *y, int absmode)
{
    int nk[3] = {N - 1, N - 1, N - 1};
    return orc_apply_rows_box(d, N, nk, c, a, u, rows, nrows, y, absmode);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
