/*
 * CPU oracle for the arbitrary-shape-surface Fresnel sum.  TEST INFRASTRUCTURE
 * ONLY: tests, the smoke check and the benchmark's CPU-baseline leg call it; the
 * product (GPU) path never links, loads or calls anything in this directory.
 *
 * What it computes (Shimobaba, Masuda, Ito, "Arbitrary shape surface Fresnel
 * diffraction", Sec. 2): the Fourier-form Fresnel diffraction from a source
 * surface displaced by d1(x1) onto a planar destination, Eq. (7), which comes
 * from the Huygens integral on the surface (Eq. (2)-(3)) through the Fresnel
 * expansion of r about r0 = z0 - d1 (Eq. (4)), the amplitude approximation
 * r^2 ~ z0^2 and the output-chirp approximation r0 -> z0 (Eq. (6)).  The
 * incident wave is a normal plane wave u_I = exp(i k d1) (the paper's choice
 * for its experiments) or u_I = 1.
 *
 * The integral over the non-uniform samples is a plain sum with unit weights;
 * callers fold any area element into u1.  The sign of the x1.x2 term is taken
 * as minus, as in Eq. (4), Eq. (5) and the transform kernel of Eq. (9) (Eq. (7)
 * prints a plus; with it, d1 = 0 would not reduce to the ordinary Fresnel
 * transform).  The destination pixel (ix, iy) sits at
 * X = x0 + p2x (ix - mx/2), Y = y0 + p2y (iy - my/2) (integer division); the
 * window centre (x0, y0) is 0 for a window on the axis.
 *
 *   u2(X, Y) = exp(i k (z0 + (X^2 + Y^2) / (2 z0))) / (i lambda z0)
 *            * sum_j u_j u_I,j exp(i k [ -d_j + (x_j^2 + y_j^2) / (2 r0_j)
 *                                          - (x_j X + y_j Y) / r0_j ])
 *
 * Everything is FP64; each term's phase is one real argument passed to sincos.
 * The loop is the plain direct sum, O(points x pixels), parallel over pixels.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <omp.h>

#define ORACLE_INCIDENT_PLANE 0
#define ORACLE_INCIDENT_NONE 1

/* Returns the number of OpenMP threads a parallel region will use. */
int asf_oracle_threads(int32_t requested)
{
    if (requested > 0) return requested;
    return omp_get_max_threads();
}

/*
 * n          number of source samples
 * x, y, d    FP64 [n]: source position x1 = (x, y) and displacement d1 (m)
 * u          FP64 [2n]: complex source field, interleaved (re, im)
 * lambda, z0 wavelength and source-to-destination distance (m)
 * p2x, p2y   destination pitch (m); mx, my destination grid size
 * x0, y0     destination window centre (m)
 * incident   0: plane wave exp(i k d1); 1: u_I = 1
 * n_eval     number of destination pixels to evaluate
 * ix, iy     int32 [n_eval]: pixel column and row
 * out        FP64 [2 n_eval]: complex u2 at those pixels, interleaved
 * threads    OpenMP threads (<= 0: default)
 * Returns 0, or -1 if some r0 = z0 - d1 <= 0 or an argument is invalid.
 */
int asf_oracle_direct(int64_t n, const double *x, const double *y, const double *d,
                      const double *u, double lambda, double z0, double p2x, double p2y,
                      double x0, double y0, int32_t mx, int32_t my, int32_t incident, int64_t n_eval,
                      const int32_t *ix, const int32_t *iy, double *out, int32_t threads)
{
    if (n < 0 || n_eval < 0 || !(lambda > 0.0) || !(z0 > 0.0)) return -1;
    for (int64_t j = 0; j < n; ++j)
        if (!(z0 - d[j] > 0.0)) return -1;

    const double pi = 3.14159265358979323846;
    const double k = 2.0 * pi / lambda;
    const int nthr = asf_oracle_threads(threads);

#pragma omp parallel for schedule(dynamic, 1) num_threads(nthr)
    for (int64_t e = 0; e < n_eval; ++e) {
        const double X = x0 + p2x * (double)(ix[e] - mx / 2);
        const double Y = y0 + p2y * (double)(iy[e] - my / 2);
        double sr = 0.0, si = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double r0 = z0 - d[j];
            double arg = k * (-d[j] + (x[j] * x[j] + y[j] * y[j]) / (2.0 * r0)
                              - (x[j] * X + y[j] * Y) / r0);
            if (incident == ORACLE_INCIDENT_PLANE) arg += k * d[j];
            double s, c;
            sincos(arg, &s, &c);
            const double ur = u[2 * j], ui = u[2 * j + 1];
            sr += ur * c - ui * s;
            si += ur * s + ui * c;
        }
        /* exp(i k (z0 + (X^2 + Y^2) / (2 z0))) * S */
        double s2, c2;
        sincos(k * (z0 + (X * X + Y * Y) / (2.0 * z0)), &s2, &c2);
        const double tr = c2 * sr - s2 * si;
        const double ti = c2 * si + s2 * sr;
        /* 1 / (i lambda z0) = -i / (lambda z0) */
        const double a = 1.0 / (lambda * z0);
        out[2 * e] = a * ti;
        out[2 * e + 1] = -a * tr;
    }
    return 0;
}

/*
 * The adjoint of the same linear map, u1 -> u2 above: for source point j
 *
 *   g1_j = sum over pixels (ix, iy) of conj(A(ix, iy; j)) g2(ix, iy),
 *
 * where A(ix, iy; j) is the coefficient that multiplies u_j in u2(X, Y):
 * the prefactor 1/(i lambda z0), exp(i k (z0 + (X^2 + Y^2)/(2 z0))) and the
 * term's own phase.  The conjugate is formed as exp(-i (sum of the phases)) times
 * i/(lambda z0), one sincos per term.
 *
 * g2         FP64 [2 mx my]: complex destination field, interleaved, row-major (iy, ix)
 * n_eval     number of source points to evaluate
 * jidx       int64 [n_eval]: their indices into x, y, d
 * out        FP64 [2 n_eval]: complex g1 at those points, interleaved
 * Other arguments as for asf_oracle_direct.  Parallel over points.
 */
int asf_oracle_adjoint(int64_t n, const double *x, const double *y, const double *d,
                       double lambda, double z0, double p2x, double p2y, double x0, double y0,
                       int32_t mx, int32_t my,
                       int32_t incident, const double *g2, int64_t n_eval, const int64_t *jidx,
                       double *out, int32_t threads)
{
    if (n < 0 || n_eval < 0 || !(lambda > 0.0) || !(z0 > 0.0) || mx < 0 || my < 0) return -1;
    for (int64_t e = 0; e < n_eval; ++e)
        if (jidx[e] < 0 || jidx[e] >= n || !(z0 - d[jidx[e]] > 0.0)) return -1;

    const double pi = 3.14159265358979323846;
    const double k = 2.0 * pi / lambda;
    const double a = 1.0 / (lambda * z0);
    const int nthr = asf_oracle_threads(threads);

#pragma omp parallel for schedule(dynamic, 1) num_threads(nthr)
    for (int64_t e = 0; e < n_eval; ++e) {
        const int64_t j = jidx[e];
        const double r0 = z0 - d[j];
        double sr = 0.0, si = 0.0;
        for (int32_t iy = 0; iy < my; ++iy) {
            const double Y = y0 + p2y * (double)(iy - my / 2);
            for (int32_t ix = 0; ix < mx; ++ix) {
                const double X = x0 + p2x * (double)(ix - mx / 2);
                double arg = k * (-d[j] + (x[j] * x[j] + y[j] * y[j]) / (2.0 * r0)
                                  - (x[j] * X + y[j] * Y) / r0);
                if (incident == ORACLE_INCIDENT_PLANE) arg += k * d[j];
                arg += k * (z0 + (X * X + Y * Y) / (2.0 * z0));
                double s, c;
                sincos(arg, &s, &c);
                /* conj(exp(i arg)) g2 = (c - i s)(gr + i gi) */
                const double gr = g2[2 * ((int64_t)iy * mx + ix)];
                const double gi = g2[2 * ((int64_t)iy * mx + ix) + 1];
                sr += c * gr + s * gi;
                si += c * gi - s * gr;
            }
        }
        /* conj(1 / (i lambda z0)) = i / (lambda z0) */
        out[2 * e] = -a * si;
        out[2 * e + 1] = a * sr;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* The exact and intermediate forms of Sec. 2, for the approximation study.   */
/* ------------------------------------------------------------------------- */

#define ORACLE_EQ5 5   /* Fresnel on the surface, Eq. (5): the exact chirp exp(i k |X|^2 / (2 r0)) */
#define ORACLE_EQ2 2   /* Huygens on the surface, Eq. (2) with r of Eq. (3) */

/*
 * u2 at pixels (ix, iy) by one of the two direct sums that precede Eq. (7):
 *
 * model 5, Eq. (5): Eq. (7) before the output-chirp approximation of Eq. (6),
 *   u2 = exp(i k z0) / (i lambda z0)
 *        * sum_j u_j u_I,j exp(i k [ -d_j + |x_j|^2 / (2 r0_j) - x_j.X / r0_j + |X|^2 / (2 r0_j) ])
 *   (the third exponential of Eq. (5) is read with its factor i k, as Eq. (6) writes it);
 *
 * model 2, Eq. (2)-(3): the Huygens sum on the surface with no expansion of r,
 *   u2 = z0 / (i lambda) * sum_j u_j u_I,j exp(i k r_j) / r_j^2,
 *   r_j = sqrt(|X - x_j|^2 + (z0 - d_j)^2).
 *
 * Same arguments, units and conventions as asf_oracle_direct (unit weights,
 * destination pixel at X = x0 + p2x (ix - mx/2)).  Returns 0, or -1 on an invalid
 * argument, an unknown model or some r0 <= 0.
 */
int asf_oracle_surface(int32_t model, int64_t n, const double *x, const double *y, const double *d,
                       const double *u, double lambda, double z0, double p2x, double p2y,
                       double x0, double y0, int32_t mx, int32_t my, int32_t incident, int64_t n_eval,
                       const int32_t *ix, const int32_t *iy, double *out, int32_t threads)
{
    if (model != ORACLE_EQ5 && model != ORACLE_EQ2) return -1;
    if (n < 0 || n_eval < 0 || !(lambda > 0.0) || !(z0 > 0.0)) return -1;
    for (int64_t j = 0; j < n; ++j)
        if (!(z0 - d[j] > 0.0)) return -1;

    const double pi = 3.14159265358979323846;
    const double k = 2.0 * pi / lambda;
    const int nthr = asf_oracle_threads(threads);

#pragma omp parallel for schedule(dynamic, 1) num_threads(nthr)
    for (int64_t e = 0; e < n_eval; ++e) {
        const double X = x0 + p2x * (double)(ix[e] - mx / 2);
        const double Y = y0 + p2y * (double)(iy[e] - my / 2);
        double sr = 0.0, si = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double r0 = z0 - d[j];
            double arg, amp;
            if (model == ORACLE_EQ5) {
                arg = k * (-d[j] + (x[j] * x[j] + y[j] * y[j]) / (2.0 * r0)
                           - (x[j] * X + y[j] * Y) / r0 + (X * X + Y * Y) / (2.0 * r0));
                amp = 1.0;
            } else {
                const double dx = X - x[j], dy = Y - y[j];
                const double r = sqrt(dx * dx + dy * dy + r0 * r0);
                arg = k * r;
                amp = 1.0 / (r * r);
            }
            if (incident == ORACLE_INCIDENT_PLANE) arg += k * d[j];
            double s, c;
            sincos(arg, &s, &c);
            const double ur = amp * u[2 * j], ui = amp * u[2 * j + 1];
            sr += ur * c - ui * s;
            si += ur * s + ui * c;
        }
        double tr, ti, a;
        if (model == ORACLE_EQ5) {
            /* exp(i k z0) / (i lambda z0) */
            double s2, c2;
            sincos(k * z0, &s2, &c2);
            tr = c2 * sr - s2 * si;
            ti = c2 * si + s2 * sr;
            a = 1.0 / (lambda * z0);
        } else {
            /* z0 / (i lambda) */
            tr = sr;
            ti = si;
            a = z0 / lambda;
        }
        /* times 1 / i = -i */
        out[2 * e] = a * ti;
        out[2 * e + 1] = -a * tr;
    }
    return 0;
}

#define ORACLE_EQ7 7   /* the Fourier form, Eq. (7) */

/*
 * The one-dimensional forms (a line source x1 with displacement d1(x1) onto a
 * line of m destination pixels at X = x0 + p2 (ix - m/2)), used by the paper's
 * profiles.  The paper does not write them; they are read as what Eq. (2), (5)
 * and (7) give for a surface and field that do not vary along y, with the
 * integral over y1 done analytically:
 *
 *  - Eq. (5) and (7): the y parts of the phase form the chirp
 *    exp(i k (y1 - Y)^2 / (2 r0)), whose integral is sqrt(i lambda r0); the
 *    amplitude approximation that turns r^2 into z0^2 turns this r0 into z0,
 *    so the 2D prefactor 1 / (i lambda z0) becomes 1 / sqrt(i lambda z0):
 *
 *    model 7:  u2 = exp(i k (z0 + X^2 / (2 z0))) / sqrt(i lambda z0)
 *                   * sum_j u_j u_I,j exp(i k [ -d_j + x_j^2 / (2 r0_j) - x_j X / r0_j ])
 *    model 5:  u2 = exp(i k z0) / sqrt(i lambda z0)
 *                   * sum_j u_j u_I,j exp(i k [ -d_j + x_j^2 / (2 r0_j) - x_j X / r0_j + X^2 / (2 r0_j) ])
 *
 *  - Eq. (2): the integral over y1 of exp(i k R) / R^2, R = sqrt(rho^2 + y1^2)
 *    with rho = sqrt((X - x)^2 + r0^2), taken by stationary phase (its leading
 *    term; the next is smaller by about 1 / (k rho), 1e-7 at rho = 1 m for
 *    visible light): sqrt(i lambda rho) exp(i k rho) / rho^2, so
 *
 *    model 2:  u2 = z0 / (i lambda) * sum_j u_j u_I,j sqrt(i lambda rho_j) exp(i k rho_j) / rho_j^2
 *                 = z0 exp(-i pi/4) / sqrt(lambda) * sum_j u_j u_I,j exp(i k rho_j) / rho_j^(3/2).
 *
 * x, d  FP64 [n]; u FP64 [2n] interleaved; ix int32 [n_eval]; out FP64 [2 n_eval].
 * Returns 0, or -1 on an invalid argument, an unknown model or some r0 <= 0.
 */
int asf_oracle_line(int32_t model, int64_t n, const double *x, const double *d, const double *u,
                    double lambda, double z0, double p2, double x0, int32_t m, int32_t incident,
                    int64_t n_eval, const int32_t *ix, double *out, int32_t threads)
{
    if (model != ORACLE_EQ7 && model != ORACLE_EQ5 && model != ORACLE_EQ2) return -1;
    if (n < 0 || n_eval < 0 || !(lambda > 0.0) || !(z0 > 0.0)) return -1;
    for (int64_t j = 0; j < n; ++j)
        if (!(z0 - d[j] > 0.0)) return -1;

    const double pi = 3.14159265358979323846;
    const double k = 2.0 * pi / lambda;
    const int nthr = asf_oracle_threads(threads);

#pragma omp parallel for schedule(dynamic, 1) num_threads(nthr)
    for (int64_t e = 0; e < n_eval; ++e) {
        const double X = x0 + p2 * (double)(ix[e] - m / 2);
        double sr = 0.0, si = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double r0 = z0 - d[j];
            double arg, amp = 1.0;
            if (model == ORACLE_EQ7) {
                arg = k * (-d[j] + x[j] * x[j] / (2.0 * r0) - x[j] * X / r0);
            } else if (model == ORACLE_EQ5) {
                arg = k * (-d[j] + x[j] * x[j] / (2.0 * r0) - x[j] * X / r0 + X * X / (2.0 * r0));
            } else {
                const double dx = X - x[j];
                const double rho = sqrt(dx * dx + r0 * r0);
                arg = k * rho;
                amp = 1.0 / (rho * sqrt(rho));
            }
            if (incident == ORACLE_INCIDENT_PLANE) arg += k * d[j];
            double s, c;
            sincos(arg, &s, &c);
            const double ur = amp * u[2 * j], ui = amp * u[2 * j + 1];
            sr += ur * c - ui * s;
            si += ur * s + ui * c;
        }
        /* common phase and amplitude: exp(i phase) * a */
        double phase, a;
        if (model == ORACLE_EQ7) {
            phase = k * (z0 + X * X / (2.0 * z0)) - pi / 4.0;
            a = 1.0 / sqrt(lambda * z0);
        } else if (model == ORACLE_EQ5) {
            phase = k * z0 - pi / 4.0;
            a = 1.0 / sqrt(lambda * z0);
        } else {
            phase = -pi / 4.0;
            a = z0 / sqrt(lambda);
        }
        double s2, c2;
        sincos(phase, &s2, &c2);
        out[2 * e] = a * (c2 * sr - s2 * si);
        out[2 * e + 1] = a * (c2 * si + s2 * sr);
    }
    return 0;
}
