/*
 * Oracle (test infrastructure only): exact MBF reactions between point-dipole
 * clouds, plain FP64, written for obviousness rather than speed.
 *
 * Only tests/, the package's smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code with the GPU library.
 *
 * Section II-A: the HARP model is built from the exact interaction between a
 * testing MBF T and a source MBF S computed on a polar grid.  With MBFs made of
 * point dipoles (moment a, unit orientation u, position rho relative to the
 * element reference point) that interaction is the Galerkin reaction
 *
 *   Z_TS(R) = -j omega mu0 sum_s sum_s' a_T,s a_S,s' u_T,s . G(d) . u_S,s'
 *   d       = R + rho_T,s - rho_S,s'
 *
 * with the free-space dyadic Green's function (time factor e^{+j omega t})
 *
 *   G(d) = g(|d|) [ A(k|d|) I + B(k|d|) dhat dhat ],   g(r) = e^{-jkr} / (4 pi r)
 *   A(x) = 1 - j/x - 1/x^2,   B(x) = -1 + 3j/x + 3/x^2.
 *
 * The -j omega mu prefactor is the one of Eq. (1), so the large-distance limit
 * of Z_TS is exactly Eq. (1).  For the self block (zero distance, Section III-A)
 * the thin-wire reduced kernel replaces |d| by s = sqrt(|d|^2 + a_w^2) in g, A
 * and B and dhat dhat by d d^T / s^2.
 */
#include <complex.h>
#include <math.h>
#include <stddef.h>

#define SAMPLE_FIELDS 8 /* x, y, z, ux, uy, uz, a_re, a_im */

static const double PI = 3.14159265358979323846;

/* u1 . G(d) . u2 for one pair of samples; reg > 0 selects the reduced kernel. */
static double complex dyadic_uu(double k, const double d[3], const double u1[3],
                                const double u2[3], double reg)
{
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double s = sqrt(r2 + reg * reg);
    double x = k * s;
    double complex g = cexp(-I * x) / (4.0 * PI * s);
    double complex A = 1.0 - I / x - 1.0 / (x * x);
    double complex B = -1.0 + 3.0 * I / x + 3.0 / (x * x);
    double u1u2 = u1[0] * u2[0] + u1[1] * u2[1] + u1[2] * u2[2];
    double u1d = u1[0] * d[0] + u1[1] * d[1] + u1[2] * d[2];
    double u2d = u2[0] * d[0] + u2[1] * d[1] + u2[2] * d[2];
    return g * (A * u1u2 + B * u1d * u2d / (s * s));
}

/* Full 3x3 dyadic at d (no regularisation), row-major complex out[9][2]. */
void oracle_dyadic(double k, double dx, double dy, double dz, double *out)
{
    double d[3] = {dx, dy, dz};
    double e[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double complex v = dyadic_uu(k, d, e[i], e[j], 0.0);
            out[2 * (3 * i + j)] = creal(v);
            out[2 * (3 * i + j) + 1] = cimag(v);
        }
}

/* Reaction between a testing cloud T (reference point at R) and a source
 * cloud S (reference point at the origin).  out = {re, im}. */
void oracle_reaction(double k, double omega_mu, int nT, const double *T, int nS,
                     const double *S, double Rx, double Ry, double Rz, double reg,
                     double *out)
{
    double complex acc = 0.0;
    for (int s = 0; s < nT; ++s) {
        const double *ts = T + (size_t)s * SAMPLE_FIELDS;
        double complex aT = ts[6] + I * ts[7];
        for (int q = 0; q < nS; ++q) {
            const double *ss = S + (size_t)q * SAMPLE_FIELDS;
            double complex aS = ss[6] + I * ss[7];
            double d[3] = {Rx + ts[0] - ss[0], Ry + ts[1] - ss[1], Rz + ts[2] - ss[2]};
            acc += aT * aS * dyadic_uu(k, d, ts + 3, ss + 3, reg);
        }
    }
    acc *= -I * omega_mu;
    out[0] = creal(acc);
    out[1] = cimag(acc);
}

/* Reactions of every ordered MBF pair (T, S) of one element with itself
 * displaced by (Rx[p], Ry[p], 0), for n_pts displacements.
 * samples: [n_mbf][n_samp][8];  out: [n_pts][n_mbf (T)][n_mbf (S)][2]. */
void oracle_reaction_grid(double k, double omega_mu, int n_mbf, int n_samp,
                          const double *samples, int n_pts, const double *Rx,
                          const double *Ry, double reg, double *out)
{
    const size_t mbf_stride = (size_t)n_samp * SAMPLE_FIELDS;
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
    for (int p = 0; p < n_pts; ++p)
        for (int t = 0; t < n_mbf; ++t)
            for (int s = 0; s < n_mbf; ++s) {
                double *o = out + 2 * (((size_t)p * n_mbf + t) * n_mbf + s);
                oracle_reaction(k, omega_mu, n_samp, samples + t * mbf_stride, n_samp,
                                samples + s * mbf_stride, Rx[p], Ry[p], 0.0, reg, o);
            }
}
