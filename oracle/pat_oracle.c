/*
 * pat_oracle.c -- FP64 direct-sum oracle for the PAT operator pair (A, A*).
 *
 * TEST INFRASTRUCTURE ONLY (see pat_oracle.h).  Plain loops, FP64, OpenMP over
 * independent outputs.  Every function follows one step of the discrete
 * operator read from eq. (1)-(3) of Sec. 2.1 and the "polar grid in the
 * spectral domain" of Sec. 2.4.1:
 *
 *   step 1  F(n,l) = h^2 sum_{i,j} m_ij f_ij e^{-i lam_n (x_j cos psi_l + y_i sin psi_l)}
 *           (the exact pixel Fourier transform at the polar points, all l)
 *   steps 2-5, plane-wave form (Jacobi-Anger summed back, so no Bessel function):
 *           g(d,j) = sum_n W_n cos(c lam_n t_j) Re[(1/Npsi) sum_l F(n,l) e^{i lam_n R cos(theta_d-psi_l)}]
 *                    + kappa * h^2 sum m f
 *
 * The exact Fourier solution of eq. (1) at a detector x_d is
 *   p(x_d,t) = (2 pi)^-2 int fhat(xi) cos(c|xi|t) e^{i x_d.xi} dxi;
 * in polar frequency coordinates xi = lam (cos psi, sin psi), dxi = lam dlam dpsi,
 * the lam-integral is the rectangle rule with nodes lam_n = n dlam (weight
 * lam_n dlam, the node lam=0 has weight 0) and the psi-integral the uniform
 * Npsi-point rule, which together give W_n = lam_n dlam / (2 pi) and 1/Npsi.
 * kappa = dlam^2/(24 pi) cancels the leading Euler-Maclaurin endpoint term of
 * that rectangle rule (the k=0 mode integrand has derivative fhat(0)/(2 pi) at 0).
 *
 * A* is the plain matrix transpose under unweighted Euclidean inner products,
 * which is what a gradient of ||A f - g||^2 needs (Sec. 2.2).
 */
#include "pat_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double PI = 3.14159265358979323846264338327950288;

static int g_threads = 0;

void oracle_set_threads(int nthreads) { g_threads = nthreads > 0 ? nthreads : 0; }

int oracle_get_threads(void)
{
#ifdef _OPENMP
    return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
    return 1;
#endif
}

/* smallest 2^a 3^b >= x */
static long smooth23_at_least(double x)
{
    long best = -1;
    for (long p2 = 1; p2 < (1L << 40); p2 *= 2) {
        for (long p = p2; ; p *= 3) {
            if ((double)p >= x) {
                if (best < 0 || p < best) best = p;
                break;
            }
        }
        if ((double)p2 >= x) break;
    }
    return best;
}

int oracle_derive(const oracle_geom* g, oracle_sizes* s)
{
    if (!g || !s) return -1;
    if (g->n < 2 || g->n_det < 1 || g->n_t < 1) return -1;
    if (!(g->dt > 0) || !(g->c > 0) || !(g->det_r > 0) || !(g->support_r > 0)) return -1;
    if (!(g->arc_span > 0) || g->arc_span > 2 * PI + 1e-12) return -1;
    if (!(g->lambda_oversample >= 1)) return -1;
    if (g->support_r > g->det_r) return -1;
    double h = 2.0 / g->n;
    s->M = (int)smooth23_at_least(g->lambda_oversample * g->n_t);
    s->dlam = PI / (s->M * g->c * g->dt);
    /* lam_max <= pi/h (pixel Nyquist): n_lam = floor((pi/h)/dlam) = floor(M c dt / h) */
    s->n_lam = (int)floor(s->M * g->c * g->dt / h + 1e-9);
    if (s->n_lam < 1) return -1;
    double z = s->n_lam * s->dlam * g->det_r;
    s->K = (int)ceil(z + 10.0 * cbrt(z) - 1e-9);
    long np = 2L * s->K + 2;
    for (;;) {
        long cand = smooth23_at_least((double)np);
        if (cand % 4 == 0) { s->n_psi = (int)cand; break; }
        np = cand + 1;
    }
    s->kappa = g->em_correction ? s->dlam * s->dlam / (24.0 * PI) : 0.0;
    return 0;
}

/* ---- grid helpers ------------------------------------------------------- */

static double pix(const oracle_geom* g, int k) { return -1.0 + (k + 0.5) * (2.0 / g->n); }

static int in_mask(const oracle_geom* g, int i, int j)
{
    double x = pix(g, j), y = pix(g, i);
    return x * x + y * y < g->support_r * g->support_r;
}

/* detector angle: explicit, or uniform on the arc (cell-centred elements) */
static double theta_det(const oracle_geom* g, int d)
{
    if (g->det_theta) return g->det_theta[d];
    return g->arc_center - 0.5 * g->arc_span + (d + 0.5) * g->arc_span / g->n_det;
}

static double psi_at(const oracle_sizes* s, int l) { return 2.0 * PI * l / s->n_psi; }
static double lam_at(const oracle_sizes* s, int n) { return n * s->dlam; }        /* n = 1..n_lam */
static double W_at(const oracle_sizes* s, int n) { return lam_at(s, n) * s->dlam / (2.0 * PI); }
static double t_at(const oracle_geom* g, int j) { return j * g->dt; }               /* j = 1..T */

static double mass_of(const oracle_geom* g, const double* f)
{
    double h = 2.0 / g->n, m = 0.0;
    for (int i = 0; i < g->n; ++i)
        for (int j = 0; j < g->n; ++j)
            if (in_mask(g, i, j)) m += f[(size_t)i * g->n + j];
    return h * h * m;
}

/* ---- step 1: polar pixel DFT --------------------------------------------- */

void oracle_polar_spectrum(const oracle_geom* g, const double* f, double* F)
{
    oracle_sizes s;
    if (oracle_derive(g, &s)) return;
    const int N = g->n;
    const double h = 2.0 / N;
    double* mf = (double*)malloc(sizeof(double) * N * N);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            mf[(size_t)i * N + j] = in_mask(g, i, j) ? f[(size_t)i * N + j] : 0.0;
    const long npairs = (long)s.n_lam * s.n_psi;
#pragma omp parallel num_threads(oracle_get_threads())
    {
        double* cx = (double*)malloc(sizeof(double) * N);
        double* sx = (double*)malloc(sizeof(double) * N);
#pragma omp for schedule(static)
        for (long q = 0; q < npairs; ++q) {
            int n = 1 + (int)(q / s.n_psi), l = (int)(q % s.n_psi);
            double lam = lam_at(&s, n), psi = psi_at(&s, l);
            double kx = lam * cos(psi), ky = lam * sin(psi);
            for (int j = 0; j < N; ++j) { cx[j] = cos(kx * pix(g, j)); sx[j] = sin(kx * pix(g, j)); }
            double re = 0.0, im = 0.0;
            for (int i = 0; i < N; ++i) {
                /* row sum: sum_j mf_ij e^{-i kx x_j} = a - i b */
                double a = 0.0, b = 0.0;
                const double* row = mf + (size_t)i * N;
#pragma omp simd reduction(+ : a, b)
                for (int j = 0; j < N; ++j) { a += row[j] * cx[j]; b += row[j] * sx[j]; }
                double cy = cos(ky * pix(g, i)), sy = sin(ky * pix(g, i));
                /* (cy - i sy)(a - i b) = (cy a - sy b) - i (sy a + cy b) */
                re += cy * a - sy * b;
                im -= sy * a + cy * b;
            }
            F[2 * q] = h * h * re;
            F[2 * q + 1] = h * h * im;
        }
        free(cx);
        free(sx);
    }
    free(mf);
}

/* ---- steps 2-5: plane-wave synthesis at the detectors -------------------- */

void oracle_polar_to_data(const oracle_geom* g, const double* F, double mass, double* out)
{
    oracle_sizes s;
    if (oracle_derive(g, &s)) return;
    const int D = g->n_det, T = g->n_t, NL = s.n_lam, NP = s.n_psi;
    /* P(n,d) = Re[(1/Npsi) sum_l F(n,l) e^{i lam_n R cos(theta_d - psi_l)}] */
    double* P = (double*)malloc(sizeof(double) * (size_t)NL * D);
#pragma omp parallel for schedule(static) num_threads(oracle_get_threads())
    for (long q = 0; q < (long)NL * D; ++q) {
        int n = 1 + (int)(q / D), d = (int)(q % D);
        double lam = lam_at(&s, n), th = theta_det(g, d), acc = 0.0;
        const double* Fn = F + 2 * (size_t)(n - 1) * NP;
        for (int l = 0; l < NP; ++l) {
            double ph = lam * g->det_r * cos(th - psi_at(&s, l));
            acc += Fn[2 * l] * cos(ph) - Fn[2 * l + 1] * sin(ph);
        }
        P[q] = acc / NP;
    }
    /* g(d,j) = sum_n W_n cos(c lam_n t_j) P(n,d) + kappa * mass */
#pragma omp parallel for schedule(static) num_threads(oracle_get_threads())
    for (long q = 0; q < (long)D * T; ++q) {
        int d = (int)(q / T), j = 1 + (int)(q % T);
        double acc = 0.0;
        for (int n = 1; n <= NL; ++n)
            acc += W_at(&s, n) * cos(g->c * lam_at(&s, n) * t_at(g, j)) * P[(size_t)(n - 1) * D + d];
        out[q] = acc + s.kappa * mass;
    }
    free(P);
}

int oracle_forward(const oracle_geom* g, const double* f, double* out)
{
    oracle_sizes s;
    if (oracle_derive(g, &s)) return -1;
    double* F = (double*)malloc(sizeof(double) * 2 * (size_t)s.n_lam * s.n_psi);
    if (!F) return -1;
    oracle_polar_spectrum(g, f, F);
    oracle_polar_to_data(g, F, mass_of(g, f), out);
    free(F);
    return 0;
}

/* ---- transposes ---------------------------------------------------------- */

/* Transpose of steps 2-5 (without the kappa term):
 *   Q(n,d)   = W_n sum_j cos(c lam_n t_j) data(d,j)
 *   Ft(n,l)  = (1/Npsi) sum_d Q(n,d) e^{-i lam_n R cos(theta_d - psi_l)}
 * (the transpose of z -> Re[z e^{i phi}] is q -> q e^{-i phi}). */
void oracle_data_to_polar(const oracle_geom* g, const double* data, double* Ft)
{
    oracle_sizes s;
    if (oracle_derive(g, &s)) return;
    const int D = g->n_det, T = g->n_t, NL = s.n_lam, NP = s.n_psi;
    double* Q = (double*)malloc(sizeof(double) * (size_t)NL * D);
#pragma omp parallel for schedule(static) num_threads(oracle_get_threads())
    for (long q = 0; q < (long)NL * D; ++q) {
        int n = 1 + (int)(q / D), d = (int)(q % D);
        double acc = 0.0;
        for (int j = 1; j <= T; ++j)
            acc += cos(g->c * lam_at(&s, n) * t_at(g, j)) * data[(size_t)d * T + (j - 1)];
        Q[q] = W_at(&s, n) * acc;
    }
#pragma omp parallel for schedule(static) num_threads(oracle_get_threads())
    for (long q = 0; q < (long)NL * NP; ++q) {
        int n = 1 + (int)(q / NP), l = (int)(q % NP);
        double lam = lam_at(&s, n), psi = psi_at(&s, l), re = 0.0, im = 0.0;
        for (int d = 0; d < D; ++d) {
            double ph = lam * g->det_r * cos(theta_det(g, d) - psi);
            double qv = Q[(size_t)(n - 1) * D + d];
            re += qv * cos(ph);
            im -= qv * sin(ph);
        }
        Ft[2 * q] = re / NP;
        Ft[2 * q + 1] = im / NP;
    }
    free(Q);
}

/* Transpose of step 1 plus the kappa term:
 *   f(i,j) = m_ij [ h^2 Re sum_{n,l} Ft(n,l) e^{+i lam_n (x_j cos psi_l + y_i sin psi_l)} + kappa h^2 data_sum ]
 * Each thread accumulates a private image over its share of (n,l); the private
 * images are added in thread order. */
void oracle_polar_to_image(const oracle_geom* g, const double* Ft, double data_sum, double* f)
{
    oracle_sizes s;
    if (oracle_derive(g, &s)) return;
    const int N = g->n, NP = s.n_psi;
    const double h = 2.0 / N;
    const long npairs = (long)s.n_lam * NP;
    const int nth = oracle_get_threads();
    double* acc = (double*)calloc((size_t)nth * N * N, sizeof(double));
#pragma omp parallel num_threads(nth)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* mine = acc + (size_t)tid * N * N;
        double* cx = (double*)malloc(sizeof(double) * N);
        double* sx = (double*)malloc(sizeof(double) * N);
#pragma omp for schedule(static)
        for (long q = 0; q < npairs; ++q) {
            int n = 1 + (int)(q / NP), l = (int)(q % NP);
            double lam = lam_at(&s, n), psi = psi_at(&s, l);
            double kx = lam * cos(psi), ky = lam * sin(psi);
            double fr = Ft[2 * q], fi = Ft[2 * q + 1];
            for (int j = 0; j < N; ++j) { cx[j] = cos(kx * pix(g, j)); sx[j] = sin(kx * pix(g, j)); }
            for (int i = 0; i < N; ++i) {
                double cy = cos(ky * pix(g, i)), sy = sin(ky * pix(g, i));
                /* u = Ft e^{i ky y_i} */
                double ur = fr * cy - fi * sy, ui = fr * sy + fi * cy;
                double* row = mine + (size_t)i * N;
                /* Re(u e^{i kx x_j}) = ur cos - ui sin */
                for (int j = 0; j < N; ++j) row[j] += ur * cx[j] - ui * sx[j];
            }
        }
        free(cx);
        free(sx);
    }
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double v = 0.0;
            for (int t = 0; t < nth; ++t) v += acc[(size_t)t * N * N + (size_t)i * N + j];
            f[(size_t)i * N + j] = in_mask(g, i, j) ? h * h * v + s.kappa * h * h * data_sum : 0.0;
        }
    free(acc);
}

static double sum_of(const double* v, long n)
{
    double a = 0.0;
    for (long k = 0; k < n; ++k) a += v[k];
    return a;
}

int oracle_adjoint(const oracle_geom* g, const double* data, double* f)
{
    oracle_sizes s;
    if (oracle_derive(g, &s)) return -1;
    double* Ft = (double*)malloc(sizeof(double) * 2 * (size_t)s.n_lam * s.n_psi);
    if (!Ft) return -1;
    oracle_data_to_polar(g, data, Ft);
    oracle_polar_to_image(g, Ft, sum_of(data, (long)g->n_det * g->n_t), f);
    free(Ft);
    return 0;
}

int oracle_adjoint_pixels(const oracle_geom* g, const double* data, int npix,
                          const int* idx, double* out)
{
    oracle_sizes s;
    if (oracle_derive(g, &s)) return -1;
    const int N = g->n, NP = s.n_psi;
    const double h = 2.0 / N;
    double* Ft = (double*)malloc(sizeof(double) * 2 * (size_t)s.n_lam * NP);
    if (!Ft) return -1;
    oracle_data_to_polar(g, data, Ft);
    double dsum = sum_of(data, (long)g->n_det * g->n_t);
#pragma omp parallel for schedule(dynamic, 1) num_threads(oracle_get_threads())
    for (int q = 0; q < npix; ++q) {
        int i = idx[q] / N, j = idx[q] % N;
        if (!in_mask(g, i, j)) { out[q] = 0.0; continue; }
        double x = pix(g, j), y = pix(g, i), acc = 0.0;
        for (int n = 1; n <= s.n_lam; ++n)
            for (int l = 0; l < NP; ++l) {
                double lam = lam_at(&s, n), psi = psi_at(&s, l);
                double ph = lam * (x * cos(psi) + y * sin(psi));
                const double* Fq = Ft + 2 * ((size_t)(n - 1) * NP + l);
                acc += Fq[0] * cos(ph) - Fq[1] * sin(ph);
            }
        out[q] = h * h * acc + s.kappa * h * h * dsum;
    }
    free(Ft);
    return 0;
}
