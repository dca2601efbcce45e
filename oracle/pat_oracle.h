/*
 * pat_oracle.h -- FP64 CPU oracle for the circular-geometry PAT operator pair.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, plain, direct-sum definition of
 * the discrete forward operator A and its transpose A*, used to check the GPU
 * library.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or constant with the
 * GPU path.
 *
 * Physics: eq. (1) (wave IVP with constant speed c, zero initial velocity) and
 * eq. (2) (boundary traces on a detector circle / arc Gamma_m, Sec. 2.1); the
 * data are g = A f (eq. (3)).  The discretisation (Sec. 2.4.1 says only "polar
 * grid computations in the spectral domain") is the documented reading:
 *
 *   F(n,l)  = h^2 sum_{i,j} m_ij f_ij exp(-i lam_n (x_j cos psi_l + y_i sin psi_l))
 *   g(d,j)  = sum_n W_n cos(c lam_n t_j) Re[(1/Npsi) sum_l F(n,l) exp(i lam_n R cos(theta_d - psi_l))]
 *             + kappa * h^2 sum m f
 *
 * evaluated by direct sums (no FFT, no Bessel function), and its exact transpose.
 */
#ifndef PAT_ORACLE_H
#define PAT_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int    n;                 /* grid side N; cell-centred pixels on [-1,1]^2     */
    double support_r;         /* rho_s: pixel kept iff x^2+y^2 < rho_s^2          */
    double det_r;             /* R: detector circle radius                         */
    int    n_det;             /* D                                                  */
    double arc_center;        /* theta_c [rad]                                      */
    double arc_span;          /* alpha in (0, 2pi]                                  */
    int    n_t;               /* T; t_j = j*dt for j = 1..T                         */
    double dt;
    double c;                 /* speed of sound                                     */
    double lambda_oversample; /* sigma_t                                            */
    int    em_correction;     /* 1: add the rank-1 endpoint (kappa) term            */
    const double* det_theta;  /* NULL, or D explicit detector angles [rad] that
                                 replace the uniform arc (arc_* then unused)       */
} oracle_geom;

typedef struct {
    int    M;       /* smallest 2^a3^b >= sigma_t*T                                 */
    double dlam;    /* pi / (M c dt)                                                */
    int    n_lam;   /* floor(M c dt / h + 1e-9)                                     */
    int    K;       /* ceil(z + 10 z^(1/3) - 1e-9), z = n_lam*dlam*R                */
    int    n_psi;   /* smallest 2^a3^b >= 2K+2 that is divisible by 4               */
    double kappa;   /* dlam^2/(24 pi) if em_correction else 0                        */
} oracle_sizes;

/* Derive the operator-defining sizes; returns 0 on success, -1 on bad input. */
int oracle_derive(const oracle_geom* g, oracle_sizes* s);

/* Number of OpenMP threads the oracle uses (0 = library default). */
void oracle_set_threads(int nthreads);
int  oracle_get_threads(void);

/* Step 1 on the full polar grid: F is [n_lam][n_psi] complex, interleaved re/im. */
void oracle_polar_spectrum(const oracle_geom* g, const double* f, double* F);
/* Steps 2-5 in plane-wave form: F (as above) and the mass h^2 sum m f -> g [D][T]. */
void oracle_polar_to_data(const oracle_geom* g, const double* F, double mass, double* out);
/* Transposes of the two steps above. */
void oracle_data_to_polar(const oracle_geom* g, const double* data, double* Ft);
void oracle_polar_to_image(const oracle_geom* g, const double* Ft, double data_sum, double* f);

/* Whole operator pair: f [N][N] (row i = y_i, column j = x_j) <-> g [D][T]. */
int oracle_forward(const oracle_geom* g, const double* f, double* out);
int oracle_adjoint(const oracle_geom* g, const double* data, double* f);
/* A* evaluated only at the listed pixels (flat index i*N+j); out[q] for idx[q]. */
int oracle_adjoint_pixels(const oracle_geom* g, const double* data, int npix,
                          const int* idx, double* out);

#ifdef __cplusplus
}
#endif
#endif
