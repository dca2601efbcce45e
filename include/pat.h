/*
 * pat.h -- C-ABI of the MI355X (gfx950) photoacoustic-tomography operator library.
 *
 * The library evaluates the forward operator A of eq. (3) (Sec. 2.1): the 2D
 * wave initial-value problem of eq. (1) with constant speed of sound c, zero
 * initial velocity and initial pressure f, observed as the boundary traces of
 * eq. (2) at detectors on a circle of radius R (or an arc of it, the limited
 * view of Sec. 2.1), and its exact discrete adjoint A* (the plain matrix
 * transpose), which the gradient-based reconstructions of eq. (4) and eq. (5)
 * call once per iteration (Sec. 2.2).  The discretisation is the "polar grid
 * in the spectral domain" of Sec. 2.4.1:
 *
 *   F(n,l) = h^2 sum m_ij f_ij exp(-i lam_n (x_j cos psi_l + y_i sin psi_l))   (polar pixel spectrum)
 *   F_k(n) = angular Fourier coefficients of F(n, .), |k| <= K
 *   b_k(n) = i^k J_k(lam_n R) W_n F_k(n),  W_n = lam_n dlam / (2 pi)
 *   B_k(j) = sum_n b_k(n) cos(c lam_n t_j)
 *   g(d,j) = Re sum_k e^{i k theta_d} B_k(j) + kappa h^2 sum m f,  kappa = dlam^2/(24 pi)
 *
 * with lam_n = n dlam (n = 1..n_lam), dlam = pi/(M c dt), M the smallest
 * 2^a 3^b >= sigma_t T, lam_{n_lam} <= pi/h, pixel centres x_j = -1 + (j+1/2) h,
 * h = 2/N, mask m_ij = [x_j^2 + y_i^2 < rho_s^2], detectors
 * theta_d = theta_c - alpha/2 + (d+1/2) alpha/D, times t_j = j dt (j = 1..T).
 *
 * Layouts (all row-major, FP32, caller-owned device memory):
 *   image f : [batch][N][N]   row i is y_i (increasing), column j is x_j
 *   data  g : [batch][D][T]   detector-major, column j-1 is t_j
 *
 * Execution model: every compute call is asynchronous and stream-ordered on
 * the HIP stream passed in (`stream`, a hipStream_t; NULL = default stream).
 * No call allocates, frees or synchronises.  All argument checks run on the
 * host before anything is enqueued, so an error return means nothing was
 * launched.  Plans own their device tables; the caller owns every tensor and
 * the workspace.  A plan may be used concurrently from several streams only
 * with distinct workspaces.
 */
#ifndef PAT_H
#define PAT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define PAT_OK               0
#define PAT_ERR_ARG         -1   /* bad argument: null pointer, size out of range, batch > capacity */
#define PAT_ERR_UNSUPPORTED -2   /* geometry outside what the kernels handle (LDS or size limits) */
#define PAT_ERR_WORKSPACE   -3   /* workspace missing or smaller than pat_workspace_size()       */
#define PAT_ERR_HIP         -4   /* a HIP runtime call failed (launch, copy, event)               */
#define PAT_ERR_ALLOC       -5   /* device allocation failed while building a plan                */

typedef struct pat_plan pat_plan;

/* Geometry and discretisation of one operator (eq. (1)-(3), Sec. 2.1 and 2.4.1). */
typedef struct {
    int    n;                 /* grid side N >= 16; cell-centred pixels on [-1,1]^2, h = 2/N         */
    double support_r;         /* rho_s in (0, det_r]: pixels with x^2+y^2 >= rho_s^2 are zero (1.0) */
    double det_r;             /* R > 0: detector circle radius (1.0)                                  */
    int    n_det;             /* D >= 1                                                               */
    double arc_center;        /* theta_c [rad] (-pi/2: the array at the bottom)                       */
    double arc_span;          /* alpha in (0, 2 pi]; 2 pi = full circle                               */
    int    n_t;               /* T >= 1; t_j = j * dt for j = 1..T                                    */
    double dt;                /* > 0                                                                  */
    double c;                 /* constant speed of sound > 0                                          */
    double lambda_oversample; /* sigma_t >= 1 (2.0); radial frequency step dlam = pi/(M c dt)         */
    int    em_correction;     /* 1: add the rank-1 endpoint term kappa*h^2*sum(m f) (default 1)       */
    int    max_batch;         /* capacity of the batch dimension (>= 1); sizes pat_workspace_size.
                                 1 also selects the single-instance work split of the adjoint's
                                 spread (more, shorter work rows while their partial rows take at
                                 most 32 MiB per instance), so plans that differ only here may
                                 differ in the last bits of A* g                                  */
    const double* det_theta;  /* NULL: the uniform arc above.  Else D explicit detector angles [rad],
                                 any order and spacing (gaps, several arcs, sparse elements), in host
                                 memory read only during pat_plan_create / pat_plan_derive (the plan
                                 keeps a copy); arc_center and arc_span are then unused.  The angular
                                 synthesis Re sum_k e^{ik theta_d} B_k of eq. (2) then runs as a dense
                                 product on the matrix cores instead of an FFT.                       */
} pat_plan_desc;

/* What a plan derived (pat_plan_query). */
typedef struct {
    int    M;                 /* length of the radial/temporal cosine grid                            */
    double dlam;              /* radial frequency step                                                */
    int    n_lam;             /* number of radial frequencies lam_n = n*dlam, n = 1..n_lam            */
    int    K;                 /* highest angular mode, ceil(z + 10 z^(1/3)), z = lam_max R            */
    int    n_psi;             /* uniform angular grid size (smallest 2^a3^b >= 2K+2, multiple of 4)    */
    double kappa;             /* endpoint-term coefficient dlam^2/(24 pi), 0 if disabled              */
    int    n_grid;            /* oversampled spectral grid side used for the polar interpolation      */
    int    n_points;          /* polar points evaluated per image (half plane, per-ring angular grids) */
    int    len_czt;           /* FFT length of the synthesis over detector angles: P when the detector
                                 pitch is 2 pi s / P (P = 2^a 3^b, integer s), else the chirp-z length
                                 >= K + D                                                             */
    int    syn_stride;        /* s in that case (detector d sits at point s d of the P-point grid),
                                 0 for the chirp-z synthesis                                          */
    int    syn_dense;         /* 1: explicit detector angles; the synthesis is the product of the
                                 (K+1)-mode coefficients with a [2(K+1)][D] cos/sin table (len_czt,
                                 syn_stride 0)                                                        */
    int    n_ring_modes;      /* sum over radial frequencies of the angular modes kept (K_n + 1)       */
    size_t workspace_per_instance; /* workspace bytes per batch instance                              */
    size_t table_bytes;       /* device bytes held by the plan's tables                               */
} pat_plan_info;

/* Build a plan: derive sizes, compute every table in FP64 on the host, upload
 * them as FP32 device tables (hipMalloc; freed by pat_plan_destroy).  The
 * current HIP device at creation is the plan's device.  Returns PAT_OK and
 * sets *out, or an error code and leaves *out untouched. */
int  pat_plan_create(const pat_plan_desc* desc, pat_plan** out);
int  pat_plan_query(const pat_plan* plan, pat_plan_info* out);
void pat_plan_destroy(pat_plan* plan);

/* Workspace bytes a forward or adjoint call needs for `batch` instances
 * (0 if plan is NULL or batch < 1).  The workspace is scratch only: its
 * contents on entry are ignored and on exit are unspecified. */
size_t pat_workspace_size(const pat_plan* plan, int batch);

/* g = A f for `batch` images (1 <= batch <= max_batch).
 * f: device [batch][N][N] FP32 (read); g: device [batch][D][T] FP32 (written).
 * ws: device workspace of at least pat_workspace_size(plan, batch) bytes.
 * The call enqueues its kernels and returns; they are ordered on `stream`.
 * A call of at least the plan's split batch (pat_plan_set_split) runs the
 * second half of its instances on a stream the plan owns, forked from and
 * joined back to `stream` by events, so the call can still be recorded into a
 * HIP graph from `stream`; calls sharing a plan from several host threads are
 * serialised for that fork-launch-join sequence only.
 * Errors: PAT_ERR_ARG (null pointer, batch out of range), PAT_ERR_WORKSPACE,
 * PAT_ERR_HIP (launch failure). */
int  pat_forward(const pat_plan* plan, const float* f, float* g, int batch,
                 void* ws, size_t ws_bytes, void* stream);

/* f = A* g (exact transpose of pat_forward under the plain Euclidean inner
 * products of R^{N x N} and R^{D x T}; this is the gradient of 0.5||A f - g||^2
 * with respect to f at residual g, Sec. 2.2).
 * g: device [batch][D][T] FP32 (read); f: device [batch][N][N] FP32 (written).
 * Same workspace and error rules as pat_forward. */
int  pat_adjoint(const pat_plan* plan, const float* g, float* f, int batch,
                 void* ws, size_t ws_bytes, void* stream);

/* g = A f without a caller workspace, for callers that cannot allocate device
 * memory (code recorded into a HIP graph, tight serving loops, harnesses that
 * forbid hipMalloc).  Same operator, kernels, launch shapes and results as
 * pat_forward (bitwise); the workspace is instead a device array of
 * PAT_NOALLOC_SCRATCH_BYTES (128 MiB) inside the library, one per GPU, held
 * from the first call on that GPU until the process ends.  f, g, batch,
 * stream: as for pat_forward; the current HIP device must be the plan's.
 * The call allocates and frees nothing (the first call on a device looks up
 * the array's device address once).  All calls on one GPU share the array:
 * calls that overlap on one GPU (other streams, other threads) race, so a
 * caller serialises them.  Errors: PAT_ERR_ARG (null pointer, batch out of
 * range, current device is not the plan's), PAT_ERR_WORKSPACE
 * (pat_workspace_size(plan, batch) exceeds PAT_NOALLOC_SCRATCH_BYTES),
 * PAT_ERR_HIP. */
#define PAT_NOALLOC_SCRATCH_BYTES (128u * 1024u * 1024u)
int  pat_forward_noalloc(const pat_plan* plan, const float* f, float* g, int batch, void* stream);

/* Smoothed isotropic total variation of eq. (4)/(5) (Sec. 2.1, 2.2):
 *   TV_eps(f) = sum_{i,j} sqrt((f_{i,j+1}-f_{i,j})^2 + (f_{i+1,j}-f_{i,j})^2 + eps^2)
 * with forward differences and zero difference across the last row/column
 * (Neumann boundary).  Writes grad = d TV_eps / d f ([batch][N][N]) and, if
 * tv is not NULL, tv[b] = TV_eps(f_b) ([batch], FP32).
 * Errors: PAT_ERR_ARG (null f/grad, n < 2, batch < 1, eps <= 0), PAT_ERR_HIP. */
int  pat_tv_grad(const float* f, float* grad, float* tv, int n, int batch, float eps,
                 void* stream);

/* One projected-gradient step of eq. (4) with smoothed TV, fused:
 *   f <- max(f - tau * (adj + lambda * tvgrad), 0)     (elementwise, in place on f)
 * f, adj, tvgrad: device [count] FP32.  Errors: PAT_ERR_ARG, PAT_ERR_HIP. */
int  pat_pgd_update(float* f, const float* adj, const float* tvgrad, long count,
                    float tau, float lambda, void* stream);

/* Residual r = A f - g_meas computed in place on `g` (g holds A f on entry),
 * and, if sq is not NULL, sq[b] = 0.5 * ||r_b||^2 per instance (FP32).
 * g, g_meas: device [batch][count_per] FP32.  Errors: PAT_ERR_ARG, PAT_ERR_HIP. */
int  pat_residual(float* g, const float* g_meas, float* sq, long count_per, int batch,
                  void* stream);

/* Primal-dual TV reconstruction (the classical baseline of Sec. 2.1:
 * min_{f >= 0} 0.5 ||A f - g||^2 + alpha TV(f), solved with the primal-dual
 * hybrid gradient method the paper cites, stopped on the relative change of
 * Sec. 2.3).  With K = (A, grad), one iteration is
 *   A fbar -> ax (pat_forward);  pat_pd_dual_data;  pat_pd_dual_tv;
 *   A* y1 -> aty (pat_adjoint);  pat_pd_primal;  [pat_pd_change]
 * with step sizes sigma tau (||A||^2 + 8) < 1.  TV is the isotropic total
 * variation with forward differences and a zero difference across the last
 * row / column (Neumann boundary).  All buffers are device FP32, [batch]-major.
 * pat_pd_dual_data: y1 <- (y1 + sigma (ax - g)) / (1 + sigma), count elements.
 * pat_pd_dual_tv:   y2 <- projection of y2 + sigma grad(xbar) onto
 *                   {|y2_ij| <= alpha}; y2 [batch][n][n][2] (x, y components).
 * pat_pd_primal:    f' = max(f - tau (aty + grad* y2), 0); xbar <- 2 f' - f;
 *                   f <- f' (f, xbar, aty [batch][n][n]; in place).
 * pat_pd_change:    out[2b] = ||xbar_b - f_b||^2 = ||f'_b - f_b(old)||^2 and
 *                   out[2b+1] = ||f_b||^2 right after pat_pd_primal (fixed-order sums).
 * Errors: PAT_ERR_ARG (NULL, n < 2, batch < 1, sigma or tau <= 0, alpha < 0), PAT_ERR_HIP. */
int  pat_pd_dual_data(float* y1, const float* ax, const float* g, long count, float sigma, void* stream);
int  pat_pd_dual_tv(float* y2, const float* xbar, int n, int batch, float sigma, float alpha, void* stream);
int  pat_pd_primal(float* f, float* xbar, const float* aty, const float* y2, int n, int batch, float tau,
                   void* stream);
int  pat_pd_change(const float* f, const float* xbar, float* out, int n, int batch, void* stream);

/* CGLS: conjugate gradients on the normal equations A* A f = A* g, the
 * iterative stand-in for the fast inverse that produces the network input of
 * the deep image prior (Sec. 2.2; the paper takes a closed-form inversion
 * from the cited literature).  From f_0: r = g - A f_0, s = A* r, p = s,
 * gamma = <s, s>; one step, with every scalar on the device (graph-capturable):
 *   q = A p (pat_forward);            pat_cg_norm2(q -> qq)
 *   pat_cg_step_fr:  alpha = gamma / qq;  f += alpha p;  r -= alpha q
 *   s = A* r (pat_adjoint);           pat_cg_norm2(s -> gamma_new)
 *   pat_cg_step_p:   p = s + (gamma_new / gamma) p
 * after which gamma_new is the next step's gamma (callers alternate two
 * buffers).  Per instance b < batch, with [batch]-major device FP32 arrays:
 * pat_cg_norm2:   out[b] = sum of x_b^2 over its `count` elements (fixed order).
 * pat_cg_step_fr: f_b, p_b have nf elements, r_b, q_b nr; gamma, qq [batch];
 *                 alpha = 0 where qq_b = 0.
 * pat_cg_step_p:  p_b, s_b have n elements; beta = 0 where gamma_b = 0.
 * Errors: PAT_ERR_ARG (NULL, counts or batch < 1), PAT_ERR_HIP. */
int  pat_cg_norm2(const float* x, float* out, long count, int batch, void* stream);
int  pat_cg_step_fr(float* f, const float* p, long nf, float* r, const float* q, long nr, const float* gamma,
                    const float* qq, int batch, void* stream);
int  pat_cg_step_p(float* p, const float* s, long n, const float* gamma_new, const float* gamma, int batch,
                   void* stream);

/* Per-kernel timing.  pat_profile_enable(plan, 1) creates HIP events; from
 * then on every pat_forward / pat_adjoint call on `plan` records an event
 * before and after each of its kernels on the call's stream (a few
 * microseconds of overhead; 0 disables and frees the events).
 * pat_profile_read waits for the last call of direction `which` (0 = forward,
 * 1 = adjoint) to finish and writes its kernel durations in milliseconds to
 * ms[0..*count-1], in launch order (forward: column pass, row pass, polar
 * interpolation, ring (angular FFT, weights, detector synthesis), cosine transform;
 * adjoint: cosine transform, ring, spread, row pass, column pass).  With
 * explicit detector angles the dense synthesis follows the ring in the forward
 * and precedes it in the adjoint (six durations per direction).  Errors: PAT_ERR_ARG (NULL, profiling off,
 * max_kernels too small), PAT_ERR_HIP. */
int  pat_profile_enable(pat_plan* plan, int enable);
int  pat_profile_read(const pat_plan* plan, int which, float* ms, int max_kernels, int* count);

/* Device copy of `bytes` bytes, the measured-bandwidth yardstick that the
 * roofline fractions of the operator kernels are quoted against (besides the
 * published 8 TB/s), and a copy of known size that calibrates the HBM byte
 * counters.  perm == NULL: dst = src, 16-byte elements (bytes, src and dst
 * multiples of 16).  perm != NULL: the 8-byte scatter dst[perm[e]] = src[e]
 * for e < bytes/8 (src, dst 8-byte aligned), perm a DEVICE array of bytes/8
 * indices in [0, bytes/8) (not inspected on the host; the caller guarantees
 * the range).  Asynchronous on `stream`.  Errors: PAT_ERR_ARG (NULL,
 * zero bytes, misaligned size or pointer), PAT_ERR_HIP. */
int  pat_stream_copy(const void* src, void* dst, size_t bytes, const int* perm, void* stream);

/* Launch shapes of a plan's kernels (tile sizes; none changes the result
 * beyond the summation order of the scalar endpoint/data sums).
 * pat_plan_create picks defaults for max_batch; pat_autotune_plan measures. */
typedef struct {
    int col_np;   /* column pairs per column-pass workgroup, 1..16                           */
    int row_rpb;  /* spectrum rows per row-pass workgroup, 1..16                             */
    int ring_rt;  /* radial frequencies (rings) per ring-kernel workgroup, 1..64             */
    int dct_dp;   /* detector pairs per cosine-transform workgroup, 1..16                    */
    int gat_cb;   /* polar-interpolation tile width in grid columns: 32, 64, 128 or 256      */
    int gat_th;   /* interpolation bands (footprint base rows) per tile: 1, 2, 4, .., 64;
                     the tile window (gat_th + 7) x (gat_cb + 7) x 8 bytes is at most 64 KB  */
    int spr_cb;   /* spread workgroup width: 64, 128, 192 or 256 columns                     */
    int spr_th;   /* spread rows (bands) per workgroup: always 8.  Each workgroup sweeps its
                     own 8 bands; a band's footprint reaches 7 rows further, and those
                     partial rows are completed in the adjoint row pass, so every grid
                     row is summed in one fixed order for every launch shape             */
    int gat_ib;   /* instances of a batch sharing one interpolation tile: 1, 2 or 4 (the
                     ES weights and indexing are shared; windows: gat_ib x the size above) */
    int spr_ib;   /* instances of a batch sharing one spread tile: 1, 2 or 4              */
} pat_launch;

/* pat_plan_get_launch copies the plan's launch shapes.  pat_plan_set_launch
 * replaces them after checking them on the host: PAT_ERR_ARG for a field out
 * of range, PAT_ERR_UNSUPPORTED if a tile needs more than the 160 KB of LDS
 * or the 1024 threads a workgroup can have; on error the plan is unchanged.
 * Calls already enqueued keep the shapes they were launched with.  The
 * workspace size does not depend on the launch shapes. */
int  pat_plan_get_launch(const pat_plan* plan, pat_launch* out);
int  pat_plan_set_launch(pat_plan* plan, const pat_launch* cfg);

/* Two-stream calls.  pat_forward / pat_adjoint calls of at least `min_batch`
 * instances run instances [0, batch/2) on the caller's stream and the rest on
 * a second stream of the plan, so that one half's kernels occupy the compute
 * units the other half's last partial waves leave idle.  The outputs are
 * bitwise those of one stream (every instance runs the same kernels and
 * tiles).  min_batch 0 or 1 turns it off; the default is 64, and
 * pat_autotune_plan times calls at its batch both ways and sets min_batch to
 * that batch if two streams are faster, else to 0.  Calls under per-kernel
 * timing (pat_profile_enable) always use one stream.
 * Errors: PAT_ERR_ARG (NULL plan or pointer, min_batch < 0). */
int  pat_plan_set_split(pat_plan* plan, int min_batch);
int  pat_plan_get_split(const pat_plan* plan, int* min_batch);

/* Heterogeneous batch: `count` instances, each with its own plan (grid size,
 * detector count and arc, time samples may all differ; a plan may appear
 * several times).  pat_batch_forward / pat_batch_adjoint evaluate every
 * instance with one launch per stage of the operator (five per call) instead
 * of five per instance; the calls allocate nothing and do not synchronise, so
 * a caller can record them into a HIP graph.  Instance i uses the FFT-stage
 * tile shapes of plans[i] as they were at pat_batch_create; the interpolation
 * and spread workgroups are common to the batch (pat_batch_set_launch).
 * The plans must outlive the batch and be on the current device.
 * pat_batch_create: PAT_ERR_ARG (NULL, count < 1 or > 65536, a NULL plan,
 * plans on different devices), PAT_ERR_ALLOC / PAT_ERR_HIP (instance table
 * upload).  The batch owns one device allocation (the instance table). */
typedef struct pat_batch pat_batch;
int  pat_batch_create(pat_plan* const* plans, int count, pat_batch** out);
void pat_batch_destroy(pat_batch* batch);

/* Workspace bytes of one batch call (the sum of the instances' workspaces,
 * each 256-byte aligned); 0 for NULL. */
size_t pat_batch_workspace_size(const pat_batch* batch);

/* g_i = A_i f_i for every instance i.  f_ptrs and g_ptrs are DEVICE arrays of
 * `count` device pointers (f_ptrs[i]: [N_i][N_i] FP32 read, g_ptrs[i]:
 * [D_i][T_i] FP32 written), as in batched BLAS interfaces; the pointed-to
 * buffers must be valid, distinct for outputs, and sized for instance i (the
 * device arrays are not inspected on the host).  ws: at least
 * pat_batch_workspace_size bytes, 256-byte aligned.
 * Errors: PAT_ERR_ARG (NULL), PAT_ERR_WORKSPACE, PAT_ERR_HIP. */
int  pat_batch_forward(const pat_batch* batch, const float* const* f_ptrs, float* const* g_ptrs,
                       void* ws, size_t ws_bytes, void* stream);
/* f_i = A_i* g_i for every instance i; same conventions (g_ptrs read, f_ptrs written). */
int  pat_batch_adjoint(const pat_batch* batch, const float* const* g_ptrs, float* const* f_ptrs,
                       void* ws, size_t ws_bytes, void* stream);

/* The batch-wide interpolation and spread shapes (gat_cb, gat_th, spr_cb,
 * spr_th of pat_launch; the instances of a heterogeneous batch never share a
 * tile; the other fields are ignored on set and returned as 0
 * on get).  pat_batch_set_launch rewrites the device instance table and
 * therefore waits for the device to be idle first.  Errors: PAT_ERR_ARG
 * (NULL, field out of range), PAT_ERR_HIP. */
int  pat_batch_get_launch(const pat_batch* batch, pat_launch* out);
int  pat_batch_set_launch(pat_batch* batch, const pat_launch* cfg);

/* Autotuner.  pat_autotune_plan times candidate launch shapes of `plan` at
 * `batch` instances (1 <= batch <= max_batch) on the null stream, choosing
 * each stage's shape by its own measured kernel time, applies the fastest,
 * then times whole forward + adjoint calls on one stream and on two (each
 * captured as a HIP graph on a stream of its own and replayed) and sets
 * the plan's split batch (pat_plan_set_split) to `batch` if two are at least
 * 1 % faster, else to 0; it records shapes and split in the JSON file
 * cache_path under a key made of the geometry, the batch and the device name.
 * When that key is already in the file the stored shapes (and split, if the
 * entry has one) are applied without timing (an entry the shape checks now
 * reject is tuned again and replaced).
 * pat_autotune_batch does the same for a batch's interpolation and spread
 * shapes.  cache_path may be NULL (no cache).  Both allocate temporary device
 * buffers and synchronise: tuning calls, not for loops or graph capture.
 * Errors: PAT_ERR_ARG, PAT_ERR_ALLOC, PAT_ERR_HIP, and PAT_ERR_ARG when the
 * cache file exists but cannot be parsed. */
int  pat_autotune_plan(pat_plan* plan, int batch, const char* cache_path);
int  pat_autotune_batch(pat_batch* batch, const char* cache_path);

/* Host-only helpers (no GPU needed).
 * pat_plan_derive: the sizes pat_plan_create would derive for `desc`, without
 * building tables (fields M, dlam, n_lam, K, n_psi, kappa, n_grid, len_czt are
 * set, the rest are 0).  Same error codes as pat_plan_create's checks.
 * pat_bessel_jn_table: out[k] = J_k(x) for k = 0..kmax in FP64 by Miller's
 * backward recurrence (the routine behind the plan's radial weights
 * i^k J_k(lam_n R) of the mode form).  PAT_ERR_ARG on kmax < 0, NULL out or
 * non-finite x. */
int  pat_plan_derive(const pat_plan_desc* desc, pat_plan_info* out);
int  pat_bessel_jn_table(int kmax, double x, double* out);

/* ---- FFT wave-propagation data simulator ---------------------------------
 * The simulation study (Sec. 2.4.1, simulations) computes its data on a finer
 * Cartesian grid with an FFT-based wave propagation method in the manner of
 * k-Wave, so that the data do not come from the reconstruction's own
 * discretisation.  Reading for a constant speed of sound c:
 *   - the fine image (desc->n pixels a side, cell centres on [-1,1]^2, h = 2/n,
 *     pixels with centre radius >= support_r dropped) is zero-padded to a
 *     periodic box of M x M cells of the same size, centred, with M the
 *     smallest even 2^a 3^b (M - n even) whose half-width L = M h / 2 meets
 *     2 L - det_r - support_r > c t_T (no wave wraps around to a detector by
 *     the last sample t_T = n_t dt) and L > det_r + 3 h;
 *   - p(t) = IFFT2[ FFT2(f) cos(c |k| t) ] (k: the box's wave vectors), the
 *     exact solution of the periodic wave equation with p_t(0) = 0;
 *   - g(d, j) = p(x_d, j dt), j = 1..n_t, at the detectors (uniform arc or
 *     det_theta, radius det_r) by separable Keys cubic convolution (a = -1/2)
 *     on the box's cell centres.
 * pat_sim_create uses desc's fields n, support_r, det_r, n_det, arc_center,
 * arc_span, det_theta, n_t, dt and c (the operator-only fields are ignored);
 * it builds the tables (FP64 on the host, device memory owned by the
 * simulator) and may allocate; errors PAT_ERR_ARG (null pointers, n < 8,
 * n_det < 1, n_t < 1, dt <= 0, c <= 0, det_r <= 0, support_r <= 0),
 * PAT_ERR_UNSUPPORTED (box side above 8192 or no FFT plan), PAT_ERR_ALLOC,
 * PAT_ERR_HIP.
 * pat_sim_query: the box side M and the workspace bytes pat_sim_run needs.
 * pat_sim_run: f_dev [n][n] f32 (rows y, columns x) -> g_dev [n_det][n_t]
 * f32, device pointers owned by the caller, with a caller-owned device
 * workspace of at least the queried size; asynchronous on `stream`
 * (hipStream_t, NULL = the null stream), allocates nothing.  Errors
 * PAT_ERR_ARG (null pointers), PAT_ERR_WORKSPACE, PAT_ERR_HIP. */
typedef struct pat_sim pat_sim;
int  pat_sim_create(const pat_plan_desc* desc, pat_sim** out);
int  pat_sim_query(const pat_sim* sim, int* box_side, size_t* workspace_bytes);
int  pat_sim_run(const pat_sim* sim, const float* f_dev, float* g_dev, void* ws_dev, size_t ws_bytes, void* stream);
void pat_sim_destroy(pat_sim* sim);

/* Human-readable text of a status code (static storage). */
const char* pat_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif
