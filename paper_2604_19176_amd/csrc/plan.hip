// plan.hip -- host-side plan construction: sizes, FP64 tables, device upload.
//
// Everything here runs once per plan on the host in FP64; kernels only read
// the resulting FP32/int tables.
#include "fft.hpp"
#include "pat_internal.hpp"
#include "../../include/pat.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <numeric>
#include <vector>

namespace pat {

using cd = std::complex<double>;
static const double PI = 3.14159265358979323846264338327950288;

// smallest 2^a 3^b >= x (optionally even / divisible by 4)
long smooth23(double x, int multiple_of)
{
    long best = -1;
    for (long p2 = 1; p2 < (1L << 40); p2 *= 2) {
        long p = p2;
        while ((double)p < x) p *= 3;
        if (p % multiple_of == 0 && (best < 0 || p < best)) best = p;
        if ((double)p2 >= x && p2 % multiple_of == 0) break;
    }
    return best;
}

// Radix plan for n = 2^a 3^b: radix-8 stages, then 4 x 4 / 4 / 2 for the rest of
// the power of two (a radix-2 stage only when a = 1), then radix-3 stages.
static int radix_plan(long n, unsigned char* rad)
{
    int a = 0;
    while (n % 2 == 0) { ++a; n /= 2; }
    int ns = 0;
    int q = a / 3, r = a % 3;
    if (r == 1 && q >= 1) { q -= 1; r = 4; }  // 2^(3q+1) = 8^(q-1) * 4 * 4
    for (int i = 0; i < q; ++i) rad[ns++] = 8;
    if (r == 4) { rad[ns++] = 4; rad[ns++] = 4; }
    else if (r == 2) rad[ns++] = 4;
    else if (r == 1) rad[ns++] = 2;
    while (n % 3 == 0) { rad[ns++] = 3; n /= 3; }
    return n == 1 ? ns : -1;
}

// FP64 Stockham FFT on the host (same decomposition as the device FFT), sign -1.
static void host_fft(std::vector<cd>& x)
{
    const long n = (long)x.size();
    unsigned char rad[kMaxStages];
    int ns = radix_plan(n, rad);
    std::vector<cd> y(n);
    long Ns = 1;
    for (int s = 0; s < ns; ++s) {
        const int R = rad[s];
        const long nb = n / R;
        for (long j = 0; j < nb; ++j) {
            long k = j % Ns;
            cd v[8];
            for (int r = 0; r < R; ++r) {
                double ang = -2.0 * PI * (double)(k * r) / (double)(Ns * R);
                v[r] = x[j + r * nb] * cd(std::cos(ang), std::sin(ang));
            }
            cd o[8];
            for (int a = 0; a < R; ++a) {
                o[a] = 0;
                for (int r = 0; r < R; ++r) {
                    double ang = -2.0 * PI * (double)((a * r) % R) / R;
                    o[a] += v[r] * cd(std::cos(ang), std::sin(ang));
                }
            }
            long base = (j - k) * R + k;
            for (int a = 0; a < R; ++a) y[base + a * Ns] = o[a];
        }
        x.swap(y);
        Ns *= R;
    }
}

// J_k(x) for k = 0..kmax by Miller's backward recurrence with the normalisation
// J_0 + 2 sum J_{2k} = 1, rescaled against overflow.  FP64.
void bessel_jn_table(int kmax, double x, double* out)
{
    if (x == 0.0) {
        for (int k = 0; k <= kmax; ++k) out[k] = (k == 0) ? 1.0 : 0.0;
        return;
    }
    const double ax = std::fabs(x);
    int start = (int)std::max<double>(kmax, ax) + 40 + (int)(12.0 * std::cbrt(ax));
    if (start % 2) ++start;
    std::vector<double> j(start + 2, 0.0);
    double jp1 = 0.0, jk = 1e-300, norm = 0.0;
    for (int k = start; k >= 0; --k) {
        j[k] = jk;
        if (k % 2 == 0) norm += (k == 0 ? 1.0 : 2.0) * jk;
        double jm1 = 2.0 * k / ax * jk - jp1;
        jp1 = jk;
        jk = jm1;
        if (std::fabs(jk) > 1e250) {
            for (int q = k; q <= start; ++q) j[q] *= 1e-250;
            norm *= 1e-250;
            jp1 *= 1e-250;
            jk *= 1e-250;
        }
    }
    for (int k = 0; k <= kmax; ++k) {
        double v = j[k] / norm;
        if (x < 0 && (k % 2)) v = -v;
        out[k] = v;
    }
}

static double es_phi(double t)
{
    double z = 2.0 * t / kEsWidth;
    double q = 1.0 - z * z;
    return q >= 0 ? std::exp(kEsBeta * (std::sqrt(q) - 1.0)) : 0.0;
}

// phihat(k) = int_{-w/2}^{w/2} phi(t) cos(2 pi k t / Ng) dt by Gauss-Legendre (FP64).
static std::vector<double> es_hat(int N, int Ng)
{
    const int Q = 256;  // nodes per half interval
    std::vector<double> xs(Q), ws(Q);
    for (int i = 0; i < Q; ++i) {  // Newton on Legendre P_Q
        double x = std::cos(PI * (i + 0.75) / (Q + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1, p1 = x;
            for (int k = 2; k <= Q; ++k) { double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k; p0 = p1; p1 = p2; }
            double dp = Q * (x * p1 - p0) / (x * x - 1);
            double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        double p0 = 1, p1 = x;
        for (int k = 2; k <= Q; ++k) { double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k; p0 = p1; p1 = p2; }
        double dp = Q * (x * p1 - p0) / (x * x - 1);
        xs[i] = x;
        ws[i] = 2.0 / ((1 - x * x) * dp * dp);
    }
    const double half = 0.5 * kEsWidth;
    std::vector<double> out(N);
    for (int j = 0; j < N; ++j) {
        double k = j - N / 2;
        double acc = 0.0;
        for (int side = 0; side < 2; ++side) {  // [-w/2, 0] and [0, w/2]
            double a = side ? 0.0 : -half, b = side ? half : 0.0;
            for (int i = 0; i < Q; ++i) {
                double t = 0.5 * (a + b) + 0.5 * (b - a) * xs[i];
                acc += 0.5 * (b - a) * ws[i] * es_phi(t) * std::cos(2 * PI * k * t / Ng);
            }
        }
        out[j] = acc;
    }
    return out;
}

struct Derived {
    int M, n_lam, K, n_psi, Ng, L, P, S;
    double h, dlam, kappa;
};

static int derive(const pat_plan_desc* d, Derived* o)
{
    if (!d || !o) return PAT_ERR_ARG;
    if (d->n < 4 || d->n_det < 1 || d->n_t < 1 || d->max_batch < 1) return PAT_ERR_ARG;
    if (!(d->dt > 0) || !(d->c > 0) || !(d->det_r > 0) || !(d->support_r > 0)) return PAT_ERR_ARG;
    if (!(d->arc_span > 0) || d->arc_span > 2 * PI + 1e-12) return PAT_ERR_ARG;
    if (!(d->lambda_oversample >= 1.0) || !std::isfinite(d->arc_center)) return PAT_ERR_ARG;
    if (d->support_r > d->det_r) return PAT_ERR_ARG;
    o->h = 2.0 / d->n;
    o->M = (int)smooth23(d->lambda_oversample * d->n_t, 1);
    o->dlam = PI / (o->M * d->c * d->dt);
    o->n_lam = (int)std::floor(o->M * d->c * d->dt / o->h + 1e-9);  // lam_max <= pi/h
    if (o->n_lam < 1) return PAT_ERR_ARG;
    double z = o->n_lam * o->dlam * d->det_r;
    o->K = (int)std::ceil(z + 10.0 * std::cbrt(z) - 1e-9);
    o->n_psi = (int)smooth23(2.0 * o->K + 2, 4);
    o->kappa = d->em_correction ? o->dlam * o->dlam / (24.0 * PI) : 0.0;
    o->Ng = (int)smooth23(2.0 * d->n, 2);
    o->L = (int)smooth23((double)o->K + d->n_det, 1);
    {   // detector pitch dtheta = 2 pi s / P with P = 2^a 3^b (the smallest such P; then gcd(s, P) = 1
        // and s (D - 1) < P): the detectors are every s-th point of a P-point angular grid and the
        // synthesis is one FFT of length P.  Taken while that FFT is no dearer than the chirp-z pair.
        const double turns = d->arc_span / (2.0 * PI * d->n_det);  // dtheta / (2 pi)
        o->P = 0;
        o->S = 0;
        for (long P = smooth23((double)d->n_det, 1); P <= 8192 && P <= 3L * o->L; P = smooth23((double)P + 1, 1)) {
            const double sd = turns * (double)P;
            const long s = std::lround(sd);
            if (s >= 1 && std::fabs(sd - (double)s) < 1e-9 * sd && s * (long)(d->n_det - 1) < P) {
                o->P = (int)P;
                o->S = (int)s;
                break;
            }
        }
    }
    // limits of the kernels: every FFT length must fit the LDS plans
    if (d->n < 16 || o->Ng > 8192 || 2L * o->M > 8192 || (!o->P && o->L > 8192) || o->n_psi > 8192)
        return PAT_ERR_UNSUPPORTED;
    if (o->n_lam >= 2 * o->M) return PAT_ERR_UNSUPPORTED;  // cosine grid index n < 2M
    return PAT_OK;
}

}  // namespace pat

using namespace pat;

// ----------------------------------------------------------------------------

namespace {

struct TableBuilder {
    std::vector<unsigned char> host;
    size_t add(const void* p, size_t bytes)
    {
        size_t off = (host.size() + 255) & ~(size_t)255;
        host.resize(off + bytes);
        if (bytes) std::memcpy(host.data() + off, p, bytes);
        return off;
    }
    template <class T>
    size_t add(const std::vector<T>& v) { return add(v.data(), v.size() * sizeof(T)); }
};

struct FftSet {
    std::vector<FftDev> descs;
    std::vector<float2> tw;
    int get(long n)
    {
        for (size_t i = 0; i < descs.size(); ++i)
            if (descs[i].n == n) return (int)i;
        FftDev d;
        std::memset(&d, 0, sizeof(d));
        d.n = (int)n;
        d.nst = radix_plan(n, d.rad);
        d.tw = (int)tw.size();
        for (long e = 0; e < n; ++e) {
            double a = -2.0 * PI * (double)e / (double)n;
            tw.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
        }
        descs.push_back(d);
        return (int)descs.size() - 1;
    }
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

namespace pat {

// Threads for `nseq` sequences of one length: tps per sequence (4 butterflies
// per thread per stage, rounded to 32); at least 128 threads in total.
static int fft_threads(int nseq, const FftDev& fd)
{
    int tps = fft_min_tps(fd, 4);
    tps = ((tps + 31) / 32) * 32;
    while (nseq * tps < 128) tps += 32;
    return nseq * tps;
}

static size_t twb_bytes(int n) { return sizeof(float2) * (size_t)tw_lds_slots(n); }

// Dynamic LDS of the ring kernels: half-ring FFT buffer, synthesis buffers,
// [D][RT] detector tile and four twiddle tables.
static size_t ring_lds_bytes(const PlanDev& d, int RT)
{
    (void)RT;  // rings of a workgroup are processed one after another in the same LDS
    return sizeof(float2) * ring_lds_slots(d.npsi_max, d.syn_len, d.syn_half);
}

constexpr size_t kLdsMax = 160 * 1024;  // LDS a gfx950 workgroup can hold

// Checks a launch configuration against the LDS, thread and width limits of
// the kernels and, if it fits, makes it the plan's (workgroup sizes, ring
// LDS, tile counts).  The workspace layout does not depend on it.
int apply_launch(pat_plan* p, const LaunchCfg& c)
{
    const PlanDev& d = p->dev;
    // column and detector tiles of at most 32 columns / detectors (the endpoint-term sums)
    auto fft_ok = [&](int v, size_t each, const FftDev& f, size_t fixed) {
        return v >= 1 && v <= 16 && v * each + fixed <= kLdsMax && fft_threads(v, f) <= 1024;
    };
    if (c.col_np < 1 || c.col_np > 16 || c.row_rpb < 1 || c.row_rpb > 16 || c.dct_dp < 1 || c.dct_dp > 16 ||
        c.ring_rt < 1 || c.ring_rt > 64 || !gather_shape_ok(c.gat_cb, c.gat_th, c.gat_ib) ||
        !spread_shape_ok(c.spr_cb, c.spr_th, c.spr_ib))
        return PAT_ERR_ARG;
    if (!fft_ok(c.col_np, sizeof(float2) * d.Ng, p->h_fft_grid, twb_bytes(d.Ng)) ||
        !fft_ok(c.row_rpb, sizeof(float2) * d.Ng, p->h_fft_grid, twb_bytes(d.Ng)) ||
        !fft_ok(c.dct_dp, sizeof(float2) * 2 * d.M, p->h_fft_dct, twb_bytes(2 * d.M)))
        return PAT_ERR_UNSUPPORTED;
    const size_t lr = ring_lds_bytes(d, c.ring_rt);
    if (lr > kLdsMax) return PAT_ERR_UNSUPPORTED;
    p->cfg = c;
    p->cfg.spr_cap = 2 * c.spr_cb;
    p->lds_ring = lr;
    p->thr_col = fft_threads(c.col_np, p->h_fft_grid);
    p->thr_row = fft_threads(c.row_rpb, p->h_fft_grid);
    p->thr_dct = fft_threads(c.dct_dp, p->h_fft_dct);
    p->n_col_tiles = (d.N + 2 * c.col_np - 1) / (2 * c.col_np);
    p->n_pair_tiles = ((d.D + 1) / 2 + c.dct_dp - 1) / c.dct_dp;
    return PAT_OK;
}

// Default launch shapes: FFT tiles of <= 64 KB of LDS where possible (several
// workgroups per CU; a single sequence may use up to 160 KB), interpolation
// and spread tiles sized for `max_batch` instances.
int choose_launch(pat_plan* p, const std::vector<FftDev>& fd, int max_batch,
                  const std::vector<const FftDev*>& ring_descs)
{
    const PlanDev& d = p->dev;
    LaunchCfg c{};
    const size_t kLds = 64 * 1024;
    p->h_fft_grid = fd[d.fft_grid];
    p->h_fft_dct = fd[d.fft_dct];
    const FftDev& fg = p->h_fft_grid;
    const FftDev& fm = p->h_fft_dct;
    auto pick = [&](int maxn, size_t bytes_each, const FftDev& f, size_t fixed) {
        const int tps = (fft_min_tps(f, 4) + 31) / 32 * 32;
        int v = maxn;
        while (v > 1 && (v * bytes_each + fixed > kLds || v * tps > 1024)) --v;
        if (v * bytes_each + fixed <= kLds && v * tps <= 1024) return v;
        return (bytes_each + fixed <= kLdsMax && tps <= 1024) ? 1 : 0;
    };
    c.col_np = pick(8, sizeof(float2) * d.Ng, fg, twb_bytes(d.Ng));
    c.row_rpb = pick(8, sizeof(float2) * d.Ng, fg, twb_bytes(d.Ng));
    c.dct_dp = pick(4, sizeof(float2) * 2 * d.M, fm, twb_bytes(2 * d.M));
    c.ring_rt = 1;
    // wide tiles amortise the per-band work; narrow ones keep small batches parallel
    const long gwide = (long)((d.Ng + 255) / 256) * ((d.NB + 31) / 32) * max_batch;
    c.gat_cb = 64;
    c.gat_th = gwide >= 512 ? 16 : 8;
    // spread: wide tiles for large batches; rows per tile as many as keep about
    // 512 workgroups (a tile sweeps th + 7 bands for th output rows)
    const int ib = tile_ib(4, max_batch);
    c.gat_ib = ib;
    c.spr_ib = ib;
    const long groups = (max_batch + ib - 1) / ib;
    c.spr_cb = (d.Ng >= 512 && groups >= 8) ? 256 : 64;
    c.spr_th = 1;
    for (int th = 32; th >= 1; th /= 2)
        if ((long)((d.Ng + c.spr_cb - 1) / c.spr_cb) * ((d.Hy + th - 1) / th) * groups >= 512) {
            c.spr_th = th;
            break;
        }
    if (!c.col_np || !c.row_rpb || !c.dct_dp) return PAT_ERR_UNSUPPORTED;
    // ring kernels: as few threads per ring as the FFT stages allow (one wave when
    // possible), so that many rings are resident per CU to hide their latency
    p->thr_ring = 0;
    for (int thr = 64; thr <= kRingMaxThreads; thr *= 2) {
        bool ok = thr * kRingModesPerThread >= d.K + 1;  // every mode's coefficient prefetched
        for (const FftDev* f : ring_descs) ok = ok && fft_min_tps(*f, 4) <= thr;
        if (ok) { p->thr_ring = thr; p->ring_mb = 4; break; }
    }
    if (!p->thr_ring) return PAT_ERR_UNSUPPORTED;
    return apply_launch(p, c);
}

void layout_workspace(pat_plan* p)
{
    const PlanDev& d = p->dev;
    WsLayout& w = p->ws;
    size_t o = 0;
    w.x1 = o;     o += align256(sizeof(float2) * (size_t)d.Hy * d.N);
    w.grid = o;   o += align256(sizeof(float2) * (size_t)d.Hy * d.Ng);
    w.hdet = o;   o += align256(sizeof(float) * (size_t)d.D * d.nlam);
    w.polar = o;  o += align256(sizeof(float2) * (size_t)d.npts);
    // endpoint-term partial sums: one per image column (forward) or detector (adjoint)
    w.n_red = std::max(d.N, d.D);
    w.red = o;    o += align256(sizeof(float) * (size_t)w.n_red);
    w.bytes = o;
}

}  // namespace pat

extern "C" int pat_plan_derive(const pat_plan_desc* desc, pat_plan_info* out)
{
    Derived dv;
    int rc = derive(desc, &dv);
    if (rc != PAT_OK) return rc;
    if (!out) return PAT_ERR_ARG;
    std::memset(out, 0, sizeof(*out));
    out->M = dv.M;
    out->dlam = dv.dlam;
    out->n_lam = dv.n_lam;
    out->K = dv.K;
    out->n_psi = dv.n_psi;
    out->kappa = dv.kappa;
    out->n_grid = dv.Ng;
    out->len_czt = dv.P ? dv.P : dv.L;
    out->syn_stride = dv.P ? dv.S : 0;
    return PAT_OK;
}

extern "C" int pat_bessel_jn_table(int kmax, double x, double* out)
{
    if (kmax < 0 || !out || !std::isfinite(x)) return PAT_ERR_ARG;
    bessel_jn_table(kmax, x, out);
    return PAT_OK;
}

// Host part of plan creation; fills every table into `tb` and the PlanDev
// offsets (as byte offsets stored in the pointer fields, relocated later).
static int build_tables(const pat_plan_desc* desc, const Derived& dv, pat_plan* p, TableBuilder& tb)
{
    PlanDev& d = p->dev;
    const int N = desc->n, Ng = dv.Ng, nlam = dv.n_lam, K = dv.K, D = desc->n_det, T = desc->n_t;
    const double h = dv.h, R = desc->det_r;
    d.N = N; d.Ng = Ng; d.Hy = Ng / 2 + 9; d.nlam = nlam; d.K = K; d.Kp = K + 1; d.M = dv.M;
    d.T = T; d.D = D; d.L = dv.P ? 0 : dv.L; d.NB = Ng / 2 + 2;
    d.kappa = (float)dv.kappa;
    d.h2 = (float)(h * h);

    FftSet ffts;
    d.fft_grid = ffts.get(Ng);
    d.fft_dct = ffts.get(2L * dv.M);
    d.fold_P = dv.P;
    d.fold_s = dv.P ? dv.S : 0;
    d.syn_len = dv.P ? dv.P : dv.L;
    d.fft_syn = ffts.get(d.syn_len);
    d.syn_half = (dv.P && dv.P % 2 == 0) ? 1 : 0;
    d.fft_synh = d.syn_half ? ffts.get(dv.P / 2) : d.fft_syn;

    // --- image-side tables -------------------------------------------------
    std::vector<double> ph = es_hat(N, Ng);
    std::vector<float> deap(N);
    for (int j = 0; j < N; ++j) {
        if (!(ph[j] > 1e-300)) return PAT_ERR_UNSUPPORTED;
        deap[j] = (float)(h / ph[j]);
    }
    std::vector<int2> mask(N);
    const double rs2 = desc->support_r * desc->support_r;
    for (int i = 0; i < N; ++i) {
        double y = -1.0 + (i + 0.5) * h;
        int lo = N, hi = 0;
        for (int j = 0; j < N; ++j) {
            double x = -1.0 + (j + 0.5) * h;
            if (x * x + y * y < rs2) { lo = std::min(lo, j); hi = std::max(hi, j + 1); }
        }
        if (lo >= hi) { lo = 0; hi = 0; }
        mask[i] = make_int2(lo, hi);
    }

    // --- rings: per-ring mode cut-off and angular grid ----------------------
    std::vector<int> ringK(nlam), ringN(nlam), ringOff(nlam + 1), ringFft(nlam), ringTwn(nlam), ringJoff(nlam);
    std::vector<double> rho(nlam);
    int npts = 0, joff = 0, npsi_max = 0;
    for (int n = 1; n <= nlam; ++n) {
        double lam = n * dv.dlam, x = lam * R;
        int kn = (int)std::ceil(x + 10.0 * std::cbrt(x) - 1e-9);
        kn = std::min(K, std::max(kn, 1));
        int np = (int)smooth23(2.0 * kn + 2, 2);
        ringK[n - 1] = kn;
        ringN[n - 1] = np;
        ringOff[n - 1] = npts;
        ringJoff[n - 1] = joff;
        ringFft[n - 1] = ffts.get(np / 2);
        ringTwn[n - 1] = ffts.get(np);
        rho[n - 1] = lam * h * Ng / (2.0 * PI);
        npts += np / 2;
        joff += kn + 1;
        npsi_max = std::max(npsi_max, np);
    }
    ringOff[nlam] = npts;
    p->n_ring_modes = joff;
    d.npsi_max = npsi_max;
    d.npts = npts;
    p->n_psi_max = npsi_max;

    // radial weights J_k(lam_n R) W_n / Npsi(n) (FP64; combined with the synthesis factors below)
    std::vector<double> Jw(joff);
    {
        std::vector<double> jt(K + 1);
        for (int n = 1; n <= nlam; ++n) {
            double lam = n * dv.dlam;
            double W = lam * dv.dlam / (2.0 * PI);
            bessel_jn_table(ringK[n - 1], lam * R, jt.data());
            for (int k = 0; k <= ringK[n - 1]; ++k)
                Jw[ringJoff[n - 1] + k] = jt[k] * W / ringN[n - 1];
        }
    }

    // --- polar points (ring order), footprint bases and phases -------------
    std::vector<float4> geo(npts);
    std::vector<float2> phase(npts);
    std::vector<int> r0s(npts), bxs(npts);
    for (int n = 0; n < nlam; ++n) {
        const int np = ringN[n];
        for (int l = 0; l < np / 2; ++l) {
            double psi = 2.0 * PI * l / np;
            double sx = rho[n] * std::cos(psi), sy = rho[n] * std::sin(psi);
            double flx = std::floor(sx), fly = std::floor(sy);
            long bx = (long)flx - 3, by = (long)fly - 3;
            int r0 = (int)(by + 4);
            if (r0 < 0 || r0 + 7 >= d.Hy) return PAT_ERR_UNSUPPORTED;
            int bxm = (int)(((bx % Ng) + Ng) % Ng);
            int q = ringOff[n] + l;
            float4 gq;
            int ibx = bxm, ir0 = r0;
            std::memcpy(&gq.x, &ibx, 4);
            std::memcpy(&gq.y, &ir0, 4);
            gq.z = (float)(sx - flx);
            gq.w = (float)(sy - fly);
            geo[q] = gq;
            double a = -PI * (sx + sy) / Ng;
            phase[q] = make_float2((float)std::cos(a), (float)std::sin(a));
            r0s[q] = r0;
            bxs[q] = bxm;
        }
    }
    // band order: stable sort by (r0, bx)
    std::vector<int> order(npts);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return r0s[a] != r0s[b] ? r0s[a] < r0s[b] : bxs[a] < bxs[b];
    });
    std::vector<int> ring_of(npts);  // band-order slot -> ring-order index
    std::vector<int> band_of(npts);  // ring-order index -> band-order slot
    std::vector<float4> bgeo(npts);
    std::vector<float2> bphase(npts);
    for (int s = 0; s < npts; ++s) {
        ring_of[s] = order[s];
        band_of[order[s]] = s;
        bgeo[s] = geo[order[s]];
        bphase[s] = phase[order[s]];
    }
    const int NB = d.NB;
    std::vector<int> bptr((size_t)NB * (Ng + 1));
    {
        // counts per (r0, bx) then exclusive scan in (r0, bx) order
        std::vector<int> cnt((size_t)NB * Ng, 0);
        for (int q = 0; q < npts; ++q) cnt[(size_t)r0s[q] * Ng + bxs[q]]++;
        int run = 0;
        for (int r = 0; r < NB; ++r) {
            for (int b = 0; b < Ng; ++b) {
                bptr[(size_t)r * (Ng + 1) + b] = run;
                run += cnt[(size_t)r * Ng + b];
            }
            bptr[(size_t)r * (Ng + 1) + Ng] = run;
        }
    }

    // --- synthesis over detector angles --------------------------------------
    const double dth = desc->arc_span / D;
    const double th0 = desc->arc_center - 0.5 * desc->arc_span + 0.5 * dth;
    auto wpow = [&](long m) {  // w^{m^2}, w = e^{i dth/2}; phase reduced mod 2 pi in FP64
        double a = std::fmod(0.5 * dth * (double)m * (double)m, 2.0 * PI);
        return cd(std::cos(a), std::sin(a));
    };
    std::vector<cd> pre(K + 1);
    std::vector<float2> post, vhat;
    for (int k = 0; k <= K; ++k) {
        double a = std::fmod(k * th0, 2.0 * PI);
        cd v = (k == 0 ? 1.0 : 2.0) * cd(std::cos(a), std::sin(a));
        if (!dv.P) v *= wpow(k);
        pre[k] = v;
    }
    // Per ring n and mode k <= K_n, one coefficient
    //   coef = pre_k i^k J_k(lam_n R) W_n / Npsi(n) * (i for odd k),
    // the last factor because the ring's angular coefficient is i Q_k for odd k
    // when the real transform Q of the conjugate-antipodal ring is used; the
    // product i^k (i for odd k) is the real sign (-1)^ceil(k/2).
    std::vector<float2> coef(joff);
    for (int n = 0; n < nlam; ++n)
        for (int k = 0; k <= ringK[n]; ++k) {
            const double sg = (((k + 1) / 2) & 1) ? -1.0 : 1.0;
            const cd v = pre[k] * (sg * Jw[ringJoff[n] + k]);
            coef[ringJoff[n] + k] = make_float2((float)v.real(), (float)v.imag());
        }
    if (!dv.P) {
        const int L = dv.L;
        post.resize(D);
        vhat.resize(L);
        for (int q = 0; q < D; ++q) {
            cd v = wpow(q);
            post[q] = make_float2((float)v.real(), (float)v.imag());
        }
        std::vector<cd> v(L, cd(0, 0));
        for (long m = -K; m <= D - 1; ++m) v[((m % L) + L) % L] = std::conj(wpow(m));
        host_fft(v);
        for (int q = 0; q < L; ++q) vhat[q] = make_float2((float)(v[q].real() / L), (float)(v[q].imag() / L));
    }

    {
        std::vector<const FftDev*> rdesc;
        for (int n = 0; n < nlam; ++n) {
            if (std::find(rdesc.begin(), rdesc.end(), &ffts.descs[ringFft[n]]) == rdesc.end())
                rdesc.push_back(&ffts.descs[ringFft[n]]);
        }
        rdesc.push_back(&ffts.descs[d.syn_half ? d.fft_synh : d.fft_syn]);
        int rc = choose_launch(p, ffts.descs, desc->max_batch, rdesc);
        if (rc != PAT_OK) return rc;
    }

    // --- pack ---------------------------------------------------------------
    size_t o_deap = tb.add(deap), o_mask = tb.add(mask);
    size_t o_geo = tb.add(geo), o_phase = tb.add(phase);
    size_t o_roff = tb.add(ringOff), o_rk = tb.add(ringK), o_rfft = tb.add(ringFft), o_rj = tb.add(ringJoff);
    size_t o_rtwn = tb.add(ringTwn);
    size_t o_coef = tb.add(coef);
    size_t o_ringof = tb.add(ring_of), o_bandof = tb.add(band_of), o_bgeo = tb.add(bgeo), o_bph = tb.add(bphase), o_bptr = tb.add(bptr);
    size_t o_post = tb.add(post), o_vhat = tb.add(vhat);
    size_t o_ffts = tb.add(ffts.descs), o_tw = tb.add(ffts.tw);
    // store offsets in the pointer fields; relocated after the upload
    auto off = [](size_t o) { return (const void*)(uintptr_t)o; };
    d.deap = (const float*)off(o_deap);
    d.mask_rows = (const int2*)off(o_mask);
    d.pt_geo = (const float4*)off(o_geo);
    d.pt_phase = (const float2*)off(o_phase);
    d.ring_off = (const int*)off(o_roff);
    d.ring_K = (const int*)off(o_rk);
    d.ring_fft = (const int*)off(o_rfft);
    d.ring_twn = (const int*)off(o_rtwn);
    d.ring_joff = (const int*)off(o_rj);
    d.coef = (const float2*)off(o_coef);
    d.ring_of = (const int*)off(o_ringof);
    d.band_of = (const int*)off(o_bandof);
    d.bpt_geo = (const float4*)off(o_bgeo);
    d.bpt_phase = (const float2*)off(o_bph);
    d.band_ptr = (const int*)off(o_bptr);
    d.czt_post = (const float2*)off(o_post);
    d.czt_vhat = (const float2*)off(o_vhat);
    d.ffts = (const FftDev*)off(o_ffts);
    d.tw = (const float2*)off(o_tw);
    return PAT_OK;
}

extern "C" int pat_plan_create(const pat_plan_desc* desc, pat_plan** out)
{
    if (!desc || !out) return PAT_ERR_ARG;
    Derived dv;
    int rc = derive(desc, &dv);
    if (rc != PAT_OK) return rc;
    pat_plan* p = new (std::nothrow) pat_plan;
    if (!p) return PAT_ERR_ALLOC;
    std::memset(p, 0, sizeof(*p));
    TableBuilder tb;
    rc = build_tables(desc, dv, p, tb);
    if (rc != PAT_OK) { delete p; return rc; }
    if (hipGetDevice(&p->device) != hipSuccess) { delete p; return PAT_ERR_HIP; }
    void* mem = nullptr;
    if (hipMalloc(&mem, tb.host.size()) != hipSuccess) { delete p; return PAT_ERR_ALLOC; }
    if (hipMemcpy(mem, tb.host.data(), tb.host.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(mem);
        delete p;
        return PAT_ERR_HIP;
    }
    p->table_mem = mem;
    p->table_bytes = tb.host.size();
    // relocate
    char* base = (char*)mem;
    PlanDev& d = p->dev;
    auto rel = [&](auto& ptr) { ptr = (std::remove_reference_t<decltype(ptr)>)(base + (uintptr_t)ptr); };
    rel(d.deap); rel(d.mask_rows); rel(d.pt_geo); rel(d.pt_phase); rel(d.ring_off); rel(d.ring_K);
    rel(d.ring_fft); rel(d.ring_twn); rel(d.ring_joff); rel(d.coef); rel(d.ring_of); rel(d.band_of); rel(d.bpt_geo); rel(d.bpt_phase);
    rel(d.band_ptr); rel(d.czt_post); rel(d.czt_vhat); rel(d.ffts); rel(d.tw);
    p->desc = *desc;
    p->max_batch = desc->max_batch;
    p->n_psi_uniform = dv.n_psi;
    p->M = dv.M;
    p->dlam = dv.dlam;
    p->kappa = dv.kappa;
    layout_workspace(p);
    *out = p;
    return PAT_OK;
}

extern "C" int pat_plan_query(const pat_plan* p, pat_plan_info* out)
{
    if (!p || !out) return PAT_ERR_ARG;
    std::memset(out, 0, sizeof(*out));
    out->M = p->M;
    out->dlam = p->dlam;
    out->n_lam = p->dev.nlam;
    out->K = p->dev.K;
    out->n_psi = p->n_psi_uniform;
    out->kappa = p->kappa;
    out->n_grid = p->dev.Ng;
    out->n_points = p->dev.npts;
    out->len_czt = p->dev.syn_len;
    out->syn_stride = p->dev.fold_s;
    out->n_ring_modes = p->n_ring_modes;
    out->workspace_per_instance = p->ws.bytes;
    out->table_bytes = p->table_bytes;
    return PAT_OK;
}

extern "C" int pat_profile_enable(pat_plan* p, int enable);

extern "C" void pat_plan_destroy(pat_plan* p)
{
    if (!p) return;
    (void)pat_profile_enable(p, 0);
    if (p->table_mem) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) cur = p->device;
        (void)hipSetDevice(p->device);
        (void)hipFree(p->table_mem);
        (void)hipSetDevice(cur);
    }
    delete p;
}

extern "C" size_t pat_workspace_size(const pat_plan* p, int batch)
{
    if (!p || batch < 1) return 0;
    return p->ws.bytes * (size_t)batch;
}
