// plan.hip -- host-side plan construction: sizes, FP64 tables, device upload.
//
// Everything here runs once per plan on the host in FP64; kernels only read
// the resulting FP32/int tables.
#include "fft.hpp"
#include "cfft.hpp"
#include "pat_internal.hpp"
#include "../../include/pat.h"

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <complex>
#include <cstring>
#include <numeric>
#include <map>
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

// Radix plan of the host's FP64 FFT (chirp-z filter spectrum) for n = 2^a 3^b:
// radix-8 stages, then 4 x 4 / 4 / 2 for the rest of the power of two (a
// radix-2 stage only when a = 1), then radix-3 stages.
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

// FP64 Stockham FFT on the host, sign -1.
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
    int dense;  // explicit detector angles: synthesis as a dense product
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
    o->P = 0;
    o->S = 0;
    o->dense = d->det_theta ? 1 : 0;
    if (o->dense)
        for (int q = 0; q < d->n_det; ++q)
            if (!std::isfinite(d->det_theta[q])) return PAT_ERR_ARG;
    if (!o->dense) {   // detector pitch dtheta = 2 pi s / P with P = 2^a 3^b (the smallest such P; then gcd(s, P) = 1
        // and s (D - 1) < P): the detectors are every s-th point of a P-point angular grid and the
        // synthesis is one FFT of length P.  Taken while that FFT is no dearer than the chirp-z pair.
        const double turns = d->arc_span / (2.0 * PI * d->n_det);  // dtheta / (2 pi)
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
    if (d->n < 16 || o->Ng > 8192 || 2L * o->M > 8192 || (!o->P && !o->dense && o->L > 8192) || o->n_psi > 8192)
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

// Pass plans of the device FFT (fft.hpp) for length n at `tps` threads per
// sequence, each thread holding at most `maxb` butterflies per pass.
//
// kFftMeasured holds the fastest plan measured on an MI355X (gfx950) for
// every length 2^a 3^b the transforms use: all plans (every multiset of
// radices {2, 3, 4, 6, 8, 9, 16} in both orders) timed in a one-workgroup-per-
// sequence kernel, for the ring kernels (maxb 2) at 64, 128 and 256 threads
// and for the fixed-length transforms (maxb 4) at their thread counts.
// Lengths outside the table use a cost model fitted to the same measurements:
// per pass, the rounds of butterflies times a per-radix cost, the LDS bank
// multiplicity of the pass's stores, the division k = j mod Ns when Ns is not
// a power of two, and a fixed cost per pass; every ordering of every multiset
// (at most two radix-16 passes) is ranked.
struct FftMeasured {
    short n, tps;
    unsigned char maxb;
    unsigned char rad[6];
};
static const FftMeasured kFftMeasured[] = {
    {8, 64, 2, {8}}, {9, 64, 2, {9}}, {12, 64, 2, {6, 2}}, {16, 64, 2, {4, 4}}, {18, 64, 2, {6, 3}},
    {24, 64, 2, {8, 3}}, {27, 64, 2, {9, 3}}, {32, 64, 2, {8, 4}}, {36, 64, 2, {6, 6}}, {48, 64, 2, {8, 6}},
    {54, 64, 2, {9, 6}}, {64, 64, 2, {8, 8}}, {72, 64, 2, {9, 8}}, {81, 64, 2, {9, 9}},
    {96, 64, 2, {4, 4, 6}}, {108, 64, 2, {6, 6, 3}}, {128, 64, 2, {8, 4, 4}}, {144, 64, 2, {8, 3, 6}},
    {162, 64, 2, {9, 6, 3}}, {192, 64, 2, {6, 8, 4}}, {216, 64, 2, {6, 6, 6}}, {243, 64, 2, {9, 9, 3}},
    {256, 64, 2, {4, 4, 4, 4}}, {288, 64, 2, {6, 6, 8}}, {324, 64, 2, {9, 6, 6}}, {384, 64, 2, {6, 8, 8}},
    {432, 64, 2, {9, 6, 8}}, {486, 64, 2, {6, 9, 9}}, {512, 64, 2, {8, 8, 8}}, {576, 64, 2, {9, 8, 8}},
    {648, 64, 2, {9, 9, 8}}, {729, 64, 2, {9, 9, 9}}, {768, 64, 2, {6, 16, 8}}, {1024, 64, 2, {8, 8, 16}},
    {8, 128, 2, {8}}, {9, 128, 2, {9}}, {12, 128, 2, {4, 3}}, {16, 128, 2, {16}}, {18, 128, 2, {6, 3}},
    {24, 128, 2, {8, 3}}, {27, 128, 2, {9, 3}}, {32, 128, 2, {8, 4}}, {36, 128, 2, {6, 6}},
    {48, 128, 2, {8, 6}}, {54, 128, 2, {9, 6}}, {64, 128, 2, {8, 8}}, {72, 128, 2, {8, 9}},
    {81, 128, 2, {9, 9}}, {96, 128, 2, {16, 6}}, {108, 128, 2, {6, 6, 3}}, {128, 128, 2, {8, 4, 4}},
    {144, 128, 2, {8, 3, 6}}, {162, 128, 2, {9, 6, 3}}, {192, 128, 2, {8, 8, 3}}, {216, 128, 2, {6, 6, 6}},
    {243, 128, 2, {9, 9, 3}}, {256, 128, 2, {8, 8, 4}}, {288, 128, 2, {8, 6, 6}}, {324, 128, 2, {9, 6, 6}},
    {384, 128, 2, {6, 8, 8}}, {432, 128, 2, {9, 6, 8}}, {486, 128, 2, {9, 9, 6}}, {512, 128, 2, {8, 8, 8}},
    {576, 128, 2, {9, 8, 8}}, {648, 128, 2, {9, 9, 8}}, {729, 128, 2, {9, 9, 9}}, {768, 128, 2, {6, 16, 8}},
    {864, 128, 2, {9, 6, 16}}, {1024, 128, 2, {8, 8, 16}}, {1152, 128, 2, {9, 16, 8}},
    {1296, 128, 2, {9, 9, 16}}, {1536, 128, 2, {6, 16, 16}}, {2048, 128, 2, {8, 16, 16}}, {8, 256, 2, {8}},
    {9, 256, 2, {9}}, {12, 256, 2, {6, 2}}, {16, 256, 2, {16}}, {18, 256, 2, {6, 3}}, {24, 256, 2, {8, 3}},
    {27, 256, 2, {9, 3}}, {32, 256, 2, {8, 4}}, {36, 256, 2, {6, 6}}, {48, 256, 2, {8, 6}},
    {54, 256, 2, {9, 6}}, {64, 256, 2, {8, 8}}, {72, 256, 2, {8, 9}}, {81, 256, 2, {9, 9}},
    {96, 256, 2, {16, 6}}, {108, 256, 2, {6, 6, 3}}, {128, 256, 2, {16, 8}}, {144, 256, 2, {8, 3, 6}},
    {162, 256, 2, {9, 6, 3}}, {192, 256, 2, {8, 8, 3}}, {216, 256, 2, {9, 6, 4}}, {243, 256, 2, {9, 9, 3}},
    {256, 256, 2, {8, 8, 4}}, {288, 256, 2, {8, 6, 6}}, {324, 256, 2, {9, 6, 6}}, {384, 256, 2, {8, 8, 6}},
    {432, 256, 2, {8, 6, 9}}, {486, 256, 2, {9, 9, 6}}, {512, 256, 2, {8, 8, 8}}, {576, 256, 2, {9, 8, 8}},
    {648, 256, 2, {9, 9, 8}}, {729, 256, 2, {9, 9, 9}}, {768, 256, 2, {6, 16, 8}}, {864, 256, 2, {9, 6, 16}},
    {972, 256, 2, {9, 6, 6, 3}}, {1024, 256, 2, {4, 4, 8, 8}}, {1152, 256, 2, {9, 16, 8}},
    {1296, 256, 2, {6, 6, 6, 6}}, {1458, 256, 2, {9, 9, 6, 3}}, {1536, 256, 2, {3, 8, 8, 8}},
    {1728, 256, 2, {9, 6, 8, 4}}, {1944, 256, 2, {9, 9, 6, 4}}, {2048, 256, 2, {4, 8, 8, 8}},
    {2304, 256, 2, {9, 16, 16}}, {2592, 256, 2, {9, 6, 6, 8}}, {2916, 256, 2, {9, 9, 6, 6}},
    {3072, 256, 2, {6, 8, 8, 8}}, {4096, 256, 2, {8, 8, 8, 8}}, {32, 32, 4, {8, 4}}, {36, 32, 4, {6, 6}},
    {48, 32, 4, {6, 8}}, {54, 32, 4, {9, 6}}, {64, 32, 4, {8, 8}}, {72, 32, 4, {6, 3, 4}},
    {96, 32, 4, {6, 4, 4}}, {108, 32, 4, {6, 6, 3}}, {128, 32, 4, {4, 4, 8}}, {144, 32, 4, {6, 6, 4}},
    {162, 32, 4, {9, 6, 3}}, {192, 32, 4, {6, 8, 4}}, {216, 32, 4, {9, 3, 8}}, {256, 32, 4, {4, 8, 8}},
    {288, 32, 4, {9, 8, 4}}, {324, 32, 4, {9, 6, 6}}, {384, 32, 4, {6, 16, 4}}, {512, 32, 4, {4, 8, 16}},
    {432, 64, 4, {9, 6, 8}}, {486, 64, 4, {6, 9, 9}}, {576, 64, 4, {9, 16, 4}}, {648, 64, 4, {3, 6, 6, 6}},
    {768, 64, 4, {6, 16, 8}}, {1024, 64, 4, {4, 16, 16}}, {864, 96, 4, {9, 6, 16}},
    {972, 96, 4, {9, 6, 6, 3}}, {1152, 96, 4, {9, 16, 8}}, {1296, 96, 4, {9, 9, 16}},
    {1458, 128, 4, {9, 9, 6, 3}}, {1536, 128, 4, {6, 16, 16}}, {2048, 128, 4, {8, 16, 16}},
    {1728, 160, 4, {6, 6, 6, 8}}, {2304, 160, 4, {9, 16, 16}}, {1944, 192, 4, {9, 6, 6, 6}},
    {2592, 192, 4, {9, 9, 8, 4}}, {2916, 192, 4, {9, 9, 9, 4}}, {3072, 256, 4, {6, 8, 8, 8}},
    {4096, 256, 4, {4, 8, 8, 16}}, {3456, 288, 4, {6, 6, 6, 16}}, {4608, 288, 4, {9, 8, 8, 8}},
    {3888, 352, 4, {9, 9, 3, 16}}, {5184, 352, 4, {9, 9, 8, 8}}, {4374, 384, 4, {6, 9, 9, 9}},
    {5832, 384, 4, {9, 9, 9, 8}}, {6144, 512, 4, {6, 16, 8, 8}}, {8192, 512, 4, {4, 8, 16, 16}},
    {6912, 576, 4, {9, 6, 16, 8}}, {7776, 672, 4, {9, 9, 6, 16}},
};

static double fft_radix_cost(int R)
{
    switch (R) {
        case 2: return 0.0408;
        case 3: return 0.0665;
        case 4: return 0.1071;
        case 6: return 0.1386;
        case 8: return 0.1963;
        case 9: return 0.2150;
        default: return 0.3514;
    }
}

// Model cost of the pass order `rad` (or a negative value if it does not fit
// tps threads holding at most maxb butterflies each)
static double fft_plan_cost(long n, int tps, int maxb, const std::vector<int>& rad)
{
    double c = 0.0;
    long Ns = 1;
    for (int R : rad) {
        const long rounds = (n / R + tps - 1) / tps;
        if (rounds > radix_max_butterflies(R, maxb)) return -1.0;
        int conf = 0;  // max stores per float2 bank slot (32 slots) in a half wave, summed over outputs r
        for (int r = 0; r < R; ++r) {
            int cnt[32] = {0}, mx = 0;
            for (long j = 0; j < std::min<long>(32, n / R); ++j) {
                const long a = (j / Ns) * Ns * R + j % Ns + r * Ns;
                mx = std::max(mx, ++cnt[a & 31]);
            }
            conf += mx;
        }
        c += rounds * (fft_radix_cost(R) + 0.0033 * conf + ((Ns & (Ns - 1)) ? 0.0086 : 0.0)) + 0.0731;
        Ns *= R;
    }
    return c;
}

// Passes of length n at tps threads per sequence, each holding at most maxb
// butterflies, into rad; returns their number or -1.
int fft_passes(long n, int tps, int maxb, unsigned char* rad)
{
    for (const FftMeasured& m : kFftMeasured)
        if (m.n == n && m.tps == tps && m.maxb == maxb) {
            std::vector<int> p;
            for (int i = 0; i < 6 && m.rad[i]; ++i) p.push_back(m.rad[i]);
            if (fft_plan_cost(n, tps, maxb, p) < 0.0) break;  // measured at more butterflies per thread
            for (size_t i = 0; i < p.size(); ++i) rad[i] = (unsigned char)p[i];
            return (int)p.size();
        }
    int a = 0, b = 0;
    long m = n;
    while (m % 2 == 0) { ++a; m /= 2; }
    while (m % 3 == 0) { ++b; m /= 3; }
    if (m != 1 || n < 2) return -1;
    double best = -1.0;
    std::vector<int> bestp;
    for (int c6 = 0; c6 <= std::min(a, b); ++c6)
        for (int c9 = 0; c9 <= (b - c6) / 2; ++c9) {
            const int c3 = b - c6 - 2 * c9, ap = a - c6;
            for (int c16 = 0; c16 <= std::min(2, ap / 4); ++c16)
                for (int c8 = 0; c8 <= (ap - 4 * c16) / 3; ++c8)
                    for (int c4 = 0; c4 <= (ap - 4 * c16 - 3 * c8) / 2; ++c4) {
                        const int c2 = ap - 4 * c16 - 3 * c8 - 2 * c4;
                        std::vector<int> p;
                        p.insert(p.end(), c2, 2);
                        p.insert(p.end(), c3, 3);
                        p.insert(p.end(), c4, 4);
                        p.insert(p.end(), c6, 6);
                        p.insert(p.end(), c8, 8);
                        p.insert(p.end(), c9, 9);
                        p.insert(p.end(), c16, 16);
                        if (p.size() > 10) continue;
                        do {
                            const double c = fft_plan_cost(n, tps, maxb, p);
                            if (c >= 0.0 && (best < 0.0 || c < best)) { best = c; bestp = p; }
                        } while (std::next_permutation(p.begin(), p.end()));
                    }
        }
    if (best < 0.0 || (int)bestp.size() > kMaxStages) return -1;
    for (size_t i = 0; i < bestp.size(); ++i) rad[i] = (unsigned char)bestp[i];
    return (int)bestp.size();
}

// Threads per sequence the fixed-length transforms (grid, cosine) are planned
// for: the smallest multiple of 32, from n/16 up (one radix-16 or two radix-8
// butterflies per thread and pass), for which a pass plan fits; 0 if none does.
static int fixed_fft_tps(long n)
{
    unsigned char rad[kMaxStages];
    for (long t = std::max<long>(32, ((n + 15) / 16 + 31) / 32 * 32); t <= 1024; t += 32)
        if (fft_passes(n, (int)t, kFftMaxButterflies, rad) >= 0) return (int)t;
    return 0;
}

struct FftSet {
    std::vector<FftDev> descs;
    std::vector<int> key_tps;
    std::vector<float2> tw;
    // descriptor of length n planned for tps threads per sequence holding at
    // most maxb butterflies each (tps = 0: only the twiddle table
    // e^{-2 pi i e/n}, no transform); -1 if no plan fits
    int get(long n, int tps, int maxb = kFftMaxButterflies)
    {
        int full = -1;
        for (size_t i = 0; i < descs.size(); ++i) {
            if (descs[i].n != n) continue;
            if (key_tps[i] == tps * 16 + maxb) return (int)i;
            full = descs[i].tw;
        }
        FftDev d;
        std::memset(&d, 0, sizeof(d));
        d.n = (int)n;
        if (tps > 0) {
            d.nst = fft_passes(n, tps, maxb, d.rad);
            if (d.nst < 0) return -1;
        }
        if (full < 0) {
            full = (int)tw.size();
            for (long e = 0; e < n; ++e) {
                double a = -2.0 * PI * (double)e / (double)n;
                tw.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
            }
        }
        d.tw = full;
        d.tb = (int)tw.size();
        long Ns = 1;
        for (int s = 0; s < d.nst; ++s) {
            const long R = d.rad[s];
            for (long k = 0; k < Ns; ++k) {
                double a = -2.0 * PI * (double)k / (double)(Ns * R);
                tw.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
            }
            d.ntb += (int)Ns;
            Ns *= R;
        }
        descs.push_back(d);
        key_tps.push_back(tps * 16 + maxb);
        return (int)descs.size() - 1;
    }
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

namespace pat {

// Threads for `nseq` sequences of one length: tps per sequence (what the
// passes need, rounded to 32); at least 128 threads in total.
static int fft_threads(int nseq, const FftDev& fd)
{
    int tps = fft_min_tps(fd);
    tps = ((tps + 31) / 32) * 32;
    while (nseq * tps < 128) tps += 32;
    return nseq * tps;
}

// LDS of a length's per-pass twiddles
static size_t twb_bytes(const FftDev& f) { return sizeof(float2) * (size_t)f.ntb; }

// A fixed-length transform of length n for another module: its descriptor,
// planned like the grid and cosine transforms, with its twiddles appended to
// `tw` (the descriptor's offsets index `tw`).  Returns the threads per
// sequence, 0 if no plan fits.
int fixed_fft_for(long n, FftDev* out, std::vector<float2>& tw)
{
    const int tps = fixed_fft_tps(n);
    if (!tps) return 0;
    FftSet s;
    const int i = s.get(n, tps);
    if (i < 0) return 0;
    FftDev d = s.descs[i];
    d.tw += (int)tw.size();
    d.tb += (int)tw.size();
    tw.insert(tw.end(), s.tw.begin(), s.tw.end());
    *out = d;
    return tps;
}

int fft_workgroup_threads(int nseq, const FftDev& fd) { return fft_threads(nseq, fd); }

// Threads of a 2D-FFT pass workgroup over `nseq` sequences of the plan's grid side
// (compile-time lengths: a tile of one sequence gets twice the transform's
// lanes, which shortens the single-instance chain; the kernels pass `wide`
// to the transform when their tile has one sequence)
int grid_threads(const pat_plan* p, int nseq)
{
    return p->dev.grid_spec ? (nseq == 1 ? 2 : nseq) * cfft_lanes(p->dev.Ng) : fft_threads(nseq, p->h_fft_grid);
}

// Dynamic LDS of the ring kernels: half-ring FFT buffer, synthesis buffers,
// [D][RT] detector tile and four twiddle tables.
static size_t ring_lds_bytes(const PlanDev& d, int RT)
{
    (void)RT;  // rings of a workgroup are processed one after another in the same LDS
    if (d.ring_spec) return sizeof(float2) * ring_spec_lds_slots(d.npsi_max, d.syn_len);
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
    auto grid_ok = [&](int v) {
        if (!d.grid_spec) return fft_ok(v, sizeof(float2) * d.Ng, p->h_fft_grid, twb_bytes(p->h_fft_grid));
        return v >= 1 && v <= 16 && v * sizeof(float2) * d.Ng + twb_bytes(p->h_fft_grid) <= kLdsMax &&
               (v == 1 ? 2 : v) * cfft_lanes(d.Ng) <= 1024;
    };
    if (c.col_np < 1 || c.col_np > 16 || c.row_rpb < 1 || c.row_rpb > 16 || c.dct_dp < 1 || c.dct_dp > 16 ||
        c.ring_rt < 1 || c.ring_rt > 64 || !gather_shape_ok(c.gat_cb, c.gat_th, c.gat_ib) ||
        !spread_shape_ok(c.spr_cb, c.spr_th, c.spr_ib))
        return PAT_ERR_ARG;
    const bool dct_ok = d.dct_spec ? (c.dct_dp * sizeof(float2) * (size_t)cfft_padded_len(2 * d.M) <= kLdsMax &&
                                      c.dct_dp * cfft_lanes(2 * d.M) <= 1024)
                                   : fft_ok(c.dct_dp, sizeof(float2) * 2 * d.M, p->h_fft_dct, twb_bytes(p->h_fft_dct));
    if (!grid_ok(c.col_np) || !grid_ok(c.row_rpb) || !dct_ok) return PAT_ERR_UNSUPPORTED;
    const size_t lr = ring_lds_bytes(d, c.ring_rt);
    if (lr > kLdsMax) return PAT_ERR_UNSUPPORTED;
    p->cfg = c;
    p->cfg.spr_cap = 2 * c.spr_cb;
    p->lds_ring = lr;
    // compile-time ring kernels: ring_rt >= 2 gives the rings of the short-length
    // group two waves each (the same arithmetic on more lanes)
    if (d.ring_spec) p->thr_ring = ring_spec_threads(d.ring_spec_grp, d.ring_spec_grp == 0 && c.ring_rt >= 2 ? 2 : 1);
    p->thr_col = grid_threads(p, c.col_np);
    p->thr_row = grid_threads(p, c.row_rpb);
    p->thr_dct = d.dct_spec ? c.dct_dp * cfft_lanes(2 * d.M) : fft_threads(c.dct_dp, p->h_fft_dct);
    p->n_col_tiles = (d.N + 2 * c.col_np - 1) / (2 * c.col_np);
    p->n_pair_tiles = ((d.D + 1) / 2 + c.dct_dp - 1) / c.dct_dp;
    return PAT_OK;
}

// Default launch shapes: FFT tiles of <= 64 KB of LDS where possible (several
// workgroups per CU; a single sequence may use up to 160 KB), interpolation
// and spread tiles sized for `max_batch` instances.
int choose_launch(pat_plan* p, const std::vector<FftDev>& fd, int max_batch)
{
    const PlanDev& d = p->dev;
    LaunchCfg c{};
    const size_t kLds = 64 * 1024;
    p->h_fft_grid = fd[d.fft_grid];
    p->h_fft_dct = fd[d.fft_dct];
    const FftDev& fg = p->h_fft_grid;
    const FftDev& fm = p->h_fft_dct;
    auto pick = [&](int maxn, size_t bytes_each, const FftDev& f, size_t fixed) {
        const int tps = (fft_min_tps(f) + 31) / 32 * 32;
        int v = maxn;
        while (v > 1 && (v * bytes_each + fixed > kLds || v * tps > 1024)) --v;
        if (v * bytes_each + fixed <= kLds && v * tps <= 1024) return v;
        return (bytes_each + fixed <= kLdsMax && tps <= 1024) ? 1 : 0;
    };
    c.col_np = pick(8, sizeof(float2) * d.Ng, fg, twb_bytes(fg));
    c.row_rpb = pick(8, sizeof(float2) * d.Ng, fg, twb_bytes(fg));
    c.dct_dp = pick(4, sizeof(float2) * 2 * d.M, fm, twb_bytes(fm));
    c.ring_rt = 1;
    // wide tiles amortise the per-band work; narrow ones keep small batches parallel
    const long gwide = (long)((d.Ng + 255) / 256) * ((d.NB + 31) / 32) * max_batch;
    c.gat_cb = 64;
    c.gat_th = gwide >= 512 ? 16 : 8;
    // spread: wide tiles for large batches, 128 columns for small ones (measured
    // at 256^2: batch 1 fastest with 128..256 columns, 64 slower)
    const int ib = tile_ib(4, max_batch);
    c.gat_ib = ib;
    c.spr_ib = ib;
    const long groups = (max_batch + ib - 1) / ib;
    c.spr_cb = (d.Ng >= 512 && groups >= 8) ? 256 : (d.Ng >= 256 ? 128 : 64);
    c.spr_th = kSpreadTh;
    if (!c.col_np || !c.row_rpb || !c.dct_dp) return PAT_ERR_UNSUPPORTED;
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
    // explicit angles: mode coefficients a_k(n) (forward) / their adjoints, [nlam][K+1]
    w.modes = o;  o += d.syn_dense ? align256(sizeof(float2) * (size_t)d.nlam * d.Kp) : 0;
    // spread: 7 partial rows per row tile; the partial rows of split row tiles' runs
    w.tail = o;   o += align256(sizeof(float2) * 7 * (size_t)d.Ng * spread_row_tiles(d.NB));
    w.slab = o;   o += align256(sizeof(float2) * (size_t)d.slab_rows * d.Ng);
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
    out->len_czt = dv.dense ? 0 : (dv.P ? dv.P : dv.L);
    out->syn_stride = dv.P ? dv.S : 0;
    out->syn_dense = dv.dense;
    return PAT_OK;
}

extern "C" int pat_bessel_jn_table(int kmax, double x, double* out)
{
    if (kmax < 0 || !out || !std::isfinite(x)) return PAT_ERR_ARG;
    bessel_jn_table(kmax, x, out);
    return PAT_OK;
}

// Spread work rows.  In band rb the lane of column c visits the points whose
// footprint base column is c - 7 .. c (mod Ng); a row tile's longest lane,
// summed over its bands, bounds its workgroup's time.  For batches: a row tile
// among the first kSpreadSplitTiles whose longest lane exceeds
// kSpreadSplitFactor times the median over the row tiles is split into the
// fewest runs S (2 or kSpreadMaxRuns) that bring every run's longest lane
// under that limit, or into kSpreadMaxRuns.  Plans for single instances
// (max_batch 1), whose spread is one wave per tile and bound by each tile's
// chain of bands, split every row tile whose longest lane exceeds
// kSpreadSplitFactorSingle times the median: more, shorter work rows, at the
// cost of the slab rows the adjoint row pass adds up, unless those would
// exceed kSpreadSlabCapSingle bytes per instance (then the batched rule).  The last row tile,
// which writes the grid's final rows itself, is never split.  Output: the work
// rows (first band, last band, first slab row or -1, row tile), per row tile
// (S, first slab row), and the slab rows in all.  The split is a property of
// the plan: every launch shape and batch size of a plan sums in its order.
constexpr double kSpreadSplitFactor = 1.5;
constexpr double kSpreadSplitFactorSingle = 0.7;
constexpr size_t kSpreadSlabCapSingle = 32u << 20;  // slab bytes per instance of a single-instance plan

static void spread_runs(const std::vector<int>& bptr, int NB, int Ng, bool single, std::vector<int4>& rows,
                        std::vector<int2>& split, int& slab_rows)
{
    const int nrt = spread_row_tiles(NB);
    std::vector<int> vis((size_t)NB * Ng);
    for (int r = 0; r < NB; ++r) {
        const int* bp = &bptr[(size_t)r * (Ng + 1)];
        for (int c = 0; c < Ng; ++c) {
            int v = 0;
            for (int dx = 0; dx < 8; ++dx) {
                const int b = ((c - dx) % Ng + Ng) % Ng;
                v += bp[b + 1] - bp[b];
            }
            vis[(size_t)r * Ng + c] = v;
        }
    }
    auto longest = [&](int t, int S) {  // longest lane over the runs of row tile t split S ways
        const int w = kSpreadTh / S, b0 = t * kSpreadTh, b1 = std::min(NB, b0 + kSpreadTh);
        int best = 0;
        for (int q = 0; q < S; ++q)
            for (int c = 0; c < Ng; ++c) {
                int v = 0;
                for (int r = b0 + q * w; r < std::min(b1, b0 + (q + 1) * w); ++r) v += vis[(size_t)r * Ng + c];
                best = std::max(best, v);
            }
        return best;
    };
    std::vector<int> whole(nrt);
    for (int t = 0; t < nrt; ++t) whole[t] = longest(t, 1);
    std::vector<int> srt(whole);
    std::sort(srt.begin(), srt.end());
    const double limit = (single ? kSpreadSplitFactorSingle : kSpreadSplitFactor) * srt[srt.size() / 2];
    // runs per row tile
    std::vector<int> runs(nrt, 1);
    long used = 0;  // slab rows
    for (int t = 0; t + 1 < nrt; ++t) {
        if (!single && t >= kSpreadSplitTiles) break;
        int S = 1;
        while (S < kSpreadMaxRuns && longest(t, S) > limit) S *= 2;
        runs[t] = S;
        if (S > 1) used += (long)S * spread_run_rows(S);
    }
    // a single-instance plan whose slab would exceed kSpreadSlabCapSingle
    // bytes per instance takes the batched rule instead (splitting only part
    // of the tiles leaves the unsplit ones as the longest chains)
    if (single && used * (long)((size_t)Ng * sizeof(float2)) > (long)kSpreadSlabCapSingle) {
        spread_runs(bptr, NB, Ng, false, rows, split, slab_rows);
        return;
    }
    rows.clear();
    split.assign(nrt, make_int2(1, -1));
    slab_rows = 0;
    for (int t = 0; t < nrt; ++t) {
        const int b0 = t * kSpreadTh, b1 = std::min(NB, b0 + kSpreadTh) - 1;
        const int S = runs[t];
        if (S == 1) {
            rows.push_back(make_int4(b0, b1, -1, t));
            continue;
        }
        const int w = kSpreadTh / S;
        split[t] = make_int2(S, slab_rows);
        for (int q = 0; q < S; ++q) {
            rows.push_back(make_int4(b0 + q * w, b0 + (q + 1) * w - 1, slab_rows, t));
            slab_rows += spread_run_rows(S);
        }
    }
}

// Host part of plan creation; fills every table into `tb` and the PlanDev
// offsets (as byte offsets stored in the pointer fields, relocated later).
static int build_tables(const pat_plan_desc* desc, const Derived& dv, pat_plan* p, TableBuilder& tb)
{
    PlanDev& d = p->dev;
    const int N = desc->n, Ng = dv.Ng, nlam = dv.n_lam, K = dv.K, D = desc->n_det, T = desc->n_t;
    const double h = dv.h, R = desc->det_r;
    d.N = N; d.Ng = Ng; d.Hy = Ng / 2 + 9; d.nlam = nlam; d.K = K; d.Kp = K + 1; d.M = dv.M;
    d.T = T; d.D = D; d.L = (dv.P || dv.dense) ? 0 : dv.L; d.NB = Ng / 2 + 2;
    d.syn_dense = dv.dense;
    d.kappa = (float)dv.kappa;
    d.h2 = (float)(h * h);

    FftSet ffts;
    const int tps_grid = fixed_fft_tps(Ng), tps_dct = fixed_fft_tps(2L * dv.M);
    if (!tps_grid || !tps_dct) return PAT_ERR_UNSUPPORTED;
    d.fft_grid = ffts.get(Ng, tps_grid);
    d.fft_dct = ffts.get(2L * dv.M, tps_dct);
    if (d.fft_grid < 0 || d.fft_dct < 0) return PAT_ERR_UNSUPPORTED;
    d.fold_P = dv.P;
    d.fold_s = dv.P ? dv.S : 0;
    d.syn_len = dv.dense ? 0 : (dv.P ? dv.P : dv.L);
    d.syn_half = (dv.P && dv.P % 2 == 0) ? 1 : 0;
    // (the synthesis transforms are planned below, once the ring kernels' threads are known)

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
        ringTwn[n - 1] = ffts.get(np, 0);
        rho[n - 1] = lam * h * Ng / (2.0 * PI);
        npts += np / 2;
        joff += kn + 1;
        npsi_max = std::max(npsi_max, np);
    }
    ringOff[nlam] = npts;
    // ring kernels: as few threads per ring as the transforms allow (one wave when
    // possible, so that many rings are resident per CU to hide their latency),
    // at least (K + 1) / kRingModesPerThread (every mode's coefficient prefetched);
    // the ring and synthesis transforms are planned for that many threads
    {
        const long syn_fft_n = d.syn_half ? dv.P / 2 : d.syn_len;
        p->thr_ring = 0;
        for (int thr = 64; thr <= kRingMaxThreads && !p->thr_ring; thr *= 2) {
            unsigned char rad[kMaxStages];
            bool ok = thr * kRingModesPerThread >= K + 1 &&
                      (dv.dense || fft_passes(syn_fft_n, thr, kRingFftMaxButterflies, rad) >= 0);
            for (int n = 0; n < nlam && ok; ++n)
                if (n == 0 || ringN[n] != ringN[n - 1])
                    ok = fft_passes(ringN[n] / 2, thr, kRingFftMaxButterflies, rad) >= 0;
            if (ok) p->thr_ring = thr;
        }
        if (!p->thr_ring) return PAT_ERR_UNSUPPORTED;
        const int thr = p->thr_ring;
        for (int n = 0; n < nlam; ++n) {
            ringFft[n] = ffts.get(ringN[n] / 2, thr, kRingFftMaxButterflies);
            if (ringFft[n] < 0) return PAT_ERR_UNSUPPORTED;
        }
        // fft_syn: length syn_len (its twiddles; the transform itself unless the
        // synthesis runs as a half-length real transform, fft_synh)
        if (dv.dense) {  // no synthesis transform (the ring kernels do not read these)
            d.fft_syn = d.fft_synh = d.fft_grid;
        } else {
            d.fft_syn = ffts.get(d.syn_len, d.syn_half ? 0 : thr, kRingFftMaxButterflies);
            d.fft_synh = d.syn_half ? ffts.get(dv.P / 2, thr, kRingFftMaxButterflies) : d.fft_syn;
        }
        if (d.fft_syn < 0 || d.fft_synh < 0) return PAT_ERR_UNSUPPORTED;
    }
    p->n_ring_modes = joff;
    d.npsi_max = npsi_max;
    d.npts = npts;
    p->n_psi_max = npsi_max;

    // ring kernels with compile-time transforms (cfft.hpp) where every length
    // has one (uniform arc with a folded synthesis of even length P): tables of the transforms (per distinct length), of the
    // real-transform unpacking twiddles w_{Npsi}^k (per distinct ring length)
    // and of the synthesis prologue/epilogue twiddles w_P^s
    std::vector<float2> ctw;
    std::vector<int> ringCtw(nlam, 0), ringUw(nlam, 0);
    std::map<int, int> tab_of, uw_of;
    d.ring_spec = 0;
    d.ring_spec_grp = 0;
    {
        const int SH = dv.P / 2;
        auto len_ok = [](int L) { return cfft_len_ok(L) || cfft_len2_ok(L); };
        bool ok = !dv.dense && dv.P > 0 && d.syn_half && len_ok(SH);
        for (int n = 0; n < nlam && ok; ++n) ok = len_ok(ringN[n] / 2);
        if (ok) {
            int lmax = SH;
            for (int n = 0; n < nlam; ++n) lmax = std::max(lmax, ringN[n] / 2);
            d.ring_spec_grp = lmax > 1024 ? 2 : (lmax > kCfftSplit ? 1 : 0);
        }
        {
            auto add_cfft = [&](int L) {
                auto it = tab_of.find(L);
                if (it != tab_of.end()) return it->second;
                const CPlan cp = make_cplan(L);
                const int o = (int)ctw.size();
                ctw.resize(ctw.size() + std::max(cp.twoff[cp.np], 1));
                for (int st = 0; st < cp.np; ++st) {
                    const int R = cp.rad[st], NS = cp.ns[st];
                    if (NS == 1) continue;
                    for (int k = 0; k < NS; ++k)
                        for (int r = 1; r < R; ++r) {
                            const double a = -2.0 * PI * (double)(k * r) / (double)(NS * R);
                            ctw[o + cp.twoff[st] + k * (R - 1) + r - 1] =
                                make_float2((float)std::cos(a), (float)std::sin(a));
                        }
                }
                tab_of[L] = o;
                return o;
            };
            auto add_pow = [&](int n, int count) {  // e^{-2 pi i e / n}, e = 0..count-1
                const int o = (int)ctw.size();
                for (int e = 0; e < count; ++e) {
                    const double a = -2.0 * PI * (double)e / (double)n;
                    ctw.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
                }
                return o;
            };
            if (ok) {
                d.syn_ctw = add_cfft(SH);
                d.syn_sw = add_pow(dv.P, SH + 1);
                for (int n = 0; n < nlam; ++n) {
                    const int Pn = ringN[n] / 2;
                    ringCtw[n] = add_cfft(Pn);
                    auto it = uw_of.find(Pn);
                    if (it == uw_of.end()) it = uw_of.emplace(Pn, add_pow(2 * Pn, Pn + 1)).first;
                    ringUw[n] = it->second;
                }
                d.ring_spec = 1;
                p->thr_ring = ring_spec_threads(d.ring_spec_grp);
            }
            // the cosine transform: compile-time length 2M for the lengths the
            // kernels instantiate
            const int n2 = 2 * dv.M;
            d.dct_spec = (n2 == 256 || n2 == 512 || n2 == 1024 || n2 == 2048 || n2 == 4096 || n2 == 8192) ? 1 : 0;
            if (d.dct_spec) d.dct_ctw = add_cfft(n2);
            // the 2D-FFT passes: compile-time grid side
            d.grid_spec = grid_len_ok(Ng) ? 1 : 0;
            if (d.grid_spec) d.grid_ctw = add_cfft(Ng);
        }
    }
    if (ctw.empty()) ctw.push_back(make_float2(0.f, 0.f));

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
            int ibx = bxm, iq = q;
            std::memcpy(&gq.x, &ibx, 4);
            std::memcpy(&gq.y, &iq, 4);
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
    std::vector<int> band_of(npts);  // ring-order index -> band-order slot
    std::vector<float4> bgeo(npts);  // geometry in band order (y: the point's ring-order index)
    std::vector<float2> bphase(npts);
    for (int s = 0; s < npts; ++s) {
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
    std::vector<int4> sprRow;
    std::vector<int2> sprSplit;
    spread_runs(bptr, NB, Ng, desc->max_batch == 1, sprRow, sprSplit, d.slab_rows);
    d.spr_rows = (int)sprRow.size();
    // the adjoint row pass looks up row tiles r / 8 and r / 8 - 1 of its grid rows r < Hy
    std::vector<unsigned> sprHead((size_t)(d.Hy + 7) / 8 + 1, 0u);
    for (size_t t = 0; t < sprSplit.size() && t < sprHead.size(); ++t) {
        const int2 e = sprSplit[t];
        int lg = 0;
        while ((1 << lg) < e.x) ++lg;
        sprHead[t] = e.x > 1 ? ((unsigned)e.y << 4) | (unsigned)lg : 0u;
    }

    // --- synthesis over detector angles --------------------------------------
    // uniform arc: theta_d = theta_0 + d dtheta; explicit angles: the phases are
    // in the dense table below (theta_0 = 0 in the coefficients)
    const double dth = desc->arc_span / D;
    const double th0 = dv.dense ? 0.0 : desc->arc_center - 0.5 * desc->arc_span + 0.5 * dth;
    auto wpow = [&](long m) {  // w^{m^2}, w = e^{i dth/2}; phase reduced mod 2 pi in FP64
        double a = std::fmod(0.5 * dth * (double)m * (double)m, 2.0 * PI);
        return cd(std::cos(a), std::sin(a));
    };
    std::vector<cd> pre(K + 1);
    std::vector<float2> post, vhat;
    for (int k = 0; k <= K; ++k) {
        double a = std::fmod(k * th0, 2.0 * PI);
        cd v = (k == 0 ? 1.0 : 2.0) * cd(std::cos(a), std::sin(a));
        if (!dv.P && !dv.dense) v *= wpow(k);
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
    // explicit angles: rows 2k and 2k + 1 of the dense synthesis table hold
    // cos(k theta_d) and -sin(k theta_d), so that Re(a_k e^{ik theta_d}) =
    // Re a_k row_2k[d] + Im a_k row_2k+1[d] (angles reduced mod 2 pi in FP64)
    std::vector<float> syn_tab;
    if (dv.dense) {
        syn_tab.resize((size_t)2 * (K + 1) * D);
        for (int k = 0; k <= K; ++k)
            for (int q = 0; q < D; ++q) {
                const double a = std::fmod((double)k * desc->det_theta[q], 2.0 * PI);
                syn_tab[(size_t)(2 * k) * D + q] = (float)std::cos(a);
                syn_tab[(size_t)(2 * k + 1) * D + q] = (float)-std::sin(a);
            }
    }

    {
        int rc = choose_launch(p, ffts.descs, desc->max_batch);
        if (rc != PAT_OK) return rc;
    }

    // --- pack ---------------------------------------------------------------
    size_t o_deap = tb.add(deap), o_mask = tb.add(mask);
    size_t o_roff = tb.add(ringOff), o_rk = tb.add(ringK), o_rfft = tb.add(ringFft), o_rj = tb.add(ringJoff);
    size_t o_rtwn = tb.add(ringTwn);
    size_t o_coef = tb.add(coef);
    size_t o_bandof = tb.add(band_of), o_bgeo = tb.add(bgeo), o_bph = tb.add(bphase), o_bptr = tb.add(bptr);
    size_t o_post = tb.add(post), o_vhat = tb.add(vhat), o_syn = tb.add(syn_tab);
    size_t o_ffts = tb.add(ffts.descs), o_tw = tb.add(ffts.tw);
    size_t o_rctw = tb.add(ringCtw), o_ruw = tb.add(ringUw), o_ctw = tb.add(ctw);
    size_t o_sprow = tb.add(sprRow);
    size_t o_sphead = tb.add(sprHead);
    // store offsets in the pointer fields; relocated after the upload
    auto off = [](size_t o) { return (const void*)(uintptr_t)o; };
    d.deap = (const float*)off(o_deap);
    d.mask_rows = (const int2*)off(o_mask);
    d.ring_off = (const int*)off(o_roff);
    d.ring_K = (const int*)off(o_rk);
    d.ring_fft = (const int*)off(o_rfft);
    d.ring_twn = (const int*)off(o_rtwn);
    d.ring_joff = (const int*)off(o_rj);
    d.coef = (const float2*)off(o_coef);
    d.band_of = (const int*)off(o_bandof);
    d.bpt_geo = (const float4*)off(o_bgeo);
    d.bpt_phase = (const float2*)off(o_bph);
    d.band_ptr = (const int*)off(o_bptr);
    d.czt_post = (const float2*)off(o_post);
    d.czt_vhat = (const float2*)off(o_vhat);
    d.syn_tab = (const float*)off(o_syn);
    d.ffts = (const FftDev*)off(o_ffts);
    d.tw = (const float2*)off(o_tw);
    d.ring_ctw = (const int*)off(o_rctw);
    d.ring_uw = (const int*)off(o_ruw);
    d.ctw = (const float2*)off(o_ctw);
    d.spr_row = (const int4*)off(o_sprow);
    d.spr_head = (const unsigned*)off(o_sphead);
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
    rel(d.deap); rel(d.mask_rows); rel(d.ring_off); rel(d.ring_K);
    rel(d.ring_fft); rel(d.ring_twn); rel(d.ring_joff); rel(d.coef); rel(d.band_of); rel(d.bpt_geo); rel(d.bpt_phase);
    rel(d.band_ptr); rel(d.czt_post); rel(d.czt_vhat); rel(d.syn_tab); rel(d.ffts); rel(d.tw);
    rel(d.ring_ctw); rel(d.ring_uw); rel(d.ctw); rel(d.spr_row); rel(d.spr_head);
    p->desc = *desc;
    if (desc->det_theta) {  // the plan keeps its own copy of the angles
        p->det_theta = (double*)std::malloc(sizeof(double) * (size_t)desc->n_det);
        if (!p->det_theta) {
            (void)hipFree(mem);
            delete p;
            return PAT_ERR_ALLOC;
        }
        std::memcpy(p->det_theta, desc->det_theta, sizeof(double) * (size_t)desc->n_det);
        p->desc.det_theta = p->det_theta;
    }
    p->max_batch = desc->max_batch;
    p->n_psi_uniform = dv.n_psi;
    p->M = dv.M;
    p->dlam = dv.dlam;
    p->kappa = dv.kappa;
    layout_workspace(p);
    // the second stream of two-stream calls (default priority, no implicit
    // synchronisation with the null stream: the calls order it by events)
    p->split_min = kSplitMinBatch;
    p->split_mu = new (std::nothrow) std::mutex;
    if (!p->split_mu || hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming) != hipSuccess) {
        pat_plan_destroy(p);
        return PAT_ERR_HIP;
    }
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
    out->syn_dense = p->dev.syn_dense;
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
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) cur = p->device;
    (void)hipSetDevice(p->device);
    if (p->side) {  // work still queued on it finishes first
        (void)hipStreamSynchronize(p->side);
        (void)hipStreamDestroy(p->side);
    }
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    if (p->ev_join) (void)hipEventDestroy(p->ev_join);
    if (p->table_mem) (void)hipFree(p->table_mem);
    (void)hipSetDevice(cur);
    delete p->split_mu;
    std::free(p->det_theta);
    delete p;
}

extern "C" size_t pat_workspace_size(const pat_plan* p, int batch)
{
    if (!p || batch < 1) return 0;
    return p->ws.bytes * (size_t)batch;
}
