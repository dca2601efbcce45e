// tune.hip -- autotuner of the launch shapes (host code only).
//
// Every stage of the operator pair has its own tile shape and its own
// kernels, so one timed forward + adjoint per round measures a candidate of
// every stage at once: round r sets the r-th candidate of each stage's list
// (when it fits the LDS/thread limits), and each stage keeps the candidate with
// its smallest kernel time.  Then whole calls at the tuned shapes are timed
// on one stream and on two (pat_plan_set_split), and two are kept if faster.
// Results are cached in a small JSON file, one entry per geometry / batch /
// device.
#include "pat_internal.hpp"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace {

constexpr int kRounds = 10;
constexpr int kReps = 3;  // timed repetitions per round (after one warm-up); the minimum is kept

const int kColNp[] = {1, 2, 4, 8, 16};
const int kRowRpb[] = {1, 2, 4, 8, 16};
const int kRingRt[] = {1, 2, 4};
const int kDctDp[] = {1, 2, 4, 8};
// (columns, rows or bands, instances per tile); a candidate whose LDS does not fit is skipped
const int kGather[][3] = {{64, 8, 4}, {64, 16, 4}, {32, 8, 4}, {64, 4, 4}, {64, 16, 2}, {128, 16, 1},
                          {64, 8, 1}, {128, 8, 2}, {64, 8, 2}, {32, 16, 4}};
const int kSpread[][3] = {{256, 8, 4}, {192, 8, 4}, {128, 8, 4}, {256, 8, 2}, {128, 8, 2}, {192, 8, 1},
                          {128, 8, 1}, {256, 8, 1}, {64, 8, 4}, {64, 8, 1}};

enum { kSCol, kSRow, kSRing, kSDct, kSGather, kSSpread, kNS };

// Sets the round-r candidate of stage s in c; false when the list is exhausted.
bool set_candidate(pat_launch& c, int s, int r)
{
    switch (s) {
        case kSCol: if (r >= 5) return false; c.col_np = kColNp[r]; return true;
        case kSRow: if (r >= 5) return false; c.row_rpb = kRowRpb[r]; return true;
        case kSRing: if (r >= 3) return false; c.ring_rt = kRingRt[r]; return true;
        case kSDct: if (r >= 4) return false; c.dct_dp = kDctDp[r]; return true;
        case kSGather:
            if (r >= 10) return false;
            c.gat_cb = kGather[r][0]; c.gat_th = kGather[r][1]; c.gat_ib = kGather[r][2];
            return true;
        default:
            if (r >= 10) return false;
            c.spr_cb = kSpread[r][0]; c.spr_th = kSpread[r][1]; c.spr_ib = kSpread[r][2];
            return true;
    }
}

void copy_stage(pat_launch& dst, const pat_launch& src, int s)
{
    switch (s) {
        case kSCol: dst.col_np = src.col_np; break;
        case kSRow: dst.row_rpb = src.row_rpb; break;
        case kSRing: dst.ring_rt = src.ring_rt; break;
        case kSDct: dst.dct_dp = src.dct_dp; break;
        case kSGather: dst.gat_cb = src.gat_cb; dst.gat_th = src.gat_th; dst.gat_ib = src.gat_ib; break;
        default: dst.spr_cb = src.spr_cb; dst.spr_th = src.spr_th; dst.spr_ib = src.spr_ib; break;
    }
}

std::string device_name()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string s(prop.gcnArchName);
    for (char& ch : s)
        if (ch == '"' || ch == '\\') ch = '_';
    return s;
}

// FNV-1a of a plan's explicit detector angles (0 for a uniform arc)
static uint64_t angles_hash(const pat_plan_desc& d)
{
    if (!d.det_theta) return 0;
    uint64_t h = 1469598103934665603ull;
    const unsigned char* c = (const unsigned char*)d.det_theta;
    for (size_t i = 0; i < sizeof(double) * (size_t)d.n_det; ++i) h = (h ^ c[i]) * 1099511628211ull;
    return h;
}

std::string plan_key(const pat_plan* p, int batch)
{
    const pat_plan_desc& d = p->desc;
    char buf[512];
    std::snprintf(buf, sizeof buf,
                  "plan n=%d D=%d T=%d arc=%.12g ctr=%.12g dt=%.12g c=%.12g R=%.12g rho=%.12g sig=%.12g em=%d "
                  "angles=%016llx batch=%d dev=%s",
                  d.n, d.n_det, d.n_t, d.arc_span, d.arc_center, d.dt, d.c, d.det_r, d.support_r,
                  d.lambda_oversample, d.em_correction, (unsigned long long)angles_hash(d), batch,
                  device_name().c_str());
    return buf;
}

// FNV-1a over the instances' geometries and FFT-stage shapes.
std::string batch_key(const pat_batch* b)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void* data, size_t n) {
        const unsigned char* c = (const unsigned char*)data;
        for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
    };
    for (const pat_plan* p : b->plans) {
        const pat_plan_desc& d = p->desc;
        const uint64_t ah = angles_hash(d);
        mix(&ah, sizeof ah);
        mix(&d.n, sizeof d.n); mix(&d.n_det, sizeof d.n_det); mix(&d.n_t, sizeof d.n_t);
        mix(&d.arc_span, sizeof d.arc_span); mix(&d.arc_center, sizeof d.arc_center); mix(&d.dt, sizeof d.dt);
        mix(&d.c, sizeof d.c); mix(&d.det_r, sizeof d.det_r); mix(&d.support_r, sizeof d.support_r);
        mix(&d.lambda_oversample, sizeof d.lambda_oversample); mix(&d.em_correction, sizeof d.em_correction);
        mix(&p->cfg.col_np, sizeof(int)); mix(&p->cfg.row_rpb, sizeof(int));
        mix(&p->cfg.ring_rt, sizeof(int)); mix(&p->cfg.dct_dp, sizeof(int));
    }
    char buf[256];
    std::snprintf(buf, sizeof buf, "batch count=%d geo=%016llx dev=%s", b->count, (unsigned long long)h,
                  device_name().c_str());
    return buf;
}

// ---- cache file: {"key": {"col_np": 1, ...}, ...} --------------------------
constexpr int kNumFields = 10;
const char* kFields[kNumFields] = {"col_np", "row_rpb", "ring_rt", "dct_dp", "gat_cb",
                                   "gat_th", "spr_cb",  "spr_th",  "gat_ib", "spr_ib"};

int* field_ptr(pat_launch& c, int i)
{
    int* f[kNumFields] = {&c.col_np, &c.row_rpb, &c.ring_rt, &c.dct_dp, &c.gat_cb,
                          &c.gat_th, &c.spr_cb,  &c.spr_th,  &c.gat_ib, &c.spr_ib};
    return f[i];
}

// 1: file present and shaped like a JSON object, 0: no file (or empty), -1: anything else.
int cache_read(const char* path, std::string& text)
{
    text.clear();
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return 0;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, fp)) > 0) text.append(buf, n);
    std::fclose(fp);
    size_t a = text.find_first_not_of(" \t\r\n");
    size_t z = text.find_last_not_of(" \t\r\n");
    if (a == std::string::npos) { text.clear(); return 0; }
    if (text[a] != '{' || text[z] != '}') return -1;
    return 1;
}

// An entry's fields; `split` (the two-stream batch, pat_plan_set_split) is
// read when the entry has it and left unchanged otherwise.
bool cache_lookup(const std::string& text, const std::string& key, pat_launch& c, int* split = nullptr)
{
    const std::string pat = "\"" + key + "\": {";
    const size_t at = text.find(pat);
    if (at == std::string::npos) return false;
    const size_t end = text.find('}', at + pat.size());
    if (end == std::string::npos) return false;
    const std::string body = text.substr(at + pat.size(), end - at - pat.size());
    for (int i = 0; i < kNumFields; ++i) {
        const std::string f = "\"" + std::string(kFields[i]) + "\": ";
        const size_t q = body.find(f);
        if (q == std::string::npos) return false;
        if (std::sscanf(body.c_str() + q + f.size(), "%d", field_ptr(c, i)) != 1) return false;
    }
    const size_t q = body.find("\"split\": ");
    if (split && q != std::string::npos && std::sscanf(body.c_str() + q + 9, "%d", split) != 1) return false;
    return true;
}

bool cache_store(const char* path, const std::string& key, const pat_launch& c0, int split = -1)
{
    pat_launch c = c0;
    std::string text;
    if (cache_read(path, text) < 0) return false;
    char entry[768];
    int o = std::snprintf(entry, sizeof entry, "\"%s\": {", key.c_str());
    for (int i = 0; i < kNumFields; ++i)
        o += std::snprintf(entry + o, sizeof entry - o, "%s\"%s\": %d", i ? ", " : "", kFields[i], *field_ptr(c, i));
    if (split >= 0) o += std::snprintf(entry + o, sizeof entry - o, ", \"split\": %d", split);
    std::snprintf(entry + o, sizeof entry - o, "}");
    const std::string pat = "\"" + key + "\": {";
    const size_t at = text.find(pat);
    if (at != std::string::npos) {
        const size_t end = text.find('}', at + pat.size());
        text.replace(at, end + 1 - at, entry);
    } else if (text.empty()) {
        text = std::string("{\n") + entry + "\n}\n";
    } else {
        const size_t z = text.find_last_of('}');
        std::string head = text.substr(0, z);
        const size_t t = head.find_last_not_of(" \t\r\n");
        head.resize(t + 1);
        text = head + (head.back() == '{' ? "\n" : ",\n") + entry + "\n}\n";
    }
    FILE* fp = std::fopen(path, "wb");
    if (!fp) return false;
    const bool ok = std::fwrite(text.data(), 1, text.size(), fp) == text.size();
    return std::fclose(fp) == 0 && ok;
}

// Device buffers of a tuning run, freed on scope exit.
struct DevBufs {
    std::vector<void*> ptrs;
    void* alloc(size_t bytes)
    {
        void* p = nullptr;
        if (hipMalloc(&p, bytes ? bytes : 256) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return p;
    }
    ~DevBufs()
    {
        (void)hipDeviceSynchronize();
        for (void* p : ptrs) (void)hipFree(p);
    }
};

// Whole forward + adjoint calls at `batch`, one stream (t1) and two (t2):
// each way, kSplitReps call pairs are captured into a HIP graph on a stream of
// the tuner (so the host's launch rate does not enter), and the graph is
// replayed in kSplitRounds alternating rounds; the best round, in
// milliseconds per pair.  Leaves the plan's split setting as it found it.
constexpr int kSplitRounds = 4, kSplitReps = 8;
constexpr float kSplitGain = 0.99f;  // two streams kept only if at least 1 % faster

int time_split(pat_plan* p, float* f, float* g, void* ws, size_t wsb, int batch, float& t1, float& t2)
{
    const int keep = p->split_min;
    hipStream_t cs = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipGraph_t gr[2] = {nullptr, nullptr};
    hipGraphExec_t ex[2] = {nullptr, nullptr};
    int rc = PAT_OK;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess)
        rc = PAT_ERR_HIP;
    for (int mode = 0; mode < 2 && rc == PAT_OK; ++mode) {
        p->split_min = mode ? 2 : 0;
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = PAT_ERR_HIP;
            break;
        }
        for (int k = 0; k < kSplitReps && rc == PAT_OK; ++k) {
            rc = pat_forward(p, f, g, batch, ws, wsb, cs);
            if (rc == PAT_OK) rc = pat_adjoint(p, g, f, batch, ws, wsb, cs);
        }
        // the capture is ended whatever the calls returned
        if (hipStreamEndCapture(cs, &gr[mode]) != hipSuccess && rc == PAT_OK) rc = PAT_ERR_HIP;
        if (rc == PAT_OK && (hipGraphInstantiate(&ex[mode], gr[mode], nullptr, nullptr, 0) != hipSuccess ||
                             hipGraphLaunch(ex[mode], cs) != hipSuccess))  // warm-up
            rc = PAT_ERR_HIP;
    }
    t1 = t2 = 3.0e38f;
    for (int r = 0; r < kSplitRounds && rc == PAT_OK; ++r) {
        for (int mode = 0; mode < 2 && rc == PAT_OK; ++mode) {
            float ms = 0.f;
            if (hipEventRecord(e0, cs) != hipSuccess || hipGraphLaunch(ex[mode], cs) != hipSuccess ||
                hipEventRecord(e1, cs) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                rc = PAT_ERR_HIP;
            float& t = mode ? t2 : t1;
            if (rc == PAT_OK) t = std::min(t, ms / kSplitReps);
        }
    }
    if (cs) (void)hipStreamSynchronize(cs);
    for (int mode = 0; mode < 2; ++mode) {
        if (ex[mode]) (void)hipGraphExecDestroy(ex[mode]);
        if (gr[mode]) (void)hipGraphDestroy(gr[mode]);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (cs) (void)hipStreamDestroy(cs);
    p->split_min = keep;
    return rc;
}

}  // namespace

extern "C" int pat_autotune_plan(pat_plan* p, int batch, const char* cache_path)
{
    if (!p || batch < 1 || batch > p->max_batch) return PAT_ERR_ARG;
    const std::string key = plan_key(p, batch);
    pat_launch def;
    pat_plan_get_launch(p, &def);
    if (cache_path) {
        std::string text;
        const int rc = cache_read(cache_path, text);
        if (rc < 0) return PAT_ERR_ARG;
        pat_launch c = def;
        // an entry the library no longer accepts (older shape rules) is re-tuned and replaced
        int split = p->split_min;
        if (rc > 0 && cache_lookup(text, key, c, &split) && pat_plan_set_launch(p, &c) == PAT_OK) {
            p->split_min = split;
            return PAT_OK;
        }
    }
    const pat_plan_desc& dsc = p->desc;
    DevBufs bufs;
    const size_t wsb = pat_workspace_size(p, batch);
    float* f = (float*)bufs.alloc(sizeof(float) * (size_t)batch * dsc.n * dsc.n);
    float* g = (float*)bufs.alloc(sizeof(float) * (size_t)batch * dsc.n_det * dsc.n_t);
    void* ws = bufs.alloc(wsb);
    if (!f || !g || !ws) return PAT_ERR_ALLOC;
    if (hipMemset(f, 0, sizeof(float) * (size_t)batch * dsc.n * dsc.n) != hipSuccess ||
        hipMemset(g, 0, sizeof(float) * (size_t)batch * dsc.n_det * dsc.n_t) != hipSuccess)
        return PAT_ERR_HIP;
    const int was_prof = p->prof;
    int rc = pat_profile_enable(p, 1);
    if (rc != PAT_OK) return rc;
    pat_launch best = def;
    float best_t[kNS];
    for (float& t : best_t) t = 3.0e38f;
    for (int r = 0; r < kRounds && rc == PAT_OK; ++r) {
        pat_launch c = def;
        bool used[kNS] = {};
        for (int s = 0; s < kNS; ++s) {
            pat_launch trial = def;
            if (!set_candidate(trial, s, r)) continue;
            if (pat_plan_set_launch(p, &trial) != PAT_OK) continue;  // does not fit: skip this candidate
            copy_stage(c, trial, s);
            used[s] = true;
        }
        if ((rc = pat_plan_set_launch(p, &c)) != PAT_OK) break;
        float fw[6], ad[6], fmin[5], amin[5];
        for (int k = 0; k < 5; ++k) fmin[k] = amin[k] = 3.0e38f;
        for (int rep = 0; rep <= kReps && rc == PAT_OK; ++rep) {
            int cf = 0, ca = 0;
            if ((rc = pat_forward(p, f, g, batch, ws, wsb, nullptr)) != PAT_OK) break;
            if ((rc = pat_profile_read(p, 0, fw, 6, &cf)) != PAT_OK) break;
            if ((rc = pat_adjoint(p, g, f, batch, ws, wsb, nullptr)) != PAT_OK) break;
            if ((rc = pat_profile_read(p, 1, ad, 6, &ca)) != PAT_OK) break;
            if (rep == 0) continue;
            if (cf == 6) {  // dense synthesis: counted with the ring stage (its shape is fixed)
                fw[3] += fw[4];
                fw[4] = fw[5];
                ad[1] += ad[2];
                for (int k = 2; k < 5; ++k) ad[k] = ad[k + 1];
            }
            for (int k = 0; k < 5; ++k) {
                fmin[k] = std::min(fmin[k], fw[k]);
                amin[k] = std::min(amin[k], ad[k]);
            }
        }
        if (rc != PAT_OK) break;
        // forward: col, row, gather, ring, dct; adjoint: dct, ring, spread, row, col
        const float t[kNS] = {fmin[0] + amin[4], fmin[1] + amin[3], fmin[3] + amin[1],
                              fmin[4] + amin[0], fmin[2], amin[2]};
        for (int s = 0; s < kNS; ++s)
            if (used[s] && t[s] < best_t[s]) {
                best_t[s] = t[s];
                copy_stage(best, c, s);
            }
    }
    if (!was_prof) (void)pat_profile_enable(p, 0);
    if (rc != PAT_OK) {
        (void)pat_plan_set_launch(p, &def);
        return rc;
    }
    if ((rc = pat_plan_set_launch(p, &best)) != PAT_OK) return rc;
    if (batch >= 2 && !p->prof) {  // two-stream calls at this batch: kept if faster
        float t1 = 0.f, t2 = 0.f;
        if ((rc = time_split(p, f, g, ws, wsb, batch, t1, t2)) != PAT_OK) return rc;
        p->split_min = t2 < kSplitGain * t1 ? batch : 0;
    }
    if (cache_path && !cache_store(cache_path, key, best, p->split_min)) return PAT_ERR_ARG;
    return PAT_OK;
}

extern "C" int pat_autotune_batch(pat_batch* b, const char* cache_path)
{
    if (!b) return PAT_ERR_ARG;
    const std::string key = batch_key(b);
    pat_launch def;
    pat_batch_get_launch(b, &def);
    if (cache_path) {
        std::string text;
        const int rc = cache_read(cache_path, text);
        if (rc < 0) return PAT_ERR_ARG;
        pat_launch c = def;
        if (rc > 0 && cache_lookup(text, key, c) && pat_batch_set_launch(b, &c) == PAT_OK) return PAT_OK;
    }
    DevBufs bufs;
    size_t nf = 0, ng = 0;
    for (const pat_plan* p : b->plans) {
        nf += (size_t)p->desc.n * p->desc.n;
        ng += (size_t)p->desc.n_det * p->desc.n_t;
    }
    float* f = (float*)bufs.alloc(sizeof(float) * nf);
    float* g = (float*)bufs.alloc(sizeof(float) * ng);
    void* ws = bufs.alloc(b->ws_bytes);
    float** fp = (float**)bufs.alloc(sizeof(float*) * b->count);
    float** gp = (float**)bufs.alloc(sizeof(float*) * b->count);
    if (!f || !g || !ws || !fp || !gp) return PAT_ERR_ALLOC;
    {
        std::vector<float*> hf(b->count), hg(b->count);
        size_t of = 0, og = 0;
        for (int i = 0; i < b->count; ++i) {
            const pat_plan* p = b->plans[i];
            hf[i] = f + of;
            hg[i] = g + og;
            of += (size_t)p->desc.n * p->desc.n;
            og += (size_t)p->desc.n_det * p->desc.n_t;
        }
        if (hipMemset(f, 0, sizeof(float) * nf) != hipSuccess || hipMemset(g, 0, sizeof(float) * ng) != hipSuccess ||
            hipMemcpy(fp, hf.data(), sizeof(float*) * b->count, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(gp, hg.data(), sizeof(float*) * b->count, hipMemcpyHostToDevice) != hipSuccess)
            return PAT_ERR_HIP;
    }
    hipEvent_t e[3];
    for (hipEvent_t& ev : e)
        if (hipEventCreate(&ev) != hipSuccess) return PAT_ERR_HIP;
    pat_launch best = def;
    float best_g = 3.0e38f, best_s = 3.0e38f;
    int rc = PAT_OK;
    for (int r = 0; r < kRounds && rc == PAT_OK; ++r) {
        pat_launch c = def;
        set_candidate(c, kSGather, r);
        set_candidate(c, kSSpread, r);
        if ((rc = pat_batch_set_launch(b, &c)) != PAT_OK) break;
        float tf = 3.0e38f, ta = 3.0e38f;
        for (int rep = 0; rep <= kReps && rc == PAT_OK; ++rep) {
            // only the interpolation changes among the forward kernels, only the spread among the adjoint ones
            if (hipEventRecord(e[0], nullptr) != hipSuccess) { rc = PAT_ERR_HIP; break; }
            if ((rc = pat_batch_forward(b, (const float* const*)fp, gp, ws, b->ws_bytes, nullptr)) != PAT_OK) break;
            if (hipEventRecord(e[1], nullptr) != hipSuccess) { rc = PAT_ERR_HIP; break; }
            if ((rc = pat_batch_adjoint(b, (const float* const*)gp, fp, ws, b->ws_bytes, nullptr)) != PAT_OK) break;
            if (hipEventRecord(e[2], nullptr) != hipSuccess || hipEventSynchronize(e[2]) != hipSuccess) {
                rc = PAT_ERR_HIP;
                break;
            }
            float m1 = 0.f, m2 = 0.f;
            if (hipEventElapsedTime(&m1, e[0], e[1]) != hipSuccess || hipEventElapsedTime(&m2, e[1], e[2]) != hipSuccess) {
                rc = PAT_ERR_HIP;
                break;
            }
            if (rep == 0) continue;
            tf = std::min(tf, m1);
            ta = std::min(ta, m2);
        }
        if (rc != PAT_OK) break;
        if (tf < best_g) { best_g = tf; copy_stage(best, c, kSGather); }
        if (ta < best_s) { best_s = ta; copy_stage(best, c, kSSpread); }
    }
    for (hipEvent_t& ev : e) (void)hipEventDestroy(ev);
    if (rc != PAT_OK) {
        (void)pat_batch_set_launch(b, &def);
        return rc;
    }
    if ((rc = pat_batch_set_launch(b, &best)) != PAT_OK) return rc;
    if (cache_path && !cache_store(cache_path, key, best)) return PAT_ERR_ARG;
    return PAT_OK;
}
