// api.hip -- the C ABI of include/mm.h: argument checking, plan memory,
// launch configuration, step driver with HIP-graph replay, timing.
#include <cmath>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <fstream>
#include <map>
#include <string>
#include <vector>

#include <unistd.h>

#include "mm_internal.hpp"

namespace mmk {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }
int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

bool length_supported(int L);
int padded_length(int n);

// ------------------------------------------------------------------ timing ---
static hipEvent_t take_event(Plan &p)
{
    if (!p.event_pool.empty()) {
        hipEvent_t e = p.event_pool.back();
        p.event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void timing_arm(Plan &p)
{
    p.tev[0] = p.tev[1] = nullptr;
    if (!p.timing) return;
    hipEvent_t e0 = take_event(p), e1 = e0 ? take_event(p) : nullptr;
    if (!e1) {
        if (e0) p.event_pool.push_back(e0);
        return;
    }
    p.tev[0] = e0;
    p.tev[1] = e1;
}

void timing_file(Plan &p, int pass)
{
    if (p.tev[0]) p.pending.push_back({pass, {p.tev[0], p.tev[1]}});
    p.tev[0] = p.tev[1] = nullptr;
}

void timing_begin(Plan &p, int pass, hipStream_t s, hipEvent_t *ev0)
{
    (void)pass;
    *ev0 = nullptr;
    if (!p.timing) return;
    hipEvent_t e = take_event(p);
    if (e && hipEventRecord(e, s) == hipSuccess) *ev0 = e;
}

void timing_end(Plan &p, int pass, hipStream_t s, hipEvent_t ev0)
{
    if (!p.timing || !ev0) return;
    hipEvent_t e1 = take_event(p);
    if (!e1 || hipEventRecord(e1, s) != hipSuccess) return;
    p.pending.push_back({pass, {ev0, e1}});
}

static int drain_timing(Plan &p)
{
    for (const TimedPair &t : p.pending) {
        MMK_HIP(hipEventSynchronize(t.second.second));
        float ms = 0.f;
        MMK_HIP(hipEventElapsedTime(&ms, t.second.first, t.second.second));
        p.acc[t.first].ms += ms;
        p.acc[t.first].n += 1;
        p.event_pool.push_back(t.second.first);
        p.event_pool.push_back(t.second.second);
    }
    p.pending.clear();
    return MM_OK;
}

static void drop_plan_graph(Plan &p)
{
    if (p.graph.exec) (void)hipGraphExecDestroy(p.graph.exec);
    if (p.graph.graph) (void)hipGraphDestroy(p.graph.graph);
    p.graph = GraphCache{};
}

// ------------------------------------------------------------------- plan ---
// Twiddle table exp(-2 pi i m / L), m < L, built in FP64 and rounded once.
static std::vector<float2> twiddle_table(int L)
{
    std::vector<float2> h((size_t)L);
    for (int m = 0; m < L; ++m) {
        const double a = -2.0 * M_PI * (double)m / (double)L;
        h[m] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    return h;
}

struct PlanOwner {
    Plan p;
};

static void free_plan(PlanOwner *o)
{
    if (!o) return;
    Plan &p = o->p;
    drop_plan_graph(p);
    if (p.cap_stream) (void)hipStreamDestroy(p.cap_stream);
    for (auto &t : p.pending) {
        (void)hipEventDestroy(t.second.first);
        (void)hipEventDestroy(t.second.second);
    }
    for (auto e : p.event_pool) (void)hipEventDestroy(e);
    delete o;
}

static bool axis_ok(int n) { return n >= 1 && n <= 512 && padded_length(n) > 0; }

static int check_grid(int nx, int ny, int nz, double dx, double dy, double dz)
{
    if (!axis_ok(nx) || !axis_ok(ny) || !axis_ok(nz))
        return fail(MM_EINVAL, "grid sizes must be 1..512 cells per axis");
    if (!(dx > 0.0) || !(dy > 0.0) || !(dz > 0.0) || !std::isfinite(dx) || !std::isfinite(dy) ||
        !std::isfinite(dz))
        return fail(MM_EINVAL, "cell sizes must be finite and > 0");
    return MM_OK;
}

// Carve the plan's workspace (base == nullptr: only measure it) and return
// its size.  Order: K~, twiddles, reduction partials and records, then the
// run-time buffers X1, X2, H, Sa, Sb, kacc.  The spectrum set-up borrows the
// run-time region for its FP64 scratch before any step runs, so the region
// is at least that large.
size_t plan_layout(Plan &p, char *base)
{
    const size_t N = (size_t)p.nx * p.ny * p.nz;
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const size_t szK = sizeof(float) * 6 * (size_t)p.nzK * (p.Ly / 2 + 1) * p.xp;
    const size_t szX1 = sizeof(float2) * 3 * (size_t)nz * ny * p.xp;
    const size_t szX2 = nz > 1 ? sizeof(float2) * 3 * (size_t)nz * x2_plane_stride(p.Ly, p.xp) : 0;
    const size_t szF = sizeof(float) * 3 * N;
    const size_t szPart = sizeof(double) * 9 * (size_t)p.red_blocks;
    const size_t szRed = sizeof(double) * 16 * (size_t)RED_LOG;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t tw = 0;
    const int Ls[3] = {p.Lx, p.Ly, nz > 1 ? p.Lz : 0};
    for (int a = 0; a < 3; ++a) tw += Ls[a] ? al(sizeof(float2) * (size_t)Ls[a]) : 0;
    const size_t run = al(szX1) + al(szX2) + 4 * al(szF);
    const size_t scratch = al(spectrum_scratch_bytes(nx, ny, nz, p.Lx, p.Ly, p.Lz));
    const size_t total = al(szK) + tw + al(szPart) + al(szRed) + (run > scratch ? run : scratch);
    if (!base) return total;
    char *cur = base;
    p.Kt = (float *)cur; cur += al(szK);
    for (int a = 0; a < 3; ++a) {
        p.tw[a] = nullptr;
        if (!Ls[a]) continue;
        p.tw[a] = (float2 *)cur;
        cur += al(sizeof(float2) * (size_t)Ls[a]);
    }
    p.part = (double *)cur; cur += al(szPart);
    p.red = (double *)cur; cur += al(szRed);
    p.run = cur;
    p.X1 = (float2 *)cur; cur += al(szX1);
    p.X2 = szX2 ? (float2 *)cur : nullptr; cur += al(szX2);
    p.H = (float *)cur; cur += al(szF);
    p.Sa = (float *)cur; cur += al(szF);
    p.Sb = (float *)cur; cur += al(szF);
    p.kacc = (float *)cur;
    return total;
}

// ------------------------------------------------------------ tune cache ---
// A JSON object with one key per line,
//   "gfx950/256cu/128x128x128": {"xfwd": 8, "yfwd": 16, ...},
// naming the device and grid and giving the tile of every pass kind.
static const char *const PASS_NAMES[MM_PASS_COUNT] = {"xfwd",  "yfwd",  "zconv",  "yinv",  "xinv",
                                                      "yconv", "stage", "reduce", "xstage"};

static std::string tune_key(const Plan &p)
{
    return p.arch + "/" + std::to_string(p.nx) + "x" + std::to_string(p.ny) + "x" + std::to_string(p.nz);
}

static std::map<std::string, std::string> tune_cache_load(const char *path)
{
    std::map<std::string, std::string> out;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t a = line.find('"');
        const size_t b = a == std::string::npos ? a : line.find('"', a + 1);
        const size_t c = b == std::string::npos ? b : line.find('{', b);
        const size_t d = c == std::string::npos ? c : line.find('}', c);
        if (d == std::string::npos) continue;
        out[line.substr(a + 1, b - a - 1)] = line.substr(c, d - c + 1);
    }
    return out;
}

// Apply a cached entry for this plan; false if absent or any tile in it is
// not launchable here.
bool tune_cache_read(Plan &p, const char *path)
{
    const auto m = tune_cache_load(path);
    const auto it = m.find(tune_key(p));
    if (it == m.end()) return false;
    int tiles[MM_PASS_COUNT];
    for (int k = 0; k < MM_PASS_COUNT; ++k) {
        const std::string pat = std::string("\"") + PASS_NAMES[k] + "\":";
        const size_t at = it->second.find(pat);
        if (at == std::string::npos) return false;
        tiles[k] = std::atoi(it->second.c_str() + at + pat.size());
        if (tiles[k] != 0 && k != MM_PASS_REDUCE && !pass_tile_valid(p, k, tiles[k])) return false;
        if (tiles[k] == 0 && k != MM_PASS_REDUCE && k != MM_PASS_XSTAGE && p.tile[k] != 0) return false;
    }
    for (int k = 0; k < MM_PASS_COUNT; ++k) p.tile[k] = tiles[k];
    return true;
}

// Add (or replace) this plan's entry; the file is rewritten through a
// temporary and renamed into place.
void tune_cache_write(const Plan &p, const char *path)
{
    auto m = tune_cache_load(path);
    std::string v = "{";
    for (int k = 0; k < MM_PASS_COUNT; ++k)
        v += std::string(k ? ", " : "") + "\"" + PASS_NAMES[k] + "\": " + std::to_string(p.tile[k]);
    v += "}";
    m[tune_key(p)] = v;
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long long)getpid());
    {
        std::ofstream f(tmp);
        f << "{\n";
        size_t i = 0;
        for (const auto &kv : m) f << "\"" << kv.first << "\": " << kv.second << (++i < m.size() ? ",\n" : "\n");
        f << "}\n";
        if (!f) return;
    }
    (void)std::rename(tmp.c_str(), path);
}

int plan_ready(const Plan *p)
{
    if (!p) return fail(MM_EINVAL, "NULL plan");
    if (!p->ws) return fail(MM_EINVAL, "plan has no workspace: call mm_plan_bind_workspace first");
    return MM_OK;
}

}  // namespace mmk

using namespace mmk;

struct mm_plan_s {
    PlanOwner *o;
};

static Plan *P(mm_plan h) { return (h && h->o) ? &h->o->p : nullptr; }
Plan *mmk::plan_of(mm_plan h) { return P(h); }

extern "C" {

const char *mm_status_string(int status)
{
    switch (status) {
    case MM_OK: return "ok";
    case MM_EINVAL: return "invalid argument";
    case MM_ENOMEM: return "out of device memory";
    case MM_ENODEV: return "no HIP device";
    case MM_EHIP: return "HIP runtime error";
    case MM_ENONFINITE: return "non-finite value in state";
    case MM_ETUNE: return "autotuner found no candidate";
    case MM_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

int mm_last_error(char *buf, size_t n)
{
    if (buf && n > 0) {
        const size_t k = g_err.size() < n - 1 ? g_err.size() : n - 1;
        std::memcpy(buf, g_err.data(), k);
        buf[k] = '\0';
    }
    return (int)g_err.size();
}

static int have_device()
{
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return fail(MM_ENODEV, "no HIP device visible");
    }
    return MM_OK;
}

int mm_demag_setup(int nx, int ny, int nz, double dx, double dy, double dz, mm_plan *out)
{
    if (!out) return fail(MM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_grid(nx, ny, nz, dx, dy, dz);
    if (rc != MM_OK) return rc;
    if ((rc = have_device()) != MM_OK) return rc;
    PlanOwner *o = new PlanOwner();
    Plan &p = o->p;
    p.nx = nx; p.ny = ny; p.nz = nz;
    p.dx = dx; p.dy = dy; p.dz = dz;
    // each axis padded to the smallest supported transform length >= 2n
    p.Lx = padded_length(nx); p.Ly = padded_length(ny); p.Lz = nz > 1 ? padded_length(nz) : 1;
    p.nxc = p.Lx / 2 + 1;
    p.xp = x_pitch(p.nxc);
    p.nzK = nz > 1 ? p.Lz / 2 + 1 : 1;
    if (hipGetDevice(&p.device) != hipSuccess) {
        free_plan(o);
        return fail(MM_EHIP, "hipGetDevice");
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, p.device) == hipSuccess) {
        p.arch = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount) + "cu";
        p.lds_limit = prop.sharedMemPerBlock;
        if (p.lds_limit > 160 * 1024) p.lds_limit = 160 * 1024;
        if (p.lds_limit < 32768) p.lds_limit = 32768;
    }
    p.nK = 6LL * p.nzK * (p.Ly / 2 + 1) * p.nxc;
    p.red_blocks = 1024;
    p.bytes = plan_layout(p, nullptr);
    const int Ls[3] = {p.Lx, p.Ly, nz > 1 ? p.Lz : 0};
    for (int a = 0; a < 3; ++a)
        if (Ls[a]) p.tw_host[a] = twiddle_table(Ls[a]);
    if ((rc = prepare_kernels(p)) != MM_OK) {
        free_plan(o);
        return rc;
    }
    for (int k = 0; k < MM_PASS_COUNT; ++k) p.tile[k] = pass_default_tile(p, k);
    if (hipStreamCreateWithFlags(&p.cap_stream, hipStreamNonBlocking) != hipSuccess) {
        free_plan(o);
        return fail(MM_EHIP, "stream create");
    }
    mm_plan h = new mm_plan_s{o};
    *out = h;
    return MM_OK;
}

int mm_plan_workspace_bytes(mm_plan plan, size_t *bytes)
{
    Plan *p = P(plan);
    if (!p || !bytes) return fail(MM_EINVAL, "NULL plan or bytes");
    *bytes = p->bytes;
    return MM_OK;
}

int mm_plan_bind_workspace(mm_plan plan, void *ws, size_t bytes)
{
    Plan *p = P(plan);
    if (!p || !ws) return fail(MM_EINVAL, "NULL plan or workspace");
    if ((uintptr_t)ws % 256 != 0) return fail(MM_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < p->bytes)
        return fail(MM_ENOMEM, "workspace of " + std::to_string(bytes) + " bytes; the plan needs " +
                                   std::to_string(p->bytes));
    drop_plan_graph(*p);
    p->ws = nullptr;
    plan_layout(*p, (char *)ws);
    for (int a = 0; a < 3; ++a)
        if (!p->tw_host[a].empty())
            MMK_HIP(hipMemcpy(p->tw[a], p->tw_host[a].data(), sizeof(float2) * p->tw_host[a].size(),
                              hipMemcpyHostToDevice));
    int rc = build_spectrum(*p, nullptr);
    if (rc != MM_OK) return rc;
    MMK_HIP(hipDeviceSynchronize());
    p->ws = (char *)ws;
    return MM_OK;
}

void mm_destroy(mm_plan plan)
{
    if (!plan) return;
    free_plan(plan->o);
    delete plan;
}

int mm_demag_apply(mm_plan plan, const float *M, float *H, void *stream)
{
    Plan *p = P(plan);
    int rc = plan_ready(p);
    if (rc != MM_OK) return rc;
    if (!M || !H) return fail(MM_EINVAL, "NULL pointer");
    if ((const void *)M == (const void *)H) return fail(MM_EINVAL, "M and H alias");
    return demag_enqueue(*p, M, H, (hipStream_t)stream);
}

static int check_params(const mm_llg_params *q)
{
    if (!q) return fail(MM_EINVAL, "params is NULL");
    if (!(q->Ms > 0.0) || !std::isfinite(q->Ms)) return fail(MM_EINVAL, "Ms must be > 0");
    if (!std::isfinite(q->dt) || !std::isfinite(q->alpha) || !std::isfinite(q->gamma0) || !std::isfinite(q->A) ||
        !std::isfinite(q->Ku))
        return fail(MM_EINVAL, "non-finite parameter");
    if (q->integrator != MM_RK4 && q->integrator != MM_EULER) return fail(MM_EINVAL, "unknown integrator");
    if (q->demag_mode != MM_EXACT && q->demag_mode != MM_SURROGATE) return fail(MM_EINVAL, "unknown demag mode");
    if (q->sur_check_every > MM_SUR_CHECK_MAX) return fail(MM_EINVAL, "sur_check_every above MM_SUR_CHECK_MAX");
    const double u2 = q->axis[0] * q->axis[0] + q->axis[1] * q->axis[1] + q->axis[2] * q->axis[2];
    if (q->Ku != 0.0 && !(std::fabs(u2 - 1.0) < 1e-6)) return fail(MM_EINVAL, "anisotropy axis must be a unit vector");
    return MM_OK;
}

// n exact steps: direct launches (timing mode, or a single step), else
// replays of a captured graph: one RK4 step, or a pair of Euler steps (M ->
// Sa -> M, no copy) with a single copying step for an odd count.
static int exact_steps(Plan &p, const mm_llg_params &q, const StageCoef &c, float *M, int n, hipStream_t s)
{
    int rc;
    static const bool no_graph = std::getenv("MM_NO_GRAPH") != nullptr;
    const bool euler = q.integrator == MM_EULER;
    const int unit = euler ? 2 : 1;  // steps per graph replay
    if (p.timing || no_graph || n < 2) {
        // direct launches (timing mode brackets every one with HIP events)
        int i = 0;
        for (; euler && i + 2 <= n; i += 2)
            if ((rc = llg_enqueue_euler_pair(p, c, M, s)) != MM_OK) return rc;
        for (; i < n; ++i)
            if ((rc = llg_enqueue_step(p, c, q.integrator, M, s)) != MM_OK) return rc;
        return MM_OK;
    }
    std::string key((const char *)&c, sizeof(c));
    key += std::string((const char *)&q.integrator, sizeof(int));
    key += std::string((const char *)p.tile, sizeof(p.tile));
    if (!p.graph.exec || p.graph.M != M || p.graph.key != key) {
        drop_plan_graph(p);
        MMK_HIP(hipStreamBeginCapture(p.cap_stream, hipStreamCaptureModeThreadLocal));
        rc = euler ? llg_enqueue_euler_pair(p, c, M, p.cap_stream) : llg_enqueue_step(p, c, q.integrator, M, p.cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(p.cap_stream, &g);
        if (rc != MM_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return rc != MM_OK ? rc : fail(MM_EHIP, std::string("capture: ") + hipGetErrorString(e));
        }
        hipGraphExec_t x = nullptr;
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return fail(MM_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
        p.graph.graph = g;
        p.graph.exec = x;
        p.graph.M = M;
        p.graph.key = key;
    }
    for (int i = 0; i + unit <= n; i += unit) MMK_HIP(hipGraphLaunch(p.graph.exec, s));
    if (n % unit) return llg_enqueue_step(p, c, q.integrator, M, s);
    return MM_OK;
}

int mm_llg_step(mm_plan plan, const mm_llg_params *params, float *M, int nsteps, mm_stats *stats, void *stream)
{
    Plan *p = P(plan);
    int rc = plan_ready(p);
    if (rc != MM_OK) return rc;
    if (!M) return fail(MM_EINVAL, "NULL M");
    if ((rc = check_params(params)) != MM_OK) return rc;
    if (nsteps < 0) return fail(MM_EINVAL, "nsteps < 0");
    const bool sur = params->demag_mode == MM_SURROGATE;
    if (sur && !p->sur) return fail(MM_EINVAL, "MM_SURROGATE needs a surrogate attached with mm_sur_attach");
    if (sur && params->integrator != MM_RK4) return fail(MM_EINVAL, "surrogate stepping needs RK4");
    hipStream_t s = (hipStream_t)stream;
    const StageCoef c = stage_coef(*p, *params);
    // chunks of `every` steps; after each one (when stats are asked for) the
    // observables of the state are reduced into a device record
    const int every = (stats && params->log_every > 0 && params->log_every < nsteps) ? params->log_every
                                                                                      : (nsteps > 0 ? nsteps : 1);
    long long done = 0, fallbacks = 0;
    int rec = 0, out = 0;
    std::vector<long long> rec_steps, rec_fb;
    auto flush = [&]() -> int {
        if (rec == 0) return MM_OK;
        std::vector<double> h((size_t)16 * rec);
        MMK_HIP(hipMemcpyAsync(h.data(), p->red, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
        MMK_HIP(hipStreamSynchronize(s));
        for (int k = 0; k < rec; ++k) {
            mm_stats &o = stats[out + k];
            stats_from_record(*p, *params, &h[(size_t)16 * k], &o);
            o.steps = rec_steps[k];
            o.fallbacks = rec_fb[k];
        }
        out += rec;
        rec = 0;
        rec_steps.clear();
        rec_fb.clear();
        return MM_OK;
    };
    do {
        const int k = (int)std::min<long long>(every, nsteps - done);
        if (k > 0) {
            if (sur) {
                mm_sur_stats st{};
                rc = mm_llg_step_surrogate(plan, (mm_sur)p->sur, params, M, k, params->sur_tol, &st, stream);
                fallbacks += st.fallbacks;
            } else {
                rc = exact_steps(*p, *params, c, M, k, s);
            }
            if (rc != MM_OK) return rc;
            done += k;
        }
        if (stats) {
            if ((rc = demag_enqueue(*p, M, p->H, s)) != MM_OK) return rc;
            if ((rc = reduce_enqueue(*p, *params, M, p->H, s, rec)) != MM_OK) return rc;
            rec_steps.push_back(done);
            rec_fb.push_back(fallbacks);
            if (++rec == RED_LOG && (rc = flush()) != MM_OK) return rc;
        }
    } while (done < nsteps);
    if (stats) {
        if ((rc = flush()) != MM_OK) return rc;
        for (int k = 0; k < out; ++k)
            if (stats[k].nonfinite > 0)
                return fail(MM_ENONFINITE, std::to_string(stats[k].nonfinite) + " non-finite cells after " +
                                               std::to_string(stats[k].steps) + " steps");
    }
    return MM_OK;
}

int mm_reduce(mm_plan plan, const mm_llg_params *params, const float *M, mm_stats *out, void *stream)
{
    Plan *p = P(plan);
    int rc = plan_ready(p);
    if (rc != MM_OK) return rc;
    if (!M || !out) return fail(MM_EINVAL, "NULL M or out");
    if ((rc = check_params(params)) != MM_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = demag_enqueue(*p, M, p->H, s)) != MM_OK) return rc;
    if ((rc = reduce_enqueue(*p, *params, M, p->H, s, 0)) != MM_OK) return rc;
    double r[16];
    MMK_HIP(hipMemcpyAsync(r, p->red, sizeof(r), hipMemcpyDeviceToHost, s));
    MMK_HIP(hipStreamSynchronize(s));
    stats_from_record(*p, *params, r, out);
    out->steps = 0;
    out->fallbacks = 0;
    if (out->nonfinite > 0) return fail(MM_ENONFINITE, std::to_string(out->nonfinite) + " non-finite cells");
    return MM_OK;
}

int mm_llg_relax(mm_plan plan, const mm_llg_params *params, float *M, double torque_tol, long long max_steps,
                 int check_every, mm_stats *out, long long *steps_taken, void *stream)
{
    Plan *p = P(plan);
    int rc = plan_ready(p);
    if (rc != MM_OK) return rc;
    if (!M || !out || !steps_taken) return fail(MM_EINVAL, "NULL M, out or steps_taken");
    if (!(torque_tol > 0.0) || max_steps < 0 || check_every < 1) return fail(MM_EINVAL, "bad relax controls");
    if ((rc = check_params(params)) != MM_OK) return rc;
    long long done = 0;
    *steps_taken = 0;
    // each check takes the observables of the state the chunk ended on
    if ((rc = mm_reduce(plan, params, M, out, stream)) != MM_OK) return rc;
    while (out->torque_max > torque_tol && done < max_steps) {
        const int k = (int)std::min<long long>(check_every, max_steps - done);
        mm_llg_params q = *params;
        q.log_every = 0;
        if ((rc = mm_llg_step(plan, &q, M, k, out, stream)) != MM_OK) return rc;
        done += k;
        *steps_taken = done;
    }
    out->steps = done;
    return MM_OK;
}

int mm_newell_tensor(int nx, int ny, int nz, double dx, double dy, double dz, double *N, void *stream)
{
    if (!N) return fail(MM_EINVAL, "N is NULL");
    if (nx < 1 || ny < 1 || nz < 1 || (long long)nx * ny * nz > (1LL << 31))
        return fail(MM_EINVAL, "bad grid");
    if (!(dx > 0.0) || !(dy > 0.0) || !(dz > 0.0)) return fail(MM_EINVAL, "cell sizes must be > 0");
    int rc = have_device();
    if (rc != MM_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = newell_octant_device(nx, ny, nz, dx, dy, dz, N, s)) != MM_OK) return rc;
    MMK_HIP(hipStreamSynchronize(s));
    return MM_OK;
}

int mm_plan_spectrum(mm_plan plan, float *Kt, long long count, void *stream)
{
    Plan *p = P(plan);
    int rc = plan_ready(p);
    if (rc != MM_OK) return rc;
    if (!Kt) return fail(MM_EINVAL, "NULL Kt");
    if (count < p->nK) return fail(MM_EINVAL, "Kt too small");
    const size_t rec = 6 * sizeof(float);
    MMK_HIP(hipMemcpy2DAsync(Kt, rec * p->nxc, p->Kt, rec * p->xp, rec * p->nxc, (size_t)p->nzK * (p->Ly / 2 + 1),
                             hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return MM_OK;
}

int mm_plan_query(mm_plan plan, mm_plan_info *info)
{
    Plan *p = P(plan);
    if (!p || !info) return fail(MM_EINVAL, "NULL plan or info");
    info->nx = p->nx; info->ny = p->ny; info->nz = p->nz;
    info->Lx = p->Lx; info->Ly = p->Ly; info->Lz = p->Lz;
    info->spectrum_count = p->nK;
    info->workspace_bytes = (long long)p->bytes;
    for (int k = 0; k < MM_PASS_COUNT; ++k) info->cfg[k] = p->tile[k];
    info->tune_source = p->tune_source;
    return MM_OK;
}

int mm_plan_set_tile(mm_plan plan, int pass, int tile)
{
    Plan *p = P(plan);
    if (!p) return fail(MM_EINVAL, "NULL plan");
    if (!pass_tile_valid(*p, pass, tile)) return fail(MM_EINVAL, "tile not launchable for this pass");
    p->tile[pass] = tile;
    p->tune_source = 0;
    return MM_OK;
}

int mm_plan_set_timing(mm_plan plan, int enable)
{
    Plan *p = P(plan);
    if (!p) return fail(MM_EINVAL, "NULL plan");
    p->timing = enable != 0;
    return MM_OK;
}

int mm_plan_timing(mm_plan plan, double *total_ms, long long *launches)
{
    Plan *p = P(plan);
    if (!p || !total_ms || !launches) return fail(MM_EINVAL, "NULL argument");
    int rc = drain_timing(*p);
    if (rc != MM_OK) return rc;
    for (int k = 0; k < MM_PASS_COUNT; ++k) {
        total_ms[k] = p->acc[k].ms;
        launches[k] = p->acc[k].n;
        p->acc[k] = TimingAcc{};
    }
    return MM_OK;
}

int mm_plan_autotune(mm_plan plan, int reps, void *stream)
{
    Plan *p = P(plan);
    if (plan_ready(p) != MM_OK) return MM_EINVAL;
    if (reps < 1) reps = 1;
    const char *cache = std::getenv("MM_TUNE_CACHE");
    if (cache && *cache && tune_cache_read(*p, cache)) {
        p->tune_source = 2;
        drop_plan_graph(*p);
        return MM_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    // Each candidate is timed as the duration of `reps` complete demag
    // evaluations (two events around the loop, none between the launches),
    // so it is judged in the cache state and launch overlap of a real step;
    // the passes are swept twice (coordinate descent).
    // inputs: a finite state in Sa (content does not change the timing)
    MMK_HIP(hipMemsetAsync(p->Sa, 0, sizeof(float) * 3 * (size_t)p->cells(), s));
    const bool was = p->timing;
    p->timing = false;
    hipEvent_t e0, e1;
    MMK_HIP(hipEventCreate(&e0));
    MMK_HIP(hipEventCreate(&e1));
    int rc = MM_OK;
    int tuned = 0;
    // time of `reps` runs of `run` (two events around the loop)
    auto time_it = [&](auto &&run, float &ms) -> int {
        if (hipEventRecord(e0, s) != hipSuccess) return fail(MM_EHIP, "event");
        for (int r = 0; r < reps; ++r) {
            const int rc2 = run();
            if (rc2 != MM_OK) return rc2;
        }
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
            return fail(MM_EHIP, "event");
        (void)hipEventElapsedTime(&ms, e0, e1);
        return MM_OK;
    };
    // Candidates are timed in three interleaved rounds and each keeps its
    // best round (one run is noisy to a few per cent, and clocks drift over
    // a tuning run: timing each candidate's repeats back to back would
    // favour whichever runs last).
    constexpr int ROUNDS = 3;
    // MM_TUNE_LOG set: every candidate's best time to stderr
    const bool tune_log = std::getenv("MM_TUNE_LOG") != nullptr;
    for (int sweep = 0; sweep < 2 && rc == MM_OK; ++sweep) {
        for (int pass = 0; pass <= MM_PASS_YCONV && rc == MM_OK; ++pass) {
            std::vector<int> cand = pass_tile_candidates(*p, pass);
            if (cand.size() < (sweep == 0 ? 1u : 2u)) continue;
            std::vector<float> best(cand.size(), 1e30f);
            auto run = [&]() { return demag_enqueue(*p, p->Sa, p->H, s); };
            for (size_t i = 0; i < cand.size() && rc == MM_OK; ++i) {  // warm-up
                p->tile[pass] = cand[i];
                rc = run();
            }
            for (int round = 0; round < ROUNDS && rc == MM_OK; ++round)
                for (size_t i = 0; i < cand.size() && rc == MM_OK; ++i) {
                    p->tile[pass] = cand[i];
                    float ms = 0.f;
                    if ((rc = time_it(run, ms)) == MM_OK) best[i] = std::min(best[i], ms);
                }
            if (rc != MM_OK) break;
            size_t bi = 0;
            for (size_t i = 0; i < cand.size(); ++i) {
                if (best[i] < best[bi]) bi = i;
                if (tune_log) std::fprintf(stderr, "mm tune: pass %d tile %d: %.4f ms / %d runs\n", pass, cand[i], best[i], reps);
            }
            p->tile[pass] = cand[bi];
            tuned += (int)cand.size();
        }
    }
    // the fused pass's tiles and the unfused path (tile 0): each candidate
    // timed as `reps` replays of a captured one-step RK4 graph (the way
    // mm_llg_step runs steps; the fused path has fewer launches, and only a
    // replayed graph shows what that saves) on a zero state held in H
    // (which the fused step never touches; the unfused one also writes its
    // field there, which changes the values but not the work)
    if (rc == MM_OK) {
        std::vector<int> cand = xstage_candidates(*p);
        cand.push_back(0);
        mm_llg_params q{};
        q.Ms = 1.0;
        q.alpha = 0.1;
        q.gamma0 = 2.211e5;
        q.dt = 1e-14;
        q.axis[0] = 1.0;
        q.integrator = MM_RK4;
        q.renorm = 1;
        const StageCoef c = stage_coef(*p, q);
        MMK_HIP(hipMemsetAsync(p->H, 0, sizeof(float) * 3 * (size_t)p->cells(), s));
        MMK_HIP(hipStreamSynchronize(s));
        std::vector<hipGraph_t> gs(cand.size(), nullptr);
        std::vector<hipGraphExec_t> xs(cand.size(), nullptr);
        std::vector<float> best(cand.size(), 1e30f);
        const int keep = p->tile[MM_PASS_XSTAGE];
        for (size_t i = 0; i < cand.size() && cand.size() > 1 && rc == MM_OK; ++i) {
            p->tile[MM_PASS_XSTAGE] = cand[i];
            if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                rc = fail(MM_EHIP, "tune capture");
                break;
            }
            rc = llg_enqueue_step(*p, c, MM_RK4, p->H, p->cap_stream);
            hipError_t e = hipStreamEndCapture(p->cap_stream, &gs[i]);
            if (rc == MM_OK && e == hipSuccess) e = hipGraphInstantiate(&xs[i], gs[i], nullptr, nullptr, 0);
            if (rc == MM_OK && e != hipSuccess) rc = fail(MM_EHIP, std::string("tune graph: ") + hipGetErrorString(e));
            if (rc == MM_OK && hipGraphLaunch(xs[i], s) != hipSuccess) rc = fail(MM_EHIP, "tune graph launch");  // warm-up
        }
        for (int round = 0; round < ROUNDS && cand.size() > 1 && rc == MM_OK; ++round)
            for (size_t i = 0; i < cand.size() && rc == MM_OK; ++i) {
                float ms = 0.f;
                auto run = [&]() {
                    return hipGraphLaunch(xs[i], s) == hipSuccess ? MM_OK : fail(MM_EHIP, "tune graph launch");
                };
                if ((rc = time_it(run, ms)) == MM_OK) best[i] = std::min(best[i], ms);
            }
        (void)hipStreamSynchronize(s);  // no replay in flight when its graph goes
        for (size_t i = 0; i < cand.size(); ++i) {
            if (xs[i]) (void)hipGraphExecDestroy(xs[i]);
            if (gs[i]) (void)hipGraphDestroy(gs[i]);
        }
        p->tile[MM_PASS_XSTAGE] = keep;
        if (rc == MM_OK && cand.size() > 1) {
            size_t bi = 0;
            for (size_t i = 0; i < cand.size(); ++i) {
                if (best[i] < best[bi]) bi = i;
                if (tune_log)
                    std::fprintf(stderr, "mm tune: stage pass tile %d: %.4f ms / %d RK4 steps\n", cand[i], best[i], reps);
            }
            p->tile[MM_PASS_XSTAGE] = cand[bi];
            tuned += (int)cand.size();
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->timing = was;
    drop_plan_graph(*p);
    if (rc != MM_OK) return rc;
    if (tuned == 0) return fail(MM_ETUNE, "no candidate ran");
    p->tune_source = 1;
    if (cache && *cache) tune_cache_write(*p, cache);
    return MM_OK;
}

}  // extern "C"
