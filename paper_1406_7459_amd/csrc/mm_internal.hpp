// mm_internal.hpp -- host-side plan state and helpers shared by the library's
// translation units (not part of the public ABI; see include/mm.h).
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "../../include/mm.h"
#include "layout.hpp"

namespace mmk {

// Observables records kept on the device per mm_llg_step call before the host
// reads them back.
constexpr int RED_LOG = 256;

// thread-local last-error detail
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
#define MMK_HIP(call)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::mmk::fail(MM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// FP32 coefficients of one LLG stage, precomputed on the host in FP64.
struct StageCoef {
    float cx, cy, cz;       // 2A/(mu0 Ms^2 d^2) per axis (0 for an axis of length 1)
    float ka;               // 2Ku/(mu0 Ms^2)
    float ux, uy, uz;       // easy axis
    float hx, hy, hz;       // applied field
    float g;                // gamma0/(1+alpha^2)
    float gd;               // alpha g / Ms
    float dt;
    float Ms;
    int renorm;
};

// FP64 coefficients of the observables reduction.
struct ReduceCoef {
    double cx, cy, cz, ka, ux, uy, uz, hx, hy, hz;
    double Ms, A, Ku, dx, dy, dz;
};

struct TimingAcc {
    double ms = 0.0;
    long long n = 0;
};

typedef std::pair<int, std::pair<hipEvent_t, hipEvent_t>> TimedPair;

struct GraphCache {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    const float *M = nullptr;
    std::string key;
};

struct Plan {
    int nx = 0, ny = 0, nz = 0;
    double dx = 0, dy = 0, dz = 0;
    int Lx = 0, Ly = 0, Lz = 0;  // padded lengths (>= 2n); Lz = 1 when nz == 1 (z collapsed)
    int nxc = 0;                 // Lx/2 + 1 half-spectrum columns
    int xp = 0;                  // x_pitch(nxc): row pitch of X1, X2 and K~
    int nzK = 0;                 // octant depth of K~: Lz/2 + 1, or 1 when nz == 1
    int device = 0;
    size_t lds_limit = 65536;

    float *Kt = nullptr;         // [nzK][Ly/2+1][xp][6], kx < nxc used
    long long nK = 0;            // 6 nzK (Ly/2+1) nxc: the exported (unpadded) count
    float2 *X1 = nullptr;        // [3][nz][ny][xp]
    float2 *X2 = nullptr;        // [3][nz] planes of Ly rows of xp, x2_plane_stride apart (nz > 1 only)
    float *H = nullptr;          // [3][N] demag field scratch for the step driver
    float *Sa = nullptr, *Sb = nullptr, *kacc = nullptr;  // stage states and RK4 accumulator
    double *part = nullptr;      // reduction partials
    double *red = nullptr;       // final reductions, RED_LOG records of 16 doubles
    int red_blocks = 0;
    float2 *tw[3] = {nullptr, nullptr, nullptr};  // twiddles per axis length
    size_t bytes = 0;            // workspace bytes the plan needs
    char *ws = nullptr;          // the caller's bound workspace (nullptr: unbound)
    char *run = nullptr;         // run-time region of the workspace (set-up scratch before)
    std::vector<float2> tw_host[3];  // twiddle tables, uploaded at bind

    // learned demag increment attached for MM_SURROGATE stepping (mm_sur_attach)
    void *sur = nullptr;

    int tile[MM_PASS_COUNT] = {0, 0, 0, 0, 0, 0, 0, 0, 0};

    int tune_source = 0;          // 0 default / by hand, 1 timed, 2 tune cache
    std::string arch;             // device architecture and compute units (tune cache key)

    bool timing = false;
    hipEvent_t tev[2] = {nullptr, nullptr};  // armed start/stop pair for the next launch
    TimingAcc acc[MM_PASS_COUNT];
    std::vector<TimedPair> pending;       // recorded, not yet read
    std::vector<hipEvent_t> event_pool;

    GraphCache graph;
    hipStream_t cap_stream = nullptr;

    long long cells() const { return (long long)nx * ny * nz; }
};

Plan *plan_of(mm_plan h);
// MM_OK if the plan has its workspace bound, else MM_EINVAL with a detail.
int plan_ready(const Plan *p);
// Persistent tuning results (file named by MM_TUNE_CACHE).
bool tune_cache_read(Plan &p, const char *path);
void tune_cache_write(const Plan &p, const char *path);
// Carve (base != nullptr) or measure (base == nullptr) the plan workspace.
size_t plan_layout(Plan &p, char *base);
// FP64 scratch bytes of the spectrum set-up (tensor.hip).
size_t spectrum_scratch_bytes(int nx, int ny, int nz, int Lx, int Ly, int Lz);

// Launch configurations by (pass, transform length) (demag.hip).
bool shape_for(int pass, int L, int tile, int &threads, size_t &lds, int &maxt);
bool tile_valid_for(int pass, int L, int tile, size_t lds_limit);
std::vector<int> tile_candidates_for(int pass, int L, size_t lds_limit);
int default_tile_for(int pass, int L, size_t lds_limit);

// Launch helpers (demag.hip).
bool pass_tile_valid(const Plan &p, int pass, int tile);
std::vector<int> pass_tile_candidates(const Plan &p, int pass);
int pass_default_tile(const Plan &p, int pass);
int prepare_kernels(Plan &p);  // raise LDS limits where needed
int demag_enqueue(Plan &p, const float *M, float *H, hipStream_t s);
int launch_pass(Plan &p, int pass, const float *M, float *H, hipStream_t s);

// Timing hooks.  A pass of one kernel arms an event pair before its launch
// and files it after; MMK_LAUNCH hands an armed pair to the dispatch itself
// (hipExtLaunchKernelGGL), so the events time the kernel's execution and not
// the command processor's handling of separate event records.  Passes of
// several kernels bracket them with recorded events instead.
void timing_arm(Plan &p);
void timing_file(Plan &p, int pass);
void timing_begin(Plan &p, int pass, hipStream_t s, hipEvent_t *ev0);
void timing_end(Plan &p, int pass, hipStream_t s, hipEvent_t ev0);

#define MMK_LAUNCH(p, kern, grid, block, lds, s, ...)                                                         \
    do {                                                                                                      \
        if ((p).tev[0])                                                                                       \
            hipExtLaunchKernelGGL(kern, grid, block, (std::uint32_t)(lds), s, (p).tev[0], (p).tev[1], 0u,    \
                                  __VA_ARGS__);                                                               \
        else                                                                                                  \
            hipLaunchKernelGGL(kern, grid, block, lds, s, __VA_ARGS__);                                        \
    } while (0)

// Tensor set-up (tensor.hip).
int newell_octant_device(int nx, int ny, int nz, double dx, double dy, double dz, double *N,
                         hipStream_t s);
int build_spectrum(Plan &p, hipStream_t s);

// Fused x-inverse / stage / x-forward pass (xstage.hip).
bool xstage_tile_valid(const Plan &p, int tile);
std::vector<int> xstage_candidates(const Plan &p);
int xstage_default_tile(const Plan &p);
int launch_xstage(Plan &p, int stage, bool fwd, const float *S, const float *Mn, float *out, const StageCoef &c,
                  hipStream_t s);
// The passes of a demag evaluation between XFWD and XINV (YFWD, ZCONV, YINV;
// or YCONV when nz = 1) (demag.hip).
int demag_mid_enqueue(Plan &p, hipStream_t s);

// LLG (llg.hip).
StageCoef stage_coef(const Plan &p, const mm_llg_params &q);
int llg_enqueue_step(Plan &p, const StageCoef &c, int integrator, float *M, hipStream_t s);
// Two explicit Euler steps M -> Sa -> M (no copy back).
int llg_enqueue_euler_pair(Plan &p, const StageCoef &c, float *M, hipStream_t s);
int llg_step_with_fields(Plan &p, const StageCoef &c, float *M, const float *H1, hipStream_t s,
                         const std::function<int(int, const float *, float *)> &field);
int reduce_enqueue(Plan &p, const mm_llg_params &q, const float *M, const float *Hd, hipStream_t s, int slot = 0);
void stats_from_record(const Plan &p, const mm_llg_params &q, const double *r, mm_stats *out);

}  // namespace mmk
