// xstage.hip -- per-plan launches of the fused x-inverse / LLG stage /
// x-forward pass (xstage_body.hpp): launch configurations and dispatch.
#include "mm_internal.hpp"
#include "xstage_body.hpp"

namespace mmk {

template <int L, int STAGE, bool FWD, int W>
__global__ __launch_bounds__(1024) void k_xstage(float2 *__restrict__ X1, const float *S, const float *Mn,
                                                 float *__restrict__ kacc, float *out, int nx, int ny, int nz,
                                                 StageCoef c, const float2 *__restrict__ tw, int lp2)
{
    // each XCD a contiguous range of row blocks: its L2 keeps the +-y and
    // +-z neighbour rows of the stage
    const int bx = (int)xcd_block(blockIdx.x, gridDim.x);
    xstage_body<L, STAGE, FWD, W>(X1, S, Mn, kacc, out, nx, ny, nz, c, tw, lp2, bx);
}

#define MMK_XS_LENGTHS(X)                                                                                \
    X(2) X(4) X(6) X(8) X(10) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(64) X(80) X(96) X(128) \
        X(160) X(192) X(256) X(320) X(384) X(512) X(640) X(768) X(1024)

// threads and LDS of tile P (row pairs per workgroup) on x length L
static bool xs_shape(int L, int P, int &threads, size_t &lds)
{
    switch (L) {
#define MMK_CASE(LEN)                                     \
    case LEN:                                             \
        threads = 3 * P * (LEN / Factors<LEN>::E);        \
        lds = xs_lds_bytes<LEN>(P);                       \
        return true;
        MMK_XS_LENGTHS(MMK_CASE)
#undef MMK_CASE
    default: return false;
    }
}

// The fused pass's tile is P + 256 w: P = 2^k row pairs per workgroup and
// the stage phase's cells per thread task W = 1, 2, 4 for w = 0, 1, 2 (nx
// % W == 0; wider tasks take more registers); 0 selects the unfused path
// (XINV, stage kernel, XFWD).
static int xs_w(int tile) { return 1 << (tile >> 8); }

bool xstage_tile_valid(const Plan &p, int tile)
{
    if (tile == 0) return true;
    const int P = tile & 255, w = tile >> 8;
    if (tile < 0 || P < 1 || (P & (P - 1)) != 0 || P > 64 || w > 2) return false;
    if (p.nx % xs_w(tile) != 0) return false;
    int threads;
    size_t lds;
    if (!xs_shape(p.Lx, P, threads, lds)) return false;
    return threads <= 1024 && lds <= p.lds_limit;
}

std::vector<int> xstage_candidates(const Plan &p)
{
    std::vector<int> out;
    for (int w = 0; w <= 2; ++w)
        for (int P = 1; P <= 64; P *= 2) {
            const int tile = P + 256 * w;
            int threads;
            size_t lds;
            if (!xstage_tile_valid(p, tile) || !xs_shape(p.Lx, P, threads, lds)) continue;
            if (threads < 64 && xstage_tile_valid(p, 2 * P + 256 * w)) continue;  // underfilled wave
            if (P > 1 && P >= p.ny * p.nz) break;  // the half tile already held every row
            out.push_back(tile);
        }
    return out;
}

// one cell per task (the fewest registers), the largest P with at most 256
// threads (at least one pair)
int xstage_default_tile(const Plan &p)
{
    int best = 0;
    for (int P = 1; P <= 64; P *= 2) {
        int threads;
        size_t lds;
        if (!xstage_tile_valid(p, P) || !xs_shape(p.Lx, P, threads, lds)) continue;
        if (best == 0 || threads <= 256) best = P;
    }
    return best;
}

template <int L, int STAGE, bool FWD, int W>
static void xs_launch(Plan &p, int P, const float *S, const float *Mn, float *out, const StageCoef &c, hipStream_t s)
{
    int lp2 = 0;
    while ((1 << lp2) < P) ++lp2;
    const int ncr = p.ny * p.nz;
    const dim3 grid((unsigned)((ncr + 2 * P - 1) / (2 * P)));
    const dim3 block((unsigned)(3 * P * (L / Factors<L>::E)));
    const size_t lds = xs_lds_bytes<L>(P);
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void *)k_xstage<L, STAGE, FWD, W>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    MMK_LAUNCH(p, (k_xstage<L, STAGE, FWD, W>), grid, block, lds, s, p.X1, S, Mn, p.kacc, out, p.nx, p.ny, p.nz, c,
               p.tw[0], lp2);
}

template <int L, int W>
static int xs_dispatch_w(Plan &p, int P, int stage, bool fwd, const float *S, const float *Mn, float *out,
                         const StageCoef &c, hipStream_t s)
{
    if (stage == 1 && fwd) xs_launch<L, 1, true, W>(p, P, S, Mn, out, c, s);
    else if (stage == 2 && fwd) xs_launch<L, 2, true, W>(p, P, S, Mn, out, c, s);
    else if (stage == 3 && fwd) xs_launch<L, 3, true, W>(p, P, S, Mn, out, c, s);
    else if (stage == 4 && !fwd) xs_launch<L, 4, false, W>(p, P, S, Mn, out, c, s);
    else if (stage == 0 && fwd) xs_launch<L, 0, true, W>(p, P, S, Mn, out, c, s);
    else if (stage == 0 && !fwd) xs_launch<L, 0, false, W>(p, P, S, Mn, out, c, s);
    else return fail(MM_EINVAL, "fused stage: unsupported stage/forward combination");
    return MM_OK;
}

template <int L>
static int xs_dispatch(Plan &p, int tile, int stage, bool fwd, const float *S, const float *Mn, float *out,
                       const StageCoef &c, hipStream_t s)
{
    const int P = tile & 255, W = xs_w(tile);
    if (W == 4) return xs_dispatch_w<L, 4>(p, P, stage, fwd, S, Mn, out, c, s);
    if (W == 2) return xs_dispatch_w<L, 2>(p, P, stage, fwd, S, Mn, out, c, s);
    return xs_dispatch_w<L, 1>(p, P, stage, fwd, S, Mn, out, c, s);
}

// The x-inverse of the field in X1, stage `stage` (0 Euler, 1..4 RK4) from
// state S with step start Mn into `out`, and (fwd) the x-forward of `out`
// into X1.
int launch_xstage(Plan &p, int stage, bool fwd, const float *S, const float *Mn, float *out, const StageCoef &c,
                  hipStream_t s)
{
    const int P = p.tile[MM_PASS_XSTAGE];  // P + 256 w
    if (P <= 0 || !xstage_tile_valid(p, P)) return fail(MM_EINVAL, "invalid fused-stage tile");
    timing_arm(p);
    int rc = MM_OK;
    switch (p.Lx) {
#define MMK_CASE(LEN) case LEN: rc = xs_dispatch<LEN>(p, P, stage, fwd, S, Mn, out, c, s); break;
        MMK_XS_LENGTHS(MMK_CASE)
#undef MMK_CASE
    default: rc = fail(MM_EINVAL, "fused stage: unsupported x length");
    }
    timing_file(p, MM_PASS_XSTAGE);
    if (rc != MM_OK) return rc;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MM_EHIP, std::string("k_xstage: ") + hipGetErrorString(e));
    return MM_OK;
}

}  // namespace mmk
