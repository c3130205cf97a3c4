// demag.hip -- per-plan launches of the demag passes (bodies in
// demag_kernels.hpp), their launch configurations ("tiles") and dispatch.
#include <cstring>

#include "demag_kernels.hpp"
#include "mm_internal.hpp"

namespace mmk {

// Coordinates of this workgroup in a column pass over `nrows` planes (ky
// rows in the z pass).  The grid holds ntm * nrows tiles and, first, any
// edge workgroups (the last kx column at P rows each, column_of; their
// strided accesses take longest, so they are dispatched first, one to each
// XCD in turn): for those the return value is nrows (the body's nedge),
// else 0.  Tiles go through the XCD mapping, logical order kx tile fastest,
// so neighbouring tiles of one row share their L2; in the z pass the two ky
// rows of a mirror pair (one K~ octant row) come first, then the tile.
__device__ __forceinline__ int column_coords(int ntm, int nrows, int &bx, int &plane)
{
    const unsigned nmain = (unsigned)ntm * (unsigned)nrows, ne = gridDim.x - nmain;
    if (blockIdx.x < ne) {
        bx = 0;
        plane = (int)blockIdx.x;
        return nrows;
    }
    const unsigned l = xcd_block(blockIdx.x - ne, nmain);
    bx = (int)(l % (unsigned)ntm);
    plane = (int)(l / (unsigned)ntm);
    return 0;
}
__device__ __forceinline__ int conv_coords(int ntm, int hy, int &bx, int &ky)
{
    const unsigned nmain = (unsigned)ntm * 2u * (unsigned)hy, ne = gridDim.x - nmain;
    if (blockIdx.x < ne) {
        bx = 0;
        ky = (int)blockIdx.x;
        return 2 * hy;
    }
    const unsigned l = xcd_block(blockIdx.x - ne, nmain);
    const unsigned r = l >> 1;
    bx = (int)(r % (unsigned)ntm);
    ky = ky_of_slot((int)(2 * (r / (unsigned)ntm) + (l & 1)), hy);
    return 0;
}

// Per-plan kernels: one launch covers one pass of one grid.
template <int L, int V>
__global__ __launch_bounds__(1024) void k_xfwd(const float *__restrict__ M, float2 *__restrict__ X1, int ncr,
                                               int nx, int lp2, const float2 *__restrict__ tw)
{
    xfwd_body<L, V>(M, X1, ncr, nx, lp2, tw, blockIdx.x);
}
template <int L, int V>
__global__ __launch_bounds__(1024) void k_yfwd(const float2 *__restrict__ X1, float2 *__restrict__ X2, int nxc,
                                               int ny, int lp2, const float2 *__restrict__ tw, int ntm, int nrows)
{
    int bx, plane;
    const int ne = column_coords(ntm, nrows, bx, plane);
    yfwd_body<L, V>(X1, X2, nxc, ny, lp2, tw, bx, plane, ne);
}
template <int L, bool ZAXIS, int O>
__global__ __launch_bounds__((conv_max_threads<L, O>())) void k_conv_reg3(float2 *__restrict__ X,
                                                                         const float *__restrict__ Kt, int nxc,
                                                                         int hy, int nlive, int lp2,
                                                                         const float2 *__restrict__ tw, int ntm)
{
    int bx, ky = 0, ne = 0;
    if constexpr (ZAXIS) ne = conv_coords(ntm, hy, bx, ky);
    else bx = (int)xcd_block(blockIdx.x, gridDim.x);
    conv_reg3_body<L, ZAXIS, O>(X, Kt, nxc, hy, nlive, lp2, tw, bx, ky, ne);
}
template <int L, int V, bool ZAXIS>
__global__ __launch_bounds__(1024) void k_conv_split(float2 *__restrict__ X, const float *__restrict__ Kt, int nxc,
                                                      int hy, int nlive, int lp2, const float2 *__restrict__ tw,
                                                      int ntm)
{
    int bx, ky = 0;
    if constexpr (ZAXIS) (void)conv_coords(ntm, hy, bx, ky);  // launched without edge workgroups
    else bx = (int)xcd_block(blockIdx.x, gridDim.x);
    conv_split_body<L, V, ZAXIS>(X, Kt, nxc, hy, nlive, lp2, tw, bx, ky);
}
template <int L, int V>
__global__ __launch_bounds__(1024) void k_yinv(const float2 *__restrict__ X2, float2 *__restrict__ X1, int nxc,
                                               int ny, int lp2, const float2 *__restrict__ tw, int ntm, int nrows)
{
    int bx, plane;
    const int ne = column_coords(ntm, nrows, bx, plane);
    yinv_body<L, V>(X2, X1, nxc, ny, lp2, tw, bx, plane, ne);
}
template <int L, int V>
__global__ __launch_bounds__(1024) void k_xinv(const float2 *__restrict__ X1, float *__restrict__ H, int ncr,
                                               int nx, int lp2, const float2 *__restrict__ tw)
{
    xinv_body<L, V>(X1, H, ncr, nx, lp2, tw, blockIdx.x);
}

// --------------------------------------------------------------- dispatch ---
// A launch configuration ("tile") is P + 256 * variant: P transforms (rows
// for x, kx columns for y/z) per workgroup, a power of two, and a schedule
// variant: for the single-component passes 0 = default values per thread E,
// 1 = 2E, 2 = radix order 1, 3 = radix order 2; for the product passes 0 =
// reg3, 1 = split (E), 2 = split (2E), 3 = reg3 in radix order 1, 4 = reg3 in
// radix order 2 (fft_engine.hpp).

static int ilog2(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

struct KInfo {
    int E0;      // default values per thread
    int E1;      // variant-1 values per thread (== E0 when 2E0 > L)
    int nstage;
    int conv_max;  // launch bound of the reg3 product kernel
    int Eo[3];     // values per thread of radix orders 0, 1, 2 (0: no such order)
    int maxo[3];   // launch bound of the reg3 kernel in each order
    int No[3];     // stages of each order (exchange buffers only when > 1)
};

template <int L, int O> static constexpr int order_e() { if constexpr (Factors<L, O>::valid) return Factors<L, O>::E; else return 0; }
template <int L, int O> static constexpr int order_max() { if constexpr (Factors<L, O>::valid) return conv_max_threads<L, O>(); else return 0; }
template <int L, int O> static constexpr int order_n() { if constexpr (Factors<L, O>::valid) return Factors<L, O>::N; else return 0; }

template <int L> static KInfo kinfo()
{
    return {Factors<L>::E, ept<L, 1>(), Factors<L>::N, conv_max_threads<L>(),
            {order_e<L, 0>(), order_e<L, 1>(), order_e<L, 2>()},
            {order_max<L, 0>(), order_max<L, 1>(), order_max<L, 2>()},
            {order_n<L, 0>(), order_n<L, 1>(), order_n<L, 2>()}};
}

#define MMK_ALL_LENGTHS(X)                                                                               \
    X(2) X(4) X(6) X(8) X(10) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(64) X(80) X(96) X(128) \
        X(160) X(192) X(256) X(320) X(384) X(512) X(640) X(768) X(1024)

bool kinfo_for(int L, KInfo &out)
{
    switch (L) {
#define MMK_CASE(LEN) case LEN: out = kinfo<LEN>(); return true;
        MMK_ALL_LENGTHS(MMK_CASE)
#undef MMK_CASE
    default: return false;
    }
}

bool length_supported(int L)
{
    KInfo k;
    return kinfo_for(L, k);
}

// Padded transform length of an axis of n cells: the smallest supported
// length >= 2n (the zero-padded convolution needs at least 2n - 1); 0 if
// none (n > 512).
int padded_length(int n)
{
    static const int lens[] = {2,  4,   6,   8,   10,  12,  16,  20,  24,  32,  40,  48,  64,
                               80, 96,  128, 160, 192, 256, 320, 384, 512, 640, 768, 1024};
    for (int L : lens)
        if (L >= 2 * n) return L;
    return 0;
}

static int pass_length(const Plan &p, int pass)
{
    switch (pass) {
    case MM_PASS_XFWD:
    case MM_PASS_XINV: return p.Lx;
    case MM_PASS_YFWD:
    case MM_PASS_YINV:
    case MM_PASS_YCONV: return p.Ly;
    case MM_PASS_ZCONV: return p.Lz;
    default: return 0;
    }
}

static bool pass_active(const Plan &p, int pass)
{
    if (pass == MM_PASS_YFWD || pass == MM_PASS_ZCONV || pass == MM_PASS_YINV) return p.nz > 1;
    if (pass == MM_PASS_YCONV) return p.nz == 1;
    return pass == MM_PASS_XFWD || pass == MM_PASS_XINV;
}

bool is_conv(int pass) { return pass == MM_PASS_ZCONV || pass == MM_PASS_YCONV; }
bool is_rows(int pass) { return pass == MM_PASS_XFWD || pass == MM_PASS_XINV; }

// threads, LDS bytes and thread limit of a launch of `pass` on length L
// with `tile`
bool shape_for(int pass, int L, int tile, int &threads, size_t &lds, int &maxt)
{
    KInfo k{};
    if (!kinfo_for(L, k)) return false;
    const int P = tile & 255, var = tile >> 8;
    // twiddles are copied to LDS whenever the default order has several
    // stages (tw_slots); exchange buffers when the schedule's own order has
    const size_t tws = k.nstage > 1 ? (size_t)L : 0;
    maxt = 1024;
    if (is_conv(pass)) {
        if (var == 0 || var == 3 || var == 4) {
            const int o = var == 0 ? 0 : var - 2;
            if (!k.Eo[o]) return false;
            threads = P * (L / k.Eo[o]);
            maxt = k.maxo[o];
            // two exchange buffers (ping-pong transforms)
            lds = (tws + (k.No[o] > 1 ? 2 * (size_t)lds_rows(L) * P : 0)) * sizeof(float2);
        } else if (var == 1 || var == 2) {
            const int E = var == 1 ? k.E0 : k.E1;
            if (var == 2 && k.E1 == k.E0) return false;
            threads = 3 * P * (L / E);
            lds = (tws + 3 * (size_t)lds_rows(L) * P) * sizeof(float2);
        } else {
            return false;
        }
    } else {
        if (var < 0 || var > 3) return false;
        if (var == 1 && k.E1 == k.E0) return false;
        if (var >= 2 && !k.Eo[var - 1]) return false;
        const int E = var == 0 ? k.E0 : (var == 1 ? k.E1 : k.Eo[var - 1]);
        threads = P * (L / E);
        // the x forward separates its packed rows through LDS even for one stage
        const bool needs = (var >= 2 ? k.No[var - 1] : k.nstage) > 1 || pass == MM_PASS_XFWD;
        lds = (tws + (needs ? (is_rows(pass) ? (size_t)P * (lds_rows(L) + 1) : (size_t)lds_rows(L) * P) : 0)) *
              sizeof(float2);
    }
    return true;
}

bool tile_valid_for(int pass, int L, int tile, size_t lds_limit)
{
    if (pass < 0 || pass > MM_PASS_YCONV) return false;
    const int P = tile & 255;
    if (tile < 1 || P < 1 || (P & (P - 1)) != 0 || P > 128) return false;
    int threads, maxt;
    size_t lds;
    if (!shape_for(pass, L, tile, threads, lds, maxt)) return false;
    return threads >= 1 && threads <= maxt && lds <= lds_limit;
}

std::vector<int> tile_candidates_for(int pass, int L, size_t lds_limit)
{
    std::vector<int> out;
    for (int var = 0; var < (is_conv(pass) ? 5 : 4); ++var)
        for (int P = 1; P <= 128; P *= 2) {
            const int tile = P + 256 * var;
            if (!tile_valid_for(pass, L, tile, lds_limit)) continue;
            int threads, maxt;
            size_t lds;
            shape_for(pass, L, tile, threads, lds, maxt);
            if (threads < 64 && tile_valid_for(pass, L, 2 * P + 256 * var, lds_limit)) continue;  // underfilled wave
            out.push_back(tile);
        }
    return out;
}

// rows: the largest P with <= 256 threads; columns: the largest P <= 16 whose
// LDS fits in 64 KiB (the product passes in the three-component register
// schedule, which the autotuner picks at every measured size)
int default_tile_for(int pass, int L, size_t lds_limit)
{
    KInfo k{};
    if (!kinfo_for(L, k)) return 0;
    const int var = 0;  // product passes: three components in registers (faster than the split)
    int best = 0;
    for (int P = 1; P <= 128; P *= 2) {
        const int tile = P + 256 * var;
        if (!tile_valid_for(pass, L, tile, lds_limit)) continue;
        int threads, maxt;
        size_t lds;
        shape_for(pass, L, tile, threads, lds, maxt);
        if (is_rows(pass)) {
            if (best == 0 || threads <= 256) best = tile;
        } else if (best == 0 || (P <= 16 && lds <= 65536)) {
            best = tile;
        }
    }
    return best;
}

// The stage kernel's "tile" is its vector width W: W consecutive cells of
// an x row per thread (1, 2 or 4; nx % W == 0).
bool pass_tile_valid(const Plan &p, int pass, int tile)
{
    if (pass == MM_PASS_STAGE) return (tile == 1 || tile == 2 || tile == 4) && p.nx % tile == 0;
    if (pass == MM_PASS_XSTAGE) return xstage_tile_valid(p, tile);
    return pass_active(p, pass) && tile_valid_for(pass, pass_length(p, pass), tile, p.lds_limit);
}

std::vector<int> pass_tile_candidates(const Plan &p, int pass)
{
    if (pass == MM_PASS_XSTAGE) return xstage_candidates(p);
    if (!pass_active(p, pass)) return {};
    return tile_candidates_for(pass, pass_length(p, pass), p.lds_limit);
}

int pass_default_tile(const Plan &p, int pass)
{
    if (pass == MM_PASS_STAGE) return p.nx % 4 == 0 ? 4 : (p.nx % 2 == 0 ? 2 : 1);
    if (pass == MM_PASS_XSTAGE) return xstage_default_tile(p);
    if (!pass_active(p, pass)) return 0;
    return default_tile_for(pass, pass_length(p, pass), p.lds_limit);
}

template <typename K>
static hipError_t raise_one(K kern, int lim)
{
    return hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
}

template <int L>
static hipError_t raise_lds(size_t limit)
{
    const int lim = (int)limit;
    const hipError_t es[] = {
        raise_one(k_xfwd<L, 0>, lim),        raise_one(k_xfwd<L, 1>, lim),
        raise_one(k_yfwd<L, 0>, lim),        raise_one(k_yfwd<L, 1>, lim),
        raise_one(k_yinv<L, 0>, lim),        raise_one(k_yinv<L, 1>, lim),
        raise_one(k_xinv<L, 0>, lim),        raise_one(k_xinv<L, 1>, lim),
        raise_one(k_conv_reg3<L, true, 0>, lim), raise_one(k_conv_reg3<L, false, 0>, lim),
        raise_one(k_conv_split<L, 0, true>, lim), raise_one(k_conv_split<L, 1, true>, lim),
        raise_one(k_conv_split<L, 0, false>, lim), raise_one(k_conv_split<L, 1, false>, lim)};
    for (hipError_t e : es)
        if (e != hipSuccess) return e;
    return hipSuccess;
}

int prepare_kernels(Plan &p)
{
    if (p.lds_limit <= 65536) return MM_OK;
    const int Ls[3] = {p.Lx, p.Ly, p.Lz};
    for (int a = 0; a < 3; ++a) {
        hipError_t e = hipSuccess;
        switch (Ls[a]) {
#define MMK_CASE(LEN) case LEN: e = raise_lds<LEN>(p.lds_limit); break;
            MMK_ALL_LENGTHS(MMK_CASE)
#undef MMK_CASE
        default: break;
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p.lds_limit = 65536;  // keep to the portable limit
            return MM_OK;
        }
    }
    return MM_OK;
}

template <typename K>
static void raise_for(K kern, size_t lds)
{
    if (lds > 65536) (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// Tiles of a column pass over nrows planes (ky rows): when P (> 1) divides
// the Lx/2 columns below the last, ntm = Lx/2 / P tiles and ne edge
// workgroups for the last column (P rows each); else ntm tiles over every
// column and none.
static void column_grid(const Plan &p, int P, int nrows, int &ntm, int &ne)
{
    const int half = p.Lx / 2;
    if (P > 1 && half % P == 0) {
        ntm = half / P;
        ne = (nrows + P - 1) / P;
    } else {
        ntm = (p.nxc + P - 1) / P;
        ne = 0;
    }
}

template <int L, int V>
static void launch_single(Plan &p, int pass, int P, size_t lds, const float *M, float *H, hipStream_t s)
{
    if constexpr (V >= 2) {
        switch (pass) {
        case MM_PASS_XFWD: raise_for(k_xfwd<L, V>, lds); break;
        case MM_PASS_YFWD: raise_for(k_yfwd<L, V>, lds); break;
        case MM_PASS_YINV: raise_for(k_yinv<L, V>, lds); break;
        case MM_PASS_XINV: raise_for(k_xinv<L, V>, lds); break;
        default: break;
        }
    }
    constexpr int Q = L / ept<L, V>();
    const int lp2 = ilog2(P);
    const dim3 block(P * Q);
    const int nxc = p.nxc;
    const int ncr = p.nz * p.ny;
    const int pairs = 3 * ((ncr + 1) / 2);
    switch (pass) {
    case MM_PASS_XFWD: {
        MMK_LAUNCH(p, (k_xfwd<L, V>), dim3((pairs + P - 1) / P), block, lds, s, M, p.X1, ncr, p.nx, lp2, p.tw[0]);
        break;
    }
    case MM_PASS_YFWD:
    case MM_PASS_YINV: {
        const int nrows = 3 * p.nz;
        int ntm, ne;
        column_grid(p, P, nrows, ntm, ne);
        const dim3 grid((unsigned)(ntm * nrows + ne));
        if (pass == MM_PASS_YFWD)
            MMK_LAUNCH(p, (k_yfwd<L, V>), grid, block, lds, s, p.X1, p.X2, nxc, p.ny, lp2, p.tw[1], ntm, nrows);
        else
            MMK_LAUNCH(p, (k_yinv<L, V>), grid, block, lds, s, p.X2, p.X1, nxc, p.ny, lp2, p.tw[1], ntm, nrows);
        break;
    }
    case MM_PASS_XINV: {
        MMK_LAUNCH(p, (k_xinv<L, V>), dim3((pairs + P - 1) / P), block, lds, s, p.X1, H, ncr, p.nx, lp2, p.tw[0]);
        break;
    }
    default: break;
    }
}

template <int L>
static void launch_conv(Plan &p, int pass, int P, int var, size_t lds, hipStream_t s)
{
    const int lp2 = ilog2(P);
    const int nxc = p.nxc;
    const bool z = pass == MM_PASS_ZCONV;
    float2 *X = z ? p.X2 : p.X1;
    const float2 *tw = z ? p.tw[2] : p.tw[1];
    const int hy = p.Ly / 2, nl = z ? p.nz : p.ny;
    // reg3 z passes take edge workgroups (column_grid); the split schedule
    // and the y product tile every column
    const bool reg3z = z && (var == 0 || var == 3 || var == 4);
    int ntm = (nxc + P - 1) / P, ne = 0;
    if (reg3z) column_grid(p, P, p.Ly, ntm, ne);
    const dim3 grid((unsigned)(z ? ntm * p.Ly + ne : ntm));
    if (var == 0) {
        const dim3 block(P * (L / Factors<L>::E));
        if (z) MMK_LAUNCH(p, (k_conv_reg3<L, true, 0>), grid, block, lds, s, X, p.Kt, nxc, hy, nl, lp2, tw, ntm);
        else MMK_LAUNCH(p, (k_conv_reg3<L, false, 0>), grid, block, lds, s, X, p.Kt, nxc, hy, nl, lp2, tw, ntm);
    } else if (var == 3 || var == 4) {
        if constexpr (Factors<L, 1>::valid || Factors<L, 2>::valid) {
            auto go = [&](auto kern, int E) {
                if (lds > 65536)
                    (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                MMK_LAUNCH(p, kern, grid, dim3(P * (L / E)), lds, s, X, p.Kt, nxc, hy, nl, lp2, tw, ntm);
            };
            if constexpr (Factors<L, 1>::valid) {
                if (var == 3) {
                    if (z) go(k_conv_reg3<L, true, 1>, Factors<L, 1>::E);
                    else go(k_conv_reg3<L, false, 1>, Factors<L, 1>::E);
                }
            }
            if constexpr (Factors<L, 2>::valid) {
                if (var == 4) {
                    if (z) go(k_conv_reg3<L, true, 2>, Factors<L, 2>::E);
                    else go(k_conv_reg3<L, false, 2>, Factors<L, 2>::E);
                }
            }
        }
    } else if (var == 1) {
        const dim3 block(3 * P * (L / ept<L, 0>()));
        if (z) MMK_LAUNCH(p, (k_conv_split<L, 0, true>), grid, block, lds, s, X, p.Kt, nxc, hy, nl, lp2, tw, ntm);
        else MMK_LAUNCH(p, (k_conv_split<L, 0, false>), grid, block, lds, s, X, p.Kt, nxc, hy, nl, lp2, tw, ntm);
    } else {
        const dim3 block(3 * P * (L / ept<L, 1>()));
        if (z) MMK_LAUNCH(p, (k_conv_split<L, 1, true>), grid, block, lds, s, X, p.Kt, nxc, hy, nl, lp2, tw, ntm);
        else MMK_LAUNCH(p, (k_conv_split<L, 1, false>), grid, block, lds, s, X, p.Kt, nxc, hy, nl, lp2, tw, ntm);
    }
}

template <int L>
static void launch_len(Plan &p, int pass, int tile, size_t lds, const float *M, float *H, hipStream_t s)
{
    const int P = tile & 255, var = tile >> 8;
    if (is_conv(pass)) launch_conv<L>(p, pass, P, var, lds, s);
    else if (var == 0) launch_single<L, 0>(p, pass, P, lds, M, H, s);
    else if (var == 1) launch_single<L, 1>(p, pass, P, lds, M, H, s);
    else if (var == 2) { if constexpr (variant_valid<L, 2>()) launch_single<L, 2>(p, pass, P, lds, M, H, s); }
    else if (var == 3) { if constexpr (variant_valid<L, 3>()) launch_single<L, 3>(p, pass, P, lds, M, H, s); }
}

int launch_pass(Plan &p, int pass, const float *M, float *H, hipStream_t s)
{
    const int L = pass_length(p, pass);
    const int tile = p.tile[pass];
    if (!pass_tile_valid(p, pass, tile)) return fail(MM_EINVAL, "invalid tile for pass");
    int threads, maxt;
    size_t lds;
    shape_for(pass, L, tile, threads, lds, maxt);
    timing_arm(p);
    switch (L) {
#define MMK_CASE(LEN) case LEN: launch_len<LEN>(p, pass, tile, lds, M, H, s); break;
        MMK_ALL_LENGTHS(MMK_CASE)
#undef MMK_CASE
    default: timing_file(p, pass); return fail(MM_EINVAL, "unsupported FFT length");
    }
    timing_file(p, pass);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MM_EHIP, std::string("demag launch: ") + hipGetErrorString(e));
    return MM_OK;
}

int demag_mid_enqueue(Plan &p, hipStream_t s)
{
    int rc;
    if (p.nz > 1) {
        if ((rc = launch_pass(p, MM_PASS_YFWD, nullptr, nullptr, s)) != MM_OK) return rc;
        if ((rc = launch_pass(p, MM_PASS_ZCONV, nullptr, nullptr, s)) != MM_OK) return rc;
        return launch_pass(p, MM_PASS_YINV, nullptr, nullptr, s);
    }
    return launch_pass(p, MM_PASS_YCONV, nullptr, nullptr, s);
}

int demag_enqueue(Plan &p, const float *M, float *H, hipStream_t s)
{
    int rc;
    if ((rc = launch_pass(p, MM_PASS_XFWD, M, H, s)) != MM_OK) return rc;
    if ((rc = demag_mid_enqueue(p, s)) != MM_OK) return rc;
    return launch_pass(p, MM_PASS_XINV, M, H, s);
}

}  // namespace mmk
