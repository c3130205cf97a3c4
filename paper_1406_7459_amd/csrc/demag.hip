// demag.hip -- the five (3-D) or three (nz = 1) passes of one demagnetising
// field evaluation: the zero-padded convolution H = K * M of the paper,
// Sec. 2 steps (1)-(5) and eq. (13)-(16), evaluated by a real-to-complex FFT
// that never touches the zero half of the padded grid (forward) nor computes
// the discarded half (inverse).
//
//   XFWD   M [3][nz][ny][nx] f32   -> X1 [3][nz][ny][nx+1] c64   x: R2C, input i < nx
//   YFWD   X1                      -> X2 [3][nz][2ny][nx+1]      y: input j < ny
//   ZCONV  X2 -> X2 in place: z forward (input k < nz), H~ = K~ . M~
//          (eq. (13)/(15), six real K~ components with parity signs),
//          z inverse, rows k < nz written back
//   YINV   X2 -> X1                                               y: keep j < ny
//   XINV   X1 -> H [3][nz][ny][nx] f32                            x: C2R, keep i < nx
// For nz = 1 the padded z axis has length 2 with the second slot zero, so the
// z transform is the identity up to a factor folded into K~; YCONV then does
// y forward, product and y inverse in one pass (XFWD, YCONV, XINV).
//
// Every pass is one launch; a workgroup owns a tile of whole 1-D transforms
// (P consecutive kx columns for y/z, P rows -- P row pairs for XINV -- for x),
// loads them coalesced straight into registers, and exchanges through LDS
// only between FFT stages (fft_engine.hpp).
#include <cstring>

#include "fft_engine.hpp"
#include "mm_internal.hpp"

namespace mmk {

// ----------------------------------------------------------------- kernels ---

// x forward: one real row of length nx, zero-padded to L = 2nx, -> nx+1 bins.
template <int L>
__global__ __launch_bounds__(1024) void k_xfwd(const float *__restrict__ M, float2 *__restrict__ X1,
                                               int nrows, int lp2, const float2 *__restrict__ tw)
{
    constexpr int E = Factors<L>::E, Q = L / E, NX = L / 2;
    extern __shared__ float2 lds[];
    const int t = threadIdx.x;
    const int q = t % Q, p = t / Q;
    const int row = (blockIdx.x << lp2) + p;
    const bool ok = row < nrows;
    const LdsView s{lds, 1, p * (L + 1)};
    float2 v[E];
    constexpr int R0 = first_radix<L, false>();
    const float *src = M + (size_t)row * NX;
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int i = q + Q * b + r * (L / R0);
            const bool upper = r * (L / R0) >= NX;  // compile-time after unrolling
            v[b * R0 + r] = (!upper && ok && i < NX) ? make_float2(src[i], 0.f) : make_float2(0.f, 0.f);
        }
    fft<L, -1, false>(v, s, q, tw);
    constexpr int RL = last_radix<L, false>();
    float2 *dst = X1 + (size_t)row * (NX + 1);
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int k = q + Q * b + r * (L / RL);
            if (ok && k <= NX) dst[k] = v[b * RL + r];
        }
}

// y forward on a tile of P kx columns of one (component, z) plane.
template <int L>
__global__ __launch_bounds__(1024) void k_yfwd(const float2 *__restrict__ X1, float2 *__restrict__ X2,
                                               int nxc, int lp2, const float2 *__restrict__ tw)
{
    constexpr int E = Factors<L>::E, Q = L / E, NY = L / 2;
    extern __shared__ float2 lds[];
    const int P = 1 << lp2;
    const int t = threadIdx.x;
    const int p = t & (P - 1), q = t >> lp2;
    const int kx = blockIdx.x * P + p;
    const int plane = blockIdx.y;
    const bool ok = kx < nxc;
    const LdsView s{lds, P + 1, p};
    float2 v[E];
    constexpr int R0 = first_radix<L, false>();
    const float2 *src = X1 + (size_t)plane * NY * nxc + kx;
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int j = q + Q * b + r * (L / R0);
            const bool upper = r * (L / R0) >= NY;
            v[b * R0 + r] = (!upper && ok && j < NY) ? src[(size_t)j * nxc] : make_float2(0.f, 0.f);
        }
    fft<L, -1, false>(v, s, q, tw);
    constexpr int RL = last_radix<L, false>();
    float2 *dst = X2 + (size_t)plane * L * nxc + kx;
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int k = q + Q * b + r * (L / RL);
            if (ok) dst[(size_t)k * nxc] = v[b * RL + r];
        }
}

// Spectral product at one frequency: H~ = K~ . M~ with K~ real and symmetric
// (eq. (13)/(15)); sxy, sxz, syz are the parity signs of the folded octant.
__device__ __forceinline__ void kdot(float2 &a, float2 &b, float2 &c, float kxx, float kyy, float kzz,
                                     float kxy, float kxz, float kyz)
{
    const float2 mx = a, my = b, mz = c;
    a = make_float2(kxx * mx.x + kxy * my.x + kxz * mz.x, kxx * mx.y + kxy * my.y + kxz * mz.y);
    b = make_float2(kxy * mx.x + kyy * my.x + kyz * mz.x, kxy * mx.y + kyy * my.y + kyz * mz.y);
    c = make_float2(kxz * mx.x + kyz * my.x + kzz * mz.x, kxz * mx.y + kyz * my.y + kzz * mz.y);
}

// z forward -> product -> z inverse for a tile of P kx columns at one ky,
// all three components; in place on X2 (rows k < nz).
// Three components stay in VGPRs across the product: cap the workgroup so
// the allocator gets 256 (E = 8) or 512 (E = 24) registers per lane.
template <int L> constexpr int conv_max_threads() { return Factors<L>::E > 8 ? 256 : 512; }

template <int L>
__global__ __launch_bounds__(conv_max_threads<L>()) void k_zconv(float2 *__restrict__ X2, const float *__restrict__ Kt,
                                                int nxc, int ny, int lp2, const float2 *__restrict__ tw)
{
    constexpr int E = Factors<L>::E, Q = L / E, NZ = L / 2;
    extern __shared__ float2 lds[];
    const int P = 1 << lp2;
    const int t = threadIdx.x;
    const int p = t & (P - 1), q = t >> lp2;
    const int kx = blockIdx.x * P + p;
    const int ky = blockIdx.y;
    const bool ok = kx < nxc;
    const LdsView s{lds, P + 1, p};
    const size_t zs = (size_t)2 * ny * nxc;      // z stride
    const size_t cs = (size_t)NZ * zs;           // component stride
    float2 *base = X2 + (size_t)ky * nxc + kx;
    float2 va[E], vb[E], vc[E];
    constexpr int R0 = first_radix<L, false>();
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int k = q + Q * b + r * (L / R0);
            const bool upper = r * (L / R0) >= NZ;
            const bool ld = !upper && ok && k < NZ;
            const float2 z = make_float2(0.f, 0.f);
            va[b * R0 + r] = ld ? base[k * zs] : z;
            vb[b * R0 + r] = ld ? base[cs + k * zs] : z;
            vc[b * R0 + r] = ld ? base[2 * cs + k * zs] : z;
        }
    fft<L, -1, false>(va, s, q, tw);
    fft<L, -1, false>(vb, s, q, tw);
    fft<L, -1, false>(vc, s, q, tw);

    constexpr int RL = last_radix<L, false>();
    const int nyk = ny + 1;
    const int kyf = ky <= ny ? ky : 2 * ny - ky;
    const float sy = ky <= ny ? 1.f : -1.f;
    const size_t kc = (size_t)(NZ + 1) * nyk * nxc;
    const float *Kb = Kt + (size_t)kyf * nxc + (ok ? kx : 0);
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int kz = q + Q * b + r * (L / RL);
            const int kzf = kz <= NZ ? kz : L - kz;
            const float sz = kz <= NZ ? 1.f : -1.f;
            const float *K = Kb + (size_t)kzf * nyk * nxc;
            const int i = b * RL + r;
            kdot(va[i], vb[i], vc[i], K[0], K[kc], K[2 * kc], sy * K[3 * kc], sz * K[4 * kc],
                 sy * sz * K[5 * kc]);
        }

    fft<L, +1, true>(va, s, q, tw);
    fft<L, +1, true>(vb, s, q, tw);
    fft<L, +1, true>(vc, s, q, tw);
    // the reversed order ends with radix R0: outputs sit where the inputs did
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int k = q + Q * b + r * (L / R0);
            const bool upper = r * (L / R0) >= NZ;
            if (!upper && ok && k < NZ) {
                base[k * zs] = va[b * R0 + r];
                base[cs + k * zs] = vb[b * R0 + r];
                base[2 * cs + k * zs] = vc[b * R0 + r];
            }
        }
}

// nz = 1: y forward -> product (xx, yy, zz, xy; xz = yz = 0) -> y inverse,
// in place on X1 (rows j < ny).
template <int L>
__global__ __launch_bounds__(conv_max_threads<L>()) void k_yconv(float2 *__restrict__ X1, const float *__restrict__ Kt,
                                                int nxc, int lp2, const float2 *__restrict__ tw)
{
    constexpr int E = Factors<L>::E, Q = L / E, NY = L / 2;
    extern __shared__ float2 lds[];
    const int P = 1 << lp2;
    const int t = threadIdx.x;
    const int p = t & (P - 1), q = t >> lp2;
    const int kx = blockIdx.x * P + p;
    const bool ok = kx < nxc;
    const LdsView s{lds, P + 1, p};
    const size_t cs = (size_t)NY * nxc;
    float2 *base = X1 + kx;
    float2 va[E], vb[E], vc[E];
    constexpr int R0 = first_radix<L, false>();
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int j = q + Q * b + r * (L / R0);
            const bool upper = r * (L / R0) >= NY;
            const bool ld = !upper && ok && j < NY;
            const float2 z = make_float2(0.f, 0.f);
            va[b * R0 + r] = ld ? base[(size_t)j * nxc] : z;
            vb[b * R0 + r] = ld ? base[cs + (size_t)j * nxc] : z;
            vc[b * R0 + r] = ld ? base[2 * cs + (size_t)j * nxc] : z;
        }
    fft<L, -1, false>(va, s, q, tw);
    fft<L, -1, false>(vb, s, q, tw);
    fft<L, -1, false>(vc, s, q, tw);
    constexpr int RL = last_radix<L, false>();
    const size_t kc = (size_t)(NY + 1) * nxc;
    const float *Kb = Kt + (ok ? kx : 0);
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int ky = q + Q * b + r * (L / RL);
            const int kyf = ky <= NY ? ky : L - ky;
            const float sy = ky <= NY ? 1.f : -1.f;
            const float *K = Kb + (size_t)kyf * nxc;
            const int i = b * RL + r;
            kdot(va[i], vb[i], vc[i], K[0], K[kc], K[2 * kc], sy * K[3 * kc], 0.f, 0.f);
        }
    fft<L, +1, true>(va, s, q, tw);
    fft<L, +1, true>(vb, s, q, tw);
    fft<L, +1, true>(vc, s, q, tw);
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int j = q + Q * b + r * (L / R0);
            const bool upper = r * (L / R0) >= NY;
            if (!upper && ok && j < NY) {
                base[(size_t)j * nxc] = va[b * R0 + r];
                base[cs + (size_t)j * nxc] = vb[b * R0 + r];
                base[2 * cs + (size_t)j * nxc] = vc[b * R0 + r];
            }
        }
}

// y inverse on a tile of P kx columns of one (component, z) plane, keep j < ny.
template <int L>
__global__ __launch_bounds__(1024) void k_yinv(const float2 *__restrict__ X2, float2 *__restrict__ X1,
                                               int nxc, int lp2, const float2 *__restrict__ tw)
{
    constexpr int E = Factors<L>::E, Q = L / E, NY = L / 2;
    extern __shared__ float2 lds[];
    const int P = 1 << lp2;
    const int t = threadIdx.x;
    const int p = t & (P - 1), q = t >> lp2;
    const int kx = blockIdx.x * P + p;
    const int plane = blockIdx.y;
    const bool ok = kx < nxc;
    const LdsView s{lds, P + 1, p};
    float2 v[E];
    constexpr int R0 = first_radix<L, false>();
    const float2 *src = X2 + (size_t)plane * L * nxc + kx;
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int k = q + Q * b + r * (L / R0);
            v[b * R0 + r] = ok ? src[(size_t)k * nxc] : make_float2(0.f, 0.f);
        }
    fft<L, +1, false>(v, s, q, tw);
    constexpr int RL = last_radix<L, false>();
    float2 *dst = X1 + (size_t)plane * NY * nxc + kx;
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int j = q + Q * b + r * (L / RL);
            const bool upper = r * (L / RL) >= NY;
            if (!upper && ok && j < NY) dst[(size_t)j * nxc] = v[b * RL + r];
        }
}

// x inverse, complex-to-real, two rows per transform: Z = A + iB with A, B
// the Hermitian half-spectra of rows 2m and 2m+1; Re/Im of the inverse are
// the two real rows.  Keep i < nx.
template <int L>
__global__ __launch_bounds__(1024) void k_xinv(const float2 *__restrict__ X1, float *__restrict__ H,
                                               int nrows, int lp2, const float2 *__restrict__ tw)
{
    constexpr int E = Factors<L>::E, Q = L / E, NX = L / 2, NXC = NX + 1;
    extern __shared__ float2 lds[];
    const int t = threadIdx.x;
    const int q = t % Q, p = t / Q;
    const int ra = ((blockIdx.x << lp2) + p) * 2, rb = ra + 1;
    const bool oka = ra < nrows, okb = rb < nrows;
    const LdsView s{lds, 1, p * (L + 1)};
    const float2 *sa = X1 + (size_t)ra * NXC;
    const float2 *sb = X1 + (size_t)rb * NXC;
    float2 v[E];
    constexpr int R0 = first_radix<L, false>();
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int k = q + Q * b + r * (L / R0);
            float2 A = make_float2(0.f, 0.f), B = make_float2(0.f, 0.f);
            if (k <= NX) {
                if (oka) A = sa[k];
                if (okb) B = sb[k];
                if (k == 0 || k == NX) {  // bins of a real row are real there
                    A.y = 0.f;
                    B.y = 0.f;
                }
            } else {
                if (oka) A = cconj(sa[L - k]);
                if (okb) B = cconj(sb[L - k]);
            }
            v[b * R0 + r] = make_float2(A.x - B.y, A.y + B.x);
        }
    fft<L, +1, false>(v, s, q, tw);
    constexpr int RL = last_radix<L, false>();
    float *da = H + (size_t)ra * NX;
    float *db = H + (size_t)rb * NX;
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int i = q + Q * b + r * (L / RL);
            const bool upper = r * (L / RL) >= NX;
            if (!upper && i < NX) {
                if (oka) da[i] = v[b * RL + r].x;
                if (okb) db[i] = v[b * RL + r].y;
            }
        }
}

// --------------------------------------------------------------- dispatch ---

static int ilog2(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}


struct KInfo {
    int E;       // values per thread
    int nstage;
    int conv_max;  // launch bound of the three-component kernels
};

template <int L> static KInfo kinfo() { return {Factors<L>::E, Factors<L>::N, conv_max_threads<L>()}; }

static bool kinfo_for(int L, KInfo &out)
{
    switch (L) {
#define MMK_CASE(LEN) case LEN: out = kinfo<LEN>(); return true;
        MMK_CASE(2) MMK_CASE(4) MMK_CASE(6) MMK_CASE(8) MMK_CASE(12) MMK_CASE(16) MMK_CASE(24) MMK_CASE(32) MMK_CASE(48) MMK_CASE(64) MMK_CASE(96) MMK_CASE(128)
        MMK_CASE(192) MMK_CASE(256) MMK_CASE(384) MMK_CASE(512) MMK_CASE(768) MMK_CASE(1024)
#undef MMK_CASE
    default: return false;
    }
}

bool length_supported(int L)
{
    KInfo k;
    return kinfo_for(L, k);
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

// threads and LDS of a launch of `pass` with tile P
static void launch_shape(const Plan &p, int pass, int P, int &threads, size_t &lds)
{
    const int L = pass_length(p, pass);
    KInfo k{};
    kinfo_for(L, k);
    const int Q = L / k.E;
    threads = P * Q;
    const bool rows = (pass == MM_PASS_XFWD || pass == MM_PASS_XINV);
    lds = k.nstage > 1 ? (rows ? (size_t)P * (L + 1) : (size_t)L * (P + 1)) * sizeof(float2) : 0;
}

bool pass_tile_valid(const Plan &p, int pass, int P)
{
    if (pass < 0 || pass > MM_PASS_YCONV || !pass_active(p, pass)) return false;
    if (P < 1 || (P & (P - 1)) != 0 || P > 256) return false;
    int threads;
    size_t lds;
    launch_shape(p, pass, P, threads, lds);
    KInfo k{};
    kinfo_for(pass_length(p, pass), k);
    const int maxt = (pass == MM_PASS_ZCONV || pass == MM_PASS_YCONV) ? k.conv_max : 1024;
    return threads >= 1 && threads <= maxt && lds <= p.lds_limit;
}

std::vector<int> pass_tile_candidates(const Plan &p, int pass)
{
    std::vector<int> out;
    for (int P = 1; P <= 256; P *= 2) {
        if (!pass_tile_valid(p, pass, P)) continue;
        int threads;
        size_t lds;
        launch_shape(p, pass, P, threads, lds);
        if (threads < 64 && pass_tile_valid(p, pass, 2 * P)) continue;  // underfilled wave
        if (threads > 1024) continue;
        out.push_back(P);
    }
    return out;
}

int pass_default_tile(const Plan &p, int pass)
{
    if (!pass_active(p, pass)) return 0;
    const bool rows = (pass == MM_PASS_XFWD || pass == MM_PASS_XINV);
    // Columns: 16 kx (128-byte segments); rows: enough rows for >= 256 threads.
    int best = 0;
    for (int P : pass_tile_candidates(p, pass)) {
        int threads;
        size_t lds;
        launch_shape(p, pass, P, threads, lds);
        if (rows) {
            if (best == 0 || threads <= 256) best = P;
        } else {
            if (best == 0 || (P <= 16 && lds <= 65536)) best = P;
        }
    }
    return best;
}

template <int L>
static hipError_t raise_lds(size_t limit)
{
    const int lim = (int)limit;
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void *)k_xfwd<L>, hipFuncAttributeMaxDynamicSharedMemorySize, lim)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void *)k_yfwd<L>, hipFuncAttributeMaxDynamicSharedMemorySize, lim)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void *)k_zconv<L>, hipFuncAttributeMaxDynamicSharedMemorySize, lim)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void *)k_yconv<L>, hipFuncAttributeMaxDynamicSharedMemorySize, lim)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void *)k_yinv<L>, hipFuncAttributeMaxDynamicSharedMemorySize, lim)) != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)k_xinv<L>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
}

int prepare_kernels(Plan &p)
{
    if (p.lds_limit <= 65536) return MM_OK;
    const int Ls[3] = {p.Lx, p.Ly, p.Lz};
    for (int a = 0; a < 3; ++a) {
        hipError_t e = hipSuccess;
        switch (Ls[a]) {
#define MMK_CASE(LEN) case LEN: e = raise_lds<LEN>(p.lds_limit); break;
            MMK_CASE(12) MMK_CASE(16) MMK_CASE(24) MMK_CASE(32) MMK_CASE(48) MMK_CASE(64) MMK_CASE(96) MMK_CASE(128) MMK_CASE(192) MMK_CASE(256)
            MMK_CASE(384) MMK_CASE(512) MMK_CASE(768) MMK_CASE(1024)
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

template <int L>
static void launch_len(Plan &p, int pass, int P, const float *M, float *H, hipStream_t s)
{
    KInfo k = kinfo<L>();
    const int Q = L / k.E;
    const int lp2 = ilog2(P);
    const dim3 block(P * Q);
    int threads;
    size_t lds;
    launch_shape(p, pass, P, threads, lds);
    const int nxc = p.nxc;
    switch (pass) {
    case MM_PASS_XFWD: {
        const int nrows = 3 * p.nz * p.ny;
        hipLaunchKernelGGL(k_xfwd<L>, dim3((nrows + P - 1) / P), block, lds, s, M, p.X1, nrows, lp2, p.tw[0]);
        break;
    }
    case MM_PASS_YFWD:
        hipLaunchKernelGGL(k_yfwd<L>, dim3((nxc + P - 1) / P, 3 * p.nz), block, lds, s, p.X1, p.X2, nxc, lp2, p.tw[1]);
        break;
    case MM_PASS_ZCONV:
        hipLaunchKernelGGL(k_zconv<L>, dim3((nxc + P - 1) / P, 2 * p.ny), block, lds, s, p.X2, p.Kt, nxc, p.ny, lp2, p.tw[2]);
        break;
    case MM_PASS_YCONV:
        hipLaunchKernelGGL(k_yconv<L>, dim3((nxc + P - 1) / P), block, lds, s, p.X1, p.Kt, nxc, lp2, p.tw[1]);
        break;
    case MM_PASS_YINV:
        hipLaunchKernelGGL(k_yinv<L>, dim3((nxc + P - 1) / P, 3 * p.nz), block, lds, s, p.X2, p.X1, nxc, lp2, p.tw[1]);
        break;
    case MM_PASS_XINV: {
        const int nrows = 3 * p.nz * p.ny;
        const int pairs = (nrows + 1) / 2;
        hipLaunchKernelGGL(k_xinv<L>, dim3((pairs + P - 1) / P), block, lds, s, p.X1, H, nrows, lp2, p.tw[0]);
        break;
    }
    default: break;
    }
}

int launch_pass(Plan &p, int pass, const float *M, float *H, hipStream_t s)
{
    const int L = pass_length(p, pass);
    const int P = p.tile[pass];
    if (!pass_tile_valid(p, pass, P)) return fail(MM_EINVAL, "invalid tile for pass");
    hipEvent_t ev0 = nullptr;
    timing_begin(p, pass, s, &ev0);
    switch (L) {
#define MMK_CASE(LEN) case LEN: launch_len<LEN>(p, pass, P, M, H, s); break;
        MMK_CASE(2) MMK_CASE(4) MMK_CASE(6) MMK_CASE(8) MMK_CASE(12) MMK_CASE(16) MMK_CASE(24) MMK_CASE(32) MMK_CASE(48) MMK_CASE(64) MMK_CASE(96) MMK_CASE(128)
        MMK_CASE(192) MMK_CASE(256) MMK_CASE(384) MMK_CASE(512) MMK_CASE(768) MMK_CASE(1024)
#undef MMK_CASE
    default: return fail(MM_EINVAL, "unsupported FFT length");
    }
    timing_end(p, pass, s, ev0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MM_EHIP, std::string("demag launch: ") + hipGetErrorString(e));
    return MM_OK;
}

int demag_enqueue(Plan &p, const float *M, float *H, hipStream_t s)
{
    int rc;
    if ((rc = launch_pass(p, MM_PASS_XFWD, M, H, s)) != MM_OK) return rc;
    if (p.nz > 1) {
        if ((rc = launch_pass(p, MM_PASS_YFWD, M, H, s)) != MM_OK) return rc;
        if ((rc = launch_pass(p, MM_PASS_ZCONV, M, H, s)) != MM_OK) return rc;
        if ((rc = launch_pass(p, MM_PASS_YINV, M, H, s)) != MM_OK) return rc;
    } else {
        if ((rc = launch_pass(p, MM_PASS_YCONV, M, H, s)) != MM_OK) return rc;
    }
    return launch_pass(p, MM_PASS_XINV, M, H, s);
}

}  // namespace mmk
