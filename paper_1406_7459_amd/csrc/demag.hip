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

// Twiddles live at the head of the dynamic LDS block (copied once per
// workgroup; the first read comes after the first exchange barrier, and a
// single-stage transform reads none).  MMK_TW_GLOBAL keeps them in global
// memory instead (for A/B timing).
template <int L> constexpr int tw_slots()
{
#ifdef MMK_TW_GLOBAL
    return 0;
#else
    return Factors<L>::N > 1 ? L : 0;
#endif
}

template <int L>
__device__ __forceinline__ const float2 *stage_twiddles(float2 *lds, const float2 *__restrict__ tw)
{
    if constexpr (tw_slots<L>() == 0) {
        return tw;
    } else {
        for (int i = threadIdx.x; i < L; i += blockDim.x) lds[i] = tw[i];
        return lds;
    }
}

// ----------------------------------------------------------------- kernels ---

// x forward: one real row of length nx, zero-padded to L = 2nx, -> nx+1 bins.
template <int L, int V>
__global__ __launch_bounds__(1024) void k_xfwd(const float *__restrict__ M, float2 *__restrict__ X1,
                                               int nrows, int lp2, const float2 *__restrict__ tw)
{
    constexpr int E = ept<L, V>(), Q = L / E, NX = L / 2;
    extern __shared__ float2 lds[];
    const float2 *twl = stage_twiddles<L>(lds, tw);
    const int t = threadIdx.x;
    const int q = t % Q, p = t / Q;
    const int row = (blockIdx.x << lp2) + p;
    const bool ok = row < nrows;
    const LdsView s{lds + tw_slots<L>(), 1, p * (L + 1)};
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
    fft_e<L, E, -1, false>(v, s, q, twl);
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
template <int L, int V>
__global__ __launch_bounds__(1024) void k_yfwd(const float2 *__restrict__ X1, float2 *__restrict__ X2,
                                               int nxc, int lp2, const float2 *__restrict__ tw)
{
    constexpr int E = ept<L, V>(), Q = L / E, NY = L / 2;
    extern __shared__ float2 lds[];
    const float2 *twl = stage_twiddles<L>(lds, tw);
    const int P = 1 << lp2;
    const int t = threadIdx.x;
    const int p = t & (P - 1), q = t >> lp2;
    const int kx = blockIdx.x * P + p;
    const int plane = blockIdx.y;
    const bool ok = kx < nxc;
    const LdsView s{lds + tw_slots<L>(), P + 1, p};
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
    fft_e<L, E, -1, false>(v, s, q, twl);
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

// One row of the product, k0 m0 + k1 m1 + k2 m2, in a fixed operation order
// shared by every schedule.
__device__ __forceinline__ float2 krow(float k0, float k1, float k2, float2 m0, float2 m1, float2 m2)
{
    return make_float2(fmaf(k2, m2.x, fmaf(k1, m1.x, k0 * m0.x)), fmaf(k2, m2.y, fmaf(k1, m1.y, k0 * m0.y)));
}

// Spectral product at one frequency: H~ = K~ . M~ with K~ real and symmetric
// (eq. (13)/(15)); the off-diagonal entries carry the parity signs of the
// folded octant.
__device__ __forceinline__ void kdot(float2 &a, float2 &b, float2 &c, float kxx, float kyy, float kzz,
                                     float kxy, float kxz, float kyz)
{
    const float2 mx = a, my = b, mz = c;
    a = krow(kxx, kxy, kxz, mx, my, mz);
    b = krow(kxy, kyy, kyz, mx, my, mz);
    c = krow(kxz, kyz, kzz, mx, my, mz);
}

// Three components stay in VGPRs across the product: cap the workgroup so
// the allocator gets 256 (E = 8) or 512 (E = 24) registers per lane.
template <int L> constexpr int conv_max_threads() { return Factors<L>::E > 8 ? 256 : 512; }

// Schedule "reg3" of the product pass.  ZAXIS: z forward -> product -> z
// inverse for P kx columns at one ky, in place on X2 (rows k < nz).  Else
// (nz = 1): the same along y on X1 (rows j < ny), with xz = yz = 0.
template <int L, bool ZAXIS>
__global__ __launch_bounds__(conv_max_threads<L>()) void k_conv_reg3(float2 *__restrict__ X, const float *__restrict__ Kt,
                                                                      int nxc, int ny, int lp2,
                                                                      const float2 *__restrict__ tw)
{
    constexpr int E = Factors<L>::E, Q = L / E, NH = L / 2;
    extern __shared__ float2 lds[];
    const float2 *twl = stage_twiddles<L>(lds, tw);
    const int P = 1 << lp2;
    const int t = threadIdx.x;
    const int p = t & (P - 1), q = t >> lp2;
    const int kx = blockIdx.x * P + p;
    const bool ok = kx < nxc;
    const LdsView s{lds + tw_slots<L>(), P + 1, p};
    const int ky = ZAXIS ? (int)blockIdx.y : 0;
    const size_t rs = ZAXIS ? (size_t)2 * ny * nxc : (size_t)nxc;  // stride along the transform
    const size_t cs = (size_t)NH * rs;                              // component stride
    float2 *base = X + (size_t)ky * nxc + kx;
    float2 va[E], vb[E], vc[E];
    constexpr int R0 = first_radix<L, false>();
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int k = q + Q * b + r * (L / R0);
            const bool upper = r * (L / R0) >= NH;
            const bool ld = !upper && ok && k < NH;
            const float2 z = make_float2(0.f, 0.f);
            va[b * R0 + r] = ld ? base[k * rs] : z;
            vb[b * R0 + r] = ld ? base[cs + k * rs] : z;
            vc[b * R0 + r] = ld ? base[2 * cs + k * rs] : z;
        }
    fft<L, -1, false>(va, s, q, twl);
    fft<L, -1, false>(vb, s, q, twl);
    fft<L, -1, false>(vc, s, q, twl);

    constexpr int RL = last_radix<L, false>();
    const int nyk = ny + 1;
    const int kyf = ky <= ny ? ky : 2 * ny - ky;
    const float sy0 = ky <= ny ? 1.f : -1.f;
    const size_t kc = ZAXIS ? (size_t)(NH + 1) * nyk * nxc : (size_t)(NH + 1) * nxc;
    const float *Kb = Kt + (ZAXIS ? (size_t)kyf * nxc : 0) + (ok ? kx : 0);
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int k = q + Q * b + r * (L / RL);
            const int kf = k <= NH ? k : L - k;
            const float sk = k <= NH ? 1.f : -1.f;
            const int i = b * RL + r;
            if constexpr (ZAXIS) {
                const float *K = Kb + (size_t)kf * nyk * nxc;
                kdot(va[i], vb[i], vc[i], K[0], K[kc], K[2 * kc], sy0 * K[3 * kc], sk * K[4 * kc],
                     sy0 * sk * K[5 * kc]);
            } else {
                const float *K = Kb + (size_t)kf * nxc;
                kdot(va[i], vb[i], vc[i], K[0], K[kc], K[2 * kc], sk * K[3 * kc], 0.f, 0.f);
            }
        }

    fft<L, +1, true>(va, s, q, twl);
    fft<L, +1, true>(vb, s, q, twl);
    fft<L, +1, true>(vc, s, q, twl);
    // the reversed order ends with radix R0: outputs sit where the inputs did
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int k = q + Q * b + r * (L / R0);
            const bool upper = r * (L / R0) >= NH;
            if (!upper && ok && k < NH) {
                base[k * rs] = va[b * R0 + r];
                base[cs + k * rs] = vb[b * R0 + r];
                base[2 * cs + k * rs] = vc[b * R0 + r];
            }
        }
}

// Schedule "split" of the product pass: three thread groups, one component
// each (the register footprint of a single-component pass).  After the
// forward transforms every thread publishes its spectrum values to LDS,
// reads the other two components at the same frequencies, forms its own row
// of K~ . M~, and inverse-transforms it.
template <int L, int V, bool ZAXIS>
__global__ __launch_bounds__(1024) void k_conv_split(float2 *__restrict__ X, const float *__restrict__ Kt,
                                                      int nxc, int ny, int lp2, const float2 *__restrict__ tw)
{
    constexpr int E = ept<L, V>(), Q = L / E, NH = L / 2;
    extern __shared__ float2 lds[];
    const float2 *twl = stage_twiddles<L>(lds, tw);
    const int P = 1 << lp2;
    const int PQ = P * Q;
    const int g = threadIdx.x / PQ;
    const int t = threadIdx.x - g * PQ;
    const int p = t & (P - 1), q = t >> lp2;
    const int kx = blockIdx.x * P + p;
    const bool ok = kx < nxc;
    const int rsl = P + 1;
    float2 *buf = lds + tw_slots<L>();
    const LdsView s{buf + (size_t)g * L * rsl, rsl, p};
    const int ky = ZAXIS ? (int)blockIdx.y : 0;
    const size_t rs = ZAXIS ? (size_t)2 * ny * nxc : (size_t)nxc;
    const size_t cs = (size_t)NH * rs;
    float2 *base = X + (size_t)g * cs + (size_t)ky * nxc + kx;
    float2 v[E];
    constexpr int R0 = first_radix<L, false>();
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int k = q + Q * b + r * (L / R0);
            const bool upper = r * (L / R0) >= NH;
            v[b * R0 + r] = (!upper && ok && k < NH) ? base[k * rs] : make_float2(0.f, 0.f);
        }
    fft_e<L, E, -1, false>(v, s, q, twl);

    constexpr int RL = last_radix<L, false>();
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int k = q + Q * b + r * (L / RL);
            buf[((size_t)g * L + k) * rsl + p] = v[b * RL + r];
        }
    __syncthreads();
    // this group's row of the symmetric tensor: (xx,xy,xz), (xy,yy,yz), (xz,yz,zz)
    const int c0 = g == 0 ? 0 : (g == 1 ? 3 : 4);
    const int c1 = g == 0 ? 3 : (g == 1 ? 1 : 5);
    const int c2 = g == 0 ? 4 : (g == 1 ? 5 : 2);
    const int nyk = ny + 1;
    const int kyf = ky <= ny ? ky : 2 * ny - ky;
    const float sy0 = ky <= ny ? 1.f : -1.f;
    const size_t kc = ZAXIS ? (size_t)(NH + 1) * nyk * nxc : (size_t)(NH + 1) * nxc;
    const float *Kb = Kt + (ZAXIS ? (size_t)kyf * nxc : 0) + (ok ? kx : 0);
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int k = q + Q * b + r * (L / RL);
            const int kf = k <= NH ? k : L - k;
            const float sk = k <= NH ? 1.f : -1.f;
            // parity signs: ZAXIS: sy on xy, sk on xz, sy*sk on yz; y only: sk on xy
            const float sxy = ZAXIS ? sy0 : sk, sxz = ZAXIS ? sk : 0.f, syz = ZAXIS ? sy0 * sk : 0.f;
            const float w0 = g == 0 ? 1.f : (g == 1 ? sxy : sxz);
            const float w1 = g == 0 ? sxy : (g == 1 ? 1.f : syz);
            const float w2 = g == 0 ? sxz : (g == 1 ? syz : 1.f);
            const float *K = Kb + (ZAXIS ? (size_t)kf * nyk * nxc : (size_t)kf * nxc);
            const float k0 = w0 * K[c0 * kc], k1 = w1 * K[c1 * kc], k2 = w2 * K[c2 * kc];
            const float2 m0 = buf[((size_t)0 * L + k) * rsl + p];
            const float2 m1 = buf[((size_t)1 * L + k) * rsl + p];
            const float2 m2 = buf[((size_t)2 * L + k) * rsl + p];
            v[b * RL + r] = krow(k0, k1, k2, m0, m1, m2);
        }
    __syncthreads();  // every product read is done before the inverse reuses LDS
    fft_e<L, E, +1, true>(v, s, q, twl);
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int k = q + Q * b + r * (L / R0);
            const bool upper = r * (L / R0) >= NH;
            if (!upper && ok && k < NH) base[k * rs] = v[b * R0 + r];
        }
}

// y inverse on a tile of P kx columns of one (component, z) plane, keep j < ny.
template <int L, int V>
__global__ __launch_bounds__(1024) void k_yinv(const float2 *__restrict__ X2, float2 *__restrict__ X1,
                                               int nxc, int lp2, const float2 *__restrict__ tw)
{
    constexpr int E = ept<L, V>(), Q = L / E, NY = L / 2;
    extern __shared__ float2 lds[];
    const float2 *twl = stage_twiddles<L>(lds, tw);
    const int P = 1 << lp2;
    const int t = threadIdx.x;
    const int p = t & (P - 1), q = t >> lp2;
    const int kx = blockIdx.x * P + p;
    const int plane = blockIdx.y;
    const bool ok = kx < nxc;
    const LdsView s{lds + tw_slots<L>(), P + 1, p};
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
    fft_e<L, E, +1, false>(v, s, q, twl);
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
template <int L, int V>
__global__ __launch_bounds__(1024) void k_xinv(const float2 *__restrict__ X1, float *__restrict__ H,
                                               int nrows, int lp2, const float2 *__restrict__ tw)
{
    constexpr int E = ept<L, V>(), Q = L / E, NX = L / 2, NXC = NX + 1;
    extern __shared__ float2 lds[];
    const float2 *twl = stage_twiddles<L>(lds, tw);
    const int t = threadIdx.x;
    const int q = t % Q, p = t / Q;
    const int ra = ((blockIdx.x << lp2) + p) * 2, rb = ra + 1;
    const bool oka = ra < nrows, okb = rb < nrows;
    const LdsView s{lds + tw_slots<L>(), 1, p * (L + 1)};
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
    fft_e<L, E, +1, false>(v, s, q, twl);
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
// A launch configuration ("tile") is P + 256 * variant: P transforms (rows
// for x, kx columns for y/z) per workgroup, a power of two, and a schedule
// variant: for the single-component passes 0 = default values per thread E,
// 1 = 2E; for the product passes 0 = reg3, 1 = split (E), 2 = split (2E).

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
};

template <int L> static KInfo kinfo()
{
    return {Factors<L>::E, ept<L, 1>(), Factors<L>::N, conv_max_threads<L>()};
}

#define MMK_ALL_LENGTHS(X)                                                                               \
    X(2) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) \
        X(768) X(1024)

static bool kinfo_for(int L, KInfo &out)
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

static bool is_conv(int pass) { return pass == MM_PASS_ZCONV || pass == MM_PASS_YCONV; }
static bool is_rows(int pass) { return pass == MM_PASS_XFWD || pass == MM_PASS_XINV; }

// threads, LDS bytes and thread limit of a launch of `pass` with `tile`
static bool launch_shape(const Plan &p, int pass, int tile, int &threads, size_t &lds, int &maxt)
{
    const int L = pass_length(p, pass);
    KInfo k{};
    if (!kinfo_for(L, k)) return false;
    const int P = tile & 255, var = tile >> 8;
    const size_t tws = k.nstage > 1 ? (size_t)L : 0;
    maxt = 1024;
    if (is_conv(pass)) {
        if (var == 0) {
            threads = P * (L / k.E0);
            maxt = k.conv_max;
            lds = (tws + (k.nstage > 1 ? (size_t)L * (P + 1) : 0)) * sizeof(float2);
        } else if (var == 1 || var == 2) {
            const int E = var == 1 ? k.E0 : k.E1;
            if (var == 2 && k.E1 == k.E0) return false;
            threads = 3 * P * (L / E);
            lds = (tws + 3 * (size_t)L * (P + 1)) * sizeof(float2);
        } else {
            return false;
        }
    } else {
        if (var != 0 && var != 1) return false;
        if (var == 1 && k.E1 == k.E0) return false;
        const int E = var == 0 ? k.E0 : k.E1;
        threads = P * (L / E);
        lds = (tws + (k.nstage > 1 ? (is_rows(pass) ? (size_t)P * (L + 1) : (size_t)L * (P + 1)) : 0)) *
              sizeof(float2);
    }
    return true;
}

bool pass_tile_valid(const Plan &p, int pass, int tile)
{
    if (pass < 0 || pass > MM_PASS_YCONV || !pass_active(p, pass)) return false;
    const int P = tile & 255;
    if (tile < 1 || P < 1 || (P & (P - 1)) != 0 || P > 128) return false;
    int threads, maxt;
    size_t lds;
    if (!launch_shape(p, pass, tile, threads, lds, maxt)) return false;
    return threads >= 1 && threads <= maxt && lds <= p.lds_limit;
}

std::vector<int> pass_tile_candidates(const Plan &p, int pass)
{
    std::vector<int> out;
    for (int var = 0; var < 3; ++var)
        for (int P = 1; P <= 128; P *= 2) {
            const int tile = P + 256 * var;
            if (!pass_tile_valid(p, pass, tile)) continue;
            int threads, maxt;
            size_t lds;
            launch_shape(p, pass, tile, threads, lds, maxt);
            if (threads < 64 && pass_tile_valid(p, pass, 2 * P + 256 * var)) continue;  // underfilled wave
            out.push_back(tile);
        }
    return out;
}

int pass_default_tile(const Plan &p, int pass)
{
    if (!pass_active(p, pass)) return 0;
    // rows: the largest P with <= 256 threads; columns: the largest P <= 16
    // whose LDS fits in 64 KiB (split schedule for the product passes when
    // the transform has several stages, reg3 otherwise)
    const int L = pass_length(p, pass);
    KInfo k{};
    kinfo_for(L, k);
    const int var = (is_conv(pass) && k.nstage > 1) ? 1 : 0;
    int best = 0;
    for (int P = 1; P <= 128; P *= 2) {
        const int tile = P + 256 * var;
        if (!pass_tile_valid(p, pass, tile)) continue;
        int threads, maxt;
        size_t lds;
        launch_shape(p, pass, tile, threads, lds, maxt);
        if (is_rows(pass)) {
            if (best == 0 || threads <= 256) best = tile;
        } else if (best == 0 || (P <= 16 && lds <= 65536)) {
            best = tile;
        }
    }
    return best;
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
        raise_one(k_conv_reg3<L, true>, lim), raise_one(k_conv_reg3<L, false>, lim),
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

template <int L, int V>
static void launch_single(Plan &p, int pass, int P, size_t lds, const float *M, float *H, hipStream_t s)
{
    constexpr int Q = L / ept<L, V>();
    const int lp2 = ilog2(P);
    const dim3 block(P * Q);
    const int nxc = p.nxc;
    const int nrows = 3 * p.nz * p.ny;
    switch (pass) {
    case MM_PASS_XFWD:
        hipLaunchKernelGGL((k_xfwd<L, V>), dim3((nrows + P - 1) / P), block, lds, s, M, p.X1, nrows, lp2, p.tw[0]);
        break;
    case MM_PASS_YFWD:
        hipLaunchKernelGGL((k_yfwd<L, V>), dim3((nxc + P - 1) / P, 3 * p.nz), block, lds, s, p.X1, p.X2, nxc, lp2,
                           p.tw[1]);
        break;
    case MM_PASS_YINV:
        hipLaunchKernelGGL((k_yinv<L, V>), dim3((nxc + P - 1) / P, 3 * p.nz), block, lds, s, p.X2, p.X1, nxc, lp2,
                           p.tw[1]);
        break;
    case MM_PASS_XINV: {
        const int pairs = (nrows + 1) / 2;
        hipLaunchKernelGGL((k_xinv<L, V>), dim3((pairs + P - 1) / P), block, lds, s, p.X1, H, nrows, lp2, p.tw[0]);
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
    const dim3 grid((nxc + P - 1) / P, z ? 2 * p.ny : 1);
    if (var == 0) {
        const dim3 block(P * (L / Factors<L>::E));
        if (z) hipLaunchKernelGGL((k_conv_reg3<L, true>), grid, block, lds, s, X, p.Kt, nxc, p.ny, lp2, tw);
        else hipLaunchKernelGGL((k_conv_reg3<L, false>), grid, block, lds, s, X, p.Kt, nxc, p.ny, lp2, tw);
    } else if (var == 1) {
        const dim3 block(3 * P * (L / ept<L, 0>()));
        if (z) hipLaunchKernelGGL((k_conv_split<L, 0, true>), grid, block, lds, s, X, p.Kt, nxc, p.ny, lp2, tw);
        else hipLaunchKernelGGL((k_conv_split<L, 0, false>), grid, block, lds, s, X, p.Kt, nxc, p.ny, lp2, tw);
    } else {
        const dim3 block(3 * P * (L / ept<L, 1>()));
        if (z) hipLaunchKernelGGL((k_conv_split<L, 1, true>), grid, block, lds, s, X, p.Kt, nxc, p.ny, lp2, tw);
        else hipLaunchKernelGGL((k_conv_split<L, 1, false>), grid, block, lds, s, X, p.Kt, nxc, p.ny, lp2, tw);
    }
}

template <int L>
static void launch_len(Plan &p, int pass, int tile, size_t lds, const float *M, float *H, hipStream_t s)
{
    const int P = tile & 255, var = tile >> 8;
    if (is_conv(pass)) launch_conv<L>(p, pass, P, var, lds, s);
    else if (var == 0) launch_single<L, 0>(p, pass, P, lds, M, H, s);
    else launch_single<L, 1>(p, pass, P, lds, M, H, s);
}

int launch_pass(Plan &p, int pass, const float *M, float *H, hipStream_t s)
{
    const int L = pass_length(p, pass);
    const int tile = p.tile[pass];
    if (!pass_tile_valid(p, pass, tile)) return fail(MM_EINVAL, "invalid tile for pass");
    int threads, maxt;
    size_t lds;
    launch_shape(p, pass, tile, threads, lds, maxt);
    hipEvent_t ev0 = nullptr;
    timing_begin(p, pass, s, &ev0);
    switch (L) {
#define MMK_CASE(LEN) case LEN: launch_len<LEN>(p, pass, tile, lds, M, H, s); break;
        MMK_ALL_LENGTHS(MMK_CASE)
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
