// demag_kernels.hpp -- device bodies of the demag passes, shared by the
// per-plan launches (demag.hip) and the batched launches (batch.hip).  Each
// body takes its workgroup's coordinates explicitly, so a batched launch can
// feed it coordinates from a task table.
//
// Passes of one demagnetising-field evaluation (the zero-padded convolution
// H = K * M of the paper, Sec. 2 steps (1)-(5), eq. (13)-(16)), evaluated by
// a real-to-complex FFT that never touches the zero half of the padded grid
// (forward) nor computes the discarded half (inverse):
//
//   XFWD   M [3][nz][ny][nx] f32   -> X1 [3][nz][ny][xp] c64     x: R2C, input i < nx
//   YFWD   X1                      -> X2 [3][nz][2ny][xp]        y: input j < ny
//   ZCONV  X2 -> X2 in place: z forward (input k < nz), H~ = K~ . M~
//          (eq. (13)/(15), six real K~ components with parity signs),
//          z inverse, rows k < nz written back
//   YINV   X2 -> X1                                               y: keep j < ny
//   XINV   X1 -> H [3][nz][ny][nx] f32                            x: C2R, keep i < nx
// (xp = x_pitch(Lx/2 + 1): rows of Lx/2 + 1 values padded to 128 bytes; the
// padding is never read or written.)  An axis of n cells is padded to a
// supported transform length L >= 2n (L = 2n when n is 2^a, 3 2^a or 5 2^a): the
// zero-padded convolution only needs L >= 2n - 1, so the live count n is a
// run-time argument of every body and L a template parameter.
// For nz = 1 the padded z axis has length 2 with the second slot zero, so the
// z transform is the identity up to a factor folded into K~; YCONV then does
// y forward, product and y inverse in one pass (XFWD, YCONV, XINV).
//
// A workgroup owns a tile of whole 1-D transforms (P consecutive kx columns
// for y/z, P rows -- P row pairs for XINV -- for x), loads them coalesced
// straight into registers, and exchanges through LDS only between FFT stages
// (fft_engine.hpp).
#pragma once
#include "fft_engine.hpp"
#include "layout.hpp"

namespace mmk {

// Twiddles live at the head of the dynamic LDS block (copied once per
// workgroup; the first read comes after the first exchange barrier, and a
// single-stage transform reads none).
template <int L> constexpr int tw_slots() { return Factors<L>::N > 1 ? L : 0; }

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

// The row passes' twiddles in the staged layout of radix order O
// (fft_engine.hpp, stage_compute): L - R0 <= L entries, in the same slots.
template <int L, int O>
__device__ __forceinline__ const float2 *row_twiddles(float2 *lds, const float2 *__restrict__ tw)
{
    if constexpr (tw_slots<L>() == 0) {
        return tw;  // one stage: no twiddles read
    } else {
        fill_staged_twiddles<L, O>(lds, tw);
        return lds;
    }
}

// ----------------------------------------------------------------- kernels ---

// Rows of the x passes are paired within a component: pair m of the
// 3 ceil(ncr/2) pairs covers rows 2mm and 2mm+1 of component m / ceil(ncr/2)
// (ncr = nz ny rows per component), the second absent for the last pair of
// an odd ncr.  The fused x-inverse/stage/x-forward pass pairs its rows the
// same way, so both paths round identically.
__device__ __forceinline__ void x_pair_rows(int m, int ncr, int &ra, bool &oka, bool &okb)
{
    const int hp = (ncr + 1) >> 1;
    const int comp = m / hp, mm = m - comp * hp;
    ra = comp * ncr + 2 * mm;
    oka = comp < 3;
    okb = oka && 2 * mm + 1 < ncr;
}

// x forward, two real rows per complex transform: z = a + i b (rows 2m and
// 2m+1, length nx, zero-padded to L = 2nx), Z = FFT(z), then
//   A_k = (Z_k + conj Z_{L-k}) / 2,   B_k = (Z_k - conj Z_{L-k}) / (2i),
// k = 0..nx; Z_{L-k} is read back through LDS.
template <int L, int V>
__device__ __forceinline__ void xfwd_body(const float *__restrict__ M, float2 *__restrict__ X1, int ncr, int nx,
                                          int lp2, const float2 *__restrict__ tw, int bx)
{
    constexpr int OV = order_of_v<V>();
    constexpr int E = ept<L, V>(), Q = L / E, NX = L / 2, XP = x_pitch(NX + 1);
    extern __shared__ float2 lds[];
    const float2 *twl = row_twiddles<L, OV>(lds, tw);
    const int t = threadIdx.x;
    const int q = t % Q, p = t / Q;
    int ra;
    bool oka, okb;
    x_pair_rows((bx << lp2) + p, ncr, ra, oka, okb);
    const int rb = ra + 1;
    constexpr int XS = lds_rows(L) + 1;  // slots per transform (odd)
    float2 *col = lds + tw_slots<L>() + p * XS;
    const LdsView s{lds + tw_slots<L>(), 1, p * XS};
    float2 v[E];
    constexpr int R0 = first_radix<L, false, OV>();
    const float *sa = M + (size_t)ra * nx;
    const float *sb = M + (size_t)rb * nx;
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int i = q + Q * b + r * (L / R0);
            const bool upper = r * (L / R0) >= NX;  // compile-time after unrolling
            const bool in = !upper && i < nx;
            v[b * R0 + r] = make_float2(in && oka ? sa[i] : 0.f, in && okb ? sb[i] : 0.f);
        }
    fft_e<L, E, -1, false, OV, true>(v, s, q, twl);
    constexpr int RL = last_radix<L, false, OV>();
    // the last exchange ended with a barrier: the column is free for Z
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) col[lds_slot(q + Q * b + r * (L / RL))] = v[b * RL + r];
    __syncthreads();
    float2 *da = X1 + (size_t)ra * XP;
    float2 *db = X1 + (size_t)rb * XP;
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int k = q + Q * b + r * (L / RL);
            if (k <= NX) {
                const float2 z = v[b * RL + r];
                const float2 w = col[lds_slot(k == 0 ? 0 : L - k)];
                const float2 sp = make_float2(z.x + w.x, z.y - w.y);  // Z + conj(Zm)
                const float2 sm = make_float2(z.x - w.x, z.y + w.y);  // Z - conj(Zm)
                if (oka) da[k] = make_float2(0.5f * sp.x, 0.5f * sp.y);
                if (okb) db[k] = make_float2(0.5f * sm.y, -0.5f * sm.x);
            }
        }
}

// Column of thread p of a column-pass workgroup.  A tile (nedge = 0): kx
// columns bx P .. bx P + P - 1 of one plane (or ky row) `slot`.  An edge
// workgroup (nedge > 0): the half spectrum's last column kx = nxc - 1 of the
// P planes (ky rows) slot P .. slot P + P - 1 of nedge.  When P divides the
// Lx/2 columns below it, edge workgroups spare the tiles a last tile with a
// single live column.
__device__ __forceinline__ bool column_of(int nxc, int P, int p, int bx, int slot, int nedge, int &kx, int &row)
{
    if (nedge > 0) {
        kx = nxc - 1;
        row = slot * P + p;
        if (row < nedge) return true;
        row = nedge - 1;  // an idle lane keeps in-range addresses
        return false;
    }
    kx = bx * P + p;
    row = slot;
    return kx < nxc;
}

// y forward on a tile of P kx columns of one (component, z) plane, or an
// edge workgroup (column_of).
template <int L, int V>
__device__ __forceinline__ void yfwd_body(const float2 *__restrict__ X1, float2 *__restrict__ X2, int nxc, int ny,
                                          int lp2, const float2 *__restrict__ tw, int bx, int slot, int nedge = 0)
{
    constexpr int OV = order_of_v<V>();
    constexpr int E = ept<L, V>(), Q = L / E, NY = L / 2;
    static_assert((Q & (Q - 1)) == 0, "threads per transform: a power of two");
    extern __shared__ float2 lds[];
    const float2 *twl = stage_twiddles<L>(lds, tw);
    const int P = 1 << lp2;
    const int t = threadIdx.x;
    const int p = t & (P - 1), q = (t >> lp2) & (Q - 1);  // t < P Q: the mask only states q < Q
    int kx, plane;
    const bool ok = column_of(nxc, P, p, bx, slot, nedge, kx, plane);
    const int xp = x_pitch(nxc);
    const LdsView s{lds + tw_slots<L>(), P, p};
    float2 v[E];
    constexpr int R0 = first_radix<L, false, OV>();
    // this thread's row q; the other rows are compile-time multiples of the
    // (uniform) row pitch away
    const float2 *src = X1 + ((size_t)plane * ny + q) * xp + kx;
    const size_t zs = x2_plane_stride(L, xp);
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int j = q + Q * b + r * (L / R0);
            const bool upper = r * (L / R0) >= NY;
            v[b * R0 + r] = (!upper && ok && j < ny) ? float2(src[(size_t)(Q * b + r * (L / R0)) * xp])
                                                     : make_float2(0.f, 0.f);
        }
    fft_e<L, E, -1, false, OV>(v, s, q, twl);
    constexpr int RL = last_radix<L, false, OV>();
    float2 *dst = X2 + (size_t)plane * zs + (size_t)q * xp + kx;
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r)
            if (ok) dst[(size_t)(Q * b + r * (L / RL)) * xp] = v[b * RL + r];
}

// One row of the product, k0 m0 + k1 m1 + k2 m2, in a fixed operation order
// shared by every schedule.
__device__ __forceinline__ float2 krow(float k0, float k1, float k2, float2 m0, float2 m1, float2 m2)
{
    return make_float2(fmaf(k2, m2.x, fmaf(k1, m1.x, k0 * m0.x)), fmaf(k2, m2.y, fmaf(k1, m1.y, k0 * m0.y)));
}

// Order of the ky rows of the z pass: 0, ny, 1, 2ny-1, 2, 2ny-2, ... so that
// a row and its mirror 2ny - ky (the same K~ octant row) run back to back.
__device__ __host__ __forceinline__ int ky_of_slot(int y, int ny)
{
    if (y == 0) return 0;
    if (y == 1) return ny;
    const int m = (y - 2) / 2 + 1;
    return (y & 1) ? 2 * ny - m : m;
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
// the allocator gets 128 (E = 4), 256 (E = 8) or 512 (E >= 12) registers
// per lane.
template <int L, int O = 0> constexpr int conv_max_threads()
{
    return Factors<L, O>::E > 8 ? 256 : (Factors<L, O>::E > 4 ? 512 : 1024);
}

// Schedule "reg3" of the product pass in radix order O.  ZAXIS: z forward
// -> product -> z inverse for P kx columns at one ky, in place on X2 (rows
// k < nz), or (nedge = 2 hy) for the last kx column at P ky rows
// (column_of).  Else (nz = 1): the same along y on X1 (rows j < ny), with
// xz = yz = 0.
template <int L, bool ZAXIS, int O = 0>
__device__ __forceinline__ void conv_reg3_body(float2 *__restrict__ X, const float *__restrict__ Kt, int nxc, int hy,
                                               int nlive, int lp2, const float2 *__restrict__ tw, int bx, int slot,
                                               int nedge = 0)
{
    constexpr int E = Factors<L, O>::E, Q = L / E, NH = L / 2;
    static_assert((Q & (Q - 1)) == 0, "threads per transform: a power of two");
    extern __shared__ float2 lds[];
    const int P = 1 << lp2;
    const int t = threadIdx.x;
    const int p = t & (P - 1), q = (t >> lp2) & (Q - 1);  // t < P Q: the mask only states q < Q
    int kx, ky;
    const bool ok = column_of(nxc, P, p, bx, slot, nedge, kx, ky);
    const int xp = x_pitch(nxc);
    // two exchange buffers (ping-pong transforms: one barrier per exchange)
    const LdsView s{lds + tw_slots<L>(), P, p};
    const LdsView s1{lds + tw_slots<L>() + lds_rows(L) * P, P, p};
    const size_t rs = ZAXIS ? (size_t)x2_plane_stride(2 * hy, xp) : (size_t)xp;  // stride along the transform
    const size_t cs = (size_t)nlive * rs;                         // component stride
    float2 *base = X + (size_t)ky * xp + kx + (size_t)q * rs;  // this thread's row q
    float2 va[E], vb[E], vc[E];
    constexpr int R0 = first_radix<L, false, O>();
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int k = q + Q * b + r * (L / R0);
            const size_t o = (size_t)(Q * b + r * (L / R0)) * rs;  // uniform
            const bool upper = r * (L / R0) >= NH;
            const bool ld = !upper && ok && k < nlive;
            // (values, not lvalues, on both sides: a select between two
            // lvalues of class type would become a flat load through a
            // selected pointer to either global or private memory)
            va[b * R0 + r] = ld ? float2(base[o]) : make_float2(0.f, 0.f);
            vb[b * R0 + r] = ld ? float2(base[cs + o]) : make_float2(0.f, 0.f);
            vc[b * R0 + r] = ld ? float2(base[2 * cs + o]) : make_float2(0.f, 0.f);
        }
    // twiddles staged after this thread's loads are issued (the table's
    // load latency overlaps them)
    const float2 *twl = stage_twiddles<L>(lds, tw);
    fft_pp<L, -1, false, O>(va, s, s1, q, twl);
    fft_pp<L, -1, false, O>(vb, s, s1, q, twl);
    fft_pp<L, -1, false, O>(vc, s, s1, q, twl);

    constexpr int RL = last_radix<L, false, O>();
    const int nyk = hy + 1;
    const int kyf = ky <= hy ? ky : 2 * hy - ky;
    const float sy0 = ky <= hy ? 1.f : -1.f;
    // K~ records of six floats (xx, yy, zz, xy, xz, yz) per octant frequency
    const float2 *Kb = reinterpret_cast<const float2 *>(Kt) +
                       3 * ((ZAXIS ? (size_t)kyf * xp : 0) + (size_t)(ok ? kx : 0));
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int k = q + Q * b + r * (L / RL);
            const int kf = k <= NH ? k : L - k;
            const float sk = k <= NH ? 1.f : -1.f;
            const int i = b * RL + r;
            const float2 *K = Kb + 3u * __umul24((unsigned)kf, ZAXIS ? (unsigned)(nyk * xp) : (unsigned)xp);
            const float2 k01 = K[0], k23 = K[1], k45 = K[2];
            if constexpr (ZAXIS) {
                kdot(va[i], vb[i], vc[i], k01.x, k01.y, k23.x, sy0 * k23.y, sk * k45.x, sy0 * sk * k45.y);
            } else {
                kdot(va[i], vb[i], vc[i], k01.x, k01.y, k23.x, sk * k23.y, 0.f, 0.f);
            }
        }

    // Keep the inverse transforms from being interleaved with the product:
    // mixing them lifts the register peak from ~106 to ~134 VGPRs at L = 256
    // (three waves per SIMD instead of four).
    __builtin_amdgcn_sched_barrier(0);
    fft_pp<L, +1, true, O>(va, s, s1, q, twl);
    fft_pp<L, +1, true, O>(vb, s, s1, q, twl);
    fft_pp<L, +1, true, O>(vc, s, s1, q, twl);
    // the reversed order ends with radix R0: outputs sit where the inputs did
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int k = q + Q * b + r * (L / R0);
            const size_t o = (size_t)(Q * b + r * (L / R0)) * rs;
            const bool upper = r * (L / R0) >= NH;
            if (!upper && ok && k < nlive) {
                base[o] = va[b * R0 + r];
                base[cs + o] = vb[b * R0 + r];
                base[2 * cs + o] = vc[b * R0 + r];
            }
        }
}

// Schedule "split" of the product pass: three thread groups, one component
// each (the register footprint of a single-component pass).  After the
// forward transforms every thread publishes its spectrum values to LDS,
// reads the other two components at the same frequencies, forms its own row
// of K~ . M~, and inverse-transforms it.
template <int L, int V, bool ZAXIS>
__device__ __forceinline__ void conv_split_body(float2 *__restrict__ X, const float *__restrict__ Kt, int nxc, int hy,
                                                int nlive, int lp2, const float2 *__restrict__ tw, int bx, int ky)
{
    constexpr int E = ept<L, V>(), Q = L / E, NH = L / 2;
    static_assert((Q & (Q - 1)) == 0, "threads per transform: a power of two");
    extern __shared__ float2 lds[];
    const int P = 1 << lp2;
    const int PQ = P * Q;
    const int g = threadIdx.x / PQ;
    const int t = threadIdx.x - g * PQ;
    const int p = t & (P - 1), q = (t >> lp2) & (Q - 1);  // t < P Q: the mask only states q < Q
    const int kx = bx * P + p;
    const bool ok = kx < nxc;
    const int xp = x_pitch(nxc);
    constexpr int GS = lds_rows(L);  // slots per component group
    float2 *buf = lds + tw_slots<L>();
    const LdsView s{buf + (size_t)g * GS * P, P, p};
    const size_t rs = ZAXIS ? (size_t)x2_plane_stride(2 * hy, xp) : (size_t)xp;
    const size_t cs = (size_t)nlive * rs;
    float2 *base = X + (size_t)g * cs + (size_t)ky * xp + kx + (size_t)q * rs;
    float2 v[E];
    constexpr int R0 = first_radix<L, false>();
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int k = q + Q * b + r * (L / R0);
            const bool upper = r * (L / R0) >= NH;
            v[b * R0 + r] = (!upper && ok && k < nlive) ? float2(base[(size_t)(Q * b + r * (L / R0)) * rs])
                                                     : make_float2(0.f, 0.f);
        }
    // this group's row of the symmetric tensor: (xx,xy,xz), (xy,yy,yz), (xz,yz,zz);
    // its K~ values do not depend on the transform: with E = 8 values per
    // thread they are loaded first and their latency passes under the
    // forward transform (with more values the registers are not there)
    constexpr int RL = last_radix<L, false>();
    constexpr bool PRE = E <= 8;
    const int c0 = g == 0 ? 0 : (g == 1 ? 3 : 4);
    const int c1 = g == 0 ? 3 : (g == 1 ? 1 : 5);
    const int c2 = g == 0 ? 4 : (g == 1 ? 5 : 2);
    const int nyk = hy + 1;
    const int kyf = ky <= hy ? ky : 2 * hy - ky;
    const float sy0 = ky <= hy ? 1.f : -1.f;
    const float *Kb = Kt + 6 * ((ZAXIS ? (size_t)kyf * xp : 0) + (size_t)(ok ? kx : 0));
    float kr[E][3];
    auto load_k = [&]() {
#pragma unroll
        for (int b = 0; b < E / RL; ++b)
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const int k = q + Q * b + r * (L / RL);
                const int kf = k <= NH ? k : L - k;
                const float *K = Kb + 6u * __umul24((unsigned)kf, ZAXIS ? (unsigned)(nyk * xp) : (unsigned)xp);
                kr[b * RL + r][0] = K[c0];
                kr[b * RL + r][1] = K[c1];
                kr[b * RL + r][2] = K[c2];
            }
    };
    if constexpr (PRE) load_k();
    // twiddles staged after this thread's loads are issued (the table's
    // load latency overlaps them)
    const float2 *twl = stage_twiddles<L>(lds, tw);
    fft_e<L, E, -1, false>(v, s, q, twl);
    if constexpr (!PRE) load_k();

#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int k = q + Q * b + r * (L / RL);
            buf[((size_t)g * GS + lds_slot(k)) * P + p] = v[b * RL + r];
        }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int k = q + Q * b + r * (L / RL);
            const float sk = k <= NH ? 1.f : -1.f;
            // parity signs: ZAXIS: sy on xy, sk on xz, sy*sk on yz; y only: sk on xy
            const float sxy = ZAXIS ? sy0 : sk, sxz = ZAXIS ? sk : 0.f, syz = ZAXIS ? sy0 * sk : 0.f;
            const float w0 = g == 0 ? 1.f : (g == 1 ? sxy : sxz);
            const float w1 = g == 0 ? sxy : (g == 1 ? 1.f : syz);
            const float w2 = g == 0 ? sxz : (g == 1 ? syz : 1.f);
            const float *kk = kr[b * RL + r];
            const float k0 = w0 * kk[0], k1 = w1 * kk[1], k2 = w2 * kk[2];
            const int ks = lds_slot(k) * P + p;
            const float2 m0 = buf[ks];
            const float2 m1 = buf[(size_t)GS * P + ks];
            const float2 m2 = buf[(size_t)2 * GS * P + ks];
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
            if (!upper && ok && k < nlive) base[(size_t)(Q * b + r * (L / R0)) * rs] = v[b * R0 + r];
        }
}

// y inverse on a tile of P kx columns of one (component, z) plane, or an
// edge workgroup (column_of); keep j < ny.
template <int L, int V>
__device__ __forceinline__ void yinv_body(const float2 *__restrict__ X2, float2 *__restrict__ X1, int nxc, int ny,
                                          int lp2, const float2 *__restrict__ tw, int bx, int slot, int nedge = 0)
{
    constexpr int OV = order_of_v<V>();
    constexpr int E = ept<L, V>(), Q = L / E, NY = L / 2;
    static_assert((Q & (Q - 1)) == 0, "threads per transform: a power of two");
    extern __shared__ float2 lds[];
    const float2 *twl = stage_twiddles<L>(lds, tw);
    const int P = 1 << lp2;
    const int t = threadIdx.x;
    const int p = t & (P - 1), q = (t >> lp2) & (Q - 1);  // t < P Q: the mask only states q < Q
    int kx, plane;
    const bool ok = column_of(nxc, P, p, bx, slot, nedge, kx, plane);
    const int xp = x_pitch(nxc);
    const LdsView s{lds + tw_slots<L>(), P, p};
    float2 v[E];
    constexpr int R0 = first_radix<L, false, OV>();
    const float2 *src = X2 + (size_t)plane * x2_plane_stride(L, xp) + (size_t)q * xp + kx;
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r)
            v[b * R0 + r] = ok ? float2(src[(size_t)(Q * b + r * (L / R0)) * xp]) : make_float2(0.f, 0.f);
    fft_e<L, E, +1, false, OV>(v, s, q, twl);
    constexpr int RL = last_radix<L, false, OV>();
    float2 *dst = X1 + ((size_t)plane * ny + q) * xp + kx;
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int j = q + Q * b + r * (L / RL);
            const bool upper = r * (L / RL) >= NY;
            if (!upper && ok && j < ny) dst[(size_t)(Q * b + r * (L / RL)) * xp] = v[b * RL + r];
        }
}

// Input of the packed x inverse at this thread's rows k = q + Q b + r L/R0:
// z_k = A_k + i B_k for the half spectra A (row a, at sa) and B (row b, at
// sb), extended Hermitian-wise (A_{L-k} = conj A_k) and with the imaginary
// parts of the k = 0 and k = L/2 bins dropped (the bins of a real row are
// real there); an absent row (ok false) enters as zeros.  Every load is
// issued before any value is used, from rows clamped into the grid and
// masked afterwards: with the loads in branches, each conjugation waited
// for its own load, so a thread's loads ran one after another.
template <int L, int E, int R0, int Q>
__device__ __forceinline__ void x_inverse_gather(const float2 *sa, const float2 *sb, bool oka, bool okb, int q,
                                                 float2 (&v)[E])
{
    constexpr int NX = L / 2;
    float2 la[E], lb[E];
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int k = q + Q * b + r * (L / R0);
            const int kk = k <= NX ? k : L - k;
            la[b * R0 + r] = sa[kk];
            lb[b * R0 + r] = sb[kk];
        }
#pragma unroll
    for (int b = 0; b < E / R0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int i = b * R0 + r;
            const int k = q + Q * b + r * (L / R0);
            float2 A = la[i], B = lb[i];
            if (k > NX) {
                A.y = -A.y;
                B.y = -B.y;
            } else if (k == 0 || k == NX) {
                A.y = 0.f;
                B.y = 0.f;
            }
            if (!oka) A = make_float2(0.f, 0.f);
            if (!okb) B = make_float2(0.f, 0.f);
            v[i] = make_float2(A.x - B.y, A.y + B.x);
        }
}

// x inverse, complex-to-real, two rows per transform: Z = A + iB with A, B
// the Hermitian half-spectra of rows 2m and 2m+1; Re/Im of the inverse are
// the two real rows.  Keep i < nx.
template <int L, int V>
__device__ __forceinline__ void xinv_body(const float2 *__restrict__ X1, float *__restrict__ H, int ncr, int nx,
                                          int lp2, const float2 *__restrict__ tw, int bx)
{
    constexpr int OV = order_of_v<V>();
    constexpr int E = ept<L, V>(), Q = L / E, NX = L / 2, XP = x_pitch(NX + 1);
    extern __shared__ float2 lds[];
    const float2 *twl = row_twiddles<L, OV>(lds, tw);
    const int t = threadIdx.x;
    const int q = t % Q, p = t / Q;
    int ra;
    bool oka, okb;
    x_pair_rows((bx << lp2) + p, ncr, ra, oka, okb);
    const int rb = ra + 1;
    const LdsView s{lds + tw_slots<L>(), 1, p * (lds_rows(L) + 1)};
    const int ca = oka ? ra : 0;  // rows clamped into the grid (masked in the gather)
    const float2 *sa = X1 + (size_t)ca * XP;
    const float2 *sb = X1 + (size_t)(okb ? rb : ca) * XP;
    float2 v[E];
    constexpr int R0 = first_radix<L, false, OV>();
    x_inverse_gather<L, E, R0, Q>(sa, sb, oka, okb, q, v);
    fft_e<L, E, +1, false, OV, true>(v, s, q, twl);
    constexpr int RL = last_radix<L, false, OV>();
    float *da = H + (size_t)ra * nx;
    float *db = H + (size_t)rb * nx;
#pragma unroll
    for (int b = 0; b < E / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int i = q + Q * b + r * (L / RL);
            const bool upper = r * (L / RL) >= NX;
            if (!upper && i < nx) {
                if (oka) da[i] = v[b * RL + r].x;
                if (okb) db[i] = v[b * RL + r].y;
            }
        }
}

}  // namespace mmk
