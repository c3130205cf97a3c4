// fft_engine.hpp -- register-resident Stockham FFT for gfx950 (wave64).
//
// A length-L transform is shared by Q = L/E threads of one workgroup; each
// thread keeps E complex values in VGPRs.  A stage of radix R lets every
// thread run E/R butterflies: butterfly j (j = q + Q*b) reads rows
// j + r*L/R and writes rows (j/Ns)*Ns*R + j%Ns + r*Ns (Stockham autosort,
// Ns = product of the radices already applied), so the result comes out in
// natural order with no bit reversal.  Between stages the values cross the
// threads through LDS; the first stage reads straight from the caller's
// registers and the last stage leaves its outputs in registers, at rows
//   q + Q*b + r*L/R_last       (value v[b*R_last + r]).
// The same row set is what the first stage of a transform in the reversed
// radix order expects, so a forward transform, a pointwise product and an
// inverse in reversed order chain with no exchange at all (the spectral
// product of the demag convolution, paper eq. (13)/(15)).
//
// Twiddles come from a per-length table exp(-2 pi i m / L), m < L, built on
// the host in FP64 and rounded once to FP32.
#pragma once
#include <hip/hip_runtime.h>

// No implicit multiply-add contraction in the transform code: every fused
// multiply-add is written out (cmul), so every schedule of a pass -- tile,
// values per thread, component split -- performs the same operations on every
// element and gives bitwise the same result.
#pragma clang fp contract(off)

namespace mmk {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// a * (-i) for the forward sign (DIR = -1), a * (+i) for the inverse.
template <int DIR>
__device__ __forceinline__ float2 mul_mi(float2 a)
{
    return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

// ------------------------------------------------------------ butterflies ---
template <int DIR>
__device__ __forceinline__ void bfly2(float2 *x)
{
    const float2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
}

template <int DIR>
__device__ __forceinline__ void bfly3(float2 *x)
{
    const float h = 0.86602540378443864676f;  // sqrt(3)/2
    const float2 t1 = cadd(x[1], x[2]);
    const float2 t2 = make_float2(fmaf(-0.5f, t1.x, x[0].x), fmaf(-0.5f, t1.y, x[0].y));
    const float2 t3 = cscale(mul_mi<DIR>(csub(x[1], x[2])), h);
    x[0] = cadd(x[0], t1);
    x[1] = cadd(t2, t3);
    x[2] = csub(t2, t3);
}

// 5-point DFT: with t1 = x1 + x4, t2 = x2 + x3, t3 = x1 - x4, t4 = x2 - x3
// and w = exp(DIR 2 pi i / 5), X1,4 = x0 + c1 t1 + c2 t2 +- DIR i (s1 t3 + s2 t4),
// X2,3 = x0 + c2 t1 + c1 t2 +- DIR i (s2 t3 - s1 t4), where c1, s1 = cos, sin
// of 2 pi/5 and c2, s2 = cos, sin of 4 pi/5 (pairing w^k with w^-k).
template <int DIR>
__device__ __forceinline__ void bfly5(float2 *x)
{
    const float c1 = 0.30901699437494742410f, s1 = 0.95105651629515357212f;
    const float c2 = -0.80901699437494742410f, s2 = 0.58778525229247312917f;
    const float2 t1 = cadd(x[1], x[4]), t2 = cadd(x[2], x[3]);
    const float2 t3 = csub(x[1], x[4]), t4 = csub(x[2], x[3]);
    const float2 a1 = make_float2(fmaf(c2, t2.x, fmaf(c1, t1.x, x[0].x)), fmaf(c2, t2.y, fmaf(c1, t1.y, x[0].y)));
    const float2 a2 = make_float2(fmaf(c1, t2.x, fmaf(c2, t1.x, x[0].x)), fmaf(c1, t2.y, fmaf(c2, t1.y, x[0].y)));
    const float2 b1 = mul_mi<DIR>(make_float2(fmaf(s2, t4.x, s1 * t3.x), fmaf(s2, t4.y, s1 * t3.y)));
    const float2 b2 = mul_mi<DIR>(make_float2(fmaf(-s1, t4.x, s2 * t3.x), fmaf(-s1, t4.y, s2 * t3.y)));
    x[0] = cadd(x[0], cadd(t1, t2));
    x[1] = cadd(a1, b1);
    x[4] = csub(a1, b1);
    x[2] = cadd(a2, b2);
    x[3] = csub(a2, b2);
}

template <int DIR>
__device__ __forceinline__ void bfly4(float2 *x)
{
    const float2 a0 = cadd(x[0], x[2]), a1 = csub(x[0], x[2]);
    const float2 a2 = cadd(x[1], x[3]), a3 = mul_mi<DIR>(csub(x[1], x[3]));
    x[0] = cadd(a0, a2);
    x[2] = csub(a0, a2);
    x[1] = cadd(a1, a3);
    x[3] = csub(a1, a3);
}

template <int DIR>
__device__ __forceinline__ void bfly8(float2 *x)
{
    const float s = 0.70710678118654752440f;
    float2 e[4] = {x[0], x[2], x[4], x[6]};
    float2 o[4] = {x[1], x[3], x[5], x[7]};
    bfly4<DIR>(e);
    bfly4<DIR>(o);
    // o[k] *= exp(DIR * 2 pi i k / 8)
    o[1] = cmul(o[1], make_float2(s, DIR * s));
    o[2] = mul_mi<DIR>(o[2]);
    o[3] = cmul(o[3], make_float2(-s, DIR * s));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        x[k] = cadd(e[k], o[k]);
        x[k + 4] = csub(e[k], o[k]);
    }
}

// 16-point DFT in natural order as 4 x 4: with n = j + 4m and k = k1 + 4k2,
// X[k] = sum_j w16^(j k1) w4^(j k2) (sum_m x[j + 4m] w4^(m k1)).
template <int DIR>
__device__ __forceinline__ void bfly16(float2 *x)
{
    const float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;  // cos, sin of pi/8
    const float h = 0.70710678118654752440f;
    float2 y[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        float2 t[4] = {x[j], x[j + 4], x[j + 8], x[j + 12]};
        bfly4<DIR>(t);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) y[j][k1] = t[k1];
    }
    // w16^(j k1) for j, k1 = 1..3: exponents 1, 2, 3, 2, 4, 6, 3, 6, 9
    const float2 w1 = make_float2(c1, DIR * s1), w2 = make_float2(h, DIR * h), w3 = make_float2(s1, DIR * c1);
    y[1][1] = cmul(y[1][1], w1);
    y[1][2] = cmul(y[1][2], w2);
    y[1][3] = cmul(y[1][3], w3);
    y[2][1] = cmul(y[2][1], w2);
    y[2][2] = mul_mi<DIR>(y[2][2]);
    y[2][3] = cmul(y[2][3], make_float2(-h, DIR * h));
    y[3][1] = cmul(y[3][1], w3);
    y[3][2] = cmul(y[3][2], make_float2(-h, DIR * h));
    y[3][3] = cmul(y[3][3], make_float2(-c1, -DIR * s1));
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        float2 t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
        bfly4<DIR>(t);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) x[k1 + 4 * k2] = t[k2];
    }
}

template <int R, int DIR>
__device__ __forceinline__ void bfly(float2 *x)
{
    if constexpr (R == 2) bfly2<DIR>(x);
    else if constexpr (R == 3) bfly3<DIR>(x);
    else if constexpr (R == 4) bfly4<DIR>(x);
    else if constexpr (R == 5) bfly5<DIR>(x);
    else if constexpr (R == 8) bfly8<DIR>(x);
    else if constexpr (R == 16) bfly16<DIR>(x);
    else static_assert(R == 2 || R == 3 || R == 4 || R == 5 || R == 8 || R == 16, "radix");
}

// ------------------------------------------------- factorisation tables ---
// Radix order O of the forward transform and values per thread E (E must
// be a multiple of every radix; Q = L/E threads share one transform).
// O = 0 is the default; O = 1 and 2 are the alternative orders the product
// pass's autotuner tries (1: radix 16 first, E = 16, for 2^a, and radix 3
// then 4s, E = 12, for 3 2^a; 2: radix 4 only, E = 4, for 2^a).  Orders
// round differently; every schedule of one order is bitwise identical.
template <int L, int O = 0> struct Factors { static constexpr bool valid = false; };
#define MMK_FACTORS(LEN, ORD, EPT, ...)                              \
    template <> struct Factors<LEN, ORD> {                           \
        static constexpr bool valid = true;                          \
        static constexpr int E = EPT;                                \
        static constexpr int R[] = {__VA_ARGS__};                    \
        static constexpr int N = sizeof(R) / sizeof(int);            \
    };
MMK_FACTORS(2, 0, 2, 2)
MMK_FACTORS(4, 0, 4, 4)
MMK_FACTORS(6, 0, 6, 3, 2)
MMK_FACTORS(8, 0, 8, 8)
MMK_FACTORS(12, 0, 12, 3, 4)
MMK_FACTORS(16, 0, 8, 8, 2)
MMK_FACTORS(24, 0, 24, 3, 8)
MMK_FACTORS(32, 0, 8, 8, 4)
MMK_FACTORS(48, 0, 24, 3, 8, 2)
MMK_FACTORS(64, 0, 8, 8, 8)
MMK_FACTORS(96, 0, 24, 3, 8, 4)
MMK_FACTORS(128, 0, 8, 8, 4, 4)
MMK_FACTORS(192, 0, 24, 3, 8, 8)
MMK_FACTORS(256, 0, 8, 8, 8, 4)
MMK_FACTORS(384, 0, 24, 3, 8, 4, 4)
MMK_FACTORS(512, 0, 8, 8, 8, 8)
MMK_FACTORS(768, 0, 24, 3, 8, 8, 4)
MMK_FACTORS(1024, 0, 8, 8, 8, 4, 4)
// 5 2^a: radix 5 then 4s (and a final 2), E = 20
MMK_FACTORS(10, 0, 10, 5, 2)
MMK_FACTORS(20, 0, 20, 5, 4)
MMK_FACTORS(40, 0, 20, 5, 4, 2)
MMK_FACTORS(80, 0, 20, 5, 4, 4)
MMK_FACTORS(160, 0, 20, 5, 4, 4, 2)
MMK_FACTORS(320, 0, 20, 5, 4, 4, 4)
MMK_FACTORS(640, 0, 20, 5, 4, 4, 4, 2)
// radix 16 first (2^a), radix 3 then 4s (3 2^a)
MMK_FACTORS(16, 1, 16, 16)
MMK_FACTORS(24, 1, 12, 3, 4, 2)
MMK_FACTORS(32, 1, 16, 16, 2)
MMK_FACTORS(48, 1, 12, 3, 4, 4)
MMK_FACTORS(64, 1, 16, 16, 4)
MMK_FACTORS(96, 1, 12, 3, 4, 4, 2)
MMK_FACTORS(128, 1, 16, 16, 8)
MMK_FACTORS(192, 1, 12, 3, 4, 4, 4)
MMK_FACTORS(256, 1, 16, 16, 16)
MMK_FACTORS(384, 1, 12, 3, 4, 4, 4, 2)
MMK_FACTORS(512, 1, 16, 16, 8, 4)
MMK_FACTORS(768, 1, 12, 3, 4, 4, 4, 4)
MMK_FACTORS(1024, 1, 16, 16, 16, 4)
// radix 4 only (2^a, E = 4)
MMK_FACTORS(16, 2, 4, 4, 4)
MMK_FACTORS(32, 2, 4, 4, 4, 2)
MMK_FACTORS(64, 2, 4, 4, 4, 4)
MMK_FACTORS(128, 2, 4, 4, 4, 4, 2)
MMK_FACTORS(256, 2, 4, 4, 4, 4, 4)
MMK_FACTORS(512, 2, 4, 4, 4, 4, 4, 2)
MMK_FACTORS(1024, 2, 4, 4, 4, 4, 4, 4)
#undef MMK_FACTORS

template <int L, bool REV, int O = 0>
__device__ __host__ constexpr int radix_at(int s)
{
    return REV ? Factors<L, O>::R[Factors<L, O>::N - 1 - s] : Factors<L, O>::R[s];
}
template <int L, bool REV, int O = 0>
__device__ __host__ constexpr int ns_before(int s)
{
    int p = 1;
    for (int i = 0; i < s; ++i) p *= radix_at<L, REV, O>(i);
    return p;
}
template <int L, bool REV, int O = 0>
__device__ __host__ constexpr int first_radix() { return radix_at<L, REV, O>(0); }
template <int L, bool REV, int O = 0>
__device__ __host__ constexpr int last_radix() { return radix_at<L, REV, O>(Factors<L, O>::N - 1); }

// LDS rows are padded: row r of a transform sits in slot r + r/8 (one spare
// slot after every 8 rows).  The exchanges write with lane strides of R*NS
// rows and read with stride 1; without the spare slots the strided writes
// fall into a few banks.  A transform of L rows takes lds_rows(L) slots.
__host__ __device__ constexpr int lds_rows(int L) { return L + L / 8; }
__device__ __forceinline__ int lds_slot(int r) { return r + (r >> 3); }

// LDS view of a tile of transforms: slot s of this thread's transform at
// base[s * rs + co].
struct LdsView {
    float2 *base;
    int rs;  // stride between slots of one transform
    int co;  // this thread's offset (its transform's column or start)
    __device__ __forceinline__ float2 &at(int slot) const { return base[slot * rs + co]; }
};

// -------------------------------------------------------------- stages ---
// Twiddles of a stage with radix R after NS points: w^(r k L/(NS R)) for
// k < NS, 1 <= r < R, with w = exp(-2 pi i / L).  Flat layout: tw[m] = w^m
// (m < L).  Staged layout (STW): the entries of each stage in the order
// [r - 1][k], stage after stage; stage S (NS > 1) starts at NS - R0 (the
// stages before it hold NS - R0 entries, R0 the first radix), L - R0 in all.
// In a row pass the lanes of a wave are consecutive k of one transform, so
// flat reads stride by r L/(NS R) slots and fall into a few LDS banks; the
// staged reads are consecutive.  Both hold the same values (staged entries
// are copies of flat ones), so the transforms agree bitwise.
template <int L, int E, int R, int NS, int DIR, bool STW = false, int R0 = 1>
__device__ __forceinline__ void stage_compute(float2 (&v)[E], int q, const float2 *__restrict__ tw)
{
    constexpr int Q = L / E;
    constexpr int NB = E / R;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        float2 *x = &v[b * R];
        if constexpr (NS > 1) {
            const int k = (q + Q * b) % NS;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 w = STW ? tw[(NS - R0) + (r - 1) * NS + k] : tw[r * k * (L / (NS * R))];
                if constexpr (DIR > 0) w.y = -w.y;
                x[r] = cmul(x[r], w);
            }
        }
        bfly<R, DIR>(x);
    }
}

// Write the outputs of a stage (radix R, NS) to LDS, then read the inputs
// of the next stage (radix R2).  TRAIL: a second barrier keeps the next
// exchange's writes from overtaking this exchange's reads (not needed when
// the next exchange writes another buffer).
// Where a thread's rows are base + c with c a compile-time offset that never
// carries base into the next group of 8 (c a multiple of 8, or base a
// multiple of R with c < R | 8), slot(base + c) = slot(base) + slot(c) and
// the per-access offsets fold into the LDS instructions.
template <int L, int E, int R, int NS, int R2, bool TRAIL = true>
__device__ __forceinline__ void exchange(float2 (&v)[E], const LdsView &s, int q)
{
    constexpr int Q = L / E;
#pragma unroll
    for (int b = 0; b < E / R; ++b) {
        const int j = q + Q * b;
        const int row = (j / NS) * NS * R + (j % NS);
        if constexpr (NS % 8 == 0 || (NS == 1 && 8 % R == 0)) {
            const int sb = lds_slot(row);
#pragma unroll
            for (int r = 0; r < R; ++r) s.at(sb + r * NS + ((r * NS) >> 3)) = v[b * R + r];
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) s.at(lds_slot(row + r * NS)) = v[b * R + r];
        }
    }
    __syncthreads();
    constexpr int ST = L / R2;
#pragma unroll
    for (int b = 0; b < E / R2; ++b) {
        const int row = q + Q * b;
        if constexpr (ST % 8 == 0) {
            const int sb = lds_slot(row);
#pragma unroll
            for (int r = 0; r < R2; ++r) v[b * R2 + r] = s.at(sb + r * ST + ((r * ST) >> 3));
        } else {
#pragma unroll
            for (int r = 0; r < R2; ++r) v[b * R2 + r] = s.at(lds_slot(row + r * ST));
        }
    }
    if constexpr (TRAIL) __syncthreads();
}

template <int L, int E, int DIR, bool REV, int S, int O = 0, bool STW = false>
__device__ __forceinline__ void run_stages(float2 (&v)[E], const LdsView &s, int q,
                                           const float2 *__restrict__ tw)
{
    constexpr int R = radix_at<L, REV, O>(S);
    constexpr int NS = ns_before<L, REV, O>(S);
    stage_compute<L, E, R, NS, DIR, STW, first_radix<L, REV, O>()>(v, q, tw);
    if constexpr (S + 1 < Factors<L, O>::N) {
        constexpr int R2 = radix_at<L, REV, O>(S + 1);
        exchange<L, E, R, NS, R2>(v, s, q);
        run_stages<L, E, DIR, REV, S + 1, O, STW>(v, s, q, tw);
    }
}

// Fill the staged twiddle table (stage_compute) of length L in radix order
// O (stages in forward order) into `out` from the flat table `tw`: every
// thread of the workgroup takes entries threadIdx.x, + blockDim.x, ...
template <int L, int O, int S = 1>
__device__ __forceinline__ void fill_staged_one(float2 *out, const float2 *__restrict__ tw, int i)
{
    if constexpr (S < Factors<L, O>::N) {
        constexpr int R = radix_at<L, false, O>(S), NS = ns_before<L, false, O>(S);
        constexpr int lo = NS - first_radix<L, false, O>(), hi = lo + NS * (R - 1);
        if (i < hi) {
            const int loc = i - lo;
            const int r = 1 + loc / NS, k = loc % NS;
            out[i] = tw[r * k * (L / (NS * R))];
        } else {
            fill_staged_one<L, O, S + 1>(out, tw, i);
        }
    }
}
template <int L, int O>
__device__ __forceinline__ void fill_staged_twiddles(float2 *out, const float2 *__restrict__ tw)
{
    for (int i = threadIdx.x; i < L - first_radix<L, false, O>(); i += blockDim.x) fill_staged_one<L, O>(out, tw, i);
}

// Ping-pong form: exchange S uses buffer S mod 2, so only one barrier per
// exchange is needed; exchange k + 2 rewrites a buffer only after every
// thread has passed exchange k + 1's barrier, which follows its reads of
// exchange k.  The last exchange keeps its trailing barrier when it uses
// buffer 0 (an odd number of exchanges), since the next transform's first
// exchange writes buffer 0 again.  The caller must not write either buffer
// between transforms without a barrier.
template <int L, int E, int DIR, bool REV, int S, int O = 0>
__device__ __forceinline__ void run_stages_pp(float2 (&v)[E], const LdsView &s0, const LdsView &s1, int q,
                                              const float2 *__restrict__ tw)
{
    constexpr int R = radix_at<L, REV, O>(S);
    constexpr int NS = ns_before<L, REV, O>(S);
    constexpr int N = Factors<L, O>::N;
    stage_compute<L, E, R, NS, DIR>(v, q, tw);
    if constexpr (S + 1 < N) {
        constexpr int R2 = radix_at<L, REV, O>(S + 1);
        constexpr bool TRAIL = S == N - 2 && S % 2 == 0;
        exchange<L, E, R, NS, R2, TRAIL>(v, S % 2 ? s1 : s0, q);
        run_stages_pp<L, E, DIR, REV, S + 1, O>(v, s0, s1, q, tw);
    }
}

template <int L, int DIR, bool REV, int O = 0, int E>
__device__ __forceinline__ void fft_pp(float2 (&v)[E], const LdsView &s0, const LdsView &s1, int q,
                                       const float2 *__restrict__ tw)
{
    static_assert(E == Factors<L, O>::E, "values per thread of the radix order");
    run_stages_pp<L, E, DIR, REV, 0, O>(v, s0, s1, q, tw);
}

// Full transform with E values per thread (E a multiple of every radix of
// L; Q = L/E threads per transform).  On entry v[b*R0 + r] holds row
// q + Q*b + r*L/R0 with R0 = first_radix<L,REV>; on exit v[b*RL + r] holds
// row q + Q*b + r*L/RL with RL = last_radix<L,REV>.  Every thread of the
// workgroup must call it (it contains barriers when the transform has more
// than one stage).
template <int L, int E, int DIR, bool REV, int O = 0, bool STW = false>
__device__ __forceinline__ void fft_e(float2 (&v)[E], const LdsView &s, int q, const float2 *__restrict__ tw)
{
    static_assert(!STW || !REV, "the staged twiddle table holds the forward stage order");
    run_stages<L, E, DIR, REV, 0, O, STW>(v, s, q, tw);
}

template <int L, int DIR, bool REV>
__device__ __forceinline__ void fft(float2 (&v)[Factors<L>::E], const LdsView &s, int q,
                                    const float2 *__restrict__ tw)
{
    run_stages<L, Factors<L>::E, DIR, REV, 0>(v, s, q, tw);
}

// Values per thread of variant V of length L: V = 0 the default E, V = 1
// twice as many (half the threads per transform, wider tiles per workgroup).
// Schedule variant V of a single-component pass: 0 = order 0 with E values
// per thread, 1 = order 0 with 2E, 2 = order 1, 3 = order 2 (each with its
// own E).  order_of_v gives the radix order, ept the values per thread.
template <int V> constexpr int order_of_v() { return V == 2 ? 1 : (V == 3 ? 2 : 0); }
template <int L, int V> constexpr int ept()
{
    if constexpr (V == 2 && Factors<L, 1>::valid) return Factors<L, 1>::E;
    else if constexpr (V == 3 && Factors<L, 2>::valid) return Factors<L, 2>::E;
    else return (V == 1 && 2 * Factors<L>::E <= L) ? 2 * Factors<L>::E : Factors<L>::E;
}
template <int L, int V> constexpr bool variant_valid()
{
    if constexpr (V == 2) return Factors<L, 1>::valid;
    else if constexpr (V == 3) return Factors<L, 2>::valid;
    else if constexpr (V == 1) return 2 * Factors<L>::E <= L;
    else return true;
}

}  // namespace mmk
