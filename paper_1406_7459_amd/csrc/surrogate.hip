// surrogate.hip -- learned demag increment for the intermediate RK stages.
//
// A stack of six 3x3x3 convolutions (3 -> 32 -> 32 -> 32 -> 32 -> 32 -> 3
// channels, zero "same" padding, a bias per output channel, GELU (tanh form)
// after all but the last) maps a magnetisation increment dm to a demag-field
// increment dh.  Demag is linear, so in RK stages 2-4 the field is taken as
//   H(M_s) = H_d(M_n) + Ms * sigma * Net((M_s - M_n) / (Ms sigma)),
// sigma = rms of the increment (the exact stage-1 field anchors it).
//
// Matrix-core path: activations are bfloat16, channel-last [cell][32]; a
// convolution is an implicit GEMM (rows = output channels, columns = 16
// cells, K = 32 input channels per tap, 27 taps) on v_mfma_f32_16x16x32_bf16
// with FP32 accumulation.  Layers with 3 channels are zero-padded to 32.
// The input gradient reuses the same kernel with the weights transposed and
// the taps mirrored (its epilogue applies the GELU derivative of the layer
// below); the weight gradient is an MFMA reduction over cells of
// channel-major copies of dZ and of the layer input.  Training keeps FP32
// master weights and Adam moments; the bfloat16 copies are refreshed after
// every update, and every reduction runs in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "mm_internal.hpp"

namespace mmk {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int SC = 32;       // padded channel count
constexpr int NT = 27;       // taps
constexpr int NLAYER = 6;
constexpr int WSZ = SC * NT * SC;  // weights per padded layer
static const int CH[NLAYER + 1] = {3, 32, 32, 32, 32, 32, 3};

// GELU, tanh form: 0.5 x (1 + tanh(u)) with u = sqrt(2/pi) (x + 0.044715 x^3),
// evaluated as x * s with s = 1 / (1 + e^(-2u)) (the same function; one
// exponential and one reciprocal instead of a tanh), and its derivative
// s + 2 x s (1 - s) u'.  e^(-2u) = 2^(x (k1 + k3 x^2)) with the constants
// folded (k1 = -2 sqrt(2/pi) log2(e), k3 = 0.044715 k1): one multiply, one
// fma and one multiply before the base-2 exponential.
__device__ __forceinline__ float gelu_s(float x, float &du)
{
    constexpr float c = 0.7978845608028654f;  // sqrt(2/pi)
    constexpr float k1 = (float)(-2.0 * 0.7978845608028654 * 1.4426950408889634);
    constexpr float k3 = (float)(0.044715 * -2.0 * 0.7978845608028654 * 1.4426950408889634);
    const float x2 = x * x;
    du = c * (1.f + 3.f * 0.044715f * x2);
    return __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(x * __builtin_fmaf(k3, x2, k1)));
}
__device__ __forceinline__ float gelu_f(float x)
{
    float du;
    return x * gelu_s(x, du);
}
__device__ __forceinline__ float gelu_d(float x)
{
    float du;
    const float s = gelu_s(x, du);
    return s + 2.f * x * s * (1.f - s) * du;
}

// EPI 0: hidden layer, Zh = bf16(acc + b) and Xn = bf16(gelu(acc + b));
// EPI 1: last layer, dh[co][cell] = s * (acc + b) for co < 3 (SoA FP32),
//        s = sig[0] if sig is given (device sigma) else scale, and (training,
//        Z given) Z[cell][co] = acc + b in [N][4];
// EPI 2: input gradient fused with the GELU derivative of the layer below:
//        dZ_prev = acc * gelu'(Zp) with Zp = Zh (read, the bf16 pre-activations
//        of the layer below), written as bf16 cell-major Xn and channel-major Xt;
// EPI 3: hidden layer for inference only, Xn = bf16(gelu(acc + b)) (no Z).
//
// A wave owns a 16-cell run along x at one y and TZ = 4 consecutive z levels
// (four column tiles), for all 32 output channels (two accumulators per
// tile).  For each in-plane offset (dx, dy) it loads the six source rows
// z0-1 .. z0+4 once and applies each to every output level it reaches
// (dz = -1, 0, 1): 13.5 activation loads per tile instead of 27, and each
// weight fragment read from LDS feeds up to eight MFMAs.  The loads of the
// next offset are issued before the current offset's MFMAs.  A block at the
// bottom (top) of the grid has no source row z0-1 (z0+4): that row is
// neither loaded nor multiplied (separate instances of the task body, so
// that the load counts stay static), and a 4-level film does 9 loads per
// tile and 5/6 of the MFMAs of an interior block.  The last layer has 3
// output channels: rows 16..31 of its weights are zero and are neither
// staged nor multiplied.  Eight waves share one copy of the layer's weights
// in LDS (55 KB, rows padded to stagger the banks), so two workgroups
// (sixteen waves) fit a CU.
constexpr int TZ = 4;
constexpr int CONV_WAVES = 8;
constexpr int WROW = NT * 4 + 1;  // 16-byte slots per output channel in LDS

// fragments travel as raw 16-byte words (a bf16 vector in a phi or a select
// is repacked element by element) and become bf16 at the MFMA
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

// Channel-major, zero-padded copies of the layer inputs and of dZ, kept for
// the weight gradient (training only).  Element (ch, x, y, z) sits at
// ch * G + f + (z + 1) pl + y xp + x with xp = roundup(nx + 1, 8) (a zero
// after every row), pl = (ny + 1) xp (a zero row after every level), a zero
// level below and above the grid and at least xp + 8 zeros at both ends:
// every neighbour of every cell and of every padding cell lies inside the
// buffer, the ones outside the grid read zero, and rows start on 16 bytes.
struct PadGeom {
    int xp, pl, f;
    long long G;  // elements per channel, a multiple of 8
};
static inline PadGeom pad_geom(int nx, int ny, int nz)
{
    PadGeom g;
    g.xp = (nx + 1 + 7) & ~7;
    g.pl = (ny + 1) * g.xp;
    g.f = g.xp + 8;
    g.G = ((long long)g.f + (long long)(nz + 2) * g.pl + g.xp + 80 + 7) & ~7LL;
    return g;
}
__device__ __forceinline__ long long pad_at(const PadGeom &g, int x, int y, int z)
{
    return g.f + (long long)(z + 1) * g.pl + (long long)y * g.xp + x;
}

// Epilogue of a hidden layer at one cell c = (x, y, z): lane group kq holds
// the accumulators of output channels 4 kq + r (a0) and 16 + 4 kq + r (a1),
// b0/b1 their biases.  Xn = bf16(gelu(acc + b)); EPI 0 (training) also
// writes the bf16 pre-activations Zh and the channel-major copy Xt of Xn.
template <int EPI>
__device__ __forceinline__ void hidden_out(const f4 &a0, const f4 &a1, const f4 &b0, const f4 &b1, long long c,
                                           int kq, __bf16 *__restrict__ Zh, __bf16 *__restrict__ Xn,
                                           __bf16 *__restrict__ Xt, const PadGeom &pg, int x, int y, int z)
{
    f4 z0v, z1v;
    bf4 g0, g1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        z0v[r] = a0[r] + b0[r];
        z1v[r] = a1[r] + b1[r];
        g0[r] = (__bf16)gelu_f(z0v[r]);
        g1[r] = (__bf16)gelu_f(z1v[r]);
    }
    if constexpr (EPI == 0) {
        bf4 h0, h1;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            h0[r] = (__bf16)z0v[r];
            h1[r] = (__bf16)z1v[r];
        }
        *reinterpret_cast<bf4 *>(Zh + c * SC + 4 * kq) = h0;
        *reinterpret_cast<bf4 *>(Zh + c * SC + 16 + 4 * kq) = h1;
        const long long pc = pad_at(pg, x, y, z);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Xt[(long long)(4 * kq + r) * pg.G + pc] = g0[r];
            Xt[(long long)(16 + 4 * kq + r) * pg.G + pc] = g1[r];
        }
    }
    *reinterpret_cast<bf4 *>(Xn + c * SC + 4 * kq) = g0;
    *reinterpret_cast<bf4 *>(Xn + c * SC + 16 + 4 * kq) = g1;
}

// One launch covers the z blocks zb0 .. zb0+nzbr-1 of one kind: ZLO (the
// block starts at z = 0) and ZHI (it reaches the top level).
template <int EPI, bool ZLO, bool ZHI>
__global__ __launch_bounds__(64 * CONV_WAVES) __attribute__((amdgpu_waves_per_eu(4))) void k_conv(
    const __bf16 *__restrict__ X, const __bf16 *__restrict__ W, const float *__restrict__ bias, float *__restrict__ Z,
    __bf16 *__restrict__ Zh, __bf16 *__restrict__ Xn, float *__restrict__ dh, float scale,
    const float *__restrict__ sig, int nx, int ny, int nz, int zb0, int nzbr, __bf16 *__restrict__ Xt, PadGeom pg)
{
    constexpr bool HALF = EPI == 1;
    constexpr int NCO = HALF ? 16 : 32;
    constexpr int J0 = ZLO ? 1 : 0, J1 = ZHI ? TZ + 1 : TZ + 2;  // source rows that exist
    __shared__ u4 wl[NCO * WROW];
    {
        // every load of the staging is issued before the first LDS write (a
        // load-wait-write loop would pay the load latency once per round)
        constexpr int NW = NCO * NT * 4, ROUNDS = (NW + 64 * CONV_WAVES - 1) / (64 * CONV_WAVES);
        const u4 *Wv = reinterpret_cast<const u4 *>(W);
        u4 tmp[ROUNDS];
#pragma unroll
        for (int k = 0; k < ROUNDS; ++k) {
            const int i = threadIdx.x + k * 64 * CONV_WAVES;
            if (i < NW) tmp[k] = Wv[i];
        }
#pragma unroll
        for (int k = 0; k < ROUNDS; ++k) {
            const int i = threadIdx.x + k * 64 * CONV_WAVES;
            const int co = i / (NT * 4);
            if (i < NW) wl[co * WROW + (i - co * NT * 4)] = tmp[k];
        }
    }
    __syncthreads();
    // the wave index is uniform: read it into a scalar so that the task
    // coordinates, the validity flags and the row offsets live in SGPRs
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int col = lane & 15, kq = lane >> 4;
    const int nxt = (nx + 15) >> 4;
    const long long ntask = (long long)nxt * ny * nzbr;
    const u4 zero = {0u, 0u, 0u, 0u};
    const u4 *wa = wl + col * WROW + kq;
    // raw buffer over the activations (byte size <= 2^31, checked by the host);
    // an offset past the end reads as zero
    const __amdgpu_buffer_rsrc_t src = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<__bf16 *>(X), 0, (int)((long long)nx * ny * nz * SC * 2), 0x00020000);
    const unsigned OUT_OF_RANGE = 0x80000000u;
    // the lane's biases are loaded once, ahead of the tasks
    f4 bia0 = {0.f, 0.f, 0.f, 0.f}, bia1 = {0.f, 0.f, 0.f, 0.f};
    if constexpr (EPI == 0 || EPI == 3) {
        bia0 = *reinterpret_cast<const f4 *>(bias + 4 * kq);
        bia1 = *reinterpret_cast<const f4 *>(bias + 16 + 4 * kq);
    } else if constexpr (EPI == 1) {
        bia0 = *reinterpret_cast<const f4 *>(bias);
    }
    // XCD-contiguous workgroup order: the rows y-1..y+1 and levels z0-1..z0+4
    // a task reads were read by its neighbours in the same L2
    for (long long task = (long long)xcd_block(blockIdx.x, gridDim.x) * CONV_WAVES + wv; task < ntask;
         task += (long long)gridDim.x * CONV_WAVES) {
        const int xt = (int)(task % nxt);
        const long long rest = task / nxt;
        const int y = (int)(rest % ny);
        const int z0 = (zb0 + (int)(rest / ny)) * TZ;
        const int x = xt * 16 + col;
        // an index the compiler cannot see through keeps the weight reads
        // inside the task loop (hoisted, 54 fragments would not fit the registers)
        int wofs = 0;
        asm volatile("" : "+v"(wofs));
        const u4 *wt = wa + wofs;
        f4 acc0[TZ], acc1[TZ];
#pragma unroll
        for (int u = 0; u < TZ; ++u) {
            acc0[u] = f4{0.f, 0.f, 0.f, 0.f};
            acc1[u] = f4{0.f, 0.f, 0.f, 0.f};
        }
        // uniform validity of the source levels z0-1+j and the rows y-1..y+1;
        // a row outside the grid loads as zero, so its MFMAs add nothing
        bool vz[TZ + 2], vy[3];
#pragma unroll
        for (int j = 0; j < TZ + 2; ++j) vz[j] = z0 - 1 + j >= 0 && z0 - 1 + j < nz;
#pragma unroll
        for (int d = 0; d < 3; ++d) vy[d] = y - 1 + d >= 0 && y - 1 + d < ny;
        // byte offset of the lane's cell within a row, per dx; a lane whose
        // neighbour lies outside the row reads past the end of the buffer
        unsigned xo[3];
        bool vx[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int xx = x - 1 + d;
            vx[d] = xx >= 0 && xx < nx;
            xo[d] = (unsigned)(xx * SC + 8 * kq) * 2u;
        }
        const int rs = nx * SC, ps = rs * ny;  // elements per row and per level
        // source rows of offset g = 3 (dy + 1) + (dx + 1), levels z0-1+j
        auto fetch = [&](int g, u4 *s) {
            const int dy = g / 3, dx = g % 3;
#pragma unroll
            for (int j = J0; j < J1; ++j) {
                const bool ok = vy[dy] && vz[j] && vx[dx];
                const unsigned row = (unsigned)((z0 - 1 + j) * ps + (y - 1 + dy) * rs) * 2u;
                s[j] = __builtin_amdgcn_raw_buffer_load_b128(src, ok ? row + xo[dx] : OUT_OF_RANGE, 0, 0);
            }
        };
        // loads run PF offsets ahead of the MFMAs, in a ring of PF + 1 row sets
        // (two ahead in the inference forms when a block loads only four
        // source rows, one otherwise: the registers of a deeper ring are not
        // there)
        constexpr int PF = (EPI == 1 || EPI == 3) && J1 - J0 <= 4 ? 2 : 1;
        u4 ring[PF + 1][TZ + 2];
#pragma unroll
        for (int g = 0; g < PF; ++g) fetch(g, ring[g]);
#pragma unroll
        for (int g = 0; g < 9; ++g) {
            if (g + PF < 9) fetch(g + PF, ring[(g + PF) % (PF + 1)]);
            const u4 *cur = ring[g % (PF + 1)];
#pragma unroll
            for (int dz = -1; dz <= 1; ++dz) {
                const int t = (dz + 1) * 9 + g;
                const bf8 a0 = __builtin_bit_cast(bf8, wt[t * 4]);
                const bf8 a1 = __builtin_bit_cast(bf8, HALF ? zero : wt[16 * WROW + t * 4]);
#pragma unroll
                for (int u = 0; u < TZ; ++u) {
                    const int j = u + dz + 1;
                    if (j < J0 || j >= J1) continue;
                    const bf8 bv = __builtin_bit_cast(bf8, cur[j]);
                    acc0[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bv, acc0[u], 0, 0, 0);
                    if (!HALF) acc1[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bv, acc1[u], 0, 0, 0);
                }
            }
            // keep the ring's distance (the scheduler would otherwise hoist
            // further loads and run out of registers)
            __builtin_amdgcn_sched_barrier(0);
        }
        if (x >= nx) continue;
        // lane holds D[co = 4 kq + r][cell] (acc0) and D[16 + 4 kq + r][cell] (acc1)
#pragma unroll
        for (int u = 0; u < TZ; ++u) {
            if (z0 + u >= nz) break;
            const long long c = ((long long)(z0 + u) * ny + y) * nx + x;
            if constexpr (EPI == 0 || EPI == 3) {
                hidden_out<EPI>(acc0[u], acc1[u], bia0, bia1, c, kq, Zh, Xn, Xt, pg, x, y, z0 + u);
            } else if constexpr (EPI == 1) {
                if (kq == 0) {
                    const long long N = (long long)nx * ny * nz;
                    const float s = sig ? sig[0] : scale;
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        const float z = acc0[u][r] + bia0[r];
                        if (Z) Z[c * 4 + r] = z;  // training only
                        dh[r * N + c] = s * z;
                    }
                }
            } else {
                const bf4 z0v = *reinterpret_cast<const bf4 *>(Zh + c * SC + 4 * kq);
                const bf4 z1v = *reinterpret_cast<const bf4 *>(Zh + c * SC + 16 + 4 * kq);
                bf4 g0, g1;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    g0[r] = (__bf16)(acc0[u][r] * gelu_d((float)z0v[r]));
                    g1[r] = (__bf16)(acc1[u][r] * gelu_d((float)z1v[r]));
                }
                *reinterpret_cast<bf4 *>(Xn + c * SC + 4 * kq) = g0;
                *reinterpret_cast<bf4 *>(Xn + c * SC + 16 + 4 * kq) = g1;
                const long long pc = pad_at(pg, x, y, z0 + u);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    Xt[(long long)(4 * kq + r) * pg.G + pc] = g0[r];
                    Xt[(long long)(16 + 4 * kq + r) * pg.G + pc] = g1[r];
                }
            }
        }
    }
}

// First layer.  Its input has 3 live channels, so a K step of 32 channels
// per tap would multiply 29 zeros; here K packs four taps of 8 channels
// (channels 0..7 of the input, 3..7 zero): lane group kq takes tap 4 s + kq
// in step s, so the 27 taps need 7 MFMA steps per output half instead of 27
// (tap 27 carries zero weights).  The input is stored zero-padded (PadGeom
// positions, 8 channels = 16 bytes each), so every neighbour of a cell,
// inside the grid or not, is one unmasked load, and a lane's 7 tap offsets
// are fixed for the whole kernel: a load is a scalar level base plus a
// constant per-lane offset.  A wave keeps its 14 weight fragments in
// registers and walks (16-cell x run, y, TZ-level block) tasks, level by
// level, with the next level's 7 loads in flight during the current level's
// 14 MFMAs.  Levels past the top of the grid (a ragged last block) reload the
// top level and store nothing; x positions past the row's end read padding or
// the next row and store nothing.
constexpr int IN_CH = 8;                 // channels per position of the padded input
constexpr int IN_KS = (NT + 3) / 4;      // K steps of the packed first layer
constexpr int IN_WAVES = 4;

template <int EPI>
__global__ __launch_bounds__(64 * IN_WAVES) void k_conv_in(const __bf16 *__restrict__ Xin,
                                                          const __bf16 *__restrict__ W,
                                                          const float *__restrict__ bias, __bf16 *__restrict__ Zh,
                                                          __bf16 *__restrict__ Xn, __bf16 *__restrict__ Xt, PadGeom pg,
                                                          int nx, int ny, int nz)
{
    static_assert(EPI == 0 || EPI == 3, "the first layer is a hidden layer");
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int col = lane & 15, kq = lane >> 4;
    const u4 zero = {0u, 0u, 0u, 0u};
    // weight fragments W[co][t][0..7] of both output halves, and the byte
    // offset of the tap's neighbour from the lane's cell, biased by
    // pl + xp + 1 positions so that it is never negative
    u4 wlo[IN_KS], whi[IN_KS];
    unsigned vo[IN_KS];
    const int bias_pos = pg.pl + pg.xp + 1;
#pragma unroll
    for (int st = 0; st < IN_KS; ++st) {
        const int t = 4 * st + kq, tc = t < NT ? t : NT - 1;
        const u4 a = *reinterpret_cast<const u4 *>(W + (long long)(col * NT + tc) * SC);
        const u4 b = *reinterpret_cast<const u4 *>(W + (long long)((16 + col) * NT + tc) * SC);
        wlo[st] = t < NT ? a : zero;
        whi[st] = t < NT ? b : zero;
        const int dz = tc / 9 - 1, dy = (tc % 9) / 3 - 1, dx = tc % 3 - 1;
        const int d = t < NT ? dz * pg.pl + dy * pg.xp + dx : 0;
        vo[st] = (unsigned)(col + d + bias_pos) * (unsigned)(IN_CH * 2);
    }
    const f4 bia0 = *reinterpret_cast<const f4 *>(bias + 4 * kq);
    const f4 bia1 = *reinterpret_cast<const f4 *>(bias + 16 + 4 * kq);
    // task indices fit 32 bits (at most one task per cell, 2^25 cells)
    const unsigned nxt = (unsigned)(nx + 15) >> 4, nzb = (unsigned)(nz + TZ - 1) / TZ;
    const unsigned ntask = nxt * (unsigned)ny * nzb;
    const char *base = reinterpret_cast<const char *>(Xin);
    for (unsigned task = xcd_block(blockIdx.x, gridDim.x) * IN_WAVES + wv; task < ntask;
         task += gridDim.x * IN_WAVES) {
        const int xt = (int)(task % nxt);
        const unsigned rest = task / nxt;
        const int y = (int)(rest % (unsigned)ny);
        const int z0 = (int)(rest / (unsigned)ny) * TZ;
        const int x = xt * 16 + col;
        // the 7 fragments of level z0 + u (clamped to the grid), from the
        // run's first position less the bias
        auto fetch = [&](int u, u4 *b) {
            const int zu = z0 + u < nz ? z0 + u : nz - 1;
            const char *lv = base + (pad_at(pg, xt * 16, y, zu) - bias_pos) * (IN_CH * 2);
#pragma unroll
            for (int st = 0; st < IN_KS; ++st) b[st] = *reinterpret_cast<const u4 *>(lv + vo[st]);
        };
        u4 ring[2][IN_KS];
        fetch(0, ring[0]);
#pragma unroll
        for (int u = 0; u < TZ; ++u) {
            if (u + 1 < TZ) fetch(u + 1, ring[(u + 1) & 1]);
            f4 a0 = {0.f, 0.f, 0.f, 0.f}, a1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int st = 0; st < IN_KS; ++st) {
                const bf8 bv = __builtin_bit_cast(bf8, ring[u & 1][st]);
                a0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, wlo[st]), bv, a0, 0, 0, 0);
                a1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, whi[st]), bv, a1, 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
            if (x < nx && z0 + u < nz)
                hidden_out<EPI>(a0, a1, bia0, bia1, ((long long)(z0 + u) * ny + y) * nx + x, kq, Zh, Xn, Xt, pg, x,
                                y, z0 + u);
        }
    }
}

// sigma = sqrt(sum / count) from the nb FP64 partials of the sum of squares
// (1 if the sum is 0 or normalisation is off), in a fixed order (a strided
// sum per thread, then a tree; 256 threads), then dm [3][N] FP32 (SoA) *
// (1/sigma) -> the first layer's zero-padded input, 8 bf16 channels at each
// PadGeom position (channels 3..7 zero; the positions outside the grid are
// zeroed once at creation and never written).
// Every workgroup forms sigma itself (4 KB of partials from L2, no extra
// launch); workgroup 0 stores sig = {sigma, 1/sigma} for the later kernels
// (the step driver never synchronises for it).
// (training: also channels 0..2 of the channel-major copy Xt)
__global__ __launch_bounds__(256) void k_to_cl_dev(const float *__restrict__ dm, __bf16 *__restrict__ X,
                                                   const double *__restrict__ part, int nb, double count,
                                                   int normalize, float *__restrict__ sig, long long N,
                                                   __bf16 *__restrict__ Xt, PadGeom pg, int nx, int ny)
{
    __shared__ double red[256];
    __shared__ float s_inv;
    double t = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) t += part[b];
    red[threadIdx.x] = t;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double sg = normalize ? sqrt(red[0] / count) : 1.0;
        if (!(sg > 0.0) || !isfinite(sg)) sg = 1.0;
        const float inv_sg = (float)(1.0 / sg);
        if (blockIdx.x == 0) {
            sig[0] = (float)sg;
            sig[1] = inv_sg;
        }
        s_inv = inv_sg;
    }
    __syncthreads();
    const float inv = s_inv;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long long)gridDim.x * blockDim.x) {
        bf8 v = {0, 0, 0, 0, 0, 0, 0, 0};
        v[0] = (__bf16)(dm[c] * inv);
        v[1] = (__bf16)(dm[N + c] * inv);
        v[2] = (__bf16)(dm[2 * N + c] * inv);
        const long long pc = pad_at(pg, (int)(c % nx), (int)((c / nx) % ny), (int)(c / ((long long)nx * ny)));
        *reinterpret_cast<bf8 *>(X + pc * IN_CH) = v;
        if (Xt) {
#pragma unroll
            for (int r = 0; r < 3; ++r) Xt[r * pg.G + pc] = v[r];
        }
    }
}

// last-layer gradient: dZ = 2 (z - target/scale) / (3N) on co < 3, as bf16
// cell-major dZb and channel-major dZt (buffers of the last layer only, whose
// padded channels are zeroed once at creation and never written); squared
// error partials (FP64) per block
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ Z, const float *__restrict__ tgt, float inv,
                                             __bf16 *__restrict__ dZb, __bf16 *__restrict__ dZt, PadGeom pg,
                                             double *__restrict__ part, int nx, int ny, long long N)
{
    double s = 0.0;
    const float w = 2.f / (3.f * (float)N);
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long long)gridDim.x * blockDim.x) {
        const long long pc = pad_at(pg, (int)(c % nx), (int)((c / nx) % ny), (int)(c / ((long long)nx * ny)));
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const float d = Z[c * 4 + r] - tgt[r * N + c] * inv;
            s += (double)d * d;
            const __bf16 g = (__bf16)(w * d);
            dZb[c * SC + r] = g;
            dZt[r * pg.G + pc] = g;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    __shared__ double sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Weight and bias gradient partials of one layer on the matrix cores:
//   part[block][co][t][ci] = sum_cells dZ[cell][co] X[cell + off(t)][ci],
//   part[block][WSZ + co] = sum_cells dZ[cell][co]
// (each workgroup's row has the layout of one layer's parameters).
// The reduction runs over cells, so the MFMA's K is a run of 32 consecutive
// padded positions of the channel-major copies (one 16-byte chunk of 8 cells
// per lane): A = dZ of 16 output channels, B = X of 16 input channels at the
// source row of (dy, dz).  The dx = -1 and +1 fragments are the dx = 0 one
// shifted by one cell, funnel-shifted from a window of cells -2 .. 9 around
// the lane's chunk (one 16-byte and one 8-byte load).  A wave owns one input
// half and one part of the taps (source rows 0-4 or 5-8, i.e. 15 or 12 taps)
// for both output halves, so each source window is loaded by two waves of a
// group and reused for two output halves (the loads, each touching 16
// channel rows, bound this kernel).  Four waves cover the 32 x 32 x 27
// block; the two groups of four in a workgroup take alternate runs of the
// workgroup's contiguous range (XCD-contiguous order) and meet in LDS.  A
// run's loads are issued one run ahead.  Padding positions carry dZ = 0, so
// whole runs need no masks.
constexpr int DW_BLOCKS = 256;
constexpr int DW_ROUND = 10;  // accumulator tiles handed over through LDS per round
// a window of cells -2 .. 9 is 4-byte aligned
typedef unsigned int u4w __attribute__((ext_vector_type(4), aligned(4)));
typedef unsigned int u2w __attribute__((ext_vector_type(2), aligned(4)));
struct DwWin {
    u4w lo;  // cells -2 .. 5
    u2w hi;  // cells 6 .. 9
};

template <int TH>
__device__ __forceinline__ void dw_wave(const __bf16 *__restrict__ dZt, const __bf16 *__restrict__ Xt,
                                        float *__restrict__ part, const PadGeom &pg, int nruns, int gq, int grp,
                                        int w, f4 (*red)[DW_ROUND][64], float (*bred)[2][4][16])
{
    constexpr int SR0 = TH ? 5 : 0, NR = TH ? 4 : 5, NTT = 3 * NR;  // source rows, taps
    const int lane = threadIdx.x & 63, m = lane & 15, kq = lane >> 4;
    const __bf16 *A0 = dZt + (long long)m * pg.G + 8 * kq;  // output channels m and 16 + m
    const __bf16 *A1 = A0 + 16 * pg.G;
    const __bf16 *B = Xt + (long long)(16 * gq + m) * pg.G + 8 * kq;
    long long roff[NR];  // source row offsets of (dz, dy)
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int sr = SR0 + i;
        roff[i] = (long long)(sr / 3 - 1) * pg.pl + (long long)(sr % 3 - 1) * pg.xp;
    }
    f4 acc[2][NTT];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh)
#pragma unroll
        for (int t = 0; t < NTT; ++t) acc[hh][t] = f4{0.f, 0.f, 0.f, 0.f};
    float bs0 = 0.f, bs1 = 0.f;
    const int per = (nruns + gridDim.x - 1) / gridDim.x;
    const int rb = (int)xcd_block(blockIdx.x, gridDim.x) * per, re = min(nruns, rb + per);
    auto fetch = [&](int r, u4 &a0, u4 &a1, DwWin *win) {
        const long long p = (long long)pg.f + pg.pl + 32LL * r;
        a0 = *reinterpret_cast<const u4 *>(A0 + p);
        a1 = *reinterpret_cast<const u4 *>(A1 + p);
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            win[i].lo = *reinterpret_cast<const u4w *>(B + p + roff[i] - 2);
            win[i].hi = *reinterpret_cast<const u2w *>(B + p + roff[i] + 6);
        }
    };
    // the next run's loads are made opaque at the end of the iteration (kept
    // in flight across this run's MFMAs, not moved to the top of the next
    // iteration); the last prefetch repeats a valid run
    int r = rb + grp;
    DwWin win[NR];
    u4 a0 = {0u, 0u, 0u, 0u}, a1 = {0u, 0u, 0u, 0u};
    if (r < re) fetch(r, a0, a1, win);
    for (; r < re; r += 2) {
        u4 an0, an1;
        DwWin nw[NR];
        fetch(min(r + 2, re - 1), an0, an1, nw);
        if (TH == 0 && gq == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                bs0 += __uint_as_float(a0[i] << 16) + __uint_as_float(a0[i] & 0xffff0000u);
                bs1 += __uint_as_float(a1[i] << 16) + __uint_as_float(a1[i] & 0xffff0000u);
            }
        }
        const bf8 av0 = __builtin_bit_cast(bf8, a0), av1 = __builtin_bit_cast(bf8, a1);
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const unsigned d0 = win[i].lo[0], d1 = win[i].lo[1], d2 = win[i].lo[2], d3 = win[i].lo[3];
            const unsigned d4 = win[i].hi[0], d5 = win[i].hi[1];
            const bf8 bc = __builtin_bit_cast(bf8, u4{d1, d2, d3, d4});
            const bf8 bm = __builtin_bit_cast(
                bf8, u4{__builtin_amdgcn_alignbit(d1, d0, 16), __builtin_amdgcn_alignbit(d2, d1, 16),
                        __builtin_amdgcn_alignbit(d3, d2, 16), __builtin_amdgcn_alignbit(d4, d3, 16)});
            const bf8 bp = __builtin_bit_cast(
                bf8, u4{__builtin_amdgcn_alignbit(d2, d1, 16), __builtin_amdgcn_alignbit(d3, d2, 16),
                        __builtin_amdgcn_alignbit(d4, d3, 16), __builtin_amdgcn_alignbit(d5, d4, 16)});
            const int t0 = 3 * i;  // local tap (dx = -1, 0, +1)
            acc[0][t0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av0, bm, acc[0][t0], 0, 0, 0);
            acc[1][t0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av1, bm, acc[1][t0], 0, 0, 0);
            acc[0][t0 + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av0, bc, acc[0][t0 + 1], 0, 0, 0);
            acc[1][t0 + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av1, bc, acc[1][t0 + 1], 0, 0, 0);
            acc[0][t0 + 2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av0, bp, acc[0][t0 + 2], 0, 0, 0);
            acc[1][t0 + 2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av1, bp, acc[1][t0 + 2], 0, 0, 0);
        }
        asm volatile("" : "+v"(an0), "+v"(an1));
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            asm volatile("" : "+v"(nw[i].lo), "+v"(nw[i].hi));
            win[i] = nw[i];
        }
        a0 = an0;
        a1 = an1;
    }
    // group 1 hands its 2 NTT tiles to group 0 through LDS, DW_ROUND at a time
    // (three rounds for either part of the taps: the barriers match)
#pragma unroll
    for (int rd = 0; rd < 3; ++rd) {
        if (grp == 1) {
#pragma unroll
            for (int i = 0; i < DW_ROUND; ++i) {
                const int k = rd * DW_ROUND + i;
                if (k < 2 * NTT) red[w & 3][i][lane] = acc[k / NTT][k % NTT];
            }
        }
        __syncthreads();
        if (grp == 0) {
#pragma unroll
            for (int i = 0; i < DW_ROUND; ++i) {
                const int k = rd * DW_ROUND + i;
                if (k < 2 * NTT) acc[k / NTT][k % NTT] += red[w][i][lane];
            }
        }
        __syncthreads();
    }
    if (TH == 0 && gq == 0) {
        bred[grp][0][kq][m] = bs0;
        bred[grp][1][kq][m] = bs1;
    }
    __syncthreads();
    if (grp == 0) {
        // lane holds D[co = 16 hh + 4 kq + i][ci = 16 gq + m] of tap 3 SR0 + t
        float *o = part + (long long)blockIdx.x * (WSZ + SC);
#pragma unroll
        for (int hh = 0; hh < 2; ++hh)
#pragma unroll
            for (int t = 0; t < NTT; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    o[((16 * hh + 4 * kq + i) * NT + 3 * SR0 + t) * SC + 16 * gq + m] = acc[hh][t][i];
    }
}

__global__ __launch_bounds__(512) void k_conv_dw(const __bf16 *__restrict__ dZt, const __bf16 *__restrict__ Xt,
                                                 float *__restrict__ part, PadGeom pg, int nruns)
{
    __shared__ f4 red[4][DW_ROUND][64];
    __shared__ float bred[2][2][4][16];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gq = w & 1, th = (w >> 1) & 1, grp = w >> 2;
    if (th == 0)
        dw_wave<0>(dZt, Xt, part, pg, nruns, gq, grp, w, red, bred);
    else
        dw_wave<1>(dZt, Xt, part, pg, nruns, gq, grp, w, red, bred);
    if (threadIdx.x < SC) {
        const int co = threadIdx.x, hh = co >> 4, mm = co & 15;
        float b = 0.f;
#pragma unroll
        for (int g2 = 0; g2 < 2; ++g2)
#pragma unroll
            for (int q = 0; q < 4; ++q) b += bred[g2][hh][q][mm];
        part[(long long)blockIdx.x * (WSZ + SC) + WSZ + co] = b;
    }
}

// fixed-order sum over chunks: g[e] = sum_b part[b][e].  A workgroup takes 64
// elements; its four waves sum a quarter of the chunks each (eight loads in
// flight per lane) and the quarters are added in order.
__global__ __launch_bounds__(256) void k_sum_chunks(const float *__restrict__ part, int nchunk, int n,
                                                    float *__restrict__ g)
{
    __shared__ double q[4][64];
    const int e = blockIdx.x * 64 + (threadIdx.x & 63), w = threadIdx.x >> 6;
    const int per = (nchunk + 3) / 4, b0 = w * per, b1 = min(nchunk, b0 + per);
    double s = 0.0;
    if (e < n) {
        int b = b0;
        for (; b + 8 <= b1; b += 8) {
            float v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = part[(long long)(b + i) * n + e];
#pragma unroll
            for (int i = 0; i < 8; ++i) s += v[i];
        }
        for (; b < b1; ++b) s += part[(long long)b * n + e];
    }
    q[w][threadIdx.x & 63] = s;
    __syncthreads();
    if (w == 0 && e < n) g[e] = (float)(((q[0][threadIdx.x] + q[1][threadIdx.x]) + q[2][threadIdx.x]) + q[3][threadIdx.x]);
}

// Adam on FP32 masters, then refresh the bf16 forward weights [co][t][ci]
// and the mirrored transpose [ci][26-t][co] used by the input gradient.
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                                              const float *__restrict__ g, int n, float lr, float b1, float b2,
                                              float c1, float c2, float eps)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    w[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

__global__ __launch_bounds__(256) void k_refresh(const float *__restrict__ w, __bf16 *__restrict__ wb,
                                                 __bf16 *__restrict__ wt, long long wstride)
{
    // layer blockIdx.y: masters at w + layer * wstride, copies at layer * WSZ
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= WSZ) return;
    w += blockIdx.y * wstride;
    wb += (long long)blockIdx.y * WSZ;
    wt += (long long)blockIdx.y * WSZ;
    const int co = e / (NT * SC), t = (e / SC) % NT, ci = e % SC;
    const __bf16 b = (__bf16)w[e];
    wb[e] = b;
    wt[(ci * NT + (NT - 1 - t)) * SC + co] = b;
}

// residual gate: sums of |a - b|^2 and |b|^2 over 3N (FP64 partials)
__global__ __launch_bounds__(256) void k_resid(const float *__restrict__ a, const float *__restrict__ b,
                                               double *__restrict__ part, long long n)
{
    double s0 = 0.0, s1 = 0.0;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const double d = (double)a[e] - (double)b[e];
        s0 += d * d;
        s1 += (double)b[e] * (double)b[e];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s0 += __shfl_down(s0, o, 64);
        s1 += __shfl_down(s1, o, 64);
    }
    __shared__ double sh[2][4];
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = s0;
        sh[1][threadIdx.x >> 6] = s1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
        part[2 * blockIdx.x + 1] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
    }
}

// r = sqrt(sum |a - b|^2 / sum |b|^2) (0 when the second sum is 0) from the
// nb pairs of k_resid partials, in a fixed order (a strided sum per thread,
// then a tree; 256 threads, one workgroup), into *r: the gate's residual
// stays on the device until the host reads a group of them.
__global__ __launch_bounds__(256) void k_resid_fin(const double *__restrict__ part, int nb, double *__restrict__ r)
{
    __shared__ double sh[2][256];
    double s0 = 0.0, s1 = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        s0 += part[2 * i];
        s1 += part[2 * i + 1];
    }
    sh[0][threadIdx.x] = s0;
    sh[1][threadIdx.x] = s1;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *r = sh[1][0] > 0.0 ? sqrt(sh[0][0] / sh[1][0]) : 0.0;
}

// Sum of squares (FP64 partials per workgroup) of d = (a - b) * s (b may be
// NULL: d = a * s), and d itself into dout when given: the increment of the
// state and its scale in one pass.
__global__ __launch_bounds__(256) void k_sumsq_diff(const float *__restrict__ a, const float *__restrict__ b, float s,
                                                    float *__restrict__ dout, double *__restrict__ part, long long n)
{
    double acc = 0.0;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const float d = (b ? a[e] - b[e] : a[e]) * s;
        if (dout) dout[e] = d;
        acc += (double)d * d;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    __shared__ double sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// d = (a - b) * s   (increment of the state, scaled)
__global__ __launch_bounds__(256) void k_axpby(const float *__restrict__ a, const float *__restrict__ b, float s,
                                               float *__restrict__ d, long long n)
{
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        d[e] = (a[e] - b[e]) * s;
}
// h = h0 + s * dh
__global__ __launch_bounds__(256) void k_anchor(const float *__restrict__ h0, const float *__restrict__ dh, float s,
                                                float *__restrict__ h, long long n)
{
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        h[e] = h0[e] + s * dh[e];
}

}  // namespace mmk

namespace mmk {

struct Sur {
    int nx, ny, nz;
    long long N;
    // FP32 masters and Adam moments, padded layout [co][t][ci] per layer, then 32 biases
    float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    __bf16 *wb = nullptr, *wt = nullptr;  // bf16 forward / mirrored-transposed copies
    __bf16 *Xin = nullptr;                // network input, zero-padded: [G][8] (PadGeom positions)
    __bf16 *X[NLAYER] = {};               // X[l]: input of layer l >= 1, [N][32] (layer 0 reads Xin)
    __bf16 *Zh[NLAYER - 1] = {};          // hidden pre-activations (training), [N][32]
    float *Zout = nullptr;                // last layer's output before the scale, [N][4] (channels 0-2)
    __bf16 *dZb[2] = {};                  // [N][32], this layer's dZ and the one below
    __bf16 *dZbL = nullptr, *dZtL = nullptr;  // the last layer's dZ, cell- and channel-major
    PadGeom pg;                           // channel-major padded copies (training)
    __bf16 *Xt[NLAYER] = {};              // layer inputs, [32][G]
    __bf16 *dZt = nullptr;                // [32][G]
    float *part = nullptr;                // weight/bias gradient partials, [workgroup][layer_stride]
    double *dpart = nullptr;              // FP64 reduction partials
    float *sig = nullptr;                 // device sigma, 1/sigma
    float *tmp = nullptr, *tmp2 = nullptr;  // [3][N] scratch
    float *H0 = nullptr, *Mprev = nullptr, *Hs = nullptr;  // step driver: anchor field, saved state, prediction
    float *Mgroup = nullptr;              // step driver: first state of a group of gated steps
    double *rlog = nullptr;               // step driver: residuals of a group, [MM_SUR_CHECK_MAX]
    int adam_t = 0;
    size_t bytes = 0;                     // workspace the buffers above live in
    char *ws = nullptr;                   // bound workspace (nullptr: unbound)
};

static const int RED_B = 512;
static long long layer_stride() { return (long long)WSZ + SC; }  // weights then biases

// Carve (base != nullptr) or measure the surrogate's buffers in one
// workspace, every buffer 256-byte aligned; returns the bytes needed.
static size_t sur_layout(Sur &s, char *base)
{
    size_t off = 0;
    auto take = [&](auto **ptr, size_t bytes) {
        if (base) *ptr = reinterpret_cast<std::remove_reference_t<decltype(**ptr)> *>(base + off);
        off += (bytes + 255) & ~(size_t)255;
    };
    const size_t P = (size_t)NLAYER * layer_stride();
    take(&s.w, P * 4);
    take(&s.m, P * 4);
    take(&s.v, P * 4);
    take(&s.g, P * 4);
    take(&s.wb, (size_t)NLAYER * WSZ * 2);
    take(&s.wt, (size_t)NLAYER * WSZ * 2);
    take(&s.Xin, (size_t)s.pg.G * IN_CH * 2);
    for (int l = 0; l < NLAYER; ++l) {
        if (l > 0) take(&s.X[l], (size_t)s.N * SC * 2);
        if (l < NLAYER - 1) take(&s.Zh[l], (size_t)s.N * SC * 2);
        take(&s.Xt[l], (size_t)s.pg.G * SC * 2);
    }
    take(&s.Zout, (size_t)s.N * 4 * 4);
    take(&s.dZt, (size_t)s.pg.G * SC * 2);
    take(&s.dZb[0], (size_t)s.N * SC * 2);
    take(&s.dZb[1], (size_t)s.N * SC * 2);
    take(&s.dZbL, (size_t)s.N * SC * 2);
    take(&s.dZtL, (size_t)s.pg.G * SC * 2);
    take(&s.part, (size_t)DW_BLOCKS * layer_stride() * 4);
    take(&s.dpart, (size_t)2 * RED_B * 8);
    take(&s.sig, 16);
    take(&s.tmp, (size_t)3 * s.N * 4);
    take(&s.tmp2, (size_t)3 * s.N * 4);
    take(&s.H0, (size_t)3 * s.N * 4);
    take(&s.Mprev, (size_t)3 * s.N * 4);
    take(&s.Hs, (size_t)3 * s.N * 4);
    take(&s.Mgroup, (size_t)3 * s.N * 4);
    take(&s.rlog, (size_t)MM_SUR_CHECK_MAX * 8);
    return off;
}

static long long flat_param_count()
{
    long long n = 0;
    for (int l = 0; l < NLAYER; ++l) n += (long long)CH[l + 1] * CH[l] * NT + CH[l + 1];
    return n;
}

static void refresh(Sur &s, hipStream_t st)
{
    hipLaunchKernelGGL(k_refresh, dim3((WSZ + 255) / 256, NLAYER), dim3(256), 0, st, s.w, s.wb, s.wt,
                       layer_stride());
}

static unsigned grid_for(long long n) { return (unsigned)std::min<long long>((n + 255) / 256, 4096); }

// A convolution over the whole grid: one launch per kind of z block (bottom,
// interior, top; a single launch when one block spans the thickness), each
// with CONV_WAVES waves per workgroup and one (16-cell x run, y, TZ-level z
// block) task per wave and pass.
template <int EPI>
static void launch_conv(const Sur &s, hipStream_t st, const __bf16 *X, const __bf16 *W, const float *bias, float *Z,
                        __bf16 *Zh, __bf16 *Xn, float *dh, const float *sig, __bf16 *Xt = nullptr)
{
    const int nzb = (s.nz + TZ - 1) / TZ;
    auto go = [&](auto kern, int zb0, int nzbr) {
        const long long tasks = (long long)((s.nx + 15) / 16) * s.ny * nzbr;
        const unsigned gb = (unsigned)std::min<long long>((tasks + CONV_WAVES - 1) / CONV_WAVES, 8192);
        hipLaunchKernelGGL(kern, dim3(gb), dim3(64 * CONV_WAVES), 0, st, X, W, bias, Z, Zh, Xn, dh, 1.f, sig, s.nx,
                           s.ny, s.nz, zb0, nzbr, Xt, s.pg);
    };
    if (nzb == 1) {
        go(k_conv<EPI, true, true>, 0, 1);
        return;
    }
    go(k_conv<EPI, true, false>, 0, 1);
    if (nzb > 2) go(k_conv<EPI, false, false>, 1, nzb - 2);
    go(k_conv<EPI, false, true>, nzb - 1, 1);
}

// the packed first layer (k_conv_in) over the whole grid
template <int EPI>
static void launch_conv_in(const Sur &s, hipStream_t st, __bf16 *Zh, __bf16 *Xt)
{
    const long long tasks = (long long)((s.nx + 15) / 16) * s.ny * ((s.nz + TZ - 1) / TZ);
    const unsigned gb = (unsigned)std::min<long long>((tasks + IN_WAVES - 1) / IN_WAVES, 8192);
    hipLaunchKernelGGL(k_conv_in<EPI>, dim3(gb), dim3(64 * IN_WAVES), 0, st, s.Xin, s.wb, s.w + WSZ, Zh,
                       s.X[1], Xt, s.pg, s.nx, s.ny, s.nz);
}

// forward of the whole stack on the padded input Xin (already filled); last layer -> dh.
// keep_z: store the pre-activations Z of the hidden layers (needed by the
// backward pass; inference skips them).
static void sur_forward(Sur &s, float *dh, hipStream_t st, bool dev_scale, bool keep_z)
{
    if (keep_z)
        launch_conv_in<0>(s, st, s.Zh[0], s.Xt[1]);
    else
        launch_conv_in<3>(s, st, nullptr, nullptr);
    for (int l = 1; l < NLAYER; ++l) {
        const __bf16 *W = s.wb + (long long)l * WSZ;
        const float *b = s.w + l * layer_stride() + WSZ;
        if (l < NLAYER - 1 && keep_z)
            launch_conv<0>(s, st, s.X[l], W, b, nullptr, s.Zh[l], s.X[l + 1], nullptr, nullptr, s.Xt[l + 1]);
        else if (l < NLAYER - 1)
            launch_conv<3>(s, st, s.X[l], W, b, nullptr, nullptr, s.X[l + 1], nullptr, nullptr);
        else  // dh = sigma * Net(...) with sigma from device memory when dev_scale
            launch_conv<1>(s, st, s.X[l], W, b, keep_z ? s.Zout : nullptr, nullptr, nullptr, dh,
                           dev_scale ? s.sig : nullptr);
    }
}

// sigma of dm (normalize) into s.sig, and Xin = bf16(dm / sigma)
// (train: also the channel-major copy Xt[0] for the weight gradient)
// (have_partials: the sum-of-squares partials of dm are already in s.dpart)
static void sur_input(Sur &s, const float *dm, int normalize, hipStream_t st, bool train = false,
                      bool have_partials = false)
{
    if (!have_partials)
        hipLaunchKernelGGL(k_sumsq_diff, dim3(RED_B), dim3(256), 0, st, dm, nullptr, 1.f, nullptr, s.dpart, 3 * s.N);
    hipLaunchKernelGGL(k_to_cl_dev, dim3(grid_for(s.N)), dim3(256), 0, st, dm, s.Xin, s.dpart, RED_B,
                       (double)(3 * s.N), normalize, s.sig, s.N, train ? s.Xt[0] : nullptr, s.pg, s.nx, s.ny);
}

// loss and gradients into s.g (masters' layout); returns the loss on the host
static int sur_backward(Sur &s, const float *dh_target, double *loss, hipStream_t st)
{
    // target is divided by sigma inside k_mse: pass 1/sigma via a host read
    float sg[2];
    MMK_HIP(hipMemcpyAsync(sg, s.sig, sizeof(sg), hipMemcpyDeviceToHost, st));
    MMK_HIP(hipStreamSynchronize(st));
    hipLaunchKernelGGL(k_mse, dim3(RED_B), dim3(256), 0, st, s.Zout, dh_target, sg[1], s.dZbL, s.dZtL, s.pg,
                       s.dpart, s.nx, s.ny, s.N);
    std::vector<double> hp(RED_B);
    MMK_HIP(hipMemcpyAsync(hp.data(), s.dpart, sizeof(double) * RED_B, hipMemcpyDeviceToHost, st));
    for (int l = NLAYER - 1; l >= 0; --l) {
        const int nruns = (int)(((long long)s.nz * s.pg.pl + 31) / 32);
        const bool last = l == NLAYER - 1;
        hipLaunchKernelGGL(k_conv_dw, dim3(DW_BLOCKS), dim3(512), 0, st, last ? s.dZtL : s.dZt, s.Xt[l], s.part, s.pg,
                           nruns);
        const int ls = (int)layer_stride();
        hipLaunchKernelGGL(k_sum_chunks, dim3((ls + 63) / 64), dim3(256), 0, st, s.part, DW_BLOCKS, ls,
                           s.g + l * layer_stride());
        if (l > 0) {
            // dZ of layer l-1 into the other dZb buffer (the convolution still
            // reads this one; layer l's is dZbL for the last layer, else
            // dZb[(NLAYER - 2 - l) & 1]) and into dZt, whose weight gradient has run
            const __bf16 *in = last ? s.dZbL : s.dZb[(NLAYER - 2 - l) & 1];
            __bf16 *out = s.dZb[(NLAYER - 1 - l) & 1];
            launch_conv<2>(s, st, in, s.wt + (long long)l * WSZ, nullptr, nullptr, s.Zh[l - 1], out, nullptr, nullptr,
                           s.dZt);
        }
    }
    MMK_HIP(hipStreamSynchronize(st));
    double tot = 0.0;
    for (double x : hp) tot += x;
    *loss = tot / (3.0 * (double)s.N);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MM_EHIP, std::string("surrogate backward: ") + hipGetErrorString(e));
    return MM_OK;
}

// host layout conversion: oracle [co][ci][kz][ky][kx] + b[co] per layer <-> padded masters
static void to_masters(const float *src, std::vector<float> &dst)
{
    dst.assign((size_t)NLAYER * layer_stride(), 0.f);
    long long o = 0;
    for (int l = 0; l < NLAYER; ++l) {
        float *W = dst.data() + l * layer_stride();
        for (int co = 0; co < CH[l + 1]; ++co)
            for (int ci = 0; ci < CH[l]; ++ci)
                for (int t = 0; t < NT; ++t) W[(co * NT + t) * SC + ci] = src[o++];
        for (int co = 0; co < CH[l + 1]; ++co) W[WSZ + co] = src[o++];
    }
}
static void from_masters(const float *src, float *dst)
{
    long long o = 0;
    for (int l = 0; l < NLAYER; ++l) {
        const float *W = src + l * layer_stride();
        for (int co = 0; co < CH[l + 1]; ++co)
            for (int ci = 0; ci < CH[l]; ++ci)
                for (int t = 0; t < NT; ++t) dst[o++] = W[(co * NT + t) * SC + ci];
        for (int co = 0; co < CH[l + 1]; ++co) dst[o++] = W[WSZ + co];
    }
}

static void free_sur(Sur *s) { delete s; }

static int sur_ready(const Sur *s)
{
    if (!s) return fail(MM_EINVAL, "NULL surrogate");
    if (!s->ws) return fail(MM_EINVAL, "surrogate has no workspace: call mm_sur_bind_workspace first");
    return MM_OK;
}

// residual of the surrogate against an exact field: |a-b|^2 / |b|^2
// relative residual |a - b| / |b| into the device double *r (no sync)
static void resid_enqueue(Sur &s, const float *a, const float *b, double *r, hipStream_t st)
{
    hipLaunchKernelGGL(k_resid, dim3(RED_B), dim3(256), 0, st, a, b, s.dpart, 3 * s.N);
    hipLaunchKernelGGL(k_resid_fin, dim3(1), dim3(256), 0, st, s.dpart, RED_B, r);
}

// H = H0 + Ms * sigma * Net((Mstage - Mn) / (Ms sigma)) on stream st (no sync)
static void sur_field(Sur &s, const float *Mstage, const float *Mn, const float *H0, float Ms, float *H, hipStream_t st)
{
    // the increment and its sum of squares in one pass
    hipLaunchKernelGGL(k_sumsq_diff, dim3(RED_B), dim3(256), 0, st, Mstage, Mn, 1.f / Ms, s.tmp, s.dpart, 3 * s.N);
    sur_input(s, s.tmp, 1, st, false, true);
    sur_forward(s, s.tmp2, st, true, false);
    hipLaunchKernelGGL(k_anchor, dim3(grid_for(3 * s.N)), dim3(256), 0, st, H0, s.tmp2, Ms, H, 3 * s.N);
}

}  // namespace mmk

using namespace mmk;

struct mm_sur_s {
    Sur *s;
};

extern "C" {

int mm_sur_create(int nx, int ny, int nz, mm_sur *out)
{
    if (!out) return fail(MM_EINVAL, "out is NULL");
    *out = nullptr;
    // the convolution addresses the bf16 activations ([cell][32], 64 bytes a
    // cell) with 32-bit buffer offsets below 2^31: at most 2^25 cells
    if (nx < 1 || ny < 1 || nz < 1 || (long long)nx * ny * nz > (1LL << 25))
        return fail(MM_EINVAL, "surrogate grid: need 1 <= nx, ny, nz and nx*ny*nz <= 2^25");
    Sur *s = new Sur();
    s->nx = nx;
    s->ny = ny;
    s->nz = nz;
    s->N = (long long)nx * ny * nz;
    s->pg = pad_geom(nx, ny, nz);
    // the first layer reaches its neighbours with 32-bit byte offsets spanning
    // two padded planes
    if ((2LL * s->pg.pl + 2LL * s->pg.xp + 32) * IN_CH * 2 >= (1LL << 32)) {
        delete s;
        return fail(MM_EINVAL, "surrogate grid: a padded x-y plane of more than 2^27 positions");
    }
    s->bytes = sur_layout(*s, nullptr);
    *out = new mm_sur_s{s};
    return MM_OK;
}

int mm_sur_workspace_bytes(mm_sur sur, size_t *bytes)
{
    if (!sur || !bytes) return fail(MM_EINVAL, "NULL surrogate or bytes");
    *bytes = sur->s->bytes;
    return MM_OK;
}

int mm_sur_bind_workspace(mm_sur sur, void *ws, size_t bytes)
{
    if (!sur || !ws) return fail(MM_EINVAL, "NULL surrogate or workspace");
    Sur &s = *sur->s;
    if ((uintptr_t)ws % 256 != 0) return fail(MM_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < s.bytes)
        return fail(MM_ENOMEM, "workspace of " + std::to_string(bytes) + " bytes; the surrogate needs " +
                                   std::to_string(s.bytes));
    s.ws = nullptr;
    sur_layout(s, (char *)ws);
    const size_t P = (size_t)NLAYER * layer_stride();
    // weights and Adam state zero; the padded input and the padded copies
    // are zero outside the grid's cells and stay so
    MMK_HIP(hipMemset(s.w, 0, P * 4));
    MMK_HIP(hipMemset(s.m, 0, P * 4));
    MMK_HIP(hipMemset(s.v, 0, P * 4));
    MMK_HIP(hipMemset(s.g, 0, P * 4));
    MMK_HIP(hipMemset(s.Xin, 0, (size_t)s.pg.G * IN_CH * 2));
    for (int l = 0; l < NLAYER; ++l) MMK_HIP(hipMemset(s.Xt[l], 0, (size_t)s.pg.G * SC * 2));
    MMK_HIP(hipMemset(s.dZt, 0, (size_t)s.pg.G * SC * 2));
    MMK_HIP(hipMemset(s.dZtL, 0, (size_t)s.pg.G * SC * 2));
    MMK_HIP(hipMemset(s.dZbL, 0, (size_t)s.N * SC * 2));
    s.adam_t = 0;
    refresh(s, nullptr);
    MMK_HIP(hipDeviceSynchronize());
    s.ws = (char *)ws;
    return MM_OK;
}

int mm_sur_attach(mm_plan plan, mm_sur sur)
{
    Plan *p = plan_of(plan);
    if (!p) return fail(MM_EINVAL, "NULL plan");
    if (!sur) {
        p->sur = nullptr;
        return MM_OK;
    }
    if (sur->s->N != p->cells() || sur->s->nx != p->nx || sur->s->ny != p->ny)
        return fail(MM_EINVAL, "surrogate and plan grids differ");
    p->sur = sur;
    return MM_OK;
}

// A training pair from the solver's own trajectory: advance M by nsteps
// exact RK4 steps; dm = (M_after - M_before) / Ms, dh = H_d(dm) (demag is
// linear, so dh is the field increment per Ms).
int mm_sur_make_pair(mm_plan plan, const mm_llg_params *params, float *M, int nsteps, float *dm, float *dh,
                     void *stream)
{
    Plan *pp = plan_of(plan);
    int rc0 = plan_ready(pp);
    if (rc0 != MM_OK) return rc0;
    if (!params || !M || !dm || !dh || dm == dh) return fail(MM_EINVAL, "NULL or aliased argument");
    if (nsteps < 1) return fail(MM_EINVAL, "nsteps < 1");
    Plan &p = *pp;
    hipStream_t st = (hipStream_t)stream;
    const size_t n3 = 3 * (size_t)p.cells();
    MMK_HIP(hipMemcpyAsync(dm, M, n3 * sizeof(float), hipMemcpyDeviceToDevice, st));
    const StageCoef c = stage_coef(p, *params);
    for (int i = 0; i < nsteps; ++i) {
        int rc = llg_enqueue_step(p, c, params->integrator, M, st);
        if (rc != MM_OK) return rc;
    }
    hipLaunchKernelGGL(k_axpby, dim3(grid_for((long long)n3)), dim3(256), 0, st, M, dm, (float)(1.0 / params->Ms),
                       dm, (long long)n3);
    return demag_enqueue(p, dm, dh, st);
}

void mm_sur_destroy(mm_sur sur)
{
    if (!sur) return;
    free_sur(sur->s);
    delete sur;
}

long long mm_sur_param_count(void) { return flat_param_count(); }

int mm_sur_set_params(mm_sur sur, const float *host, long long n)
{
    if (sur_ready(sur ? sur->s : nullptr) != MM_OK) return MM_EINVAL;
    if (!host || n != flat_param_count()) return fail(MM_EINVAL, "surrogate params: bad pointer or count");
    Sur &s = *sur->s;
    std::vector<float> w;
    to_masters(host, w);
    MMK_HIP(hipMemcpy(s.w, w.data(), w.size() * 4, hipMemcpyHostToDevice));
    MMK_HIP(hipMemset(s.m, 0, w.size() * 4));
    MMK_HIP(hipMemset(s.v, 0, w.size() * 4));
    s.adam_t = 0;
    refresh(s, nullptr);
    MMK_HIP(hipDeviceSynchronize());
    return MM_OK;
}

int mm_sur_get_params(mm_sur sur, float *host, long long n)
{
    if (sur_ready(sur ? sur->s : nullptr) != MM_OK) return MM_EINVAL;
    if (!host || n != flat_param_count()) return fail(MM_EINVAL, "surrogate params: bad pointer or count");
    Sur &s = *sur->s;
    std::vector<float> w((size_t)NLAYER * layer_stride());
    MMK_HIP(hipDeviceSynchronize());
    MMK_HIP(hipMemcpy(w.data(), s.w, w.size() * 4, hipMemcpyDeviceToHost));
    from_masters(w.data(), host);
    return MM_OK;
}

int mm_sur_forward(mm_sur sur, const float *dm, float *dh, int normalize, void *stream)
{
    if (sur_ready(sur ? sur->s : nullptr) != MM_OK) return MM_EINVAL;
    if (!dm || !dh) return fail(MM_EINVAL, "NULL surrogate or field");
    Sur &s = *sur->s;
    hipStream_t st = (hipStream_t)stream;
    sur_input(s, dm, normalize, st);
    sur_forward(s, dh, st, true, false);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MM_OK : fail(MM_EHIP, std::string("surrogate forward: ") + hipGetErrorString(e));
}

int mm_sur_gradients(mm_sur sur, const float *dm, const float *dh, int normalize, double *loss, float *grads,
                     long long n, void *stream)
{
    if (sur_ready(sur ? sur->s : nullptr) != MM_OK) return MM_EINVAL;
    if (!dm || !dh || !loss) return fail(MM_EINVAL, "NULL surrogate argument");
    if (grads && n != flat_param_count()) return fail(MM_EINVAL, "gradient count");
    Sur &s = *sur->s;
    hipStream_t st = (hipStream_t)stream;
    sur_input(s, dm, normalize, st, true);
    sur_forward(s, s.tmp2, st, false, true);
    int rc = sur_backward(s, dh, loss, st);
    if (rc != MM_OK || !grads) return rc;
    std::vector<float> g((size_t)NLAYER * layer_stride());
    MMK_HIP(hipMemcpy(g.data(), s.g, g.size() * 4, hipMemcpyDeviceToHost));
    from_masters(g.data(), grads);
    return MM_OK;
}

int mm_sur_train_step(mm_sur sur, const float *dm, const float *dh, float lr, int normalize, double *loss,
                      void *stream)
{
    if (sur_ready(sur ? sur->s : nullptr) != MM_OK) return MM_EINVAL;
    if (!dm || !dh || !loss) return fail(MM_EINVAL, "NULL surrogate argument");
    if (!(lr > 0.f)) return fail(MM_EINVAL, "learning rate must be > 0");
    Sur &s = *sur->s;
    hipStream_t st = (hipStream_t)stream;
    sur_input(s, dm, normalize, st, true);
    sur_forward(s, s.tmp2, st, false, true);
    int rc = sur_backward(s, dh, loss, st);
    if (rc != MM_OK) return rc;
    s.adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - std::pow(0.9, s.adam_t)), c2 = (float)(1.0 - std::pow(0.999, s.adam_t));
    const int P = (int)(NLAYER * layer_stride());
    hipLaunchKernelGGL(k_adam, dim3((P + 255) / 256), dim3(256), 0, st, s.w, s.m, s.v, s.g, P, lr, b1, b2, c1, c2,
                       1e-8f);
    refresh(s, st);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MM_OK : fail(MM_EHIP, std::string("surrogate train: ") + hipGetErrorString(e));
}

int mm_sur_zero(mm_sur sur)
{
    if (sur_ready(sur ? sur->s : nullptr) != MM_OK) return MM_EINVAL;
    Sur &s = *sur->s;
    const size_t P = (size_t)NLAYER * layer_stride();
    MMK_HIP(hipMemset(s.w, 0, P * 4));
    refresh(s, nullptr);
    MMK_HIP(hipDeviceSynchronize());
    return MM_OK;
}

// Steps with the learned increment in RK stages 2-4, exact demag at stage 1,
// and every accepted state judged on the device against the exact field of
// that state (the next step's stage-1 field).  The steps run in groups of
// k = sur_check_every; after a group the host reads its k residuals, and one
// above `tol` redoes the group from its first state with exact demag and
// keeps the surrogate off for one step.
int mm_llg_step_surrogate(mm_plan plan, mm_sur sur, const mm_llg_params *params, float *M, int nsteps, double tol,
                          mm_sur_stats *stats, void *stream)
{
    Plan *pp = plan_of(plan);
    if (plan_ready(pp) != MM_OK || sur_ready(sur ? sur->s : nullptr) != MM_OK) return MM_EINVAL;
    if (!params || !M) return fail(MM_EINVAL, "NULL params or M");
    if (params->integrator != MM_RK4) return fail(MM_EINVAL, "surrogate stepping needs RK4");
    if (nsteps < 0) return fail(MM_EINVAL, "nsteps < 0");
    if (params->sur_check_every > MM_SUR_CHECK_MAX) return fail(MM_EINVAL, "sur_check_every above MM_SUR_CHECK_MAX");
    Plan &p = *pp;
    Sur &s = *sur->s;
    if (s.N != p.cells()) return fail(MM_EINVAL, "surrogate and plan grids differ");
    hipStream_t st = (hipStream_t)stream;
    const StageCoef c = stage_coef(p, *params);
    const size_t bytes = sizeof(float) * 3 * (size_t)p.cells();
    const int K = params->sur_check_every > 1 ? params->sur_check_every : 1;
    float *H0 = s.H0, *Mprev = s.Mprev, *Hs = s.Hs;
    mm_sur_stats acc{};
    std::vector<double> r((size_t)K);
    bool use = true;
    // exact field of the current state
    int rc = demag_enqueue(p, M, H0, st);
    for (int n = 0; n < nsteps && rc == MM_OK;) {
        if (!use) {  // the step after a redone group
            rc = llg_enqueue_step(p, c, MM_RK4, M, st);
            if (rc == MM_OK) rc = demag_enqueue(p, M, H0, st);
            use = true;
            acc.steps += 1;
            n += 1;
            continue;
        }
        const int k = std::min(K, nsteps - n);
        // the group's first state (a one-step group has it in Mprev)
        if (k > 1) (void)hipMemcpyAsync(s.Mgroup, M, bytes, hipMemcpyDeviceToDevice, st);
        for (int j = 0; j < k && rc == MM_OK; ++j) {
            (void)hipMemcpyAsync(Mprev, M, bytes, hipMemcpyDeviceToDevice, st);
            rc = llg_step_with_fields(p, c, M, H0, st, [&](int stage, const float *Sstate, float *Hout) {
                (void)stage;
                sur_field(s, Sstate, Mprev, H0, c.Ms, Hout, st);
                return MM_OK;
            });
            // judge the accepted state: exact H of M_{n+1} against the network's
            if (rc == MM_OK) rc = demag_enqueue(p, M, p.H, st);
            if (rc == MM_OK) {
                sur_field(s, M, Mprev, H0, c.Ms, Hs, st);
                resid_enqueue(s, Hs, p.H, s.rlog + j, st);
                (void)hipMemcpyAsync(H0, p.H, bytes, hipMemcpyDeviceToDevice, st);
            }
        }
        if (rc != MM_OK) break;
        MMK_HIP(hipMemcpyAsync(r.data(), s.rlog, sizeof(double) * k, hipMemcpyDeviceToHost, st));
        MMK_HIP(hipStreamSynchronize(st));
        bool redo = false;
        for (int j = 0; j < k; ++j) {
            acc.last_residual = r[j];
            acc.max_residual = r[j] > acc.max_residual ? r[j] : acc.max_residual;
            acc.sum_residual += r[j];
            acc.checked += 1;
            if (tol >= 0.0 && !(r[j] <= tol)) redo = true;
        }
        if (redo) {
            // the whole group again with exact demag from its first state
            acc.fallbacks += k;
            (void)hipMemcpyAsync(M, k > 1 ? s.Mgroup : Mprev, bytes, hipMemcpyDeviceToDevice, st);
            for (int j = 0; j < k && rc == MM_OK; ++j) rc = llg_enqueue_step(p, c, MM_RK4, M, st);
            if (rc == MM_OK) rc = demag_enqueue(p, M, H0, st);
            use = false;
        }
        acc.steps += k;
        n += k;
    }
    if (stats) *stats = acc;
    if (rc == MM_OK) {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = fail(MM_EHIP, std::string("surrogate step: ") + hipGetErrorString(e));
    }
    return rc;
}

}  // extern "C"
