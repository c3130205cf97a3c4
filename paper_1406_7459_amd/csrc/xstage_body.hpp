// xstage_body.hpp -- the x-inverse of one demag evaluation, the LLG stage
// that consumes its field and the x-forward of the stage's result, fused in
// one pass over the rows of the grid.
//
// Per stage the unfused path runs XINV (half spectrum -> H), the stage
// kernel (H, S, Mn, kacc -> S', kacc) and the next evaluation's XFWD
// (S' -> half spectrum), moving H out and back and S' back in.  Here a
// workgroup owns 2P consecutive cell rows (r = k ny + j) of all three
// components:
//   1. inverse C2R of its rows (xinv_body's arithmetic, one component per
//      thread group) -> H of its cells in LDS;
//   2. the stage on its cells (stage_cell, the same per-cell arithmetic as
//      the stage kernel), H from LDS, neighbours and the rest from global
//      memory; S' to global memory and into LDS in place of H;
//   3. (FWD) forward R2C of S' from LDS (xfwd_body's arithmetic) -> X1.
// X1 rows are read and rewritten by their owning workgroup only.  Every
// value is computed by the same operations as on the unfused path, so the
// states are bitwise those of XINV + stage + XFWD.
#pragma once
#include "demag_kernels.hpp"
#include "stage_body.hpp"

namespace mmk {

// LDS layout: twiddles | 3P transforms of XS slots (float2).  The H/S' rows
// [3][2P][nx] (float) share the transforms' space: they are written after
// the inverse transforms' last exchange (whose trailing barrier every thread
// has passed) and read into registers, behind a barrier, before the forward
// transforms' first exchange; 3 2P nx floats never exceed the 6P XS floats.
// Sharing leaves room for more resident workgroups per CU.
template <int L> constexpr int xs_slots() { return lds_rows(L) + 1; }
template <int L> __host__ __device__ constexpr size_t xs_rows_offset(int)
{
    return (size_t)tw_slots<L>() * sizeof(float2);  // 16-byte aligned: L is even
}
template <int L> __host__ __device__ constexpr size_t xs_lds_bytes(int P)
{
    return ((size_t)tw_slots<L>() + 3 * (size_t)P * xs_slots<L>()) * sizeof(float2);
}

// Inputs of one stage task: W consecutive cells of a row, their stage
// state, its four y/z neighbour rows and the two x neighbours outside the
// group, the step's start state and the RK4 accumulator.
template <int W> struct XsTask {
    float m[3][W], y0[3][W], y1[3][W], z0[3][W], z1[3][W], mn[3][W], ka[3][W];
    float left[3], right[3];
    unsigned id, i;
};

// W: cells per thread task of the stage phase (nx % W == 0).
template <int L, int STAGE, bool FWD, int W>
__device__ __forceinline__ void xstage_body(float2 *__restrict__ X1, const float *S, const float *Mn,
                                            float *__restrict__ kacc, float *out, int nx_, int ny, int nz,
                                            const StageCoef &c, const float2 *__restrict__ tw, int lp2, int bx)
{
    constexpr int E = Factors<L>::E, Q = L / E, NX = L / 2, XP = x_pitch(NX + 1);
    extern __shared__ float2 lds[];
    const float2 *twl = row_twiddles<L, 0>(lds, tw);
    const int P = 1 << lp2;
    const int PQ = P * Q;
    const int t = threadIdx.x;
    const int g = t / PQ;  // component of this thread's transforms
    const unsigned tt = (unsigned)(t - g * PQ);  // in [0, PQ): unsigned, so the compiler sees q < Q
    const int q = (int)(tt % Q), p = (int)(tt / Q);
    const int ncr = nz * ny;  // cell rows per component
    const int r0 = bx * 2 * P;
    const int ra = r0 + 2 * p, rb = ra + 1;
    const bool oka = ra < ncr, okb = rb < ncr;
    constexpr int XS = xs_slots<L>();
    float2 *fbuf = lds + tw_slots<L>();
    float *rows = reinterpret_cast<float *>(reinterpret_cast<char *>(lds) + xs_rows_offset<L>(P));
    const int rstride = 2 * P * nx_;  // floats per component in `rows`
    const LdsView s{fbuf, 1, (g * P + p) * XS};

    // stage tasks: cells [r0 nx, (r0 + 2P) nx), W consecutive cells of a row
    // per task (as stage_body_vec, with the field from LDS)
    const unsigned nx = (unsigned)nx_, nxy = (unsigned)nx_ * (unsigned)ny;
    const unsigned n = nxy * (unsigned)nz;
    const unsigned cbase = (unsigned)r0 * nx;
    auto load_task = [&](unsigned e, XsTask<W> &T) -> bool {
        const unsigned id = cbase + e;
        if (e >= (unsigned)rstride || id >= n) return false;
        const unsigned k = id / nxy;
        const unsigned rem = id - k * nxy;
        const unsigned j = rem / nx;
        const unsigned i = rem - j * nx;
        const unsigned ym = j > 0 ? id - nx : id, yp = j + 1 < (unsigned)ny ? id + nx : id;
        const unsigned zm = k > 0 ? id - nxy : id, zp = k + 1 < (unsigned)nz ? id + nxy : id;
        T.id = id;
        T.i = i;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float *sc = S + (size_t)a * n;
            const float *mc = Mn + (size_t)a * n;
            const float *kc = kacc + (size_t)a * n;
            if constexpr (W == 1) {
                T.m[a][0] = ld32(sc, id);
                T.y0[a][0] = ld32(sc, ym);
                T.y1[a][0] = ld32(sc, yp);
                T.z0[a][0] = ld32(sc, zm);
                T.z1[a][0] = ld32(sc, zp);
                T.mn[a][0] = ld32(mc, id);
                T.ka[a][0] = (STAGE == 2 || STAGE == 3 || STAGE == 4) ? ld32(kc, id) : 0.f;
            } else {
                typedef typename VecOf<W>::T V;
                const V vm = ldv32<V>(sc, id), vy0 = ldv32<V>(sc, ym), vy1 = ldv32<V>(sc, yp);
                const V vz0 = ldv32<V>(sc, zm), vz1 = ldv32<V>(sc, zp), vmn = ldv32<V>(mc, id);
                V vka;
                if constexpr (STAGE == 2 || STAGE == 3 || STAGE == 4) vka = ldv32<V>(kc, id);
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    T.m[a][w] = lane_of<W>(vm, w);
                    T.y0[a][w] = lane_of<W>(vy0, w);
                    T.y1[a][w] = lane_of<W>(vy1, w);
                    T.z0[a][w] = lane_of<W>(vz0, w);
                    T.z1[a][w] = lane_of<W>(vz1, w);
                    T.mn[a][w] = lane_of<W>(vmn, w);
                    T.ka[a][w] = (STAGE == 2 || STAGE == 3 || STAGE == 4) ? lane_of<W>(vka, w) : 0.f;
                }
            }
            // at a free edge the task's own end cell, read again: no load
            // waits on another
            T.left[a] = ld32(sc, i > 0 ? id - 1 : id);
            T.right[a] = ld32(sc, i + W < nx ? id + W : id + W - 1);
        }
        return true;
    };
    auto stage_task = [&](unsigned e, const XsTask<W> &T) {
        if (e >= (unsigned)rstride || T.id >= n) return;
        float o[3][W], kn[3][W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            float mm[3], xm[3], xp[3], a0[3], a1[3], b0[3], b1[3], h[3], mnn[3], kk[3], oo[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                mm[a] = T.m[a][w];
                xm[a] = w > 0 ? T.m[a][w - 1] : T.left[a];
                xp[a] = w + 1 < W ? T.m[a][w + 1] : T.right[a];
                a0[a] = T.y0[a][w];
                a1[a] = T.y1[a][w];
                b0[a] = T.z0[a][w];
                b1[a] = T.z1[a][w];
                h[a] = rows[a * rstride + e + w];
                mnn[a] = T.mn[a][w];
                kk[a] = T.ka[a][w];
            }
            stage_cell<STAGE>(mm, xm, xp, a0, a1, b0, b1, h, mnn, kk, oo, c);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                o[a][w] = oo[a];
                kn[a][w] = kk[a];
            }
        }
        const unsigned id = T.id;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float *oc = out + (size_t)a * n;
            float *kc = kacc + (size_t)a * n;
            float *hc = rows + a * rstride + e;
            if constexpr (W == 1) {
                if constexpr (STAGE == 1 || STAGE == 2 || STAGE == 3) st32(kc, id, kn[a][0]);
                st32(oc, id, o[a][0]);
                if constexpr (FWD) hc[0] = o[a][0];
            } else {
                typedef typename VecOf<W>::T V;
                V vo, vk;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    set_lane<W>(vo, w, o[a][w]);
                    set_lane<W>(vk, w, kn[a][w]);
                }
                if constexpr (STAGE == 1 || STAGE == 2 || STAGE == 3) stv32<V>(kc, id, vk);
                stv32<V>(oc, id, vo);
                if constexpr (FWD) *reinterpret_cast<V *>(hc) = vo;
            }
        }
    };
    // the first task's loads are in flight during the inverse transform
    const unsigned e0 = (unsigned)t * W;
    XsTask<W> T0;
    T0.id = n;
    (void)load_task(e0, T0);

    // 1. inverse C2R of rows ra, rb of component g (as xinv_body)
    {
        const size_t ca = (size_t)g * ncr + (oka ? ra : 0);  // rows clamped into the grid (masked in the gather)
        const float2 *sa = X1 + ca * XP;
        const float2 *sb = X1 + (okb ? ca + 1 : ca) * XP;
        float2 v[E];
        constexpr int R0 = first_radix<L, false>();
        x_inverse_gather<L, E, R0, Q>(sa, sb, oka, okb, q, v);
        fft_e<L, E, +1, false, 0, true>(v, s, q, twl);
        constexpr int RL = last_radix<L, false>();
        float *ha = rows + g * rstride + 2 * p * nx_;
#pragma unroll
        for (int b = 0; b < E / RL; ++b)
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const int i = q + Q * b + r * (L / RL);
                const bool upper = r * (L / RL) >= NX;
                if (!upper && i < nx_) {
                    ha[i] = v[b * RL + r].x;
                    ha[nx_ + i] = v[b * RL + r].y;
                }
            }
    }
    __syncthreads();

    // 2. the stage on this thread's tasks; the first task's inputs were
    // loaded before the inverse transform
    stage_task(e0, T0);
    for (unsigned e = e0 + blockDim.x * W; e < (unsigned)rstride; e += blockDim.x * W) {
        XsTask<W> T;
        if (!load_task(e, T)) break;
        stage_task(e, T);
    }
    if constexpr (!FWD) return;

    __syncthreads();
    // 3. forward R2C of the new state's rows ra, rb of component g (as
    // xfwd_body; a row past the grid enters as zeros)
    {
        const float *za = rows + g * rstride + 2 * p * nx_;
        const float *zb = za + nx_;
        float2 v[E];
        constexpr int R0 = first_radix<L, false>();
#pragma unroll
        for (int b = 0; b < E / R0; ++b)
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                const int i = q + Q * b + r * (L / R0);
                const bool upper = r * (L / R0) >= NX;
                const bool in = !upper && i < nx_;
                v[b * R0 + r] = make_float2(in && oka ? za[i] : 0.f, in && okb ? zb[i] : 0.f);
            }
        __syncthreads();  // every row read before the transforms reuse the space
        fft_e<L, E, -1, false, 0, true>(v, s, q, twl);
        constexpr int RL = last_radix<L, false>();
        float2 *col = fbuf + (g * P + p) * XS;
#pragma unroll
        for (int b = 0; b < E / RL; ++b)
#pragma unroll
            for (int r = 0; r < RL; ++r) col[lds_slot(q + Q * b + r * (L / RL))] = v[b * RL + r];
        __syncthreads();
        float2 *da = X1 + ((size_t)g * ncr + ra) * XP;
        float2 *db = da + XP;
#pragma unroll
        for (int b = 0; b < E / RL; ++b)
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const int k = q + Q * b + r * (L / RL);
                if (k <= NX) {
                    const float2 z = v[b * RL + r];
                    const float2 w = col[lds_slot(k == 0 ? 0 : L - k)];
                    const float2 sp = make_float2(z.x + w.x, z.y - w.y);
                    const float2 sm = make_float2(z.x - w.x, z.y + w.y);
                    if (oka) da[k] = make_float2(0.5f * sp.x, 0.5f * sp.y);
                    if (okb) db[k] = make_float2(0.5f * sm.y, -0.5f * sm.x);
                }
            }
    }
}

}  // namespace mmk
