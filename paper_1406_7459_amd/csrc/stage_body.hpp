// stage_body.hpp -- per-cell part of a time step, shared by the per-plan and
// the batched launches: effective field of eq. (2) (exchange eq. (3)-(4)
// with free boundaries, uniaxial anisotropy eq. (5) in easy-axis form,
// Zeeman, plus the demag field), the Landau-Lifshitz right-hand side of
// eq. (6), and one stage of classical RK4 or an explicit Euler step.
#pragma once
#include <hip/hip_runtime.h>

#include "mm_internal.hpp"

namespace mmk {

// STAGE 1..4: RK4 stages; 0: Euler.  One cell: its stage state m, the six
// neighbours (xm, xp, ym, yp, zm, zp; a missing neighbour is the cell
// itself, the free boundary), the demag field hd of the stage state, the
// step's start state mn and the accumulator ka (read by stages 2-4, written
// by stages 1-3) -> the next stage state (stage 4 / Euler: the new state,
// renormalised if requested) in o.
template <int STAGE>
__device__ __forceinline__ void stage_cell(const float (&m)[3], const float (&xm)[3], const float (&xp)[3],
                                           const float (&ym)[3], const float (&yp)[3], const float (&zm)[3],
                                           const float (&zp)[3], const float (&hd)[3], const float (&mn)[3],
                                           float (&ka)[3], float (&o)[3], const StageCoef &c)
{
    // fixed arithmetic in every file and every launch shape that uses this
    // cell (per-plan, vectorised and batched launches give bitwise the same
    // states)
#pragma clang fp contract(off)
    float h[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        h[a] = c.cx * (xm[a] + xp[a] - 2.f * m[a]) + c.cy * (ym[a] + yp[a] - 2.f * m[a]) +
               c.cz * (zm[a] + zp[a] - 2.f * m[a]) + hd[a];
    const float um = c.ka * (c.ux * m[0] + c.uy * m[1] + c.uz * m[2]);
    h[0] += um * c.ux + c.hx;
    h[1] += um * c.uy + c.hy;
    h[2] += um * c.uz + c.hz;
    // f = -g m x h - gd m x (m x h)
    const float t0 = m[1] * h[2] - m[2] * h[1];
    const float t1 = m[2] * h[0] - m[0] * h[2];
    const float t2 = m[0] * h[1] - m[1] * h[0];
    const float d0 = m[1] * t2 - m[2] * t1;
    const float d1 = m[2] * t0 - m[0] * t2;
    const float d2 = m[0] * t1 - m[1] * t0;
    const float f[3] = {-c.g * t0 - c.gd * d0, -c.g * t1 - c.gd * d1, -c.g * t2 - c.gd * d2};
    if constexpr (STAGE == 1 || STAGE == 2 || STAGE == 3) {
        const float step = STAGE == 3 ? c.dt : 0.5f * c.dt;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ka[a] = STAGE == 1 ? f[a] : ka[a] + 2.f * f[a];
            o[a] = mn[a] + step * f[a];
        }
    } else {
        if constexpr (STAGE == 4) {
            const float w = c.dt * (1.f / 6.f);
#pragma unroll
            for (int a = 0; a < 3; ++a) o[a] = mn[a] + w * (ka[a] + f[a]);
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) o[a] = mn[a] + c.dt * f[a];
        }
        if (c.renorm) {
            const float nn = sqrtf(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
            const float sc = nn > 0.f ? c.Ms / nn : 1.f;
#pragma unroll
            for (int a = 0; a < 3; ++a) o[a] *= sc;
        }
    }
}

// Element idx of a float array through a 32-bit byte offset from a uniform
// base: the load/store takes the scalar-base form (base in SGPRs, one 32-bit
// VGPR offset) instead of a 64-bit per-lane address.  Byte offsets stay
// below 2^32 (at most 512^3 cells per component).
__device__ __forceinline__ float ld32(const float *base, unsigned idx)
{
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(base) + (idx << 2));
}
__device__ __forceinline__ void st32(float *base, unsigned idx, float v)
{
    *reinterpret_cast<float *>(reinterpret_cast<char *>(base) + (idx << 2)) = v;
}

// One cell per thread: reads the stage state S (with its six neighbours),
// the demag field Hd of S, the step's start state Mn and the accumulator;
// writes the accumulator and the next stage state `out`.
// Indices are 32-bit (a grid holds at most 512^3 cells, so byte offsets of
// one component stay below 2^32) and every array is addressed as a uniform
// per-component base plus one of seven per-thread offsets.
template <int STAGE>
__device__ __forceinline__ void stage_body(const float *S, const float *__restrict__ Hd, const float *Mn,
                                           float *__restrict__ kacc, float *out, int nx, int ny, int nz,
                                           const StageCoef &c, unsigned id)
{
    const unsigned nxy = (unsigned)nx * (unsigned)ny;
    const unsigned n = nxy * (unsigned)nz;
    if (id >= n) return;
    const unsigned k = id / nxy;
    const unsigned rem = id - k * nxy;
    const unsigned j = rem / (unsigned)nx;
    const unsigned i = rem - j * (unsigned)nx;
    const unsigned xm = i > 0 ? id - 1 : id, xp = i + 1 < (unsigned)nx ? id + 1 : id;
    const unsigned ym = j > 0 ? id - nx : id, yp = j + 1 < (unsigned)ny ? id + nx : id;
    const unsigned zm = k > 0 ? id - nxy : id, zp = k + 1 < (unsigned)nz ? id + nxy : id;
    float m[3], vxm[3], vxp[3], vym[3], vyp[3], vzm[3], vzp[3], hd[3], mn[3], ka[3], o[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float *s = S + (size_t)a * n;
        m[a] = ld32(s, id);
        vxm[a] = ld32(s, xm);
        vxp[a] = ld32(s, xp);
        vym[a] = ld32(s, ym);
        vyp[a] = ld32(s, yp);
        vzm[a] = ld32(s, zm);
        vzp[a] = ld32(s, zp);
        hd[a] = ld32(Hd + (size_t)a * n, id);
        mn[a] = ld32(Mn + (size_t)a * n, id);
        ka[a] = (STAGE == 2 || STAGE == 3 || STAGE == 4) ? ld32(kacc + (size_t)a * n, id) : 0.f;
    }
    stage_cell<STAGE>(m, vxm, vxp, vym, vyp, vzm, vzp, hd, mn, ka, o, c);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if constexpr (STAGE == 1 || STAGE == 2 || STAGE == 3) st32(kacc + (size_t)a * n, id, ka[a]);
        st32(out + (size_t)a * n, id, o[a]);
    }
}

// W consecutive cells of one x row per thread (W = 2 or 4, nx % W == 0):
// every array is read and written with W-wide vector accesses; the x
// neighbours inside the group come from the group itself, the two outside
// it from single loads.  Same arithmetic per cell as stage_body.
template <int W> struct VecOf;
template <> struct VecOf<2> { typedef float2 T; };
template <> struct VecOf<4> { typedef float4 T; };

template <typename V>
__device__ __forceinline__ V ldv32(const float *base, unsigned idx)
{
    return *reinterpret_cast<const V *>(reinterpret_cast<const char *>(base) + (idx << 2));
}
template <typename V>
__device__ __forceinline__ void stv32(float *base, unsigned idx, const V &v)
{
    *reinterpret_cast<V *>(reinterpret_cast<char *>(base) + (idx << 2)) = v;
}

template <int W>
__device__ __forceinline__ float lane_of(const typename VecOf<W>::T &v, int e)
{
    if constexpr (W == 2) return e == 0 ? v.x : v.y;
    else return e == 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w));
}
template <int W>
__device__ __forceinline__ void set_lane(typename VecOf<W>::T &v, int e, float x)
{
    if constexpr (W == 2) { if (e == 0) v.x = x; else v.y = x; }
    else { if (e == 0) v.x = x; else if (e == 1) v.y = x; else if (e == 2) v.z = x; else v.w = x; }
}

template <int STAGE, int W>
__device__ __forceinline__ void stage_body_vec(const float *S, const float *__restrict__ Hd, const float *Mn,
                                               float *__restrict__ kacc, float *out, int nx, int ny, int nz,
                                               const StageCoef &c, unsigned g)
{
    typedef typename VecOf<W>::T V;
    const unsigned nxy = (unsigned)nx * (unsigned)ny;
    const unsigned n = nxy * (unsigned)nz;
    const unsigned id = g * W;  // first cell of the group
    if (id >= n) return;
    const unsigned k = id / nxy;
    const unsigned rem = id - k * nxy;
    const unsigned j = rem / (unsigned)nx;
    const unsigned i = rem - j * (unsigned)nx;
    const unsigned ym = j > 0 ? id - nx : id, yp = j + 1 < (unsigned)ny ? id + nx : id;
    const unsigned zm = k > 0 ? id - nxy : id, zp = k + 1 < (unsigned)nz ? id + nxy : id;
    V vs[3], vym[3], vyp[3], vzm[3], vzp[3], vhd[3], vmn[3], vka[3];
    float left[3], right[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float *s = S + (size_t)a * n;
        vs[a] = ldv32<V>(s, id);
        vym[a] = ldv32<V>(s, ym);
        vyp[a] = ldv32<V>(s, yp);
        vzm[a] = ldv32<V>(s, zm);
        vzp[a] = ldv32<V>(s, zp);
        // x neighbours outside the group: at a free edge the group's own end
        // cell, read again (not selected from vs, so the load is issued
        // unconditionally and never waits on vs)
        left[a] = ld32(s, i > 0 ? id - 1 : id);
        right[a] = ld32(s, i + W < (unsigned)nx ? id + W : id + W - 1);
        vhd[a] = ldv32<V>(Hd + (size_t)a * n, id);
        vmn[a] = ldv32<V>(Mn + (size_t)a * n, id);
        if constexpr (STAGE == 2 || STAGE == 3 || STAGE == 4) vka[a] = ldv32<V>(kacc + (size_t)a * n, id);
    }
    V vo[3], vk[3];
#pragma unroll
    for (int e = 0; e < W; ++e) {
        float m[3], xm[3], xp[3], y0[3], y1[3], z0[3], z1[3], hd[3], mn[3], ka[3], o[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            m[a] = lane_of<W>(vs[a], e);
            xm[a] = e > 0 ? lane_of<W>(vs[a], e - 1) : left[a];
            xp[a] = e + 1 < W ? lane_of<W>(vs[a], e + 1) : right[a];
            y0[a] = lane_of<W>(vym[a], e);
            y1[a] = lane_of<W>(vyp[a], e);
            z0[a] = lane_of<W>(vzm[a], e);
            z1[a] = lane_of<W>(vzp[a], e);
            hd[a] = lane_of<W>(vhd[a], e);
            mn[a] = lane_of<W>(vmn[a], e);
            ka[a] = (STAGE == 2 || STAGE == 3 || STAGE == 4) ? lane_of<W>(vka[a], e) : 0.f;
        }
        stage_cell<STAGE>(m, xm, xp, y0, y1, z0, z1, hd, mn, ka, o, c);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            set_lane<W>(vo[a], e, o[a]);
            set_lane<W>(vk[a], e, ka[a]);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if constexpr (STAGE == 1 || STAGE == 2 || STAGE == 3) stv32<V>(kacc + (size_t)a * n, id, vk[a]);
        stv32<V>(out + (size_t)a * n, id, vo[a]);
    }
}

}  // namespace mmk
