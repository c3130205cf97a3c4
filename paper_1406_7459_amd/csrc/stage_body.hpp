// stage_body.hpp -- per-cell part of a time step, shared by the per-plan and
// the batched launches: effective field of eq. (2) (exchange eq. (3)-(4)
// with free boundaries, uniaxial anisotropy eq. (5) in easy-axis form,
// Zeeman, plus the demag field), the Landau-Lifshitz right-hand side of
// eq. (6), and one stage of classical RK4 or an explicit Euler step.
#pragma once
#include <hip/hip_runtime.h>

#include "mm_internal.hpp"

namespace mmk {

// STAGE 1..4: RK4 stages; 0: Euler.  Reads the stage state S (with its six
// neighbours), the demag field Hd of S, the step's start state Mn and the
// accumulator; writes the accumulator and the next stage state `out`
// (stage 4 / Euler: the new state, renormalised if requested).
// Indices are 32-bit (a grid holds at most 512^3 cells, so byte offsets of
// one component stay below 2^32) and every array is addressed as a uniform
// per-component base plus one of seven per-thread offsets: the loads take
// the scalar-base form and the index arithmetic stays off the 64-bit path.
template <int STAGE>
__device__ __forceinline__ void stage_body(const float *S, const float *__restrict__ Hd, const float *Mn,
                                           float *__restrict__ kacc, float *out, int nx, int ny, int nz,
                                           const StageCoef &c, unsigned id)
{
    // fixed arithmetic in every file that includes this body (per-plan and
    // batched launches give bitwise the same states)
#pragma clang fp contract(off)
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
    float m[3], h[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float *s = S + (size_t)a * n;
        const float mc = s[id];
        m[a] = mc;
        h[a] = c.cx * (s[xm] + s[xp] - 2.f * mc) + c.cy * (s[ym] + s[yp] - 2.f * mc) +
               c.cz * (s[zm] + s[zp] - 2.f * mc) + (Hd + (size_t)a * n)[id];
    }
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
    float mn[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) mn[a] = (Mn + (size_t)a * n)[id];
    if constexpr (STAGE == 1 || STAGE == 2 || STAGE == 3) {
        const float step = STAGE == 3 ? c.dt : 0.5f * c.dt;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float *ka = kacc + (size_t)a * n;
            const float acc = STAGE == 1 ? f[a] : ka[id] + 2.f * f[a];
            ka[id] = acc;
            (out + (size_t)a * n)[id] = mn[a] + step * f[a];
        }
    } else {
        float r[3];
        if constexpr (STAGE == 4) {
            const float w = c.dt * (1.f / 6.f);
#pragma unroll
            for (int a = 0; a < 3; ++a) r[a] = mn[a] + w * ((kacc + (size_t)a * n)[id] + f[a]);
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) r[a] = mn[a] + c.dt * f[a];
        }
        if (c.renorm) {
            const float nn = sqrtf(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
            const float sc = nn > 0.f ? c.Ms / nn : 1.f;
#pragma unroll
            for (int a = 0; a < 3; ++a) r[a] *= sc;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) (out + (size_t)a * n)[id] = r[a];
    }
}

}  // namespace mmk
