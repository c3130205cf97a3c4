// llg.hip -- the per-cell part of a time step: effective field of eq. (2)
// (exchange eq. (3)-(4) with free boundaries, uniaxial anisotropy eq. (5) in
// easy-axis form, Zeeman, plus the demag field computed by demag.hip), the
// Landau-Lifshitz right-hand side of eq. (6) and one stage of classical RK4
// (or an explicit Euler step, the integrator of the paper's timings), fused
// into one memory-bound kernel; and the FP64 observables reduction.
#include <cmath>

#include "mm_internal.hpp"
#include "stage_body.hpp"

namespace mmk {

template <int STAGE>
__global__ __launch_bounds__(256) void k_stage(const float *S, const float *__restrict__ Hd, const float *Mn,
                                               float *__restrict__ kacc, float *out, int nx, int ny, int nz,
                                               StageCoef c)
{
    const unsigned b = xcd_block(blockIdx.x, gridDim.x);  // each XCD a slab of cells
    stage_body<STAGE>(S, Hd, Mn, kacc, out, nx, ny, nz, c, b * blockDim.x + threadIdx.x);
}

template <int STAGE, int W>
__global__ __launch_bounds__(256) void k_stage_vec(const float *S, const float *__restrict__ Hd, const float *Mn,
                                                   float *__restrict__ kacc, float *out, int nx, int ny, int nz,
                                                   StageCoef c)
{
    const unsigned b = xcd_block(blockIdx.x, gridDim.x);
    stage_body_vec<STAGE, W>(S, Hd, Mn, kacc, out, nx, ny, nz, c, b * blockDim.x + threadIdx.x);
}

StageCoef stage_coef(const Plan &p, const mm_llg_params &q)
{
    const double mu0 = 4e-7 * M_PI;
    const double ex = 2.0 * q.A / (mu0 * q.Ms * q.Ms);
    StageCoef c{};
    c.cx = p.nx > 1 ? (float)(ex / (p.dx * p.dx)) : 0.f;
    c.cy = p.ny > 1 ? (float)(ex / (p.dy * p.dy)) : 0.f;
    c.cz = p.nz > 1 ? (float)(ex / (p.dz * p.dz)) : 0.f;
    c.ka = (float)(2.0 * q.Ku / (mu0 * q.Ms * q.Ms));
    c.ux = (float)q.axis[0];
    c.uy = (float)q.axis[1];
    c.uz = (float)q.axis[2];
    c.hx = (float)q.Hext[0];
    c.hy = (float)q.Hext[1];
    c.hz = (float)q.Hext[2];
    const double g = q.gamma0 / (1.0 + q.alpha * q.alpha);
    c.g = (float)g;
    c.gd = (float)(q.alpha * g / q.Ms);
    c.dt = (float)q.dt;
    c.Ms = (float)q.Ms;
    c.renorm = q.renorm;
    return c;
}

template <int STAGE>
static int launch_stage(Plan &p, const float *S, const float *Mn, float *out, const StageCoef &c, hipStream_t s,
                        const float *Hd = nullptr)
{
    if (!Hd) Hd = p.H;
    const size_t n = (size_t)p.cells();
    const int bs = 256;
    // vector width: the plan's stage tile, if every array is aligned for it
    int W = p.tile[MM_PASS_STAGE];
    auto aligned = [](const void *q, int w) { return ((uintptr_t)q % (sizeof(float) * w)) == 0; };
    while (W > 1 && (p.nx % W != 0 || !aligned(S, W) || !aligned(Hd, W) || !aligned(Mn, W) || !aligned(out, W) ||
                     !aligned(p.kacc, W)))
        W /= 2;
    const size_t threads = (n + W - 1) / W;
    const dim3 grid((unsigned)((threads + bs - 1) / bs));
    timing_arm(p);
    if (W == 4)
        MMK_LAUNCH(p, (k_stage_vec<STAGE, 4>), grid, dim3(bs), 0, s, S, Hd, Mn, p.kacc, out, p.nx, p.ny, p.nz, c);
    else if (W == 2)
        MMK_LAUNCH(p, (k_stage_vec<STAGE, 2>), grid, dim3(bs), 0, s, S, Hd, Mn, p.kacc, out, p.nx, p.ny, p.nz, c);
    else
        MMK_LAUNCH(p, k_stage<STAGE>, grid, dim3(bs), 0, s, S, Hd, Mn, p.kacc, out, p.nx, p.ny, p.nz, c);
    timing_file(p, MM_PASS_STAGE);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MM_EHIP, std::string("k_stage: ") + hipGetErrorString(e));
    return MM_OK;
}

// One step; on return M holds the new state.  RK4: S_1 = M, S_2 = Sa,
// S_3 = Sb, S_4 = Sa; stage 4 writes M in place (each cell reads only its own
// M there, neighbours come from Sa).  Euler: M -> Sa, then Sa is copied back
// (a pair of Euler steps, llg_enqueue_euler_pair, needs no copy).
// With the fused pass (tile of MM_PASS_XSTAGE > 0) a stage's field never
// leaves the chip: XFWD(M), then per stage the middle demag passes and one
// fused x-inverse / stage / x-forward launch (the last stage without the
// forward part).
int llg_enqueue_step(Plan &p, const StageCoef &c, int integrator, float *M, hipStream_t s)
{
    int rc;
    const size_t bytes = sizeof(float) * 3 * (size_t)p.cells();
    const bool fused = p.tile[MM_PASS_XSTAGE] > 0;
    if (integrator == MM_EULER) {
        if (fused) {
            if ((rc = launch_pass(p, MM_PASS_XFWD, M, nullptr, s)) != MM_OK) return rc;
            if ((rc = demag_mid_enqueue(p, s)) != MM_OK) return rc;
            if ((rc = launch_xstage(p, 0, false, M, M, p.Sa, c, s)) != MM_OK) return rc;
        } else {
            if ((rc = demag_enqueue(p, M, p.H, s)) != MM_OK) return rc;
            if ((rc = launch_stage<0>(p, M, M, p.Sa, c, s)) != MM_OK) return rc;
        }
        MMK_HIP(hipMemcpyAsync(M, p.Sa, bytes, hipMemcpyDeviceToDevice, s));
        return MM_OK;
    }
    if (fused) {
        if ((rc = launch_pass(p, MM_PASS_XFWD, M, nullptr, s)) != MM_OK) return rc;
        if ((rc = demag_mid_enqueue(p, s)) != MM_OK) return rc;
        if ((rc = launch_xstage(p, 1, true, M, M, p.Sa, c, s)) != MM_OK) return rc;
        if ((rc = demag_mid_enqueue(p, s)) != MM_OK) return rc;
        if ((rc = launch_xstage(p, 2, true, p.Sa, M, p.Sb, c, s)) != MM_OK) return rc;
        if ((rc = demag_mid_enqueue(p, s)) != MM_OK) return rc;
        if ((rc = launch_xstage(p, 3, true, p.Sb, M, p.Sa, c, s)) != MM_OK) return rc;
        if ((rc = demag_mid_enqueue(p, s)) != MM_OK) return rc;
        return launch_xstage(p, 4, false, p.Sa, M, M, c, s);
    }
    if ((rc = demag_enqueue(p, M, p.H, s)) != MM_OK) return rc;
    if ((rc = launch_stage<1>(p, M, M, p.Sa, c, s)) != MM_OK) return rc;
    if ((rc = demag_enqueue(p, p.Sa, p.H, s)) != MM_OK) return rc;
    if ((rc = launch_stage<2>(p, p.Sa, M, p.Sb, c, s)) != MM_OK) return rc;
    if ((rc = demag_enqueue(p, p.Sb, p.H, s)) != MM_OK) return rc;
    if ((rc = launch_stage<3>(p, p.Sb, M, p.Sa, c, s)) != MM_OK) return rc;
    if ((rc = demag_enqueue(p, p.Sa, p.H, s)) != MM_OK) return rc;
    return launch_stage<4>(p, p.Sa, M, M, c, s);
}

// Two explicit Euler steps, M -> Sa -> M: the state alternates between the
// two buffers and nothing is copied.
int llg_enqueue_euler_pair(Plan &p, const StageCoef &c, float *M, hipStream_t s)
{
    int rc;
    if (p.tile[MM_PASS_XSTAGE] > 0) {
        if ((rc = launch_pass(p, MM_PASS_XFWD, M, nullptr, s)) != MM_OK) return rc;
        if ((rc = demag_mid_enqueue(p, s)) != MM_OK) return rc;
        if ((rc = launch_xstage(p, 0, true, M, M, p.Sa, c, s)) != MM_OK) return rc;
        if ((rc = demag_mid_enqueue(p, s)) != MM_OK) return rc;
        return launch_xstage(p, 0, false, p.Sa, p.Sa, M, c, s);
    }
    if ((rc = demag_enqueue(p, M, p.H, s)) != MM_OK) return rc;
    if ((rc = launch_stage<0>(p, M, M, p.Sa, c, s)) != MM_OK) return rc;
    if ((rc = demag_enqueue(p, p.Sa, p.H, s)) != MM_OK) return rc;
    return launch_stage<0>(p, p.Sa, p.Sa, M, c, s);
}

// RK4 step whose stage-1 field is given (H1, the field of M) and whose
// stage 2-4 fields come from `field(stage, S, H)` (written into p.H).
int llg_step_with_fields(Plan &p, const StageCoef &c, float *M, const float *H1, hipStream_t s,
                         const std::function<int(int, const float *, float *)> &field)
{
    int rc;
    if ((rc = launch_stage<1>(p, M, M, p.Sa, c, s, H1)) != MM_OK) return rc;
    if ((rc = field(2, p.Sa, p.H)) != MM_OK) return rc;
    if ((rc = launch_stage<2>(p, p.Sa, M, p.Sb, c, s)) != MM_OK) return rc;
    if ((rc = field(3, p.Sb, p.H)) != MM_OK) return rc;
    if ((rc = launch_stage<3>(p, p.Sb, M, p.Sa, c, s)) != MM_OK) return rc;
    if ((rc = field(4, p.Sa, p.H)) != MM_OK) return rc;
    return launch_stage<4>(p, p.Sa, M, M, c, s);
}

// ------------------------------------------------------------- reduction ---
// Per cell, in FP64 from the FP32 state: exchange link energy (+x, +y, +z
// links inside the sample), anisotropy Ku(|m|^2 - (u.m)^2), H_d.M, H_ext.M,
// |M x H_eff|/Ms, M/Ms, and a non-finite count.  Wave64 shuffles, then one
// partial per block; a single-block pass combines the partials in a fixed
// order (no float atomics: bitwise reproducible).
constexpr int RED_VALS = 9;  // ex, an, d, z, mx, my, mz, nonfinite, torque_max

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_down(v, o, 64);
        v = (w > v || w != w) ? w : v;
    }
    return v;
}

__global__ __launch_bounds__(256) void k_reduce_cells(const float *__restrict__ M, const float *__restrict__ Hd,
                                                      double *__restrict__ part, int nx, int ny, int nz,
                                                      ReduceCoef c)
{
    const size_t n = (size_t)nx * ny * nz;
    double acc[RED_VALS] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const double iMs = 1.0 / c.Ms;
    for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(id % nx);
        const int j = (int)((id / nx) % ny);
        const int k = (int)(id / ((size_t)nx * ny));
        const size_t sy = nx, sz = (size_t)nx * ny;
        double m[3], mxp[3], myp[3], mzp[3], lap[3];
        bool finite = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float *s = M + a * n;
            const float v = s[id];
            finite = finite && isfinite(v);
            m[a] = v;
            // a missing neighbour reads the cell itself (clamped index: every
            // load is issued unconditionally)
            const double xm = s[i > 0 ? id - 1 : id], xp = s[i < nx - 1 ? id + 1 : id];
            const double ym = s[j > 0 ? id - sy : id], yp = s[j < ny - 1 ? id + sy : id];
            const double zm = s[k > 0 ? id - sz : id], zp = s[k < nz - 1 ? id + sz : id];
            mxp[a] = xp;
            myp[a] = yp;
            mzp[a] = zp;
            lap[a] = c.cx * (xp + xm - 2.0 * m[a]) + c.cy * (yp + ym - 2.0 * m[a]) + c.cz * (zp + zm - 2.0 * m[a]);
        }
        double ex = 0.0;
        if (i < nx - 1) {
            double t = 0;
            for (int a = 0; a < 3; ++a) t += (mxp[a] - m[a]) * (mxp[a] - m[a]);
            ex += t / (c.dx * c.dx);
        }
        if (j < ny - 1) {
            double t = 0;
            for (int a = 0; a < 3; ++a) t += (myp[a] - m[a]) * (myp[a] - m[a]);
            ex += t / (c.dy * c.dy);
        }
        if (k < nz - 1) {
            double t = 0;
            for (int a = 0; a < 3; ++a) t += (mzp[a] - m[a]) * (mzp[a] - m[a]);
            ex += t / (c.dz * c.dz);
        }
        const double hd[3] = {Hd[id], Hd[n + id], Hd[2 * n + id]};
        const double um = c.ux * m[0] + c.uy * m[1] + c.uz * m[2];
        const double mm = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
        const double h0 = lap[0] + c.ka * um * c.ux + hd[0] + c.hx;
        const double h1 = lap[1] + c.ka * um * c.uy + hd[1] + c.hy;
        const double h2 = lap[2] + c.ka * um * c.uz + hd[2] + c.hz;
        const double t0 = m[1] * h2 - m[2] * h1, t1 = m[2] * h0 - m[0] * h2, t2 = m[0] * h1 - m[1] * h0;
        const double tq = sqrt(t0 * t0 + t1 * t1 + t2 * t2) * iMs;
        acc[0] += ex * iMs * iMs;
        acc[1] += c.Ku * (mm - um * um) * iMs * iMs;
        acc[2] += hd[0] * m[0] + hd[1] * m[1] + hd[2] * m[2];
        acc[3] += c.hx * m[0] + c.hy * m[1] + c.hz * m[2];
        acc[4] += m[0] * iMs;
        acc[5] += m[1] * iMs;
        acc[6] += m[2] * iMs;
        acc[7] += finite ? 0.0 : 1.0;
        acc[8] = (tq > acc[8] || tq != tq) ? tq : acc[8];
    }
    __shared__ double sh[RED_VALS][4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < RED_VALS; ++v) {
        const double r = v == 8 ? wave_max(acc[v]) : wave_sum(acc[v]);
        if (lane == 0) sh[v][wid] = r;
    }
    __syncthreads();
    if (threadIdx.x < RED_VALS) {
        const int v = threadIdx.x;
        double r = sh[v][0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
            const double x = sh[v][w];
            r = v == 8 ? ((x > r || x != x) ? x : r) : r + x;
        }
        part[(size_t)blockIdx.x * RED_VALS + v] = r;
    }
}

// One wave per quantity: lane l sums partials l, l+64, ... in order, then a
// fixed shuffle tree -- the same order on every run.
__global__ __launch_bounds__(64 * RED_VALS) void k_reduce_final(const double *__restrict__ part, int nblocks,
                                                                double *__restrict__ out)
{
    const int v = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double r = v == 8 ? 0.0 : 0.0;
    for (int b = lane; b < nblocks; b += 64) {
        const double x = part[(size_t)b * RED_VALS + v];
        r = v == 8 ? ((x > r || x != x) ? x : r) : r + x;
    }
    r = v == 8 ? wave_max(r) : wave_sum(r);
    if (lane == 0) out[v] = r;
}

int reduce_enqueue(Plan &p, const mm_llg_params &q, const float *M, const float *Hd, hipStream_t s, int slot)
{
    const double mu0 = 4e-7 * M_PI;
    const double ex = 2.0 * q.A / (mu0 * q.Ms * q.Ms);
    ReduceCoef c{};
    c.cx = p.nx > 1 ? ex / (p.dx * p.dx) : 0.0;
    c.cy = p.ny > 1 ? ex / (p.dy * p.dy) : 0.0;
    c.cz = p.nz > 1 ? ex / (p.dz * p.dz) : 0.0;
    c.ka = 2.0 * q.Ku / (mu0 * q.Ms * q.Ms);
    c.ux = q.axis[0];
    c.uy = q.axis[1];
    c.uz = q.axis[2];
    c.hx = q.Hext[0];
    c.hy = q.Hext[1];
    c.hz = q.Hext[2];
    c.Ms = q.Ms;
    c.A = q.A;
    c.Ku = q.Ku;
    c.dx = p.dx;
    c.dy = p.dy;
    c.dz = p.dz;
    hipEvent_t ev0 = nullptr;
    timing_begin(p, MM_PASS_REDUCE, s, &ev0);
    hipLaunchKernelGGL(k_reduce_cells, dim3(p.red_blocks), dim3(256), 0, s, M, Hd, p.part, p.nx, p.ny, p.nz, c);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(64 * RED_VALS), 0, s, p.part, p.red_blocks,
                       p.red + 16 * (size_t)slot);
    timing_end(p, MM_PASS_REDUCE, s, ev0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MM_EHIP, std::string("reduce: ") + hipGetErrorString(e));
    return MM_OK;
}

// Observables (eq. (1) energies with V = dx dy dz per cell, max torque, <m>,
// non-finite count) from one reduction record of RED_VALS sums.
void stats_from_record(const Plan &p, const mm_llg_params &q, const double *r, mm_stats *out)
{
    const double mu0 = 4e-7 * M_PI;
    const double V = p.dx * p.dy * p.dz;
    const double N = (double)p.cells();
    out->E_ex = q.A * V * r[0];
    out->E_an = V * r[1];
    out->E_d = -0.5 * mu0 * V * r[2];
    out->E_z = -mu0 * V * r[3];
    out->E_tot = out->E_ex + out->E_an + out->E_d + out->E_z;
    out->m_avg[0] = r[4] / N;
    out->m_avg[1] = r[5] / N;
    out->m_avg[2] = r[6] / N;
    out->nonfinite = (long long)r[7];
    out->torque_max = r[8];
}

}  // namespace mmk
