// tensor.hip -- set-up of the demag kernel K = -N and of its transform
// (paper Sec. 2, eq. (7)/(12); the transform is taken once, remark after
// eq. (16)).  All of it runs in FP64 on the GPU:
//
//  1. N(i dx, j dy, k dz) on the octant i<nx, j<ny, k<nz, six components,
//     from the Newell-Williams-Dunlop closed form (27-point second
//     difference of f and g) for centre distances below 8 times the largest
//     cell edge, and beyond that from the pair-average of the point-dipole
//     kernel (tent weight, 4 Gauss-Legendre nodes per half-axis), where the
//     closed form loses digits to cancellation.
//  2. The transform of the padded, wrapped K over Lx x Ly x Lz (each L >= 2n;
//     L = 2n when n is 2^a, 3 2^a or 5 2^a): every component is even or odd in each
//     axis (N(-r) = N(r) componentwise up to the sign of the odd axes), so it
//     is real and equals separable cosine sums (even axes) and sine sums (odd
//     axes) over the octant of offsets X < n:
//       even:  K~(k) = K(0) + 2 sum_{1<=X<n} K(X) cos(2 pi k X / L)
//       odd:   K~(k) = -2i sum_{1<=X<n} K(X) sin(2 pi k X / L)
//     with the slots of offsets n .. L-n zero.  Each off-diagonal component
//     is odd in exactly two axes, so (-i)^2 = -1 makes it real too.  Three
//     dense FP64 contractions (x, then y, then z) produce the octant
//     0..L/2 of every axis, which holds the whole spectrum by parity.
//  3. K~ is scaled by the inverse-transform normalisation 1/(Lx Ly Lz)
//     (for nz = 1 the trivial z axis is dropped and 1/(Lx Ly) is used),
//     rounded once to FP32 and stored as a six-float record per octant
//     frequency, [kz][ky][kx][xx yy zz xy xz yz]: the spectral product reads
//     one 24-byte record per frequency.
#include <cmath>

#include "mm_internal.hpp"

namespace mmk {

// ----------------------------------------------------------- Newell f, g ---
// f(x,y,z): even in all arguments.
__device__ static double nw_f(double x, double y, double z)
{
    x = fabs(x);
    y = fabs(y);
    z = fabs(z);
    const double xx = x * x, yy = y * y, zz = z * z;
    const double rr = sqrt(xx + yy + zz);
    double acc = (2.0 * xx - yy - zz) * rr * (1.0 / 6.0);
    const double sxz = xx + zz, sxy = xx + yy;
    if (y > 0.0 && sxz > 0.0) acc += 0.5 * y * (zz - xx) * asinh(y / sqrt(sxz));
    if (z > 0.0 && sxy > 0.0) acc += 0.5 * z * (yy - xx) * asinh(z / sqrt(sxy));
    if (x > 0.0 && y > 0.0 && z > 0.0) acc -= x * y * z * atan((y * z) / (x * rr));
    return acc;
}

// g(x,y,z): odd in x and y, even in z.
__device__ static double nw_g(double x, double y, double z)
{
    double sgn = 1.0;
    if (x < 0.0) { sgn = -sgn; x = -x; }
    if (y < 0.0) { sgn = -sgn; y = -y; }
    z = fabs(z);
    const double xx = x * x, yy = y * y, zz = z * z;
    const double rr = sqrt(xx + yy + zz);
    double acc = -x * y * rr * (1.0 / 3.0);
    if (x > 0.0) acc += x * (3.0 * zz - xx) * (1.0 / 6.0) * asinh(y / sqrt(xx + zz));
    if (y > 0.0) acc += y * (3.0 * zz - yy) * (1.0 / 6.0) * asinh(x / sqrt(yy + zz));
    if (x > 0.0 && y > 0.0 && z > 0.0) {
        acc += x * y * z * asinh(z / sqrt(xx + yy));
        acc -= zz * z * (1.0 / 6.0) * atan((x * y) / (z * rr));
        acc -= 0.5 * z * yy * atan((x * z) / (y * rr));
        acc -= 0.5 * z * xx * atan((y * z) / (x * rr));
    }
    return sgn * acc;
}

// 27-point second difference of F around (X,Y,Z) with steps (a,b,c):
// weights -1, 2, -1 per axis, divided by 4 pi a b c.
template <bool USE_G>
__device__ static double nw_diff(double X, double Y, double Z, double a, double b, double c)
{
    double fv[27];
#pragma unroll
    for (int n = 0; n < 27; ++n) {
        const int i = n % 3 - 1, j = (n / 3) % 3 - 1, k = n / 9 - 1;
        fv[n] = USE_G ? nw_g(X + i * a, Y + j * b, Z + k * c) : nw_f(X + i * a, Y + j * b, Z + k * c);
    }
    double s = 0.0;
#pragma unroll
    for (int n = 0; n < 27; ++n) {
        const int i = n % 3, j = (n / 3) % 3, k = n / 9;
        const double w = (i == 1 ? 2.0 : -1.0) * (j == 1 ? 2.0 : -1.0) * (k == 1 ? 2.0 : -1.0);
        s += w * fv[n];
    }
    return s / (4.0 * M_PI * a * b * c);
}

// Pair-average of the point-dipole kernel over two cells at centre offset R:
// tent-weighted Gauss-Legendre, 4 nodes on each half [-d,0], [0,d] per axis.
__device__ static void nw_far(double X, double Y, double Z, double dx, double dy, double dz, double *out)
{
    const double gx[4] = {-0.86113631159405257522, -0.33998104358485626480, 0.33998104358485626480,
                          0.86113631159405257522};
    const double gw[4] = {0.34785484513745385737, 0.65214515486254614263, 0.65214515486254614263,
                          0.34785484513745385737};
    double ux[8], wx[8], uy[8], wy[8], uz[8], wz[8];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const double t = 0.5 * (gx[n] + 1.0);  // node in (0,1)
        const double tw = 0.5 * gw[n] * (1.0 - t);  // GL weight on [0,1] times tent
        ux[n] = t * dx;  ux[n + 4] = -t * dx;  wx[n] = wx[n + 4] = tw;
        uy[n] = t * dy;  uy[n + 4] = -t * dy;  wy[n] = wy[n + 4] = tw;
        uz[n] = t * dz;  uz[n + 4] = -t * dz;  wz[n] = wz[n + 4] = tw;
    }
    double sxx = 0, syy = 0, szz = 0, sxy = 0, sxz = 0, syz = 0;
    for (int a = 0; a < 8; ++a) {
        const double rx = X + ux[a];
        for (int b = 0; b < 8; ++b) {
            const double ry = Y + uy[b];
            const double wab = wx[a] * wy[b];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const double rz = Z + uz[c];
                const double r2 = rx * rx + ry * ry + rz * rz;
                const double ir = rsqrt(r2);
                const double ir2 = ir * ir;
                const double w = wab * wz[c] * ir2 * ir2 * ir;  // weight / r^5
                sxx += w * (r2 - 3.0 * rx * rx);
                syy += w * (r2 - 3.0 * ry * ry);
                szz += w * (r2 - 3.0 * rz * rz);
                sxy -= w * 3.0 * rx * ry;
                sxz -= w * 3.0 * rx * rz;
                syz -= w * 3.0 * ry * rz;
            }
        }
    }
    const double pre = dx * dy * dz / (4.0 * M_PI);
    out[0] = pre * sxx;
    out[1] = pre * syy;
    out[2] = pre * szz;
    out[3] = pre * sxy;
    out[4] = pre * sxz;
    out[5] = pre * syz;
}

__global__ void k_newell(double *__restrict__ N, int nx, int ny, int nz, double dx, double dy, double dz)
{
    const size_t n = (size_t)nx * ny * nz;
    const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    const int i = (int)(id % nx), j = (int)((id / nx) % ny), k = (int)(id / ((size_t)nx * ny));
    const double X = i * dx, Y = j * dy, Z = k * dz;
    const double dmax = fmax(dx, fmax(dy, dz));
    double t[6];
    if (X * X + Y * Y + Z * Z < 64.0 * dmax * dmax) {
        t[0] = nw_diff<false>(X, Y, Z, dx, dy, dz);
        t[1] = nw_diff<false>(Y, X, Z, dy, dx, dz);
        t[2] = nw_diff<false>(Z, Y, X, dz, dy, dx);
        t[3] = nw_diff<true>(X, Y, Z, dx, dy, dz);
        t[4] = nw_diff<true>(X, Z, Y, dx, dz, dy);
        t[5] = nw_diff<true>(Y, Z, X, dy, dz, dx);
    } else {
        nw_far(X, Y, Z, dx, dy, dz, t);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) N[c * n + id] = t[c];
}

// ------------------------------------------------- separable transforms ---
// component c is odd along axis a for these (c, a) pairs
__device__ __host__ static inline bool odd_axis(int c, int a)
{
    return (c == 3 && (a == 0 || a == 1)) || (c == 4 && (a == 0 || a == 2)) || (c == 5 && (a == 1 || a == 2));
}

// Contract the innermost-but-`stride` axis of n live offsets (octant
// 0..n-1) to the L/2 + 1 octant frequencies of the padded length L:
// out[.., k, ..] = sum_X w(k,X) in[.., X, ..].  Layout: `in` is
// [6][outer][n][inner], `out` is [6][outer][L/2+1][inner]; one thread per
// output element.  The trig table for the axis sits in LDS.
__global__ void k_axis_transform(const double *__restrict__ in, double *__restrict__ out, int n, int L,
                                 long long outer, long long inner, int axis)
{
    extern __shared__ double tab[];  // cos then sin of 2 pi m / L, m < L
    for (int m = threadIdx.x; m < L; m += blockDim.x) {
        double sv, cv;
        sincospi(2.0 * (double)m / (double)L, &sv, &cv);
        tab[m] = cv;
        tab[L + m] = sv;
    }
    __syncthreads();
    const int nk = L / 2 + 1;
    const long long per_c = outer * (long long)nk * inner;
    const long long total = 6 * per_c;
    for (long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x; id < total;
         id += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(id / per_c);
        long long r = id - c * per_c;
        const long long o = r / ((long long)nk * inner);
        r -= o * (long long)nk * inner;
        const int k = (int)(r / inner);
        const long long e = r - (long long)k * inner;
        const double *src = in + ((long long)c * outer + o) * (long long)n * inner + e;
        double acc = 0.0;
        if (odd_axis(c, axis)) {
            for (int X = 1; X < n; ++X) acc += 2.0 * tab[L + (int)(((long long)k * X) % L)] * src[(long long)X * inner];
        } else {
            acc = src[0];
            for (int X = 1; X < n; ++X) acc += 2.0 * tab[(int)(((long long)k * X) % L)] * src[(long long)X * inner];
        }
        out[id] = acc;
    }
}

// K~ = sign * scale * D in FP32; sign -1 for the diagonal (K = -N, all-cosine
// sums), +1 for the off-diagonals ((-i)^2 from the two sine axes times -1).
// For nz = 1 the odd-in-z components vanish identically and are written 0.
__global__ void k_spectrum_store(const double *__restrict__ D, float *__restrict__ Kt, long long per_c, int nxc,
                                 int xp, double scale, int zero_xz_yz)
{
    const long long total = 6 * per_c;
    for (long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x; id < total;
         id += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(id / per_c);
        const long long f = id - (long long)c * per_c;  // octant frequency
        const double sgn = c < 3 ? -1.0 : 1.0;
        double v = sgn * scale * D[id];
        if (zero_xz_yz && c >= 4) v = 0.0;
        const long long row = f / nxc;
        Kt[6 * (row * xp + (f - row * nxc)) + c] = (float)v;  // six-float record per frequency
    }
}

int newell_octant_device(int nx, int ny, int nz, double dx, double dy, double dz, double *N,
                         hipStream_t s)
{
    const size_t n = (size_t)nx * ny * nz;
    const int bs = 128;
    hipLaunchKernelGGL(k_newell, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, N, nx, ny, nz, dx, dy, dz);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MM_EHIP, std::string("k_newell: ") + hipGetErrorString(e));
    return MM_OK;
}

static int axis_transform(const double *in, double *out, int n, int L, long long outer, long long inner, int axis,
                          hipStream_t s)
{
    const long long total = 6 * outer * (long long)(L / 2 + 1) * inner;
    const int bs = 256;
    long long blocks = (total + bs - 1) / bs;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_axis_transform, dim3((unsigned)blocks), dim3(bs), 2 * L * sizeof(double), s, in, out,
                       n, L, outer, inner, axis);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MM_EHIP, std::string("k_axis_transform: ") + hipGetErrorString(e));
    return MM_OK;
}

// Two FP64 scratch arrays: A holds the tensor octant and the x-y transform,
// B the x transform and the z transform.
static void scratch_sizes(int nx, int ny, int nz, int Lx, int Ly, int Lz, size_t &big, size_t &big2)
{
    const size_t n = (size_t)nx * ny * nz;
    const size_t kx = Lx / 2 + 1, ky = Ly / 2 + 1, kz = nz > 1 ? Lz / 2 + 1 : 1;
    const size_t sz_a = 6 * n;
    const size_t sz_b = 6 * (size_t)nz * ny * kx;
    const size_t sz_c = 6 * (size_t)nz * ky * kx;
    const size_t sz_d = 6 * kz * ky * kx;
    big = sz_a > sz_c ? sz_a : sz_c;
    big2 = sz_b > sz_d ? sz_b : sz_d;
}

size_t spectrum_scratch_bytes(int nx, int ny, int nz, int Lx, int Ly, int Lz)
{
    size_t big, big2;
    scratch_sizes(nx, ny, nz, Lx, Ly, Lz, big, big2);
    return (((big * sizeof(double)) + 255) & ~(size_t)255) + big2 * sizeof(double);
}

// K~ into p.Kt, with the FP64 scratch in the plan's run-time region (the
// workspace is bound and no step has run yet).
int build_spectrum(Plan &p, hipStream_t s)
{
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int kx = p.Lx / 2 + 1, ky = p.Ly / 2 + 1;
    size_t big, big2;
    scratch_sizes(nx, ny, nz, p.Lx, p.Ly, p.Lz, big, big2);
    double *A = reinterpret_cast<double *>(p.run);
    double *B = reinterpret_cast<double *>(p.run + (((big * sizeof(double)) + 255) & ~(size_t)255));
    int rc = newell_octant_device(nx, ny, nz, p.dx, p.dy, p.dz, A, s);
    // x: A[6][nz*ny][nx] -> B[6][nz*ny][kx]
    if (rc == MM_OK) rc = axis_transform(A, B, nx, p.Lx, (long long)nz * ny, 1, 0, s);
    // y: B[6][nz][ny][kx] -> A[6][nz][ky][kx]
    if (rc == MM_OK) rc = axis_transform(B, A, ny, p.Ly, nz, kx, 1, s);
    const double *D = A;
    double scale;
    if (nz > 1) {
        // z: A[6][nz][ky kx] -> B[6][Lz/2+1][ky kx]
        if (rc == MM_OK) rc = axis_transform(A, B, nz, p.Lz, 1, (long long)ky * kx, 2, s);
        D = B;
        scale = 1.0 / ((double)p.Lx * p.Ly * p.Lz);
    } else {
        scale = 1.0 / ((double)p.Lx * p.Ly);
    }
    if (rc == MM_OK) {
        const long long per_c = (long long)p.nzK * ky * kx;
        long long blocks = (6 * per_c + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(k_spectrum_store, dim3((unsigned)blocks), dim3(256), 0, s, D, p.Kt, per_c, kx, p.xp, scale,
                           nz == 1 ? 1 : 0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) rc = fail(MM_EHIP, std::string("k_spectrum_store: ") + hipGetErrorString(e));
    }
    hipError_t e = hipStreamSynchronize(s);
    if (rc == MM_OK && e != hipSuccess) rc = fail(MM_EHIP, std::string("spectrum sync: ") + hipGetErrorString(e));
    return rc;
}

}  // namespace mmk
