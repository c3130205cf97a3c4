/*
 * mm_oracle.c -- plain, slow, single-threaded FP64 CPU reference for the
 * per-step hot path of a finite-difference micromagnetic solver: the
 * zero-padded FFT demagnetising field and the Landau-Lifshitz-Gilbert update
 * (R. Zhu, "Speedup of Micromagnetic Simulations with C++ AMP on Graphics
 * Processing Units", arXiv:1406.7459).
 *
 * THIS FILE IS TEST INFRASTRUCTURE.  Only the test suite, the smoke entry
 * point and the CPU-baseline leg of the benchmark may load it.  The GPU
 * library never links, includes or calls it, and it shares no code, header,
 * table or constant generator with the GPU library.
 *
 * Every routine follows the definition it cites as directly as possible:
 * no blocking, no fusion, no pruning, no symmetry folding beyond what the
 * cited passage states.  Where the paper is silent the reading adopted is
 * named in the comment (readings R1..R22 of the design notes).
 *
 * Layout: every field is an array [3][nz][ny][nx] of doubles, x fastest,
 * cells zero-indexed (paper, Sec. 2, cell labelling).
 * Units: SI, fields in A/m, lengths in m, energies in J.
 */
#include <complex.h>
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PI_D 3.14159265358979323846264338327950288
#define MU0 (4.0e-7 * PI_D) /* vacuum permeability, N/A^2 */

/* ------------------------------------------------------------------------ */
/* Newell, Williams & Dunlop (1993) cell-averaged demagnetising tensor.      */
/* The paper defers the tensor formula to its refs. [10], [11] (Sec. 2,      */
/* eq. (7) and (12)); the cell-averaged Newell tensor is the reading used    */
/* (R8) with K = -N.                                                         */
/* ------------------------------------------------------------------------ */

/* f(x,y,z), even in every argument.  Terms whose prefactor vanishes are 0. */
static double newell_f(double x, double y, double z)
{
    x = fabs(x); y = fabs(y); z = fabs(z);
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = sqrt(x2 + y2 + z2);
    double r = 0.0;
    if (y > 0.0 && x2 + z2 > 0.0) r += 0.5 * y * (z2 - x2) * asinh(y / sqrt(x2 + z2));
    if (z > 0.0 && x2 + y2 > 0.0) r += 0.5 * z * (y2 - x2) * asinh(z / sqrt(x2 + y2));
    if (x > 0.0 && y > 0.0 && z > 0.0) r -= x * y * z * atan(y * z / (x * R));
    r += (2.0 * x2 - y2 - z2) * R / 6.0;
    return r;
}

/* g(x,y,z), odd in x and in y, even in z. */
static double newell_g(double x, double y, double z)
{
    const double s = (x < 0.0 ? -1.0 : 1.0) * (y < 0.0 ? -1.0 : 1.0);
    x = fabs(x); y = fabs(y); z = fabs(z);
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = sqrt(x2 + y2 + z2);
    double r = 0.0;
    if (x > 0.0 && y > 0.0 && z > 0.0) r += x * y * z * asinh(z / sqrt(x2 + y2));
    if (y > 0.0) r += y / 6.0 * (3.0 * z2 - y2) * asinh(x / sqrt(y2 + z2));
    if (x > 0.0) r += x / 6.0 * (3.0 * z2 - x2) * asinh(y / sqrt(x2 + z2));
    if (z > 0.0 && x > 0.0 && y > 0.0) r -= z2 * z / 6.0 * atan(x * y / (z * R));
    if (z > 0.0 && y > 0.0 && x > 0.0) r -= z * y2 / 2.0 * atan(x * z / (y * R));
    if (z > 0.0 && x > 0.0 && y > 0.0) r -= z * x2 / 2.0 * atan(y * z / (x * R));
    r -= x * y * R / 3.0;
    return s * r;
}

/* 27-point second difference with weights 2 (centre), -1 (+-1) per axis. */
static const double W3[3] = {-1.0, 2.0, -1.0};

static double newell_xx(double X, double Y, double Z, double dx, double dy, double dz)
{
    double acc = 0.0;
    for (int a = -1; a <= 1; a++)
        for (int b = -1; b <= 1; b++)
            for (int c = -1; c <= 1; c++)
                acc += W3[a + 1] * W3[b + 1] * W3[c + 1] *
                       newell_f(X + a * dx, Y + b * dy, Z + c * dz);
    return acc / (4.0 * PI_D * dx * dy * dz);
}

static double newell_xy(double X, double Y, double Z, double dx, double dy, double dz)
{
    double acc = 0.0;
    for (int a = -1; a <= 1; a++)
        for (int b = -1; b <= 1; b++)
            for (int c = -1; c <= 1; c++)
                acc += W3[a + 1] * W3[b + 1] * W3[c + 1] *
                       newell_g(X + a * dx, Y + b * dy, Z + c * dz);
    return acc / (4.0 * PI_D * dx * dy * dz);
}

/* Component order everywhere: xx, yy, zz, xy, xz, yz. */
void oracle_newell_exact(double X, double Y, double Z, double dx, double dy, double dz,
                         double N[6])
{
    N[0] = newell_xx(X, Y, Z, dx, dy, dz);
    N[1] = newell_xx(Y, X, Z, dy, dx, dz);
    N[2] = newell_xx(Z, Y, X, dz, dy, dx);
    N[3] = newell_xy(X, Y, Z, dx, dy, dz);
    N[4] = newell_xy(X, Z, Y, dx, dz, dy);
    N[5] = newell_xy(Y, Z, X, dy, dz, dx);
}

/* Same f/g/second-difference, evaluated in binary128 (ground truth for pins). */
static __float128 qf(__float128 x, __float128 y, __float128 z)
{
    x = fabsq(x); y = fabsq(y); z = fabsq(z);
    const __float128 x2 = x * x, y2 = y * y, z2 = z * z;
    const __float128 R = sqrtq(x2 + y2 + z2);
    __float128 r = 0;
    if (y > 0 && x2 + z2 > 0) r += y / 2 * (z2 - x2) * asinhq(y / sqrtq(x2 + z2));
    if (z > 0 && x2 + y2 > 0) r += z / 2 * (y2 - x2) * asinhq(z / sqrtq(x2 + y2));
    if (x > 0 && y > 0 && z > 0) r -= x * y * z * atanq(y * z / (x * R));
    r += (2 * x2 - y2 - z2) * R / 6;
    return r;
}

static __float128 qg(__float128 x, __float128 y, __float128 z)
{
    const __float128 s = (x < 0 ? -1 : 1) * (y < 0 ? -1 : 1);
    x = fabsq(x); y = fabsq(y); z = fabsq(z);
    const __float128 x2 = x * x, y2 = y * y, z2 = z * z;
    const __float128 R = sqrtq(x2 + y2 + z2);
    __float128 r = 0;
    if (x > 0 && y > 0 && z > 0) r += x * y * z * asinhq(z / sqrtq(x2 + y2));
    if (y > 0) r += y / 6 * (3 * z2 - y2) * asinhq(x / sqrtq(y2 + z2));
    if (x > 0) r += x / 6 * (3 * z2 - x2) * asinhq(y / sqrtq(x2 + z2));
    if (z > 0 && x > 0 && y > 0) r -= z2 * z / 6 * atanq(x * y / (z * R));
    if (z > 0 && y > 0 && x > 0) r -= z * y2 / 2 * atanq(x * z / (y * R));
    if (z > 0 && x > 0 && y > 0) r -= z * x2 / 2 * atanq(y * z / (x * R));
    r -= x * y * R / 3;
    return s * r;
}

static double q_xx(double X, double Y, double Z, double dx, double dy, double dz, int use_g)
{
    __float128 acc = 0;
    for (int a = -1; a <= 1; a++)
        for (int b = -1; b <= 1; b++)
            for (int c = -1; c <= 1; c++) {
                const __float128 x = (__float128)X + a * (__float128)dx;
                const __float128 y = (__float128)Y + b * (__float128)dy;
                const __float128 z = (__float128)Z + c * (__float128)dz;
                acc += (__float128)(W3[a + 1] * W3[b + 1] * W3[c + 1]) *
                       (use_g ? qg(x, y, z) : qf(x, y, z));
            }
    return (double)(acc / (4 * M_PIq * (__float128)dx * (__float128)dy * (__float128)dz));
}

void oracle_newell_q128(double X, double Y, double Z, double dx, double dy, double dz,
                        double N[6])
{
    N[0] = q_xx(X, Y, Z, dx, dy, dz, 0);
    N[1] = q_xx(Y, X, Z, dy, dx, dz, 0);
    N[2] = q_xx(Z, Y, X, dz, dy, dx, 0);
    N[3] = q_xx(X, Y, Z, dx, dy, dz, 1);
    N[4] = q_xx(X, Z, Y, dx, dz, dy, 1);
    N[5] = q_xx(Y, Z, X, dy, dz, dx, 1);
}

/* Gauss-Legendre nodes/weights on [-1,1] by Newton iteration on P_p. */
static void gauss_legendre(int p, double *xs, double *ws)
{
    for (int i = 0; i < p; i++) {
        double x = cos(PI_D * (i + 0.75) / (p + 0.5));
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= p; k++) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            /* p1 = P_p(x), p0 = P_{p-1}(x) */
            const double dp = p * (x * p1 - p0) / (x * x - 1.0);
            const double dxn = p1 / dp;
            x -= dxn;
            if (fabs(dxn) < 1e-16) break;
        }
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= p; k++) {
            const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        const double dp = p * (x * p1 - p0) / (x * x - 1.0);
        xs[i] = x;
        ws[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

/*
 * Far field: the cell-pair average of the point-dipole kernel.  The average
 * over source and observer positions uniformly distributed in two cells is an
 * integral of D(R+u) against the tent weight T(u) = prod_a (1-|u_a|/d_a)/d_a on
 * [-d_a, d_a]; it is done with p Gauss-Legendre nodes on each half [-d,0],
 * [0,d] of every axis.  D_ij(r) = V (delta_ij r^2 - 3 r_i r_j) / (4 pi r^5).
 */
void oracle_newell_far(double X, double Y, double Z, double dx, double dy, double dz,
                       int p, double N[6])
{
    double gx[16], gw[16];
    if (p < 1) p = 1;
    if (p > 16) p = 16;
    gauss_legendre(p, gx, gw);
    const double d[3] = {dx, dy, dz};
    double u[3][32], w[3][32];
    for (int a = 0; a < 3; a++) {
        for (int i = 0; i < p; i++) {
            /* [0, d]: u = d (x+1)/2, du = d/2 dx */
            const double up = 0.5 * d[a] * (gx[i] + 1.0);
            const double tw = (1.0 - up / d[a]) / d[a];
            u[a][i] = up;
            w[a][i] = 0.5 * d[a] * gw[i] * tw;
            u[a][p + i] = -up;
            w[a][p + i] = 0.5 * d[a] * gw[i] * tw;
        }
    }
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int i = 0; i < 2 * p; i++)
        for (int j = 0; j < 2 * p; j++)
            for (int k = 0; k < 2 * p; k++) {
                const double rx = X + u[0][i], ry = Y + u[1][j], rz = Z + u[2][k];
                const double r2 = rx * rx + ry * ry + rz * rz;
                const double r = sqrt(r2);
                const double inv5 = 1.0 / (r2 * r2 * r);
                const double wt = w[0][i] * w[1][j] * w[2][k];
                acc[0] += wt * (r2 - 3.0 * rx * rx) * inv5;
                acc[1] += wt * (r2 - 3.0 * ry * ry) * inv5;
                acc[2] += wt * (r2 - 3.0 * rz * rz) * inv5;
                acc[3] += wt * (-3.0 * rx * ry) * inv5;
                acc[4] += wt * (-3.0 * rx * rz) * inv5;
                acc[5] += wt * (-3.0 * ry * rz) * inv5;
            }
    const double V = dx * dy * dz;
    for (int c = 0; c < 6; c++) N[c] = V * acc[c] / (4.0 * PI_D);
}

/* Switch radius (in units of the largest cell edge) and quadrature order. */
static const double ORACLE_RC = 8.0;
static const int ORACLE_P = 4;

/* Production form of the tensor at one signed offset (X,Y,Z) in metres: the
 * exact f/g form near the origin, where it is accurate in FP64, and the
 * tent-weighted quadrature beyond, where the 27-term sum cancels badly. */
void oracle_newell(double X, double Y, double Z, double dx, double dy, double dz,
                   double N[6])
{
    double dmax = dx;
    if (dy > dmax) dmax = dy;
    if (dz > dmax) dmax = dz;
    const double R = sqrt(X * X + Y * Y + Z * Z);
    if (R < ORACLE_RC * dmax)
        oracle_newell_exact(X, Y, Z, dx, dy, dz, N);
    else
        oracle_newell_far(X, Y, Z, dx, dy, dz, ORACLE_P, N);
}

/* Octant table N[6][nz][ny][nx] at offsets (i dx, j dy, k dz), i,j,k >= 0. */
void oracle_tensor_octant(int nx, int ny, int nz, double dx, double dy, double dz,
                          double *N)
{
    const size_t n = (size_t)nx * ny * nz;
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                double t[6];
                oracle_newell(i * dx, j * dy, k * dz, dx, dy, dz, t);
                const size_t idx = ((size_t)k * ny + j) * nx + i;
                for (int c = 0; c < 6; c++) N[c * n + idx] = t[c];
            }
}

/* ------------------------------------------------------------------------ */
/* Demagnetising field by the direct O(N^2) sum (paper Sec. 2, eq. (11)-(12), */
/* with K = -N, self term included).                                         */
/* ------------------------------------------------------------------------ */

static inline void apply_N(const double t[6], double mx, double my, double mz, double h[3])
{
    h[0] -= t[0] * mx + t[3] * my + t[4] * mz;
    h[1] -= t[3] * mx + t[1] * my + t[5] * mz;
    h[2] -= t[4] * mx + t[5] * my + t[2] * mz;
}

/* Full signed-offset table, evaluated directly at every offset (no parity). */
static double *signed_table(int nx, int ny, int nz, double dx, double dy, double dz)
{
    const int sx = 2 * nx - 1, sy = 2 * ny - 1, sz = 2 * nz - 1;
    double *T = (double *)malloc(sizeof(double) * 6 * (size_t)sx * sy * sz);
    if (!T) return NULL;
    for (int c = 0; c < sz; c++)
        for (int b = 0; b < sy; b++)
            for (int a = 0; a < sx; a++) {
                const size_t o = ((size_t)c * sy + b) * sx + a;
                oracle_newell((a - (nx - 1)) * dx, (b - (ny - 1)) * dy,
                              (c - (nz - 1)) * dz, dx, dy, dz, T + 6 * o);
            }
    return T;
}

int oracle_demag_direct(int nx, int ny, int nz, double dx, double dy, double dz,
                        const double *M, double *H)
{
    const size_t n = (size_t)nx * ny * nz;
    const int sx = 2 * nx - 1, sy = 2 * ny - 1;
    double *T = signed_table(nx, ny, nz, dx, dy, dz);
    if (!T) return -1;
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                double h[3] = {0, 0, 0};
                for (int n3 = 0; n3 < nz; n3++)
                    for (int m = 0; m < ny; m++)
                        for (int l = 0; l < nx; l++) {
                            /* offset observer - source = (i-l, j-m, k-n3) */
                            const size_t o = ((size_t)(k - n3 + nz - 1) * sy +
                                              (j - m + ny - 1)) * sx + (i - l + nx - 1);
                            const size_t s = ((size_t)n3 * ny + m) * nx + l;
                            apply_N(T + 6 * o, M[s], M[n + s], M[2 * n + s], h);
                        }
                const size_t d = ((size_t)k * ny + j) * nx + i;
                H[d] = h[0];
                H[n + d] = h[1];
                H[2 * n + d] = h[2];
            }
    free(T);
    return 0;
}

/* Direct sum at selected observer cells (flat indices obs[]) over the source
 * cells whose M is not exactly zero; H is [3][nobs].  The tensor is evaluated
 * per pair at the signed offset. */
int oracle_demag_direct_at(int nx, int ny, int nz, double dx, double dy, double dz,
                           const double *M, int nobs, const int64_t *obs, double *H)
{
    const size_t n = (size_t)nx * ny * nz;
    size_t nsrc = 0;
    for (size_t s = 0; s < n; s++)
        if (M[s] != 0.0 || M[n + s] != 0.0 || M[2 * n + s] != 0.0) nsrc++;
    size_t *src = (size_t *)malloc(sizeof(size_t) * (nsrc ? nsrc : 1));
    if (!src) return -1;
    nsrc = 0;
    for (size_t s = 0; s < n; s++)
        if (M[s] != 0.0 || M[n + s] != 0.0 || M[2 * n + s] != 0.0) src[nsrc++] = s;
    for (int q = 0; q < nobs; q++) {
        const int64_t d = obs[q];
        const int i = (int)(d % nx), j = (int)((d / nx) % ny), k = (int)(d / ((int64_t)nx * ny));
        double h[3] = {0, 0, 0};
        for (size_t t = 0; t < nsrc; t++) {
            const size_t s = src[t];
            const int l = (int)(s % nx), m = (int)((s / nx) % ny), n3 = (int)(s / ((size_t)nx * ny));
            double tn[6];
            oracle_newell((i - l) * dx, (j - m) * dy, (k - n3) * dz, dx, dy, dz, tn);
            apply_N(tn, M[s], M[n + s], M[2 * n + s], h);
        }
        H[q] = h[0];
        H[nobs + q] = h[1];
        H[2 * nobs + q] = h[2];
    }
    free(src);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Textbook FFT: recursive mixed-radix decimation in time, any length (each  */
/* prime factor p is combined by a plain p-point DFT).  sign = -1 forward,   */
/* +1 inverse; unnormalised.                                                 */
/* ------------------------------------------------------------------------ */

typedef double complex cplx;

static int smallest_factor(int n)
{
    if (n % 2 == 0) return 2;
    for (int p = 3; p * p <= n; p += 2)
        if (n % p == 0) return p;
    return n;
}

/* tw[e * tws] = exp(sign 2 pi i e / n) for the current length n; tmp holds
 * n values of scratch, shared by all levels (a level uses it only after its
 * sub-transforms have returned). */
static void fft_rec(int n, const cplx *in, size_t stride, cplx *out, const cplx *tw, size_t tws,
                    cplx *tmp)
{
    if (n == 1) {
        out[0] = in[0];
        return;
    }
    const int p = smallest_factor(n);
    const int m = n / p;
    for (int r = 0; r < p; r++)
        fft_rec(m, in + r * stride, stride * p, out + (size_t)r * m, tw, tws * p, tmp);
    for (int k = 0; k < m; k++)
        for (int q = 0; q < p; q++) {
            const int kk = k + m * q;
            cplx acc = 0;
            for (int r = 0; r < p; r++) {
                const long e = ((long)r * kk) % n; /* exact integer reduction of the angle */
                acc += out[(size_t)r * m + k] * tw[(size_t)e * tws];
            }
            tmp[kk] = acc;
        }
    memcpy(out, tmp, sizeof(cplx) * (size_t)n);
}

/* Twiddle table exp(sign 2 pi i e / n), e < n. */
static cplx *twiddles(int n, int sign)
{
    cplx *tw = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    for (int e = 0; e < n; e++) {
        const double ang = sign * 2.0 * PI_D * (double)e / (double)n;
        tw[e] = cos(ang) + I * sin(ang);
    }
    return tw;
}

/* In-place length-n transform of (re, im). */
void oracle_fft(int n, double *re, double *im, int sign)
{
    cplx *a = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *b = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *t = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *tw = twiddles(n, sign);
    for (int i = 0; i < n; i++) a[i] = re[i] + I * im[i];
    fft_rec(n, a, 1, b, tw, 1, t);
    for (int i = 0; i < n; i++) {
        re[i] = creal(b[i]);
        im[i] = cimag(b[i]);
    }
    free(a);
    free(b);
    free(t);
    free(tw);
}

/* 3-D transform of a [Pz][Py][Px] complex array, one axis at a time. */
static void fft3(cplx *a, int Px, int Py, int Pz, int sign)
{
    int mx = Px > Py ? Px : Py;
    if (Pz > mx) mx = Pz;
    cplx *line = (cplx *)malloc(sizeof(cplx) * (size_t)mx);
    cplx *res = (cplx *)malloc(sizeof(cplx) * (size_t)mx);
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)mx);
    cplx *tx = twiddles(Px, sign), *ty = twiddles(Py, sign), *tz = twiddles(Pz, sign);
    for (int z = 0; z < Pz; z++)
        for (int y = 0; y < Py; y++) {
            cplx *row = a + ((size_t)z * Py + y) * Px;
            fft_rec(Px, row, 1, res, tx, 1, tmp);
            memcpy(row, res, sizeof(cplx) * (size_t)Px);
        }
    for (int z = 0; z < Pz; z++)
        for (int x = 0; x < Px; x++) {
            for (int y = 0; y < Py; y++) line[y] = a[((size_t)z * Py + y) * Px + x];
            fft_rec(Py, line, 1, res, ty, 1, tmp);
            for (int y = 0; y < Py; y++) a[((size_t)z * Py + y) * Px + x] = res[y];
        }
    for (int y = 0; y < Py; y++)
        for (int x = 0; x < Px; x++) {
            for (int z = 0; z < Pz; z++) line[z] = a[((size_t)z * Py + y) * Px + x];
            fft_rec(Pz, line, 1, res, tz, 1, tmp);
            for (int z = 0; z < Pz; z++) a[((size_t)z * Py + y) * Px + x] = res[z];
        }
    free(line);
    free(res);
    free(tmp);
    free(tx);
    free(ty);
    free(tz);
}

/* ------------------------------------------------------------------------ */
/* Demagnetising field by zero-padded FFT convolution, paper Sec. 2 steps    */
/* (1)-(5) and eq. (13)-(16): full 2nx x 2ny x 2nz complex arrays, no R2C,   */
/* no pruning, no symmetry folding.  The spare slot at offset +-n of every   */
/* axis is 0 (reading R10); forward unnormalised, 1/(8 nx ny nz) on the      */
/* inverse (R12); the first nx x ny x nz of the inverse is kept (R11).       */
/* ------------------------------------------------------------------------ */

typedef struct {
    int nx, ny, nz;
    double dx, dy, dz;
    int Px, Py, Pz;
    size_t P;
    cplx *Kt[6]; /* FFT of K = -N in wrap layout */
    cplx *work[3];
} oracle_demag;

static int wrap_offset(int idx, int n)
{
    /* padded index -> signed offset; index n is the spare slot (returns a
     * sentinel that the caller maps to zero) */
    if (idx < n) return idx;
    if (idx == n) return 1 << 30;
    return idx - 2 * n;
}

oracle_demag *oracle_demag_create(int nx, int ny, int nz, double dx, double dy, double dz)
{
    oracle_demag *c = (oracle_demag *)calloc(1, sizeof(oracle_demag));
    if (!c) return NULL;
    c->nx = nx; c->ny = ny; c->nz = nz;
    c->dx = dx; c->dy = dy; c->dz = dz;
    c->Px = 2 * nx; c->Py = 2 * ny; c->Pz = 2 * nz;
    c->P = (size_t)c->Px * c->Py * c->Pz;
    for (int q = 0; q < 6; q++) c->Kt[q] = (cplx *)calloc(c->P, sizeof(cplx));
    for (int q = 0; q < 3; q++) c->work[q] = (cplx *)calloc(c->P, sizeof(cplx));
    for (int z = 0; z < c->Pz; z++)
        for (int y = 0; y < c->Py; y++)
            for (int x = 0; x < c->Px; x++) {
                const int X = wrap_offset(x, nx), Y = wrap_offset(y, ny), Z = wrap_offset(z, nz);
                if (X == (1 << 30) || Y == (1 << 30) || Z == (1 << 30)) continue; /* spare slot */
                double t[6];
                oracle_newell(X * dx, Y * dy, Z * dz, dx, dy, dz, t);
                const size_t o = ((size_t)z * c->Py + y) * c->Px + x;
                for (int q = 0; q < 6; q++) c->Kt[q][o] = -t[q]; /* K = -N */
            }
    for (int q = 0; q < 6; q++) fft3(c->Kt[q], c->Px, c->Py, c->Pz, -1);
    return c;
}

void oracle_demag_destroy(oracle_demag *c)
{
    if (!c) return;
    for (int q = 0; q < 6; q++) free(c->Kt[q]);
    for (int q = 0; q < 3; q++) free(c->work[q]);
    free(c);
}

void oracle_demag_fft(oracle_demag *c, const double *M, double *H)
{
    const int nx = c->nx, ny = c->ny, nz = c->nz;
    const size_t n = (size_t)nx * ny * nz;
    /* step (1): zero-pad M */
    for (int q = 0; q < 3; q++) {
        memset(c->work[q], 0, sizeof(cplx) * c->P);
        for (int k = 0; k < nz; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++)
                    c->work[q][((size_t)k * c->Py + j) * c->Px + i] =
                        M[q * n + ((size_t)k * ny + j) * nx + i];
        /* step (3) / eq. (14) */
        fft3(c->work[q], c->Px, c->Py, c->Pz, -1);
    }
    /* step (4) / eq. (13), (15): symmetric tensor times vector */
    cplx **K = c->Kt;
    for (size_t o = 0; o < c->P; o++) {
        const cplx mx = c->work[0][o], my = c->work[1][o], mz = c->work[2][o];
        c->work[0][o] = K[0][o] * mx + K[3][o] * my + K[4][o] * mz;
        c->work[1][o] = K[3][o] * mx + K[1][o] * my + K[5][o] * mz;
        c->work[2][o] = K[4][o] * mx + K[5][o] * my + K[2][o] * mz;
    }
    /* step (5) / eq. (10), (16): inverse, normalise, keep the first half */
    const double scale = 1.0 / (double)c->P;
    for (int q = 0; q < 3; q++) {
        fft3(c->work[q], c->Px, c->Py, c->Pz, +1);
        for (int k = 0; k < nz; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++)
                    H[q * n + ((size_t)k * ny + j) * nx + i] =
                        creal(c->work[q][((size_t)k * c->Py + j) * c->Px + i]) * scale;
    }
}

/* ------------------------------------------------------------------------ */
/* Local fields, LLG right-hand side, integrators, observables.              */
/* ------------------------------------------------------------------------ */

typedef struct {
    double Ms, A, Ku;
    double ax, ay, az;     /* anisotropy easy axis (unit vector), paper: x */
    double alpha, gamma0;  /* gamma0 = gamma mu0 in m/(A s) (reading R5)  */
    double hx, hy, hz;     /* applied field, A/m */
    double dt;
    int integrator;        /* 0 classical RK4, 1 explicit Euler */
    int renorm;            /* 1: M <- Ms M/|M| after every accepted step */
} oracle_params;

/* Exchange field, eq. (3)-(4) with coefficient 2A/(mu0 Ms^2) (R3) and free
 * (Neumann) boundaries: a neighbour outside the sample is replaced by the
 * cell itself (R7), so it contributes nothing. */
void oracle_exchange(int nx, int ny, int nz, double dx, double dy, double dz, double Ms,
                     double A, const double *M, double *H)
{
    const size_t n = (size_t)nx * ny * nz;
    const double pre = 2.0 * A / (MU0 * Ms * Ms);
    for (int q = 0; q < 3; q++) {
        const double *m = M + q * n;
        for (int k = 0; k < nz; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) {
                    const size_t c = ((size_t)k * ny + j) * nx + i;
                    const double mc = m[c];
                    const double xm = i > 0 ? m[c - 1] : mc;
                    const double xp = i < nx - 1 ? m[c + 1] : mc;
                    const double ym = j > 0 ? m[c - nx] : mc;
                    const double yp = j < ny - 1 ? m[c + nx] : mc;
                    const double zm = k > 0 ? m[c - (size_t)nx * ny] : mc;
                    const double zp = k < nz - 1 ? m[c + (size_t)nx * ny] : mc;
                    H[q * n + c] = pre * ((xp - 2.0 * mc + xm) / (dx * dx) +
                                          (yp - 2.0 * mc + ym) / (dy * dy) +
                                          (zp - 2.0 * mc + zm) / (dz * dz));
                }
    }
}

/* H_eff = H_exch + H_anis + H_demag + H_extern (eq. (2)); anisotropy in the
 * easy-axis form 2Ku/(mu0 Ms^2) (u.M) u (reading R4). */
void oracle_heff(oracle_demag *c, const oracle_params *p, const double *M, double *Hd,
                 double *Heff)
{
    const int nx = c->nx, ny = c->ny, nz = c->nz;
    const size_t n = (size_t)nx * ny * nz;
    oracle_demag_fft(c, M, Hd);
    oracle_exchange(nx, ny, nz, c->dx, c->dy, c->dz, p->Ms, p->A, M, Heff);
    const double ka = 2.0 * p->Ku / (MU0 * p->Ms * p->Ms);
    for (size_t s = 0; s < n; s++) {
        const double um = p->ax * M[s] + p->ay * M[n + s] + p->az * M[2 * n + s];
        Heff[s] += ka * um * p->ax + Hd[s] + p->hx;
        Heff[n + s] += ka * um * p->ay + Hd[n + s] + p->hy;
        Heff[2 * n + s] += ka * um * p->az + Hd[2 * n + s] + p->hz;
    }
}

/* Landau-Lifshitz form, eq. (6), with gamma mu0 read as gamma0 (R5):
 * dM/dt = -g/(1+a^2) M x H - a g/((1+a^2) Ms) M x (M x H). */
static void llg_rhs_point(const oracle_params *p, double mx, double my, double mz, double hx,
                          double hy, double hz, double out[3])
{
    const double g = p->gamma0 / (1.0 + p->alpha * p->alpha);
    const double cx = my * hz - mz * hy, cy = mz * hx - mx * hz, cz = mx * hy - my * hx;
    const double dx = my * cz - mz * cy, dy = mz * cx - mx * cz, dz = mx * cy - my * cx;
    const double d = p->alpha * g / p->Ms;
    out[0] = -g * cx - d * dx;
    out[1] = -g * cy - d * dy;
    out[2] = -g * cz - d * dz;
}

void oracle_llg_rhs(oracle_demag *c, const oracle_params *p, const double *M, double *dMdt)
{
    const size_t n = (size_t)c->nx * c->ny * c->nz;
    double *Hd = (double *)malloc(sizeof(double) * 3 * n);
    double *He = (double *)malloc(sizeof(double) * 3 * n);
    oracle_heff(c, p, M, Hd, He);
    for (size_t s = 0; s < n; s++) {
        double o[3];
        llg_rhs_point(p, M[s], M[n + s], M[2 * n + s], He[s], He[n + s], He[2 * n + s], o);
        dMdt[s] = o[0];
        dMdt[n + s] = o[1];
        dMdt[2 * n + s] = o[2];
    }
    free(Hd);
    free(He);
}

static void renormalise(size_t n, double Ms, double *M)
{
    for (size_t s = 0; s < n; s++) {
        const double r = sqrt(M[s] * M[s] + M[n + s] * M[n + s] + M[2 * n + s] * M[2 * n + s]);
        if (r > 0.0) {
            M[s] *= Ms / r;
            M[n + s] *= Ms / r;
            M[2 * n + s] *= Ms / r;
        }
    }
}

/* Advance nsteps with classical RK4 (four H evaluations per step) or explicit
 * Euler (one; the integrator of the paper's timings, Table 1).  If mavg_log is
 * non-null, <m> = (1/N) sum M/Ms is stored before the first step and after
 * every log_every-th step ([nlog][3]). */
int oracle_llg_run(oracle_demag *c, const oracle_params *p, double *M, int nsteps,
                   int log_every, double *mavg_log)
{
    const size_t n = (size_t)c->nx * c->ny * c->nz, n3 = 3 * n;
    double *k1 = (double *)malloc(sizeof(double) * n3);
    double *k2 = (double *)malloc(sizeof(double) * n3);
    double *k3 = (double *)malloc(sizeof(double) * n3);
    double *k4 = (double *)malloc(sizeof(double) * n3);
    double *Y = (double *)malloc(sizeof(double) * n3);
    if (!k1 || !k2 || !k3 || !k4 || !Y) return -1;
    int nlog = 0;
    if (mavg_log) {
        for (int q = 0; q < 3; q++) {
            double s = 0;
            for (size_t t = 0; t < n; t++) s += M[q * n + t];
            mavg_log[q] = s / (double)n / p->Ms;
        }
        nlog = 1;
    }
    const double dt = p->dt;
    for (int step = 0; step < nsteps; step++) {
        if (p->integrator == 1) {
            oracle_llg_rhs(c, p, M, k1);
            for (size_t t = 0; t < n3; t++) M[t] += dt * k1[t];
        } else {
            oracle_llg_rhs(c, p, M, k1);
            for (size_t t = 0; t < n3; t++) Y[t] = M[t] + 0.5 * dt * k1[t];
            oracle_llg_rhs(c, p, Y, k2);
            for (size_t t = 0; t < n3; t++) Y[t] = M[t] + 0.5 * dt * k2[t];
            oracle_llg_rhs(c, p, Y, k3);
            for (size_t t = 0; t < n3; t++) Y[t] = M[t] + dt * k3[t];
            oracle_llg_rhs(c, p, Y, k4);
            for (size_t t = 0; t < n3; t++)
                M[t] += dt / 6.0 * (k1[t] + 2.0 * k2[t] + 2.0 * k3[t] + k4[t]);
        }
        if (p->renorm) renormalise(n, p->Ms, M);
        if (mavg_log && log_every > 0 && (step + 1) % log_every == 0) {
            for (int q = 0; q < 3; q++) {
                double s = 0;
                for (size_t t = 0; t < n; t++) s += M[q * n + t];
                mavg_log[3 * nlog + q] = s / (double)n / p->Ms;
            }
            nlog++;
        }
    }
    free(k1); free(k2); free(k3); free(k4); free(Y);
    return nlog;
}

/*
 * Observables at state M, out[9] = {E_ex, E_an, E_d, E_z, E_tot, tau_max,
 * <mx>, <my>, <mz>}.  Energies from eq. (1) with V = dx dy dz per cell:
 *   E_ex = A V sum_links |m_i - m_j|^2 / d_link^2  (R1; each nearest-neighbour
 *          pair inside the sample once, which is the discrete form of the
 *          gradient term under free boundaries),
 *   E_an = V sum Ku (|m|^2 - (u.m)^2)  (eq. (1): Ku (My^2+Mz^2)/Ms^2 for u = x),
 *   E_d  = -1/2 mu0 V sum H_d . M,   E_z = -mu0 V sum H_ext . M,
 *   tau_max = max_i |M_i x H_eff,i| / Ms,  <m> = (1/N) sum M_i / Ms.
 */
void oracle_observables(oracle_demag *c, const oracle_params *p, const double *M, double *out)
{
    const int nx = c->nx, ny = c->ny, nz = c->nz;
    const size_t n = (size_t)nx * ny * nz;
    const double V = c->dx * c->dy * c->dz, Ms = p->Ms;
    double *Hd = (double *)malloc(sizeof(double) * 3 * n);
    double *He = (double *)malloc(sizeof(double) * 3 * n);
    oracle_heff(c, p, M, Hd, He);
    double Eex = 0, Ean = 0, Ed = 0, Ez = 0, tau = 0, ms[3] = {0, 0, 0};
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                const size_t s = ((size_t)k * ny + j) * nx + i;
                const double mx = M[s] / Ms, my = M[n + s] / Ms, mz = M[2 * n + s] / Ms;
                if (i + 1 < nx) {
                    const size_t t = s + 1;
                    const double a = M[t] / Ms - mx, b = M[n + t] / Ms - my, cc = M[2 * n + t] / Ms - mz;
                    Eex += (a * a + b * b + cc * cc) / (c->dx * c->dx);
                }
                if (j + 1 < ny) {
                    const size_t t = s + nx;
                    const double a = M[t] / Ms - mx, b = M[n + t] / Ms - my, cc = M[2 * n + t] / Ms - mz;
                    Eex += (a * a + b * b + cc * cc) / (c->dy * c->dy);
                }
                if (k + 1 < nz) {
                    const size_t t = s + (size_t)nx * ny;
                    const double a = M[t] / Ms - mx, b = M[n + t] / Ms - my, cc = M[2 * n + t] / Ms - mz;
                    Eex += (a * a + b * b + cc * cc) / (c->dz * c->dz);
                }
                const double um = p->ax * mx + p->ay * my + p->az * mz;
                Ean += p->Ku * (mx * mx + my * my + mz * mz - um * um);
                Ed += Hd[s] * M[s] + Hd[n + s] * M[n + s] + Hd[2 * n + s] * M[2 * n + s];
                Ez += p->hx * M[s] + p->hy * M[n + s] + p->hz * M[2 * n + s];
                const double Mx = M[s], My = M[n + s], Mz = M[2 * n + s];
                const double hx = He[s], hy = He[n + s], hz = He[2 * n + s];
                const double tx = My * hz - Mz * hy, ty = Mz * hx - Mx * hz, tz = Mx * hy - My * hx;
                const double tn = sqrt(tx * tx + ty * ty + tz * tz) / Ms;
                if (tn > tau || tn != tn) tau = tn;
                ms[0] += mx;
                ms[1] += my;
                ms[2] += mz;
            }
    out[0] = p->A * V * Eex;
    out[1] = V * Ean;
    out[2] = -0.5 * MU0 * V * Ed;
    out[3] = -MU0 * V * Ez;
    out[4] = out[0] + out[1] + out[2] + out[3];
    out[5] = tau;
    out[6] = ms[0] / (double)n;
    out[7] = ms[1] / (double)n;
    out[8] = ms[2] / (double)n;
    free(Hd);
    free(He);
}

double oracle_mu0(void) { return MU0; }
