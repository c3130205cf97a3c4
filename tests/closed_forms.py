"""Closed forms and independent quadratures used to pin the oracle.

Nothing here calls the oracle or the GPU library: these are textbook results
(Aharoni's prism demagnetising factors, the point-dipole field, a plain 6-D
Gauss-Legendre cell-pair average, the discrete Neumann Laplacian spectrum and
the macrospin precession solution) written independently of it.
"""
import math

import numpy as np


def aharoni_dz(lx: float, ly: float, lz: float) -> float:
    """Demagnetising factor along z of a uniformly magnetised rectangular prism
    lx x ly x lz (A. Aharoni, J. Appl. Phys. 83, 3432 (1998), with half-edges
    a, b, c)."""
    a, b, c = lx / 2.0, ly / 2.0, lz / 2.0
    r = math.sqrt(a * a + b * b + c * c)
    ab = math.sqrt(a * a + b * b)
    bc = math.sqrt(b * b + c * c)
    ac = math.sqrt(a * a + c * c)
    t = 0.0
    t += (b * b - c * c) / (2 * b * c) * math.log((r - a) / (r + a))
    t += (a * a - c * c) / (2 * a * c) * math.log((r - b) / (r + b))
    t += b / (2 * c) * math.log((ab + a) / (ab - a))
    t += a / (2 * c) * math.log((ab + b) / (ab - b))
    t += c / (2 * a) * math.log((bc - b) / (bc + b))
    t += c / (2 * b) * math.log((ac - a) / (ac + a))
    t += 2 * math.atan(a * b / (c * r))
    t += (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
    t += (a * a + b * b - 2 * c * c) / (3 * a * b * c) * r
    t += c / (a * b) * (ac + bc)
    t -= (ab ** 3 + bc ** 3 + ac ** 3) / (3 * a * b * c)
    return t / math.pi


def aharoni_diag(lx, ly, lz):
    """(Dx, Dy, Dz) of the prism by permuting the axes of aharoni_dz."""
    return (aharoni_dz(ly, lz, lx), aharoni_dz(lz, lx, ly), aharoni_dz(lx, ly, lz))


def dipole_tensor(R, V):
    """Point-dipole demag tensor V (delta r^2 - 3 r r) / (4 pi r^5),
    order xx,yy,zz,xy,xz,yz."""
    x, y, z = R
    r2 = x * x + y * y + z * z
    r5 = r2 * r2 * math.sqrt(r2)
    f = V / (4 * math.pi * r5)
    return np.array([f * (r2 - 3 * x * x), f * (r2 - 3 * y * y), f * (r2 - 3 * z * z),
                     -3 * f * x * y, -3 * f * x * z, -3 * f * y * z])


def cellpair_gl(R, d, n=8):
    """Cell-pair average of the point-dipole kernel by a plain 6-D
    Gauss-Legendre rule (n nodes per dimension over both cells).  Valid for
    cells that do not touch (the integrand is then smooth)."""
    xg, wg = np.polynomial.legendre.leggauss(n)
    acc = np.zeros(6)
    # relative coordinate s_a = R_a + (u_obs - u_src) d_a, u in [-1/2, 1/2]
    u = 0.5 * xg
    w = 0.5 * wg
    s_axes = []
    w_axes = []
    for a in range(3):
        s = R[a] + (u[:, None] - u[None, :]).ravel() * d[a]
        ww = (w[:, None] * w[None, :]).ravel()
        s_axes.append(s)
        w_axes.append(ww)
    sx, sy, sz = np.meshgrid(*s_axes, indexing="ij")
    W = w_axes[0][:, None, None] * w_axes[1][None, :, None] * w_axes[2][None, None, :]
    r2 = sx * sx + sy * sy + sz * sz
    r5 = r2 * r2 * np.sqrt(r2)
    V = d[0] * d[1] * d[2]
    pre = V / (4 * math.pi) * W / r5
    acc[0] = (pre * (r2 - 3 * sx * sx)).sum()
    acc[1] = (pre * (r2 - 3 * sy * sy)).sum()
    acc[2] = (pre * (r2 - 3 * sz * sz)).sum()
    acc[3] = (pre * (-3 * sx * sy)).sum()
    acc[4] = (pre * (-3 * sx * sz)).sum()
    acc[5] = (pre * (-3 * sy * sz)).sum()
    return acc


def neumann_eigenvalue(k: int, n: int, d: float) -> float:
    """Eigenvalue of the 1-D second difference with free ends on n cells for
    the mode cos(pi k (i + 1/2) / n)."""
    return -4.0 / (d * d) * math.sin(math.pi * k / (2 * n)) ** 2


def macrospin(theta0, phi0, H, alpha, gamma0, t):
    """Closed-form LL precession of a single moment in a static field H along z:
    tan(theta/2) = tan(theta0/2) exp(-alpha g H t), phi = phi0 + g H t,
    g = gamma0 / (1 + alpha^2).  Returns the unit vector."""
    g = gamma0 / (1 + alpha * alpha)
    th = 2 * math.atan(math.tan(theta0 / 2) * math.exp(-alpha * g * H * t))
    ph = phi0 + g * H * t
    return np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
