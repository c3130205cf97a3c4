"""Seeded synthetic inputs and run parameters for the benchmark workloads.

This module only draws random numbers and holds parameter tables: it
contains none of the method's arithmetic, so both the GPU path and the CPU
oracle take their inputs from it.  All generators use numpy's PCG64.

Workloads (shapes and materials of the paper's cube benchmark, Sec. 4, and of
thin films; synthetic stand-ins, no published reference solution is used):

* ``film32``   32x32x1 cells of 4 nm, Ms 8e5, A 1.3e-11, alpha 0.5, isotropic
  random unit M (seed 1), RK4, dt 1e-14 s, 2000 steps.
* ``film128``  128x32x1 cells of 3.90625x3.90625x3 nm, Ms 8e5, A 1.3e-11;
  M along (1,1,1)/sqrt(3) tilted by up to 5 degrees per cell (seed 2); relax
  with alpha 1 for 20000 steps at dt 5e-14, then mu0 H = (-24.6, 4.3, 0) mT
  with alpha 0.02 for 1 ns.
* ``cube{n}``  n^3 cubes of 2 nm cells (n = 64, 128, 256), Ms 1e6, A 1.5e-11,
  Ku 5e4 along x, alpha 0.1, isotropic random M (seed 3000+n), dt 1e-14.
* ``sweep64``  64 films, nx, ny from {64,96,128,192,256,384,512}, nz from
  {1,2,4,8} (seed 4), 4x4x2 nm cells, Ms 8e5, A 1.3e-11, alpha 0.5, applied
  field along x evenly spaced over [-100, +100] mT, dt 2e-14.
* ``film256``  256x256x4 cells of 4 nm, Ms 8e5, A 1.3e-11, alpha 0.1,
  in-plane applied field |mu0 H| <= 50 mT at a random angle.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MU0 = 4e-7 * math.pi  # N/A^2; converts mT to A/m as H = B / mu0


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_unit(nx: int, ny: int, nz: int, seed: int) -> np.ndarray:
    """Isotropic random unit vectors, [3][nz][ny][nx] float64: three i.i.d.
    normal draws per cell scaled to length 1 (uniform on the sphere)."""
    g = rng(seed).standard_normal((3, nz, ny, nx))
    return g / np.sqrt((g * g).sum(axis=0, keepdims=True))


def tilted_unit(nx: int, ny: int, nz: int, seed: int, direction=(1.0, 1.0, 1.0),
                max_deg: float = 5.0) -> np.ndarray:
    """Unit vectors tilted from ``direction`` by theta ~ U[0, max_deg] degrees,
    about an axis at azimuth phi ~ U[0, 2 pi) in the plane normal to it."""
    r = rng(seed)
    u = np.asarray(direction, dtype=np.float64)
    u = u / np.linalg.norm(u)
    a = np.array([1.0, 0.0, 0.0]) if abs(u[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(u, a)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(u, e1)
    th = np.deg2rad(r.uniform(0.0, max_deg, (nz, ny, nx)))
    ph = r.uniform(0.0, 2 * math.pi, (nz, ny, nx))
    v = (np.cos(th)[None] * u[:, None, None, None]
         + (np.sin(th) * np.cos(ph))[None] * e1[:, None, None, None]
         + (np.sin(th) * np.sin(ph))[None] * e2[:, None, None, None])
    return v / np.sqrt((v * v).sum(axis=0, keepdims=True))


def sparse_sources(nx: int, ny: int, nz: int, count: int, seed: int) -> np.ndarray:
    """M that is zero except at ``count`` random cells holding random unit
    vectors; used where a dense direct sum would be too slow."""
    r = rng(seed)
    M = np.zeros((3, nz, ny, nx))
    n = nx * ny * nz
    idx = r.choice(n, size=min(count, n), replace=False)
    g = r.standard_normal((3, idx.size))
    g /= np.sqrt((g * g).sum(axis=0, keepdims=True))
    flat = M.reshape(3, n)
    flat[:, idx] = g
    return M


def sample_cells(n: int, count: int, seed: int) -> np.ndarray:
    """Sorted distinct flat cell indices, always including the first and last."""
    r = rng(seed)
    idx = set(r.choice(n, size=min(count, n), replace=False).tolist())
    idx.update({0, n - 1})
    return np.array(sorted(idx), dtype=np.int64)


@dataclass
class Material:
    Ms: float
    A: float
    Ku: float = 0.0
    axis: tuple = (1.0, 0.0, 0.0)
    alpha: float = 0.5
    gamma0: float = 2.211e5
    Hext: tuple = (0.0, 0.0, 0.0)
    dt: float = 1e-14


@dataclass
class Workload:
    name: str
    shape: tuple            # (nx, ny, nz)
    cell: tuple             # (dx, dy, dz) in m
    mat: Material
    seed: int
    steps: int
    extra: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz

    def initial_unit(self) -> np.ndarray:
        nx, ny, nz = self.shape
        if self.name == "film128":
            return tilted_unit(nx, ny, nz, self.seed)
        return random_unit(nx, ny, nz, self.seed)


def film32() -> Workload:
    return Workload("film32", (32, 32, 1), (4e-9, 4e-9, 4e-9),
                    Material(Ms=8.0e5, A=1.3e-11, alpha=0.5, dt=1e-14), seed=1, steps=2000)


def film128() -> Workload:
    h = (-24.6e-3 / MU0, 4.3e-3 / MU0, 0.0)
    return Workload("film128", (128, 32, 1), (3.90625e-9, 3.90625e-9, 3e-9),
                    Material(Ms=8.0e5, A=1.3e-11, alpha=1.0, dt=5e-14), seed=2, steps=20000,
                    extra=dict(relax_steps=20000, relax_alpha=1.0, switch_Hext=h,
                               switch_alpha=0.02, switch_steps=20000, log_every=20))


def cube(n: int) -> Workload:
    return Workload("cube%d" % n, (n, n, n), (2e-9, 2e-9, 2e-9),
                    Material(Ms=1.0e6, A=1.5e-11, Ku=5e4, alpha=0.1, dt=1e-14),
                    seed=3000 + n, steps=100)


SWEEP_SIZES = (64, 96, 128, 192, 256, 384, 512)
SWEEP_NZ = (1, 2, 4, 8)


def sweep64(count: int = 64) -> list:
    """The field-sweep batch: per-instance Workloads, seeds 4000+i."""
    r = rng(4)
    nx = r.choice(SWEEP_SIZES, size=count)
    ny = r.choice(SWEEP_SIZES, size=count)
    nz = r.choice(SWEEP_NZ, size=count)
    hx = np.linspace(-100e-3, 100e-3, count) / MU0
    out = []
    for i in range(count):
        m = Material(Ms=8.0e5, A=1.3e-11, alpha=0.5, dt=2e-14, Hext=(float(hx[i]), 0.0, 0.0))
        out.append(Workload("sweep64[%d]" % i, (int(nx[i]), int(ny[i]), int(nz[i])),
                            (4e-9, 4e-9, 2e-9), m, seed=4000 + i, steps=5000))
    return out


def film256(traj: int = 0) -> Workload:
    r = rng(5000 + traj)
    b = r.uniform(0.0, 50e-3)
    ang = r.uniform(0.0, 2 * math.pi)
    h = (b * math.cos(ang) / MU0, b * math.sin(ang) / MU0, 0.0)
    return Workload("film256", (256, 256, 4), (4e-9, 4e-9, 4e-9),
                    Material(Ms=8.0e5, A=1.3e-11, alpha=0.1, dt=1e-14, Hext=h),
                    seed=5000 + traj, steps=100)
