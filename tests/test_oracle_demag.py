"""Pins of the oracle's demagnetising field (no GPU): the zero-padded FFT route
(paper Sec. 2 steps (1)-(5), eq. (13)-(16)) against the direct O(N^2) sum
(eq. (11)-(12)), the oracle FFT against numpy, and closed forms."""
import numpy as np
import pytest

import oracle
from closed_forms import aharoni_diag
from paper_1406_7459_amd import workloads as W


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8, 12, 16, 18, 64, 96, 128, 192, 250, 384])
def test_fft_matches_numpy(n):
    x = W.rng(n).standard_normal(n) + 1j * W.rng(n + 1).standard_normal(n)
    assert np.allclose(oracle.fft(x, -1), np.fft.fft(x), rtol=0, atol=1e-12 * max(1, n))
    assert np.allclose(oracle.fft(x, +1), np.fft.ifft(x) * n, rtol=0, atol=1e-12 * max(1, n))


def rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


GRIDS = [((4, 3, 2), (1e-9, 1e-9, 1e-9)), ((5, 7, 3), (4e-9, 4e-9, 2e-9)),
         ((8, 8, 1), (4e-9, 4e-9, 4e-9)), ((3, 5, 4), (1e-9, 1.3e-9, 0.7e-9)),
         ((6, 1, 1), (2e-9, 2e-9, 2e-9)), ((1, 1, 1), (2e-9, 3e-9, 1e-9)),
         ((9, 6, 2), (3.90625e-9, 3.90625e-9, 3e-9))]


@pytest.mark.parametrize("grid,d", GRIDS)
def test_fft_route_equals_direct_sum(grid, d):
    nx, ny, nz = grid
    M = 8e5 * W.random_unit(nx, ny, nz, seed=11 + nx)
    Hf = oracle.Demag(nx, ny, nz, *d).apply(M)
    Hd = oracle.demag_direct(M, d)
    assert rel_l2(Hf, Hd) < 1e-12


def test_fft_route_equals_direct_sum_film32():
    wl = W.film32()
    nx, ny, nz = wl.shape
    M = wl.mat.Ms * wl.initial_unit()
    Hf = oracle.Demag(nx, ny, nz, *wl.cell).apply(M)
    Hd = oracle.demag_direct(M, wl.cell)
    assert rel_l2(Hf, Hd) < 1e-12


def test_direct_at_matches_full_direct():
    nx, ny, nz = 6, 5, 3
    d = (2e-9, 2e-9, 2e-9)
    M = W.random_unit(nx, ny, nz, seed=3)
    M[:, 1, 2, :] = 0.0   # some zero sources
    H = oracle.demag_direct(M, d).reshape(3, -1)
    obs = W.sample_cells(nx * ny * nz, 20, seed=5)
    Ha = oracle.demag_direct_at(M, d, obs)
    assert np.allclose(Ha, H[:, obs], rtol=0, atol=1e-13 * np.abs(H).max())


def test_linearity():
    nx, ny, nz = 6, 4, 3
    d = (4e-9, 4e-9, 2e-9)
    dm = oracle.Demag(nx, ny, nz, *d)
    a = W.random_unit(nx, ny, nz, 1)
    b = W.random_unit(nx, ny, nz, 2)
    lhs = dm.apply(2.5 * a - 0.75 * b)
    rhs = 2.5 * dm.apply(a) - 0.75 * dm.apply(b)
    assert rel_l2(lhs, rhs) < 1e-13


@pytest.mark.parametrize("grid,d", [((4, 4, 4), (1.0, 1.0, 1.0)), ((8, 4, 2), (1.0, 1.3, 0.7)),
                                    ((16, 16, 1), (4e-9, 4e-9, 4e-9))])
def test_uniform_prism_mean_field_is_minus_DM(grid, d):
    """Uniform M: the cell-average of H_d is -D M with D the prism's
    demagnetising tensor (Aharoni), for each direction of M."""
    nx, ny, nz = grid
    dm = oracle.Demag(nx, ny, nz, *d)
    D = aharoni_diag(nx * d[0], ny * d[1], nz * d[2])
    for a in range(3):
        M = np.zeros((3, nz, ny, nx))
        M[a] = 1.0
        Hm = dm.apply(M).reshape(3, -1).mean(axis=1)
        ref = np.zeros(3)
        ref[a] = -D[a]
        # tolerance: the tensor quadrature beyond 8 cells is accurate to ~1e-10
        assert np.allclose(Hm, ref, rtol=0, atol=1e-9)


def test_translation_invariance_of_pair_field():
    """The field of one source cell at a fixed offset does not depend on where
    the pair sits in the grid (convolution)."""
    nx, ny, nz = 7, 5, 3
    d = (1e-9, 1e-9, 1e-9)
    dm = oracle.Demag(nx, ny, nz, *d)
    vals = []
    for (i, j, k) in [(0, 0, 0), (2, 1, 1), (3, 2, 0)]:
        M = np.zeros((3, nz, ny, nx))
        M[:, k, j, i] = (0.3, -0.5, 0.8)
        H = dm.apply(M)
        vals.append(H[:, k + 1, j + 2, i + 3])
    assert np.allclose(vals[0], vals[1], atol=1e-14) and np.allclose(vals[0], vals[2], atol=1e-14)
