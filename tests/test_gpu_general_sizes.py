"""Grids of any size per axis (1..512 cells): each axis is zero-padded to the
smallest supported transform length L >= 2n.  The paper pads to 2n (Sec. 2,
zero-padding steps (1)-(5)); the linear convolution only needs L >= 2n - 1,
so any such L gives the same field.  Parity against the FP64 oracle (its own
padded FFT route on 2n, itself pinned to the direct sum) on grids with prime
factors 5, 7, 11 and 13, films and single-cell axes; the stored spectrum
against a library FFT of the oracle's tensor on the padded grid; LLG steps
and the batched form on such grids."""
import numpy as np
import pytest

import oracle
from gpucommon import rel_l2, say, to_dev, to_host
from paper_1406_7459_amd import workloads as W

pytestmark = pytest.mark.gpu
LENGTHS = [2, 4, 6, 8, 10, 12, 16, 20, 24, 32, 40, 48, 64, 80, 96, 128, 160, 192, 256, 320, 384, 512, 640, 768,
           1024]


def _padded(n):
    return min(L for L in LENGTHS if L >= 2 * n)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 9, 10, 13, 20, 40, 50, 80, 100, 125, 129, 160, 257, 300, 320, 500, 512])
def test_padded_lengths(n):
    from paper_1406_7459_amd import mm
    plan = mm.Plan(n, 1, 1, 1e-9, 1e-9, 1e-9)
    inf = plan.info()
    assert inf["Lx"] == _padded(n) and inf["Ly"] == 2 and inf["Lz"] == 1
    plan.close()


def test_sizes_beyond_512_are_rejected():
    from paper_1406_7459_amd import mm
    with pytest.raises(mm.MMError):
        mm.Plan(513, 4, 4, 1e-9, 1e-9, 1e-9)


GRIDS = [
    ((5, 7, 3), (2e-9, 3e-9, 1e-9)),
    ((10, 20, 1), (4e-9, 4e-9, 3e-9)),
    ((13, 11, 9), (2e-9, 2e-9, 2e-9)),
    ((50, 20, 4), (4e-9, 4e-9, 2e-9)),
    ((100, 7, 1), (3e-9, 3e-9, 3e-9)),
    ((25, 1, 1), (2e-9, 2e-9, 2e-9)),
    ((1, 1, 7), (1e-9, 2e-9, 1.5e-9)),
    ((7, 9, 5), (1e-9, 1e-9, 1e-9)),
    ((33, 17, 2), (2e-9, 2e-9, 2e-9)),
    # radix-5 lengths 10, 20, 40, 80 (n = 5 2^a pads to exactly 2n)
    ((5, 10, 20), (2e-9, 2e-9, 2e-9)),
    ((40, 20, 1), (3e-9, 3e-9, 2e-9)),
    ((20, 5, 10), (1e-9, 2e-9, 1e-9)),
]


@pytest.mark.parametrize("grid,d", GRIDS)
def test_demag_matches_oracle_any_size(grid, d):
    from paper_1406_7459_amd import mm
    nx, ny, nz = grid
    say("general demag", grid)
    M = 8e5 * W.random_unit(nx, ny, nz, seed=300 + nx + 3 * ny + 7 * nz)
    plan = mm.Plan(nx, ny, nz, *d)
    Hg = to_host(plan.demag(to_dev(M)))
    Ho = oracle.Demag(nx, ny, nz, *d).apply(M)
    err = rel_l2(Hg, Ho)
    say("  padded", plan.info()["Lx"], plan.info()["Ly"], plan.info()["Lz"], "rel L2", err)
    assert err <= 1e-5
    plan.close()


def _expected_spectrum(nx, ny, nz, d, Lx, Ly, Lz):
    """K~ from the oracle: K = -N at every signed offset |X| < n of the
    wrapped Lx x Ly x Lz grid (every other slot zero), library FFT, real
    part, octant, scaled by the inverse normalisation (nz = 1: a z axis of
    two slots whose equal bins the inverse sums, hence the factor 2)."""
    Pz = Lz if nz > 1 else 2
    Wt = np.zeros((6, Pz, Ly, Lx))

    def off(i, n, L):
        return i if i < n else (i - L if i > L - n else None)

    for z in range(Pz):
        Z = off(z, nz, Pz)
        for y in range(Ly):
            Y = off(y, ny, Ly)
            for x in range(Lx):
                X = off(x, nx, Lx)
                if X is None or Y is None or Z is None:
                    continue
                Wt[:, z, y, x] = -oracle.newell(X * d[0], Y * d[1], Z * d[2], *d)
    F = np.fft.fftn(Wt, axes=(1, 2, 3))
    assert np.abs(F.imag).max() <= 1e-9 * np.abs(F).max()
    if nz > 1:
        return F.real[:, : Lz // 2 + 1, : Ly // 2 + 1, : Lx // 2 + 1] / (Lx * Ly * Lz)
    return F.real[:, :1, : Ly // 2 + 1, : Lx // 2 + 1] * 2 / (Lx * Ly * 2)


@pytest.mark.parametrize("grid,d", [((5, 3, 3), (1e-9, 1.3e-9, 0.7e-9)), ((7, 10, 1), (4e-9, 4e-9, 3e-9))])
def test_stored_spectrum_on_padded_grid(grid, d):
    from paper_1406_7459_amd import mm
    nx, ny, nz = grid
    plan = mm.Plan(nx, ny, nz, *d)
    inf = plan.info()
    Kg = np.moveaxis(to_host(plan.spectrum()), -1, 0)
    Ke = _expected_spectrum(nx, ny, nz, d, inf["Lx"], inf["Ly"], inf["Lz"])
    assert Kg.shape == Ke.shape
    assert np.abs(Kg - Ke).max() <= 1e-6 * np.abs(Ke).max()
    plan.close()


@pytest.mark.parametrize("integrator", ["rk4", "euler"])
@pytest.mark.parametrize("grid", [(10, 5, 3), (13, 7, 1), (5, 6, 7)])
def test_steps_match_oracle_any_size(grid, integrator):
    """1 + 4 steps on a general grid against the oracle, with the fused
    stage pass (default) and bitwise equal to the unfused path."""
    from paper_1406_7459_amd import mm
    nx, ny, nz = grid
    d = (3e-9, 2e-9, 2.5e-9)
    mat = W.Material(Ms=8e5, A=1.3e-11, Ku=2e4, axis=(0.6, 0.0, 0.8), alpha=0.3, Hext=(1e4, -5e3, 2e4))
    kw = dict(Ms=mat.Ms, A=mat.A, Ku=mat.Ku, axis=mat.axis, alpha=mat.alpha, gamma0=mat.gamma0,
              Hext=mat.Hext, dt=mat.dt)
    pg = mm.LLGParams.make(integrator=integrator, **kw)
    po = oracle.Params(integrator=integrator, **kw)
    M0 = mat.Ms * W.random_unit(nx, ny, nz, seed=61)
    plan = mm.Plan(nx, ny, nz, *d)
    dm = oracle.Demag(nx, ny, nz, *d)
    Mg = to_dev(M0)
    Mu = to_dev(M0)
    Mo = M0
    for n in (1, 4):
        plan.step(pg, Mg, n)
        plan.set_tile("xstage", 0)
        plan.step(pg, Mu, n)
        plan.set_tile("xstage", plan.info()["tiles"]["xstage"] or 1)
        Mo, _ = dm.run(po, Mo, n)
        assert rel_l2(to_host(Mg), Mo) < 2e-6
        assert np.array_equal(to_host(Mg), to_host(Mu))
    plan.close()


def test_batch_with_general_sizes_matches_oracle():
    from paper_1406_7459_amd import mm
    # (7, 5, 1): a y product of length 10; (6, 4, 5): a z product of length
    # 10 (the merged launches' slot of 5 2^a products)
    shapes = [(10, 6, 2), (7, 5, 1), (16, 8, 4), (13, 3, 3), (6, 4, 5)]
    cells = [(2e-9, 2e-9, 2e-9), (4e-9, 4e-9, 3e-9), (2e-9, 3e-9, 2e-9), (1e-9, 1e-9, 1e-9), (2e-9, 2e-9, 3e-9)]
    b = mm.Batch(shapes, cells)
    Ms = [to_dev(8e5 * W.random_unit(*s, seed=70 + i)) for i, s in enumerate(shapes)]
    Hs = b.demag(Ms)
    for s, c, M, H in zip(shapes, cells, Ms, Hs):
        Ho = oracle.Demag(*s, *c).apply(to_host(M))
        assert rel_l2(to_host(H), Ho) <= 1e-5, s
    b.close()
