"""Parity at the full workload sizes, in the launch configuration the
benchmark times (autotuned tiles): sampled outputs against the oracle's
direct sum, and properties that hold at any size."""
import numpy as np
import pytest

import oracle
from closed_forms import aharoni_diag
from gpucommon import rel_l2, say, to_dev, to_host
from paper_1406_7459_amd import workloads as W

pytestmark = pytest.mark.gpu

FULL = [("cube128", (128, 128, 128), (2e-9, 2e-9, 2e-9)),
        ("cube256", (256, 256, 256), (2e-9, 2e-9, 2e-9)),
        ("film256", (256, 256, 4), (4e-9, 4e-9, 4e-9)),
        ("sweep-512x384x8", (512, 384, 8), (4e-9, 4e-9, 2e-9)),
        ("sweep-96x192x1", (96, 192, 1), (4e-9, 4e-9, 2e-9)),
        ("sweep-384x64x2", (384, 64, 2), (4e-9, 4e-9, 2e-9)),
        ("film128", (128, 32, 1), (3.90625e-9, 3.90625e-9, 3e-9)),
        # the largest supported axis (512 cells, transform length 1024) along z and y
        ("max-z-16x8x512", (16, 8, 512), (2e-9, 2e-9, 2e-9)),
        ("max-y-12x512x6", (12, 512, 6), (2e-9, 2e-9, 2e-9))]


@pytest.mark.parametrize("name,grid,d", FULL)
def test_sparse_sources_sampled_against_direct_sum(name, grid, d):
    from paper_1406_7459_amd import mm
    say("full-size sampled", name)
    nx, ny, nz = grid
    plan = mm.Plan(nx, ny, nz, *d)
    plan.autotune(reps=2)
    M = 8e5 * W.sparse_sources(nx, ny, nz, 32, seed=len(name))
    src = np.flatnonzero(np.abs(M).sum(axis=0).ravel())
    obs = np.unique(np.concatenate([src, W.sample_cells(nx * ny * nz, 160, seed=3)]))
    Hg = to_host(plan.demag(to_dev(M))).reshape(3, -1)[:, obs]
    Ho = oracle.demag_direct_at(M, d, obs)
    err = rel_l2(Hg, Ho)
    say("  rel L2", err)
    assert err <= 1e-5
    plan.close()


@pytest.mark.parametrize("name,grid,d", FULL[:3])
def test_uniform_state_mean_field_is_prism_factor(name, grid, d):
    from paper_1406_7459_amd import mm
    say("uniform", name)
    nx, ny, nz = grid
    plan = mm.Plan(nx, ny, nz, *d)
    plan.autotune(reps=2)
    D = aharoni_diag(nx * d[0], ny * d[1], nz * d[2])
    m = np.array([0.36, 0.48, 0.8])
    M = np.empty((3, nz, ny, nx), dtype=np.float32)
    for a in range(3):
        M[a] = 1e6 * m[a]
    H = plan.demag(to_dev(M))
    import torch
    mean = H.double().mean(dim=(1, 2, 3)).cpu().numpy()
    ref = -np.array(D) * 1e6 * m
    assert np.abs(mean - ref).max() <= 1e-5 * 1e6
    plan.close()


def test_cube64_dense_against_oracle():
    from paper_1406_7459_amd import mm
    wl = W.cube(64)
    nx, ny, nz = wl.shape
    plan = mm.Plan(nx, ny, nz, *wl.cell)
    plan.autotune(reps=2)
    M = wl.mat.Ms * wl.initial_unit()
    Hg = to_host(plan.demag(to_dev(M)))
    say("oracle cube64 ...")
    Ho = oracle.Demag(nx, ny, nz, *wl.cell).apply(M)
    err = rel_l2(Hg, Ho)
    say("  rel L2", err)
    assert err <= 1e-5
    plan.close()


def test_cube128_steps_dissipate_energy_and_keep_norm():
    from paper_1406_7459_amd import mm
    wl = W.cube(128)
    nx, ny, nz = wl.shape
    m = wl.mat
    plan = mm.Plan(nx, ny, nz, *wl.cell)
    plan.autotune(reps=2)
    p = mm.LLGParams.make(Ms=m.Ms, A=m.A, Ku=m.Ku, axis=m.axis, alpha=m.alpha, dt=m.dt)
    M = to_dev(m.Ms * wl.initial_unit())
    E = [plan.reduce(p, M)["E_tot"]]
    for _ in range(5):
        plan.step(p, M, 4)
        E.append(plan.reduce(p, M)["E_tot"])
    say("energies", E)
    assert all(E[i + 1] < E[i] for i in range(len(E) - 1))
    nrm = (M.double() ** 2).sum(dim=0).sqrt() / m.Ms
    assert float((nrm - 1).abs().max()) < 1e-6
    plan.close()
