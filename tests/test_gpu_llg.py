"""GPU LLG parity: the fused H_eff + LL right-hand side + RK4/Euler stage
kernels (paper Sec. 2 eq. (2)-(6)) and the FP64 observables reduction, against
the FP64 oracle and closed forms."""
import math

import numpy as np
import pytest

import oracle
from closed_forms import macrospin
from gpucommon import rel_l2, say, to_dev, to_host
from paper_1406_7459_amd import workloads as W

pytestmark = pytest.mark.gpu


def _params(mm, mat, **kw):
    d = dict(Ms=mat.Ms, A=mat.A, Ku=mat.Ku, axis=mat.axis, alpha=mat.alpha, gamma0=mat.gamma0,
             Hext=mat.Hext, dt=mat.dt)
    d.update(kw)
    return mm.LLGParams.make(**d), oracle.Params(**{k: v for k, v in d.items() if k != "integrator"},
                                                 integrator=kw.get("integrator", "rk4"))


CASES = [
    ("film32", W.film32().shape, W.film32().cell, W.film32().mat),
    ("cube16", (16, 16, 16), (2e-9, 2e-9, 2e-9), W.cube(16).mat),
    ("ragged", (24, 12, 3), (4e-9, 4e-9, 2e-9),
     W.Material(Ms=8e5, A=1.3e-11, Ku=2e4, axis=(0.6, 0.0, 0.8), alpha=0.3, Hext=(1e4, -5e3, 2e4))),
]


@pytest.mark.parametrize("integrator", ["rk4", "euler"])
@pytest.mark.parametrize("name,grid,d,mat", CASES)
def test_steps_match_oracle(name, grid, d, mat, integrator):
    from paper_1406_7459_amd import mm
    say("llg", name, integrator)
    nx, ny, nz = grid
    pg, po = _params(mm, mat, integrator=integrator)
    M0 = mat.Ms * W.random_unit(nx, ny, nz, seed=21)
    plan = mm.Plan(nx, ny, nz, *d)
    dm = oracle.Demag(nx, ny, nz, *d)
    Mg = to_dev(M0)
    for nsteps in (1, 9):
        plan.step(pg, Mg, nsteps)
        M0, _ = dm.run(po, M0, nsteps)
        g = to_host(Mg)
        # the state itself and the change over the run, relative to the oracle
        assert rel_l2(g, M0) < 2e-6
    plan.close()


def test_single_step_increment_matches_oracle():
    from paper_1406_7459_amd import mm
    wl = W.film32()
    nx, ny, nz = wl.shape
    pg, po = _params(mm, wl.mat)
    M0 = wl.mat.Ms * wl.initial_unit()
    plan = mm.Plan(nx, ny, nz, *wl.cell)
    Mg = to_dev(M0)
    start = to_host(Mg)
    plan.step(pg, Mg, 1)
    dg = to_host(Mg) - start
    Mo, _ = oracle.Demag(nx, ny, nz, *wl.cell).run(po, start, 1)
    assert rel_l2(dg, Mo - start) < 1e-4


def test_macrospin_precession_on_gpu():
    from paper_1406_7459_amd import mm
    d = 2e-9
    H = 1e5
    pg = mm.LLGParams.make(Ms=8e5, A=1.3e-11, alpha=0.1, Hext=(0, 0, H), dt=1e-12)
    th0, ph0 = 1.0, 0.3
    m0 = np.array([math.sin(th0) * math.cos(ph0), math.sin(th0) * math.sin(ph0), math.cos(th0)])
    plan = mm.Plan(1, 1, 1, d, d, d)
    Mg = to_dev((8e5 * m0).reshape(3, 1, 1, 1))
    plan.step(pg, Mg, 100)
    m = to_host(Mg).ravel() / 8e5
    ref = macrospin(th0, ph0, H, 0.1, 2.211e5, 1e-10)
    assert np.abs(m - ref).max() < 2e-6


def test_reduce_matches_oracle_observables():
    from paper_1406_7459_amd import mm
    nx, ny, nz = 24, 12, 6
    d = (2e-9, 3e-9, 1.5e-9)
    mat = W.Material(Ms=1e6, A=1.5e-11, Ku=5e4, axis=(1, 0, 0), alpha=0.1, Hext=(2e4, 1e4, -3e4))
    pg, po = _params(mm, mat)
    M = mat.Ms * W.random_unit(nx, ny, nz, seed=5)
    Mq = to_host(to_dev(M))  # the FP32 state the GPU sees
    plan = mm.Plan(nx, ny, nz, *d)
    st = plan.reduce(pg, to_dev(M))
    ob = oracle.Demag(nx, ny, nz, *d).observables(po, Mq)
    for k in ("E_ex", "E_an", "E_d", "E_z", "E_tot"):
        assert st[k] == pytest.approx(ob[k], rel=1e-5, abs=1e-8 * abs(ob["E_tot"])), k
    assert st["torque_max"] == pytest.approx(ob["torque_max"], rel=1e-4)
    assert np.allclose(st["m_avg"], ob["m_avg"], atol=1e-9)
    assert st["nonfinite"] == 0


def test_nonfinite_state_is_reported():
    import torch
    from paper_1406_7459_amd import mm
    plan = mm.Plan(8, 8, 2, 2e-9, 2e-9, 2e-9)
    pg = mm.LLGParams.make(Ms=8e5, A=1.3e-11)
    M = to_dev(8e5 * W.random_unit(8, 8, 2, 3))
    M[1, 1, 3, 4] = float("nan")
    with pytest.raises(mm.MMError) as ei:
        plan.reduce(pg, M)
    assert ei.value.code == mm.MM_ENONFINITE
    st = plan.reduce(pg, M, allow_nonfinite=True)
    assert st["nonfinite"] == 1


def test_graph_replay_is_bitwise_identical_to_direct_launches():
    from paper_1406_7459_amd import mm
    nx, ny, nz = 32, 16, 4
    d = (2e-9, 2e-9, 2e-9)
    pg = mm.LLGParams.make(Ms=8e5, A=1.3e-11, alpha=0.2, dt=1e-14)
    plan = mm.Plan(nx, ny, nz, *d)
    M0 = to_dev(8e5 * W.random_unit(nx, ny, nz, 9))
    a = M0.clone()
    b = M0.clone()
    plan.step(pg, a, 12)            # one call: captured graph, replayed
    for _ in range(12):
        plan.step(pg, b, 1)         # single steps: direct launches
    assert np.array_equal(to_host(a), to_host(b))
    c = M0.clone()
    plan.step(pg, c, 5)
    plan.step(pg, c, 7)             # graph reused across calls
    assert np.array_equal(to_host(a), to_host(c))


def test_renorm_keeps_unit_length_and_off_lets_it_drift():
    from paper_1406_7459_amd import mm
    nx, ny, nz = 16, 16, 1
    d = (4e-9, 4e-9, 4e-9)
    plan = mm.Plan(nx, ny, nz, *d)
    M = to_dev(8e5 * W.random_unit(nx, ny, nz, 4))
    plan.step(mm.LLGParams.make(Ms=8e5, A=1.3e-11, dt=1e-14), M, 50)
    n = np.sqrt((to_host(M) ** 2).sum(axis=0)) / 8e5
    assert np.abs(n - 1).max() < 1e-6


def test_energy_decreases_film32_full_run():
    """The film check: 2000 FP32 RK4 steps, energy monotone under damping
    with no applied field."""
    from paper_1406_7459_amd import mm
    wl = W.film32()
    nx, ny, nz = wl.shape
    pg, _ = _params(mm, wl.mat)
    plan = mm.Plan(nx, ny, nz, *wl.cell)
    M = to_dev(wl.mat.Ms * wl.initial_unit())
    E = [plan.reduce(pg, M)["E_tot"]]
    for _ in range(200):
        plan.step(pg, M, 10)
        E.append(plan.reduce(pg, M)["E_tot"])
    E = np.array(E)
    assert np.all(np.diff(E) <= 1e-6 * np.abs(E[:-1]))
    assert E[-1] < E[0]


def test_relax_reaches_torque_tolerance_and_lowers_energy():
    from paper_1406_7459_amd import mm
    nx, ny, nz = 16, 16, 16
    d = (2e-9, 2e-9, 2e-9)
    mat = W.cube(16).mat
    plan = mm.Plan(nx, ny, nz, *d)
    p = mm.LLGParams.make(Ms=mat.Ms, A=mat.A, Ku=mat.Ku, alpha=1.0, dt=1e-14)
    M = to_dev(mat.Ms * W.random_unit(nx, ny, nz, 31))
    e0 = plan.reduce(p, M)["E_tot"]
    st = plan.relax(p, M, torque_tol=1e3, max_steps=200000, check_every=500)
    say("relax", st["steps"], "steps, torque", st["torque_max"], "E", st["E_tot"])
    assert st["torque_max"] <= 1e3
    assert st["E_tot"] < e0


@pytest.mark.parametrize("fused", [True, False])
def test_timing_mode_counts_every_kernel_and_matches_untimed(fused):
    from paper_1406_7459_amd import mm
    nx, ny, nz = 32, 16, 4
    d = (2e-9, 2e-9, 2e-9)
    p = mm.LLGParams.make(Ms=8e5, A=1.3e-11, alpha=0.2, dt=1e-14)
    plan = mm.Plan(nx, ny, nz, *d)
    if not fused:
        plan.set_tile("xstage", 0)
    M0 = to_dev(8e5 * W.random_unit(nx, ny, nz, 12))
    a = M0.clone()
    plan.step(p, a, 10)
    b = M0.clone()
    plan.set_timing(True)
    plan.timing()
    plan.step(p, b, 10)
    t = plan.timing()
    plan.set_timing(False)
    assert np.array_equal(to_host(a), to_host(b))
    if fused:
        expect = dict(xfwd=10, yfwd=40, zconv=40, yinv=40, xstage=40, xinv=0, stage=0)
    else:
        expect = dict(xfwd=40, yfwd=40, zconv=40, yinv=40, xinv=40, stage=40, xstage=0)
    for k, n in expect.items():
        assert t[k][1] == n, (k, t[k])
        assert (t[k][0] > 0.0) == (n > 0)


FUSED_GRIDS = [(24, 12, 3), (6, 3, 3), (32, 16, 1), (64, 32, 8), (16, 8, 2), (3, 4, 6), (1, 1, 1), (48, 24, 12)]


@pytest.mark.parametrize("integrator", ["rk4", "euler"])
@pytest.mark.parametrize("grid", FUSED_GRIDS)
def test_fused_stage_pass_is_bitwise_the_unfused_path(grid, integrator):
    """The fused x-inverse / stage / x-forward pass (every tile) gives
    bitwise the states of XINV + stage kernel + XFWD, including grids with an
    odd number of rows per component, films and a single cell; odd and even
    step counts (Euler pairs and the copying single step)."""
    from paper_1406_7459_amd import mm
    nx, ny, nz = grid
    mat = W.Material(Ms=8e5, A=1.3e-11, Ku=2e4, axis=(0.6, 0.0, 0.8), alpha=0.3, Hext=(1e4, -5e3, 2e4))
    pg, _ = _params(mm, mat, integrator=integrator)
    plan = mm.Plan(nx, ny, nz, 4e-9, 4e-9, 2e-9)
    assert plan.info()["tiles"]["xstage"] > 0  # fused by default
    M0 = to_dev(mat.Ms * W.random_unit(nx, ny, nz, seed=34))
    plan.set_tile("xstage", 0)
    ref = {}
    for n in (1, 2, 5):
        M = M0.clone()
        plan.step(pg, M, n)
        ref[n] = to_host(M)
    tiles = []
    for P in [P + 256 * w for w in (0, 1, 2) for P in (1, 2, 4, 8, 16, 32, 64)]:
        try:
            plan.set_tile("xstage", P)
        except mm.MMError:
            continue
        tiles.append(P)
        for n in (1, 2, 5):
            M = M0.clone()
            plan.step(pg, M, n)
            assert np.array_equal(to_host(M), ref[n]), (P, n)
    say("fused tiles", grid, tiles)
    assert tiles


@pytest.mark.parametrize("integrator", ["rk4", "euler"])
@pytest.mark.parametrize("grid", [(24, 12, 3), (6, 4, 3), (64, 32, 8)])
def test_stage_vector_widths_are_bitwise_identical(grid, integrator):
    """The stage kernel with 1, 2 or 4 cells per thread (its tile) computes
    bitwise the same states, including at the x boundaries of every group,
    and a width that does not divide nx is rejected."""
    from paper_1406_7459_amd import mm
    nx, ny, nz = grid
    mat = W.Material(Ms=8e5, A=1.3e-11, Ku=2e4, axis=(0.6, 0.0, 0.8), alpha=0.3, Hext=(1e4, -5e3, 2e4))
    pg, _ = _params(mm, mat, integrator=integrator)
    plan = mm.Plan(nx, ny, nz, 4e-9, 4e-9, 2e-9)
    M0 = to_dev(mat.Ms * W.random_unit(nx, ny, nz, seed=33))
    out = {}
    for w in (1, 2, 4):
        if nx % w:
            with pytest.raises(mm.MMError):
                plan.set_tile("stage", w)
            continue
        plan.set_tile("stage", w)
        M = M0.clone()
        plan.step(pg, M, 3)
        out[w] = to_host(M)
    ws = sorted(out)
    say("stage widths", ws)
    assert len(ws) >= 2 or nx % 2
    for w in ws[1:]:
        assert np.array_equal(out[w], out[ws[0]])


def test_relax_matches_oracle_trajectory():
    """mm_llg_relax on an 8^3 cube with uniaxial anisotropy (the structure of
    the paper's cube benchmark, Sec. 4: relax to the minimum-energy state)
    against the oracle run for the same number of steps from the same FP32
    start: the state, E_tot and <m> agree, and the oracle's torque at that
    state is below the tolerance the GPU stopped at."""
    from paper_1406_7459_amd import mm
    n = 8
    d = (2e-9, 2e-9, 2e-9)
    mat = W.Material(Ms=1e6, A=1.5e-11, Ku=5e4, axis=(1, 0, 0), alpha=1.0, Hext=(0.0, 0.0, 0.0))
    pg, po = _params(mm, mat, dt=5e-14)
    plan = mm.Plan(n, n, n, *d)
    M0 = to_host(to_dev(mat.Ms * W.random_unit(n, n, n, seed=41)))
    M = to_dev(M0)
    tol = 1e5
    st = plan.relax(pg, M, torque_tol=tol, max_steps=5000, check_every=50)
    steps = st["steps"]
    say("relax 8^3", steps, "steps, torque", st["torque_max"], "E", st["E_tot"])
    assert 0 < steps < 5000 and steps % 50 == 0
    dm = oracle.Demag(n, n, n, *d)
    # one check interval before the stop the oracle's torque is still above
    # the tolerance; at the stop it is below it (up to FP32 rounding)
    Mp, _ = dm.run(po, M0, steps - 50)
    assert dm.observables(po, Mp)["torque_max"] > 0.95 * tol
    Mo, _ = dm.run(po, Mp, 50)
    g = to_host(M)
    err = rel_l2(g, Mo)
    ob = dm.observables(po, Mo)
    say("  state rel L2", err, "oracle E", ob["E_tot"], "oracle torque", ob["torque_max"])
    assert err < 1e-4
    assert st["E_tot"] == pytest.approx(ob["E_tot"], rel=1e-5)
    assert np.allclose(st["m_avg"], ob["m_avg"], atol=1e-5)
    assert st["torque_max"] <= tol
    assert ob["torque_max"] <= 1.05 * tol
