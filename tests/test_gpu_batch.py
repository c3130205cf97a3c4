"""Batched form: many grids of uneven sizes stepped by merged launches (one
per pass kind) or grouped launches (one per pass kind and length) must give
bitwise the per-instance results when the per-instance plans run the same
radix orders (same kernel bodies, same arithmetic)."""
import numpy as np
import pytest

from gpucommon import say, to_dev, to_host
from paper_1406_7459_amd import workloads as W

pytestmark = pytest.mark.gpu

SMALL = [((16, 24, 1), (4e-9, 4e-9, 2e-9)), ((32, 16, 2), (4e-9, 4e-9, 2e-9)),
         ((24, 48, 4), (4e-9, 4e-9, 2e-9)), ((16, 16, 8), (4e-9, 4e-9, 2e-9)),
         ((48, 32, 1), (4e-9, 4e-9, 2e-9)), ((32, 32, 2), (2e-9, 2e-9, 2e-9)),
         ((12, 6, 3), (1e-9, 1.3e-9, 0.7e-9)), ((64, 8, 1), (4e-9, 4e-9, 2e-9)),
         ((1, 1, 1), (2e-9, 2e-9, 2e-9)), ((96, 12, 12), (2e-9, 2e-9, 2e-9))]


def _params(mm, i, integrator="rk4"):
    return mm.LLGParams.make(Ms=8e5, A=1.3e-11, Ku=1e4 * (i % 3), alpha=0.3 + 0.05 * i,
                             Hext=(1e4 * (i - 4), 2e3 * i, -5e3), dt=1e-14, integrator=integrator)


def _alt(L):
    return L >= 24 and L % 3 == 0


def _set_variant(mm, plan, pname, var):
    for P in (16, 8, 4, 2, 1, 32, 64, 128):
        try:
            plan.set_tile(pname, P + 256 * var)
            return
        except mm.MMError:
            continue
    raise AssertionError("no tile of variant %d for %s" % (var, pname))


def _plan(mm, s, d, mode):
    """A per-instance plan running the radix orders the batch's mode runs:
    merged launches take order 1 for transform lengths 3 * 2^a >= 24, and
    in the y passes also for 2^a lengths >= 512."""
    plan = mm.Plan(*s, *d)
    if mode == "merged":
        inf = plan.info()
        if _alt(inf["Lx"]):
            plan.set_tile("xstage", 0)
            _set_variant(mm, plan, "xfwd", 2)
            _set_variant(mm, plan, "xinv", 2)
        if s[2] > 1:
            if _alt(inf["Ly"]) or (inf["Ly"] >= 512 and (inf["Ly"] & (inf["Ly"] - 1)) == 0):
                _set_variant(mm, plan, "yfwd", 2)
                _set_variant(mm, plan, "yinv", 2)
            if _alt(inf["Lz"]):
                _set_variant(mm, plan, "zconv", 3)
        elif _alt(inf["Ly"]):
            _set_variant(mm, plan, "yconv", 3)
    return plan


@pytest.mark.parametrize("mode", ["merged", "grouped"])
def test_batched_demag_is_bitwise_per_instance(mode):
    from paper_1406_7459_amd import mm
    b = mm.Batch([s for s, _ in SMALL], [d for _, d in SMALL])
    b.set_mode(mode)
    Ms = [to_dev(8e5 * W.random_unit(*s, seed=i)) for i, (s, _) in enumerate(SMALL)]
    Hb = [to_host(h) for h in b.demag(Ms)]
    for i, (s, d) in enumerate(SMALL):
        plan = _plan(mm, s, d, mode)
        Hp = to_host(plan.demag(Ms[i]))
        assert np.array_equal(Hb[i], Hp), (s, mode)
        plan.close()
    b.autotune(reps=2)
    Hb2 = [to_host(h) for h in b.demag(Ms)]
    for i in range(len(SMALL)):
        assert np.array_equal(Hb2[i], Hb[i])
    b.close()


@pytest.mark.parametrize("mode", ["merged", "grouped"])
@pytest.mark.parametrize("integrator", ["rk4", "euler"])
def test_batched_steps_are_bitwise_per_instance(integrator, mode):
    from paper_1406_7459_amd import mm
    b = mm.Batch([s for s, _ in SMALL], [d for _, d in SMALL])
    b.set_mode(mode)
    M0 = [8e5 * W.random_unit(*s, seed=10 + i) for i, (s, _) in enumerate(SMALL)]
    Mb = [to_dev(m) for m in M0]
    params = [_params(mm, i, integrator) for i in range(len(SMALL))]
    b.step(params, Mb, 7)
    for i, (s, d) in enumerate(SMALL):
        plan = _plan(mm, s, d, mode)
        Mp = to_dev(M0[i])
        plan.step(params[i], Mp, 7)
        assert np.array_equal(to_host(Mb[i]), to_host(Mp)), (s, integrator, mode)
        plan.close()
    b.close()


def test_merged_and_grouped_modes_agree():
    """The two launch modes differ only in the radix orders of 3 * 2^a
    lengths: their fields agree to rounding."""
    from paper_1406_7459_amd import mm
    b = mm.Batch([s for s, _ in SMALL], [d for _, d in SMALL])
    Ms = [to_dev(8e5 * W.random_unit(*s, seed=20 + i)) for i, (s, _) in enumerate(SMALL)]
    b.set_mode("merged")
    Hm = [to_host(h) for h in b.demag(Ms)]
    b.set_mode("grouped")
    Hg = [to_host(h) for h in b.demag(Ms)]
    for a, c in zip(Hm, Hg):
        assert np.linalg.norm(a - c) <= 1e-6 * np.linalg.norm(c)
    b.close()


def test_sweep_batch_full_size_matches_per_instance():
    """The 64-film field sweep at full size: at most one launch per pass kind
    and stage (4 x 7 per RK4 step) in the merged mode, and a few instances
    checked bitwise after two batched steps."""
    from paper_1406_7459_amd import mm
    wls = W.sweep64()
    b = mm.Batch([w.shape for w in wls], [w.cell for w in wls])
    q = b.query()
    say("sweep64 merged", q)
    assert q["launches_per_step"] <= 4 * (6 + 1)
    Ms = [to_dev(w.mat.Ms * w.initial_unit()) for w in wls]
    M0 = [m.clone() for m in Ms]
    params = [mm.LLGParams.make(Ms=w.mat.Ms, A=w.mat.A, alpha=w.mat.alpha, Hext=w.mat.Hext, dt=w.mat.dt)
              for w in wls]
    b.step(params, Ms, 2)
    for i in (0, 17, 40, 63):
        plan = _plan(mm, wls[i].shape, wls[i].cell, "merged")
        m = M0[i].clone()
        plan.step(params[i], m, 2)
        assert np.array_equal(to_host(Ms[i]), to_host(m)), wls[i].shape
        plan.close()
    b.close()


def test_batch_rejects_bad_input():
    import torch
    from paper_1406_7459_amd import mm
    b = mm.Batch([(8, 8, 2)], [(1e-9, 1e-9, 1e-9)])
    M = torch.zeros((3, 2, 8, 8), device="cuda")
    with pytest.raises(mm.MMError):
        b.demag([M], [M])
    with pytest.raises(ValueError):
        b.step([], [M], 1)
    with pytest.raises(mm.MMError):
        mm.Batch([(513, 8, 2)], [(1e-9, 1e-9, 1e-9)])
    b.close()


# ------------------------------------------------------------------------
# The batched form against the oracle itself (not only against the
# per-instance plans): nine uneven instances with nz in {1, 2, 3, 4, 8},
# padded lengths with a factor 3 (6, 12, 24, 48, 96) and a single cell.
def _oracle_params(i, integrator="rk4"):
    import oracle
    return oracle.Params(Ms=8e5, A=1.3e-11, Ku=1e4 * (i % 3), alpha=0.3 + 0.05 * i,
                         Hext=(1e4 * (i - 4), 2e3 * i, -5e3), dt=1e-14, integrator=integrator)


def test_batched_demag_matches_oracle():
    """mm_batch_demag of every instance against the oracle's zero-padded FFT
    convolution (paper Sec. 2 steps (1)-(5)); bar: relative L2 <= 1e-5."""
    import oracle
    from gpucommon import rel_l2
    from paper_1406_7459_amd import mm
    b = mm.Batch([s for s, _ in SMALL], [d for _, d in SMALL])
    M0 = [8e5 * W.random_unit(*s, seed=200 + i) for i, (s, _) in enumerate(SMALL)]
    Hb = [to_host(h) for h in b.demag([to_dev(m) for m in M0])]
    for i, (s, d) in enumerate(SMALL):
        Mq = to_host(to_dev(M0[i]))  # the FP32 input the GPU saw
        Ho = oracle.Demag(*s, *d).apply(Mq)
        err = rel_l2(Hb[i], Ho)
        say("batch demag vs oracle", s, err)
        assert err <= 1e-5, s
    b.close()


@pytest.mark.parametrize("integrator", ["rk4", "euler"])
def test_batched_steps_match_oracle(integrator):
    """1 + 4 batched steps of every instance against the oracle's RK4 / Euler
    (eq. (6)), element by element through the relative L2 of the state."""
    import oracle
    from gpucommon import rel_l2
    from paper_1406_7459_amd import mm
    b = mm.Batch([s for s, _ in SMALL], [d for _, d in SMALL])
    M0 = [to_host(to_dev(8e5 * W.random_unit(*s, seed=300 + i))) for i, (s, _) in enumerate(SMALL)]
    Mb = [to_dev(m) for m in M0]
    params = [_params(mm, i, integrator) for i in range(len(SMALL))]
    Mo = list(M0)
    for nsteps in (1, 4):
        b.step(params, Mb, nsteps)
        for i, (s, d) in enumerate(SMALL):
            Mo[i], _ = oracle.Demag(*s, *d).run(_oracle_params(i, integrator), Mo[i], nsteps)
            err = rel_l2(to_host(Mb[i]), Mo[i])
            say("batch", integrator, s, nsteps, err)
            assert err < 2e-6, (s, nsteps)
    b.close()
