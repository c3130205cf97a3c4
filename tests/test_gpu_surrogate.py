"""Learned demag increment: the bfloat16 matrix-core convolution stack, its
gradients and training against the FP64 reference (oracle/surrogate.py), the
residual gate, and what the trained network gains over no network."""
import numpy as np
import pytest
import torch

from gpucommon import rel_l2, say, to_dev, to_host
from oracle import surrogate as S
from paper_1406_7459_amd import workloads as W

pytestmark = pytest.mark.gpu


def flat(params):
    out = []
    for w, b in params:
        out.append(w.numpy().ravel())
        out.append(b.numpy())
    return np.concatenate(out).astype(np.float32)


def unflat(vec):
    out, o = [], 0
    for cin, cout in zip(S.CHANNELS[:-1], S.CHANNELS[1:]):
        n = cout * cin * 27
        w = torch.from_numpy(vec[o:o + n].astype(np.float64).reshape(cout, cin, 3, 3, 3))
        o += n
        b = torch.from_numpy(vec[o:o + cout].astype(np.float64))
        o += cout
        out.append((w, b))
    return out


def ref_params(seed):
    """Oracle initialisation with weights rounded to bfloat16 and biases made
    nonzero and rounded to float32 (the GPU's operand precisions)."""
    ps = S.init_params(seed)
    g = np.random.default_rng(seed)
    out = []
    for w, b in ps:
        bb = torch.from_numpy(g.uniform(-0.05, 0.05, b.shape)).float().double()
        out.append((S.bf16(w), bb))
    return out


@pytest.mark.parametrize("grid", [(16, 12, 4), (10, 6, 3), (33, 5, 2), (20, 7, 9), (48, 3, 6), (7, 5, 1), (1, 9, 5),
                                  (17, 2, 4)])
def test_forward_matches_reference(grid):
    from paper_1406_7459_amd import mm
    nx, ny, nz = grid
    sur = mm.Surrogate(nx, ny, nz)
    ps = ref_params(1)
    sur.set_params(flat(ps))
    assert np.array_equal(sur.get_params(), flat(ps))
    dm = S.bf16(torch.from_numpy(W.random_unit(nx, ny, nz, 3)))
    out = to_host(sur.forward(to_dev(dm.numpy())))
    ref, _ = S.forward(ps, dm, bf16_between=True)
    err = rel_l2(out, ref.numpy())
    say("forward", grid, "rel L2", err)
    # the reference rounds to bf16 where the kernels store (layer inputs);
    # FP32 accumulation in another order and the GELU's FP32 exponential flip
    # a few of those roundings by one bf16 ulp: observed <= 2e-4 over these grids
    assert err < 1e-3
    sur.close()


@pytest.mark.parametrize("grid", [(12, 8, 3), (10, 6, 9)])
def test_gradients_match_reference(grid):
    # (10, 6, 9): three z blocks, so the bottom, interior and top instances of
    # the training forward and the input gradient run, and the weight
    # gradient's runs cross several levels
    from paper_1406_7459_amd import mm
    nx, ny, nz = grid
    sur = mm.Surrogate(nx, ny, nz)
    ps = ref_params(2)
    sur.set_params(flat(ps))
    dm = S.bf16(torch.from_numpy(W.random_unit(nx, ny, nz, 4)))
    dh = torch.from_numpy(0.3 * W.random_unit(nx, ny, nz, 5)).float().double()
    loss_g, g = sur.gradients(to_dev(dm.numpy()), to_dev(dh.numpy()))
    # reference: the same bf16 operands, FP64 arithmetic, and bf16 rounding at
    # the points where the matrix-core path stores a tensor (layer inputs,
    # pre-activations as the GELU derivative's argument, every dZ)
    loss, gr = S.loss_and_grads_rounded(ps, dm, dh, rnd=S.bf16)
    gref = flat(gr)
    assert loss_g == pytest.approx(loss, rel=1e-2)
    o = 0
    worst = 0.0
    for li, (w, b) in enumerate(ps):
        n = w.numel() + b.numel()
        e = rel_l2(g[o:o + n], gref[o:o + n])
        say("layer", li, "grad rel L2", e)
        worst = max(worst, e)
        o += n
    # FP32 accumulation against FP64 moves a few bf16 roundings by one ulp
    # (2^-8): the gradients agree far below that per layer
    assert worst < 1e-2


def test_gradients_are_deterministic():
    # fixed-order partial sums: the same inputs give bitwise the same gradients
    from paper_1406_7459_amd import mm
    nx, ny, nz = 20, 7, 9
    sur = mm.Surrogate(nx, ny, nz)
    ps = ref_params(3)
    sur.set_params(flat(ps))
    dm = to_dev(S.bf16(torch.from_numpy(W.random_unit(nx, ny, nz, 6))).numpy())
    dh = to_dev((0.3 * W.random_unit(nx, ny, nz, 7)).astype(np.float32))
    l1, g1 = sur.gradients(dm, dh)
    l2, g2 = sur.gradients(dm, dh)
    say("gradients twice: loss", l1, l2)
    assert l1 == l2
    assert np.array_equal(g1, g2)
    sur.close()


def test_training_reduces_loss_on_solver_pairs():
    from paper_1406_7459_amd import mm
    nx, ny, nz = 32, 32, 2
    d = (4e-9, 4e-9, 4e-9)
    plan = mm.Plan(nx, ny, nz, *d)
    sur = mm.Surrogate(nx, ny, nz)
    sur.set_params(flat(S.init_params(7)))
    p = mm.LLGParams.make(Ms=8e5, A=1.3e-11, alpha=0.1, dt=1e-14)
    M = to_dev(8e5 * W.random_unit(nx, ny, nz, 8))
    plan.step(p, M, 20)
    pairs = [mm.Surrogate.make_pair(plan, p, M, 1) for _ in range(8)]
    first = [sur.train_step(dm, dh, 2e-3) for dm, dh in pairs]
    for _ in range(40):
        for dm, dh in pairs:
            sur.train_step(dm, dh, 2e-3)
    last = [sur.gradients(dm, dh, normalize=True)[0] for dm, dh in pairs]
    say("loss first", np.mean(first), "last", np.mean(last))
    assert np.mean(last) < 0.3 * np.mean(first)


def test_gate_at_zero_tolerance_is_the_exact_path():
    from paper_1406_7459_amd import mm
    nx, ny, nz = 32, 16, 4
    d = (4e-9, 4e-9, 4e-9)
    plan = mm.Plan(nx, ny, nz, *d)
    sur = mm.Surrogate(nx, ny, nz)
    sur.set_params(flat(S.init_params(9)))
    p = mm.LLGParams.make(Ms=8e5, A=1.3e-11, alpha=0.1, dt=1e-14, Hext=(1e4, 0, 0))
    M0 = to_dev(8e5 * W.random_unit(nx, ny, nz, 10))
    a = M0.clone()
    st = sur.step(plan, p, a, 6, tol=0.0)
    b = M0.clone()
    plan.step(p, b, 6)
    assert np.array_equal(to_host(a), to_host(b))
    assert st["steps"] == 6 and st["fallbacks"] == st["checked"]
    c = M0.clone()
    st2 = sur.step(plan, p, c, 6, tol=-1.0)
    assert st2["fallbacks"] == 0 and st2["checked"] == 6 and np.isfinite(st2["max_residual"])
    assert np.isfinite(to_host(c)).all()


def test_grouped_gate_matches_per_step_gate():
    """Residuals judged on the device and read back once per group of 4
    steps: with nothing redone the state and the residual statistics equal
    those of per-step read-back bitwise; at tol = 0 every group is redone
    from its first state and the state is the exact path's; a group longer
    than MM_SUR_CHECK_MAX is refused."""
    from paper_1406_7459_amd import mm
    nx, ny, nz = 32, 16, 4
    d = (4e-9, 4e-9, 4e-9)
    plan = mm.Plan(nx, ny, nz, *d)
    sur = mm.Surrogate(nx, ny, nz)
    sur.set_params(flat(S.init_params(9)))
    kw = dict(Ms=8e5, A=1.3e-11, alpha=0.1, dt=1e-14, Hext=(1e4, 0, 0))
    p1 = mm.LLGParams.make(**kw)
    p4 = mm.LLGParams.make(**kw, sur_check_every=4)
    M0 = to_dev(8e5 * W.random_unit(nx, ny, nz, 12))
    a, b = M0.clone(), M0.clone()
    sa = sur.step(plan, p1, a, 10, tol=-1.0)
    sb = sur.step(plan, p4, b, 10, tol=-1.0)  # groups of 4, 4 and 2 steps
    assert np.array_equal(to_host(a), to_host(b))
    assert sa == sb and sb["checked"] == 10 and sb["fallbacks"] == 0
    c, e = M0.clone(), M0.clone()
    sc = sur.step(plan, p4, c, 10, tol=0.0)
    plan.step(p1, e, 10)
    assert np.array_equal(to_host(c), to_host(e))
    # a group of 4 redone, one exact step, a group of 4 redone, one exact step
    assert sc["steps"] == 10 and sc["checked"] == 8 and sc["fallbacks"] == 8
    with pytest.raises(Exception):
        sur.step(plan, mm.LLGParams.make(**kw, sur_check_every=mm.MM_SUR_CHECK_MAX + 1), M0.clone(), 2, tol=1.0)
    sur.close()
    plan.close()


def test_trained_network_beats_no_network_at_the_gate():
    """Train online on solver pairs of a 64x64x4 film (a few hundred Adam
    steps), then step a held-out trajectory through the gate: the residual of
    the trained network's field at every accepted state is a fraction of the
    residual with no network (the stage-1 field reused), and its accepted
    state stays close to the exact path's."""
    from paper_1406_7459_amd import mm
    from paper_1406_7459_amd.surrogate_train import init_params
    nx, ny, nz = 64, 64, 4
    d = (4e-9, 4e-9, 4e-9)
    plan = mm.Plan(nx, ny, nz, *d)
    sur = mm.Surrogate(nx, ny, nz)
    sur.set_params(init_params(6, 5000))
    p = mm.LLGParams.make(Ms=8e5, A=1.3e-11, alpha=0.1, dt=1e-14, Hext=(2e4, 1e4, 0))
    dm = torch.empty((3, nz, ny, nx), device="cuda")
    dh = torch.empty_like(dm)
    losses = []
    for traj in range(6):
        M = to_dev(8e5 * W.random_unit(nx, ny, nz, 300 + traj))
        plan.step(p, M, 20)
        for _ in range(100):
            mm.Surrogate.make_pair(plan, p, M, 1, dm, dh)
            losses.append(sur.train_step(dm, dh, 3e-4))
    trained = sur.get_params()
    M0 = to_dev(8e5 * W.random_unit(nx, ny, nz, 399))
    plan.step(p, M0, 20)
    exact = M0.clone()
    plan.step(p, exact, 10)
    a = M0.clone()
    st_t = sur.step(plan, p, a, 10, tol=-1.0)  # never fall back: judge every step
    sur.zero()
    b = M0.clone()
    st_z = sur.step(plan, p, b, 10, tol=-1.0)
    sur.set_params(trained)
    say("loss first", np.mean(losses[:20]), "last", np.mean(losses[-20:]),
        "residual trained", st_t["mean_residual"], "no network", st_z["mean_residual"],
        "state err trained", rel_l2(to_host(a), to_host(exact)), "no network", rel_l2(to_host(b), to_host(exact)))
    assert np.mean(losses[-20:]) < 0.1 * np.mean(losses[:20])
    assert st_t["checked"] == 10 and st_z["checked"] == 10
    assert st_t["mean_residual"] < 0.3 * st_z["mean_residual"]
    assert rel_l2(to_host(a), to_host(exact)) < rel_l2(to_host(b), to_host(exact))
