"""Long FP32 GPU trajectories against stored FP64 oracle trajectories
(tests/golden/, written by tests/golden/make_golden.py from the oracle only).
Bar for the film dynamics: time-averaged <m> within 1e-3 per component."""
import json
import os

import numpy as np
import pytest

from gpucommon import say, to_dev
from paper_1406_7459_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_film32_trajectory():
    from paper_1406_7459_amd import mm
    g = _load("film32.json")
    wl = W.film32()
    nx, ny, nz = wl.shape
    m = wl.mat
    p = mm.LLGParams.make(Ms=m.Ms, A=m.A, alpha=m.alpha, dt=m.dt)
    plan = mm.Plan(nx, ny, nz, *wl.cell)
    M = to_dev(m.Ms * wl.initial_unit())
    got = []
    for rec in g["records"]:
        st = plan.reduce(p, M)
        got.append(st)
        if rec["step"] < g["steps"]:
            plan.step(p, M, g["record_every"])
    ref_m = np.array([r["m_avg"] for r in g["records"]])
    got_m = np.array([s["m_avg"] for s in got])
    ref_E = np.array([r["E_tot"] for r in g["records"]])
    got_E = np.array([s["E_tot"] for s in got])
    say("film32 max |d<m>|", np.abs(got_m - ref_m).max(), "max rel dE", np.abs(got_E / ref_E - 1).max())
    assert np.abs(got_m.mean(axis=0) - ref_m.mean(axis=0)).max() <= 1e-3
    assert np.abs(got_E / ref_E - 1).max() <= 1e-3


def test_film128_relax_and_switch():
    from paper_1406_7459_amd import mm
    g = _load("film128.json")
    wl = W.film128()
    nx, ny, nz = wl.shape
    m = wl.mat
    ex = wl.extra
    plan = mm.Plan(nx, ny, nz, *wl.cell)
    M = to_dev(m.Ms * wl.initial_unit())
    le = g["log_every"]

    def run(params, nsteps):
        log = [plan.reduce(params, M)["m_avg"]]
        for _ in range(nsteps // le):
            plan.step(params, M, le)
            log.append(plan.reduce(params, M)["m_avg"])
        return np.array(log)

    pr = mm.LLGParams.make(Ms=m.Ms, A=m.A, alpha=ex["relax_alpha"], dt=m.dt)
    relax = run(pr, g["relax_steps"])
    ps = mm.LLGParams.make(Ms=m.Ms, A=m.A, alpha=ex["switch_alpha"], dt=m.dt, Hext=ex["switch_Hext"])
    sw = run(ps, g["switch_steps"])
    ref_r = np.array(g["relax_mavg"])
    ref_s = np.array(g["switch_mavg"])
    assert relax.shape == ref_r.shape and sw.shape == ref_s.shape
    d_avg = np.abs(sw.mean(axis=0) - ref_s.mean(axis=0))
    say("film128 relax end <m>", relax[-1], "ref", ref_r[-1])
    say("film128 switch time-avg |d<m>|", d_avg, "max_t |d<m>|", np.abs(sw - ref_s).max())
    assert np.abs(relax[-1] - ref_r[-1]).max() <= 1e-3
    assert d_avg.max() <= 1e-3
