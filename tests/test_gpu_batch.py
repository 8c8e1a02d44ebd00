"""Batched persistent launch: every run equals its solo run and the oracle."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import grid, lgl, rk  # noqa: E402
from paper_2202_13532_amd import dg, inputs, workloads  # noqa: E402

pytestmark = pytest.mark.gpu

SMALL = [
    # nv, n, nelem, lo, hi, wc
    (1, 4, [5, 21], [0.0, -6.0], [4 * math.pi, 6.0], 0.0),
    (2, 8, [3, 4, 11], [0.0, -8.0, -8.0], [2 * math.pi, 8.0, 8.0], 1.0),
    (1, 7, [3, 10], [0.0, -5.0], [6.0, 5.0], 0.0),
    (2, 5, [2, 3, 13], [0.0, -6.0, -6.0], [5.0, 6.0, 6.0], 0.5),
    (2, 9, [2, 2, 8], [0.0, -8.0, -8.0], [20.0, 8.0, 8.0], 0.0),
    (1, 2, [4, 70], [0.0, -4.0], [3.0, 4.0], 0.0),
    (2, 11, [2, 2, 6], [0.0, -6.0, -6.0], [6.0, 6.0, 6.0], 1.0),
    (1, 12, [2, 9], [0.0, -5.0], [4.0, 5.0], 0.0),
]


def _state(case, seed):
    nv, n, nelem, lo, hi, wc = case
    g = grid.PhaseGrid(nv, n, nelem, lo, hi, wc)
    c = g.coords()
    k = 2 * math.pi / (hi[0] - lo[0])
    if nv == 1:
        f = inputs.maxwellian_1d(c[1], 1.0) * (1 + 0.05 * np.cos(k * c[0]))
    else:
        f = inputs.maxwellian_2d(c[1], c[2], 1.2) * (1 + 0.05 * np.cos(k * c[0]))
    f = np.broadcast_to(f, g.shape) * (1 + 0.01 * inputs.random_nodal(g.shape, seed))
    return g, np.ascontiguousarray(f)


def test_batch_equals_solo_runs_and_oracle():
    cfgs = [dg.make_config(nv, n, ne, lo, hi, wc) for nv, n, ne, lo, hi, wc in SMALL]
    B = dg.Batch(cfgs)
    grids, host, dev, dts = [], [], [], []
    for i, case in enumerate(SMALL):
        g, f = _state(case, 10 + i)
        grids.append(g)
        host.append(f)
        dev.append(torch.from_numpy(f).float().cuda())
        s = dg.Solver(*case[:6])
        dts.append(0.4 * s.dt_max(0.2))
        s.close()
    solo = [d.clone() for d in dev]
    B.step(dev, dts, 2)
    for i, case in enumerate(SMALL):
        s = dg.Solver(*case[:6])
        s.step(solo[i], dts[i], 2)
        s.close()
        a, b = dev[i].cpu().numpy().astype(np.float64), solo[i].cpu().numpy().astype(np.float64)
        assert np.max(np.abs(a - b)) <= 1e-6 * np.max(np.abs(b)), i
        # oracle: two FP64 steps from the FP32-rounded initial state
        f0 = torch.from_numpy(host[i]).float().double().numpy()
        ref = f0
        for _ in range(2):
            ref = rk.ssprk3_step(grids[i], lgl.operators(case[1]), ref, dts[i])
        assert np.linalg.norm(a - ref) / np.linalg.norm(ref) < 1e-5, i
    B.close()


def test_batch_bitwise_equal_to_solo():
    case = SMALL[1]
    cfg = dg.make_config(*case[:6])
    B = dg.Batch([cfg])
    g, f = _state(case, 3)
    a = torch.from_numpy(f).float().cuda()
    b = a.clone()
    s = dg.Solver(*case[:6])
    dt = 0.4 * s.dt_max(0.2)
    B.step([a], [dt], 3)
    s.step(b, dt, 3)
    assert torch.equal(a, b)
    s.close()
    B.close()


def test_batch_diagnostics_and_cfl_errors():
    cfgs = [dg.make_config(*c[:6]) for c in SMALL[:3]]
    B = dg.Batch(cfgs)
    dev, dts = [], []
    for i, case in enumerate(SMALL[:3]):
        _, f = _state(case, 20 + i)
        dev.append(torch.from_numpy(f).float().cuda())
        s = dg.Solver(*case[:6])
        dts.append(0.4 * s.dt_max(0.2))
        s.close()
    m0 = [None] * 3
    recs = B.step(dev, dts, 4, diag=True)
    assert len(recs) == 3 and all(len(r) == 4 for r in recs)
    for r in recs:
        assert all(x["finite"] == 1 for x in r)
        ms = [x["mass"] for x in r]
        assert max(ms) - min(ms) < 1e-6 * abs(ms[0])
    bad = list(dts)
    bad[1] = 100.0
    with pytest.raises(dg.DGError) as e:
        B.step(dev, bad, 1)
    assert e.value.status == dg.DG_ERR_CFL
    best = B.tune(dev, dts, 1)
    assert best > 0 and B.grid > 0
    B.close()


def test_uneven_sweep_64_runs_conserves_mass():
    wls = workloads.uneven_sweep(64)
    cfgs = [dg.make_config(w.nv, w.n, w.nelem, w.lo, w.hi, w.omega_c) for w in wls]
    B = dg.Batch(cfgs)
    dev, dts = [], []
    for w in wls:
        s = dg.Solver(w.nv, w.n, w.nelem, w.lo, w.hi, w.omega_c)
        nodes = [torch.from_numpy(s.nodes(a)).cuda() for a in range(1 + w.nv)]
        dev.append(workloads.initial_state(w, nodes, torch).float().contiguous())
        dts.append(0.9 * s.dt_max(0.05))
        s.close()
    recs = B.step(dev, dts, 2, diag=True)
    for r, w in zip(recs, wls):
        assert r[-1]["finite"] == 1
        assert abs(r[-1]["mass"] - r[0]["mass"]) < 1e-6 * abs(r[0]["mass"]), w.name
    B.close()


def _check_kinds(choice, cases):
    """One launch per 1D2V n, in decreasing n, then one for all 1D1V runs,
    reported as (n, nv) = (0, 1)."""
    kinds = [(k["n"], k["nv"]) for k in choice["kinds"]]
    want = [(n, 2) for n in sorted({c[1] for c in cases if c[0] == 2}, reverse=True)]
    if any(c[0] == 1 for c in cases):
        want.append((0, 1))
    assert kinds == want


@pytest.mark.parametrize("which", ["1d1v_only", "1d1v_with_n5", "all"])
def test_batch_1d1v_launch_forms_bitwise_equal_to_solo(which):
    """1D1V runs of several n share one launch: alone, next to one 1D2V kind
    and next to several; every run equals its solo run bit for bit."""
    if which == "1d1v_only":
        cases = [c for c in SMALL if c[0] == 1]
    elif which == "1d1v_with_n5":
        cases = [c for c in SMALL if c[0] == 1 or c[1] == 5]
    else:
        cases = SMALL
    print("batch launch forms", which, flush=True)
    B = dg.Batch([dg.make_config(*c[:6]) for c in cases])
    _check_kinds(B.choice, cases)
    states, solo, dts, sols = [], [], [], []
    for i, c in enumerate(cases):
        _, f = _state(c, 40 + i)
        states.append(torch.from_numpy(f).float().cuda())
        solo.append(states[-1].clone())
        sols.append(dg.Solver(*c[:6]))
        dts.append(0.4 * sols[-1].dt_max(0.2))
    B.step(states, dts, 2)
    for so, f, dt in zip(sols, solo, dts):
        so.step(f, dt, 2)
    for i, (a, b) in enumerate(zip(states, solo)):
        assert torch.equal(a, b), (which, i)
    B.close()
    for so in sols:
        so.close()


def _launch_form_check(concurrent_forms):
    cases = SMALL
    cfgs = [dg.make_config(*c[:6]) for c in cases]
    B = dg.Batch(cfgs)
    solos = [dg.Solver(*c[:6]) for c in cases]
    init = [torch.from_numpy(_state(c, 10 + i)[1]).float().cuda() for i, c in enumerate(cases)]
    dts = [0.4 * so.dt_max(0.2) for so in solos]
    ref = [f.clone() for f in init]
    for so, f, dt in zip(solos, ref, dts):
        so.step(f, dt, 2)
    base = B.choice
    _check_kinds(base, cases)
    for conc in concurrent_forms:
        for order in ("cost-sorted", "run-interleaved"):
            ch = {"concurrent": conc, "order": order,
                  "kinds": [dict(k, wg_per_cu=i % 3) for i, k in enumerate(base["kinds"])]}
            B.choice = ch
            got = B.choice
            assert got["concurrent"] == conc and got["order"] == order
            states = [f.clone() for f in init]
            B.step(states, dts, 2)
            for a, b in zip(states, ref):
                assert torch.equal(a, b), (conc, order)
    return B, solos, init, dts, ref, base


def test_batch_orders_grids_and_tuner_keep_bitwise_equality():
    """Both work-list orders, any per-kind launch shape (persistent grids of
    1 or 2 work-groups per CU, one work-group per tile) and the tuner's choice
    give the solo runs' results bit for bit."""
    B, solos, init, dts, ref, base = _launch_form_check([False])
    scratch = [f.clone() for f in init]          # the tuner advances the states it times
    ms = B.tune(scratch, dts, 1)
    assert ms > 0
    states = [f.clone() for f in init]
    B.step(states, dts, 2)
    for a, b in zip(states, ref):
        assert torch.equal(a, b)
    with pytest.raises(dg.DGError):
        B.choice = dict(base, kinds=base["kinds"][:-1])
    with pytest.raises(dg.DGError) as ex:
        B.choice = dict(base, concurrent=True)
    assert ex.value.status == dg.DG_ERR_UNSUPPORTED
    B.close()
    for so in solos:
        so.close()


@pytest.mark.skip(reason="concurrent kind launches (per-kind streams forked into the captured step graph) "
                         "are switched off: a run of the tuner over that form ended in a host segmentation "
                         "fault whose cause is not established")
def test_batch_concurrent_kind_launches_keep_bitwise_equality():
    B, solos, _, _, _, _ = _launch_form_check([True])
    B.close()
    for so in solos:
        so.close()
