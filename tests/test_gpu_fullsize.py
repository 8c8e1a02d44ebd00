"""Full-size checks in the launch configuration the benchmark times.

* 1D2V ring, 32^3 elements, n = 8 (16.8 M DOF) and 1D2V Maxwellian with 8
  modes, 64 x 48 x 48 elements, n = 9 (107.5 M DOF):
  - FP32 vs FP64 storage over 10 SSP-RK3 steps from the same state: the
    relative L2 difference of the states after every step <= 1e-5 (the FP32
    bound; both runs in the benchmark's launch configuration);
  - the oracle on a 1/8 x-subdomain: x elements [0, Nx/8) plus one halo
    element on each side are cut out of the GPU's input state, E comes from
    the oracle's own full-domain Poisson solve (checked against the GPU's E),
    and the oracle's FP64 RHS on the interior elements is compared with the
    GPU's FP64 full-domain RHS there (1e-12 of the size |f| |a| J of its
    terms, which nearly cancel for these states).  The
    FP32 RHS is not compared: for these near-equilibrium states the RHS is a
    small difference of large terms, so FP32 is judged on the state.
* The 64-run uneven sweep: four sampled runs of the batch equal their solo
  runs bit for bit after two steps.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import grid, lgl, poisson, rhs  # noqa: E402
from paper_2202_13532_amd import dg, workloads  # noqa: E402

pytestmark = pytest.mark.gpu


def _state(wl, s, dtype):
    nodes = [torch.from_numpy(s.nodes(a)).cuda() for a in range(1 + wl.nv)]
    f = workloads.initial_state(wl, nodes, torch)
    return f.to(torch.float32).to(dtype).contiguous()   # FP64 runs start from the FP32 values


def _subdomain_rhs(wl, f_full, E_full):
    """Oracle RHS on x elements [0, Nx/8) from the full FP64 state (halo of one
    element each side, periodic wrap of the cut-out domain; only the interior
    elements are returned)."""
    n, (Nx, Nu, Nv) = wl.n, wl.nelem
    m = Nx // 8
    idx = [(i % Nx) for i in range(-1, m + 1)]
    sub = f_full[idx]                                   # (m + 2, n, Nu, n, Nv, n)
    dx = (wl.hi[0] - wl.lo[0]) / Nx
    g = grid.PhaseGrid(2, n, [m + 2, Nu, Nv], [wl.lo[0] - dx, wl.lo[1], wl.lo[2]],
                       [wl.lo[0] + (m + 1) * dx, wl.hi[1], wl.hi[2]], wl.omega_c)
    Es = E_full.reshape(Nx, n)[idx]
    r = rhs.rhs(g, lgl.operators(n), sub, Es)
    return r[1:m + 1]


@pytest.mark.parametrize("name", ["ring_1d2v_n8", "maxwell_1d2v_n9"])
def test_fullsize_fp32_vs_fp64_and_oracle_subdomain(name):
    print("full size", name, flush=True)
    wl = workloads.ring_1d2v_n8() if name == "ring_1d2v_n8" else workloads.maxwell_1d2v_n9()
    s32 = dg.Solver(wl.nv, wl.n, wl.nelem, wl.lo, wl.hi, wl.omega_c, 0, "f32")
    s64 = dg.Solver(wl.nv, wl.n, wl.nelem, wl.lo, wl.hi, wl.omega_c, 0, "f64")
    f32 = _state(wl, s32, torch.float32)
    f64 = f32.to(torch.float64).contiguous()
    # FP64 RHS and field at the initial state
    r64 = s64.rhs(f64)
    E64 = s64.poisson(f64)
    fh = f64.cpu().numpy()
    gfull = grid.PhaseGrid(2, wl.n, wl.nelem, wl.lo, wl.hi, wl.omega_c)
    nd = rhs.density(gfull, fh)
    Eo, _ = poisson.field_from_density(gfull, nd)
    Eo = np.asarray(Eo).ravel()
    assert np.max(np.abs(E64.cpu().numpy() - Eo)) <= 1e-10 * np.max(np.abs(Eo))
    ref = _subdomain_rhs(wl, fh, Eo)
    m = wl.nelem[0] // 8
    g64 = r64[:m].cpu().numpy()
    # the RHS of a near-equilibrium state is a small difference of terms of
    # size |f| |a| J; rounding is relative to those terms
    dxs = [(wl.hi[a] - wl.lo[a]) / wl.nelem[a] for a in range(3)]
    vmax = max(abs(wl.lo[1]), abs(wl.hi[1]))
    term = np.max(np.abs(fh[:m + 1])) * (vmax * 2 / dxs[0] + (np.max(np.abs(Eo)) + vmax * wl.omega_c) * 2 / dxs[1]
                                         + vmax * wl.omega_c * 2 / dxs[2])
    print("FP64 RHS vs oracle:", np.max(np.abs(g64 - ref)), "term scale", term, flush=True)
    assert np.max(np.abs(g64 - ref)) <= 1e-12 * term
    del r64, g64, ref, nd
    del fh
    # FP32 vs FP64, every step
    dt = wl.cfl_fraction * s64.dt_max(max(float(E64.abs().max()), 0.05))
    worst = 0.0
    for _ in range(10):
        s32.step(f32, dt, 1)
        s64.step(f64, dt, 1)
        diff = float(torch.linalg.vector_norm(f32.double() - f64) / torch.linalg.vector_norm(f64))
        worst = max(worst, diff)
    print("FP32 vs FP64, worst step over 10:", worst, flush=True)
    assert worst < 1e-5
    s32.close()
    s64.close()


def test_uneven_sweep_sampled_runs_equal_solo():
    runs = workloads.uneven_sweep(64)
    cfgs = [dg.make_config(w.nv, w.n, w.nelem, w.lo, w.hi, w.omega_c) for w in runs]
    solos, states, dts = [], [], []
    for w in runs:
        so = dg.Solver(w.nv, w.n, w.nelem, w.lo, w.hi, w.omega_c)
        f = _state(w, so, torch.float32)
        dts.append(w.cfl_fraction * so.dt_max(max(float(so.poisson(f).abs().max()), 0.05)))
        states.append(f)
        solos.append(so)
    picks = [0, 17, 40, 63]
    copies = [states[r].clone() for r in picks]
    b = dg.Batch(cfgs)
    b.step(states, dts, 2)
    for r, c in zip(picks, copies):
        solos[r].step(c, dts[r], 2)
        assert torch.equal(c, states[r]), r
    b.close()
    for so in solos:
        so.close()
