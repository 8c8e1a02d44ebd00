"""delta-f storage (dg_set_background) against the FP64 oracle on f0 + g.

The state holds g = f - f0 for an x-uniform background f0; the library adds
L(f0) = -E G_u + G_b from FP64 tables.  The oracle never sees the split: it
computes on the whole f = f0 + g (Sec. 2, eq. weak).  Bars as the whole-f
parity tests: FP64 element-wise 1e-12 of the largest magnitude (1e-11 for the
bare RHS), FP32 relative L2 1e-5.

Precision: on the fine learned-correction grid (32^3 elements, n = 8, ring /
Maxwellian mixture with a 1e-3 perturbation, omega_c = 1) an FP32 run is
compared with the FP64 whole-f run over 14 000 steps by the relative L2
distance of the field-energy histories: whole-f FP32 storage drifts by
percents (the perturbation is 1e-3 of f, FP32 rounds f to 6e-8 of itself at
every stage), delta-f FP32 storage must stay within 0.1 %.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import diagnostics, grid, lgl, poisson, rhs, rk  # noqa: E402
from paper_2202_13532_amd import dg, inputs, workloads  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [
    # nv, n, nelem, lo, hi, wc, layout
    (2, 8, [3, 4, 11], [0.0, -8.0, -8.0], [4 * math.pi, 8.0, 8.0], 1.0, "dense"),
    (2, 9, [2, 3, 10], [0.0, -8.0, -8.0], [20.0, 8.0, 8.0], 0.7, "vpad"),
    (2, 5, [3, 2, 13], [0.0, -6.0, -6.0], [6.0, 6.0, 6.0], -1.1, "dense"),
    (1, 6, [5, 21], [0.0, -7.0], [4 * math.pi, 7.0], 0.0, "dense"),
]


def _background(g, nv):
    """x-uniform f0 at the velocity nodes: ring/Maxwellian mixture (1D2V),
    Maxwellian (1D1V); symmetric, so equal at the periodic wrap."""
    if nv == 2:
        u = g.axes[1].flat_nodes()[:, None]
        v = g.axes[2].flat_nodes()[None, :]
        return 0.4 * inputs.ring(u, v) + 0.6 * inputs.maxwellian_2d(u, v, 1.1)
    return inputs.maxwellian_1d(g.axes[1].flat_nodes(), 1.0)


def _full(f0, g_state, nv):
    if nv == 2:
        Nu, n, Nv = g_state.shape[2], g_state.shape[3], g_state.shape[4]
        return g_state + f0.reshape(1, 1, Nu, n, Nv, n)
    Nv, n = g_state.shape[2], g_state.shape[3]
    return g_state + f0.reshape(1, 1, Nv, n)


def _make(case, storage):
    nv, n, nelem, lo, hi, wc, layout = case
    s = dg.Solver(nv, n, nelem, lo, hi, wc, 0, storage, layout=layout)
    g = grid.PhaseGrid(nv, n, nelem, lo, hi, wc)
    return s, g


def _ids(c):
    return "nv%d_n%d_%s" % (c[0], c[1], c[6])


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_deltaf_rhs_and_step_match_oracle(case, storage):
    nv, n, nelem = case[0], case[1], case[2]
    print("delta-f parity", case, storage, flush=True)
    s, g = _make(case, storage)
    f0 = _background(g, nv)
    s.set_background(f0)
    c = g.coords()
    k = 2 * math.pi / (g.axes[0].hi - g.axes[0].lo)
    # perturbation: a smooth x mode plus small random noise (non-equilibrium)
    gx = np.broadcast_to(_full(f0, np.zeros(g.shape), nv) * 0.01 * np.cos(k * c[0]), g.shape)
    gh = np.ascontiguousarray(gx + 1e-3 * inputs.random_nodal(g.shape, 3 + n))
    gd = s.pack(torch.from_numpy(gh).to("cuda", s.dtype))
    gh = s.unpack(gd).double().cpu().numpy()           # the values the GPU holds
    fh = _full(f0, gh, nv)
    ops = lgl.operators(n)
    # RHS with a given field and with the solved one
    E = inputs.random_field(nelem[0] * n, 17)
    out = s.unpack(s.rhs(gd, torch.from_numpy(E).cuda())).double().cpu().numpy()
    ref = rhs.rhs(g, ops, fh, E.reshape(nelem[0], n))
    Eg = s.poisson(gd).cpu().numpy()
    Eo, _ = poisson.field_from_density(g, rhs.density(g, fh))
    assert np.max(np.abs(Eg - np.asarray(Eo).ravel())) <= 1e-11 * max(1.0, np.max(np.abs(Eo)))
    if storage == "f64":
        assert np.max(np.abs(out - ref)) <= 1e-11 * np.max(np.abs(ref))
    else:
        assert np.linalg.norm(out - ref) <= 1e-5 * np.linalg.norm(ref)
    # one SSP-RK3 step: g advances like f
    dt = 0.5 * s.dt_max(0.1)
    s.step(gd, dt, 1)
    gnew = s.unpack(gd).double().cpu().numpy()
    fref = rk.ssprk3_step(g, ops, fh, dt)
    gref = fref - _full(f0, np.zeros(g.shape), nv)
    if storage == "f64":
        assert np.max(np.abs(gnew - gref)) <= 1e-12 * np.max(np.abs(fref))
    else:
        assert np.linalg.norm(gnew - gref) <= 1e-5 * np.linalg.norm(gref)
    # diagnostics are those of f0 + g
    d = s.diagnostics(gd)
    fn = _full(f0, gnew, nv)
    Ef, _ = poisson.field_from_density(g, rhs.density(g, fn))
    tol = 1e-12 if storage == "f64" else 1e-6
    assert abs(d["mass"] / diagnostics.mass(g, fn) - 1) < tol
    assert abs(d["l2sq"] / diagnostics.l2sq(g, fn) - 1) < tol
    if nv == 2:
        assert abs(d["kinetic_energy"] / diagnostics.kinetic_energy(g, fn) - 1) < tol
    assert abs(d["field_energy"] / diagnostics.field_energy(g, Ef) - 1) < (1e-9 if storage == "f64" else 1e-4)
    # back to whole-f states: the same context gives the whole-f RHS of f
    s.set_background(None)
    fd = s.pack(torch.from_numpy(np.ascontiguousarray(fn)).to("cuda", s.dtype))
    out2 = s.unpack(s.rhs(fd, torch.from_numpy(E).cuda())).double().cpu().numpy()
    ref2 = rhs.rhs(g, ops, s.unpack(fd).double().cpu().numpy(), E.reshape(nelem[0], n))
    assert np.linalg.norm(out2 - ref2) <= 1e-5 * np.linalg.norm(ref2)
    s.close()


def test_background_errors():
    s = dg.Solver(2, 4, [2, 3, 5], [0.0, -4.0, -4.0], [3.0, 4.0, 4.0], 1.0, 0, "f32")
    g = grid.PhaseGrid(2, 4, [2, 3, 5], [0.0, -4.0, -4.0], [3.0, 4.0, 4.0], 1.0)
    f0 = _background(g, 2)
    bad = f0.copy()
    bad[5, 7] += 0.1 * np.max(f0)      # u node 5 is interior: its element's face values stay equal...
    bad[3, 7] += 0.1 * np.max(f0)      # ...node 3 is the last node of element 0: a jump across a u face
    with pytest.raises(dg.DGError) as ex:
        s.set_background(bad)
    assert ex.value.status == dg.DG_ERR_INVALID and "face" in str(ex.value)
    with pytest.raises(dg.DGError):
        s.set_background(np.full_like(f0, np.nan))
    s.close()
    z = dg.Solver(2, 4, [2, 3, 5], [0.0, -4.0, -4.0], [3.0, 4.0, 4.0], 1.0, 0, "f32", "zero_inflow")
    with pytest.raises(dg.DGError) as ex:
        z.set_background(f0)
    assert ex.value.status == dg.DG_ERR_UNSUPPORTED
    z.close()


def _field_history(s, f, dt, nsteps):
    recs = s.step(f, dt, nsteps, diag=True)
    return np.array([r["field_energy"] for r in recs])


def test_deltaf_fp32_follows_fp64_field_energy_history():
    """14 000 steps on the fine learned-correction grid: FP32 delta-f within
    0.1 % of the FP64 field-energy history, whole-f FP32 not."""
    wl = workloads.fine_1d2v_n8(1.0)
    wl.ic_args = {"a": 0.5, "vt": 1.0, "k1": 0.5, "eps": 1e-3}
    nsteps = 14000
    sols = {m: dg.Solver(wl.nv, wl.n, wl.nelem, wl.lo, wl.hi, wl.omega_c, 0, st)
            for m, st in [("f64", "f64"), ("f32", "f32"), ("f32_df", "f32")]}
    s64 = sols["f64"]
    nodes = [torch.from_numpy(s64.nodes(a)).cuda() for a in range(3)]
    f_full = workloads.initial_state(wl, nodes, torch).to(torch.float64).contiguous()
    u = s64.nodes(1).reshape(-1)[:, None]
    v = s64.nodes(2).reshape(-1)[None, :]
    f0 = 0.5 * inputs.ring(u, v) + 0.5 * inputs.maxwellian_2d(u, v, 1.0)
    f0d = torch.from_numpy(np.ascontiguousarray(f0)).cuda().reshape(1, 1, 32, 8, 32, 8)
    g = (f_full - f0d).contiguous()
    dt = wl.cfl_fraction * s64.dt_max(0.05)
    W = {}
    W["f64"] = _field_history(s64, f_full.clone(), dt, nsteps)
    W["f32"] = _field_history(sols["f32"], f_full.float().contiguous(), dt, nsteps)
    sols["f32_df"].set_background(f0)
    W["f32_df"] = _field_history(sols["f32_df"], g.float().contiguous(), dt, nsteps)
    err = {m: float(np.linalg.norm(W[m] - W["f64"]) / np.linalg.norm(W["f64"])) for m in ("f32", "f32_df")}
    print("field-energy history vs FP64 over %d steps: whole-f FP32 %.3e, delta-f FP32 %.3e"
          % (nsteps, err["f32"], err["f32_df"]), flush=True)
    assert err["f32_df"] < 1e-3
    assert err["f32"] > 10 * err["f32_df"]
    for so in sols.values():
        so.close()
