"""Padded v-row state layout (DG_LAYOUT_VPAD) against the dense layout.

The padded layout only moves the v chunks of every row to 64-value
boundaries; each lane of the stage, density and moment kernels performs the
same arithmetic in the same order, so every result must be bit-identical to
the dense layout's (and hence to what the dense parity tests compare with the
oracle), and the unused slots of every written state must hold zeros.  One
ragged case is also compared with the oracle directly.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import grid, lgl, rhs  # noqa: E402
from paper_2202_13532_amd import dg, inputs, workloads  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [
    # n, nelem, lo, hi, wc, vbc  (1D2V; Nv ragged against floor(64/n) where it can be)
    (9, [2, 3, 10], [0.0, -8.0, -7.0], [20.0, 8.0, 7.0], 1.0, "periodic"),
    (9, [3, 2, 7], [0.0, -6.0, -6.0], [6.0, 6.0, 6.0], 0.8, "zero_inflow"),
    (8, [3, 4, 11], [0.0, -8.0, -8.0], [2 * math.pi, 8.0, 8.0], 1.0, "periodic"),
    (3, [2, 2, 23], [0.0, -4.0, -4.0], [3.0, 4.0, 4.0], 0.7, "zero_inflow"),
    (5, [1, 2, 13], [0.0, -3.0, -3.0], [1.0, 3.0, 3.0], 2.0, "periodic"),
    (6, [2, 3, 11], [0.0, -5.0, -4.0], [4.0, 5.0, 4.0], -1.3, "periodic"),
    (7, [2, 2, 4], [0.0, -4.0, -4.0], [4.0, 4.0, 4.0], 0.0, "periodic"),
    (10, [2, 2, 13], [0.0, -6.0, -6.0], [5.0, 6.0, 6.0], 1.0, "periodic"),
    (11, [2, 3, 7], [0.0, -5.0, -5.0], [4.0, 5.0, 5.0], -0.9, "zero_inflow"),
    (12, [1, 2, 11], [0.0, -6.0, -6.0], [3.0, 6.0, 6.0], 1.0, "periodic"),
]


def _ids(c):
    return "n%d_%s_%s" % (c[0], "x".join(map(str, c[1])), c[5])


def _pad_numpy(dense, n, Nv):
    """Reference placement of a dense state's v rows into padded rows."""
    tv = 64 // n
    C = -(-Nv // tv)
    rows = dense.reshape(-1, Nv * n)
    out = np.zeros((rows.shape[0], 64 * C), dtype=dense.dtype)
    for c in range(C):
        w = min(tv, Nv - c * tv) * n
        out[:, 64 * c:64 * c + w] = rows[:, c * tv * n:c * tv * n + w]
    return out


def _pair(case, storage):
    n, nelem, lo, hi, wc, vbc = case
    d = dg.Solver(2, n, nelem, lo, hi, wc, 0, storage, vbc)
    p = dg.Solver(2, n, nelem, lo, hi, wc, 0, storage, vbc, layout="vpad")
    return d, p


def _state(case, s, seed):
    n, nelem = case[0], case[1]
    f = inputs.random_nodal([nelem[0], n, nelem[1], n, nelem[2], n], seed)
    return torch.from_numpy(f).to(device="cuda", dtype=s.dtype).contiguous()


@pytest.mark.parametrize("storage", ["f32", "f64"])
@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_pack_unpack_roundtrip(case, storage):
    print("pack/unpack", case, storage, flush=True)
    d, p = _pair(case, storage)
    f = _state(case, d, 11)
    fp = p.pack(f)
    n, Nv = case[0], case[1][2]
    assert dg.dg_state_elems(p.ctx) == fp.numel()
    assert dg.dg_state_elems(d.ctx) == f.numel()
    ref = _pad_numpy(f.cpu().numpy(), n, Nv)
    assert np.array_equal(fp.cpu().numpy().reshape(ref.shape), ref)
    assert torch.equal(p.unpack(fp), f)
    assert torch.equal(d.pack(f), f) and torch.equal(d.unpack(f), f)
    d.close()
    p.close()


@pytest.mark.parametrize("storage", ["f32", "f64"])
@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_vpad_bitwise_equal_to_dense(case, storage):
    print("vpad vs dense", case, storage, flush=True)
    d, p = _pair(case, storage)
    f = _state(case, d, 1000 + case[0])
    fp = p.pack(f)
    # RHS with a given field and with its own Poisson solve
    E = torch.from_numpy(inputs.random_field(case[1][0] * case[0], 5)).cuda()
    assert torch.equal(p.unpack(p.rhs(fp, E)), d.rhs(f, E))
    assert torch.equal(p.unpack(p.rhs(fp)), d.rhs(f))
    Ed, cd = d.poisson(f, coeffs=True)
    Ep, cp = p.poisson(fp, coeffs=True)
    assert torch.equal(Ed, Ep) and torch.equal(cd, cp)
    assert d.diagnostics(f) == p.diagnostics(fp)
    # three graph-replayed SSP-RK3 steps with diagnostics records
    dt = 0.5 * d.dt_max(float(Ed.abs().max()))
    rd = d.step(f, dt, 3, diag=True)
    rp = p.step(fp, dt, 3, diag=True)
    assert rd == rp
    assert torch.equal(p.unpack(fp), f)
    assert torch.equal(fp, p.pack(f))                 # unused slots written as zeros
    r = p.rhs(fp)
    assert torch.equal(r, p.pack(p.unpack(r)))
    d.close()
    p.close()


def test_vpad_rhs_matches_oracle_ragged_n9():
    case = CASES[0]
    n, nelem, lo, hi, wc, vbc = case
    p = dg.Solver(2, n, nelem, lo, hi, wc, 0, "f64", vbc, layout="vpad")
    g = grid.PhaseGrid(2, n, nelem, lo, hi, wc, vbc)
    f = inputs.random_nodal(g.shape, 77)
    E = inputs.random_field(nelem[0] * n, 78)
    out = p.unpack(p.rhs(p.pack(torch.from_numpy(f).cuda()), torch.from_numpy(E).cuda())).cpu().numpy()
    ref = rhs.rhs(g, lgl.operators(n), f, E.reshape(nelem[0], n))
    assert np.max(np.abs(out - ref)) <= 1e-11 * np.max(np.abs(ref))
    p.close()


def test_batch_mixed_layouts_equal_solo():
    cfgs, solos, states = [], [], []
    for i, case in enumerate(CASES):
        n, nelem, lo, hi, wc, vbc = case
        lay = "vpad" if i % 2 == 0 else "dense"
        cfgs.append(dg.make_config(2, n, nelem, lo, hi, wc, 0, "f32", vbc, lay))
        so = dg.Solver(2, n, nelem, lo, hi, wc, 0, "f32", vbc, layout=lay)
        solos.append(so)
        states.append(so.pack(_state(case, so, 300 + i)))
    dts = [0.4 * so.dt_max(float(so.poisson(f).abs().max())) for so, f in zip(solos, states)]
    copies = [f.clone() for f in states]
    b = dg.Batch(cfgs)
    b.step(states, dts, 2)
    for so, c, f, dt in zip(solos, copies, states, dts):
        so.step(c, dt, 2)
        assert torch.equal(c, f)
    b.close()
    for so in solos:
        so.close()


def test_fullsize_maxwell_n9_vpad_equals_dense():
    wl = workloads.maxwell_1d2v_n9()
    print("full size vpad", wl.name, flush=True)
    d = dg.Solver(wl.nv, wl.n, wl.nelem, wl.lo, wl.hi, wl.omega_c, 0, "f32")
    p = dg.Solver(wl.nv, wl.n, wl.nelem, wl.lo, wl.hi, wl.omega_c, 0, "f32", layout="vpad")
    nodes = [torch.from_numpy(d.nodes(a)).cuda() for a in range(1 + wl.nv)]
    f = workloads.initial_state(wl, nodes, torch).to(torch.float32).contiguous()
    fp = p.pack(f)
    dt = wl.cfl_fraction * d.dt_max(max(float(d.poisson(f).abs().max()), 0.05))
    rd = d.step(f, dt, 2, diag=True)
    rp = p.step(fp, dt, 2, diag=True)
    assert rd == rp
    assert torch.equal(p.unpack(fp), f)
    assert torch.equal(fp, p.pack(f))
    d.close()
    p.close()


def test_vpad_rejected_by_learned_correction_calls():
    case = CASES[2]
    n, nelem, lo, hi, wc, vbc = case
    p = dg.Solver(2, n, nelem, lo, hi, wc, 0, "f32", "periodic", layout="vpad")
    f = p.pack(_state(case, p, 3))
    E = p.poisson(f)
    out = torch.empty(nelem[0] * nelem[1] * nelem[2] * (7 * n ** 3 + n), dtype=torch.float32, device="cuda")
    with pytest.raises(dg.DGError, match="DG_LAYOUT_DENSE"):
        dg.dg_nn_features_raw(p.ctx, f, E, out)
    p.close()


def test_layout_calls_reject_bad_arguments():
    case = CASES[0]
    n, nelem, lo, hi, wc, vbc = case
    p = dg.Solver(2, n, nelem, lo, hi, wc, 0, "f32", vbc, layout="vpad")
    f = _state(case, p, 5)
    with pytest.raises(dg.DGError, match="NULL"):
        dg.dg_state_pack(p.ctx, None, p.empty_state())
    with pytest.raises(dg.DGError, match="NULL"):
        dg.dg_state_unpack(p.ctx, p.pack(f), None)
    with pytest.raises(dg.DGError):
        p.pack(f[:, :, :, :, :-1].contiguous())          # wrong dense shape
    with pytest.raises(dg.DGError):
        p.step(f, 1e-3, 1)                              # a dense array is not a padded state
    p.close()


def test_copy_references_copy_the_state_and_time_a_launch():
    """The bandwidth references: the streaming copy and the tile-pattern copy
    (also held to the stage kernel's residency) reproduce a padded 1D2V
    state exactly (pad slots are zero in a packed state); the empty-launch
    reference leaves its buffers alone."""
    s = dg.Solver(2, 5, [3, 4, 13], [0.0, -6.0, -6.0], [5.0, 6.0, 6.0], 0.5, layout="vpad")
    f = s.pack(torch.rand(s.dense_shape, dtype=torch.float32, device="cuda") + 0.1)
    for pattern in (0, 1, 3):
        out = s.empty_state()
        out.fill_(-1.0)
        ms = dg.dg_profile_copy(s.ctx, f, out, pattern, 2)
        assert ms > 0
        nb = f.numel() * f.element_size() // 16 * 16 // f.element_size()
        assert torch.equal(out.flatten()[:nb], f.flatten()[:nb]), pattern
    out = s.empty_state()
    out.fill_(-1.0)
    before = f.clone()
    assert dg.dg_profile_copy(s.ctx, f, out, 2, 5) > 0
    assert torch.equal(f, before) and bool((out == -1.0).all())
    with pytest.raises(dg.DGError):
        dg.dg_profile_copy(s.ctx, f, out, 4, 1)
    s.close()
