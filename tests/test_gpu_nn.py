"""GPU parity of the learned-correction path (calls through the C ABI).

* MFMA GEMM: integer-valued BF16 operands make every product and partial sum
  exact in FP32, so a one-layer network X W + b must equal the integer matmul
  bit for bit (ragged rows, inputs and outputs), through the fused inference
  kernel and through the per-layer GEMM.
* Fused inference: against the per-layer form and the FP64 oracle MLP, and
  after parameter updates.
* Forward / gradients: against the FP64 oracle MLP evaluated on the same
  BF16-rounded inputs and weights.  The device rounds every hidden activation
  and back-propagated gradient to BF16 (unit roundoff 2^-9 = 1.95e-3); over
  four layers forward and back that gives relative L2 errors of a few 1e-3,
  so the bar is relative L2 <= 2e-2 per tensor with cosine >= 0.999.
* AdamW: FP32 update against the oracle step from the same gradients,
  absolute 1e-6 (parameters O(1), FP32 rounding ~1e-7).
* Projection, feature gather, element reordering and column statistics:
  against their definitions (projection FP64 from FP32 input, result FP32:
  relative 1e-6; copies and reorderings bit-exact).
* Corrected coarse step: one SSP-RK3 step with L(u) + s NN(u) against the
  oracle RHS plus the FP64 oracle network (same BF16 weights); the increment
  f1 - f0 within relative L2 2e-2 (the BF16 network error), and with a zero
  network the plain FP32 bar 1e-5.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import grid, lgl, mlp, projection, rhs, rk  # noqa: E402
from paper_2202_13532_amd import dg, inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def bf16_bits(x):
    """Round-to-nearest-even FP32 -> BF16 bit patterns (uint16)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def bf16_values(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _x_tensor(vals, ld):
    rows, cols = vals.shape
    b = np.zeros((rows, ld), dtype=np.uint16)
    b[:, :cols] = bf16_bits(vals)
    return torch.from_numpy(b.view(np.int16)).cuda(), bf16_values(b[:, :cols])


def _he_params(sizes, seed):
    rng = np.random.default_rng(seed)
    ps = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        ps.append(rng.standard_normal((a, b)) * math.sqrt(2.0 / a))
        ps.append(rng.standard_normal(b) * 0.1)
    return ps


def _round_weights(ps):
    """Weights as the device uses them (BF16), biases FP32."""
    out = []
    for i, p in enumerate(ps):
        p32 = np.asarray(p, dtype=np.float32)
        out.append(bf16_values(bf16_bits(p32)).reshape(p32.shape) if i % 2 == 0 else p32.astype(np.float64))
    return out


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _cos(a, b):
    return float(np.dot(a.ravel(), b.ravel()) / (np.linalg.norm(a) * np.linalg.norm(b)))


# (16384, 452, 128) takes the 64-row tiles, the others the 32-row tiles
# fused: the whole-network kernel (one 16-row block per work-group, weights
# transposed); else the per-layer GEMM
@pytest.mark.parametrize("fused", [True, False], ids=["fused", "layerwise"])
@pytest.mark.parametrize("rows,k,n", [(37, 40, 24), (1000, 452, 128), (4133, 128, 64), (5, 3, 1), (16384, 452, 128),
                                      (77, 1000, 100)])
def test_mfma_gemm_exact_on_integer_operands(rows, k, n, fused):
    print("gemm exact", rows, k, n, fused, flush=True)
    rng = np.random.default_rng(rows + k + n)
    X = rng.integers(-4, 5, size=(rows, k)).astype(np.float32)
    W = rng.integers(-3, 4, size=(k, n)).astype(np.float32)
    b = rng.integers(-8, 9, size=n).astype(np.float32)
    net = dg.Network([k, n], rows)
    net.set_fused(fused)
    net.set_params(dg.Network.flatten([W, b]))
    Xd, _ = _x_tensor(X, net.ld)
    Y = net.forward(Xd).cpu().numpy()
    ref = (X.astype(np.int64) @ W.astype(np.int64) + b.astype(np.int64)).astype(np.float32)
    assert np.array_equal(Y, ref)
    net.close()


# (8192, 452, 128): 64-row tiles and 16 k slices of 512 rows
@pytest.mark.parametrize("rows,k,n", [(256, 40, 32), (1024, 452, 64), (128, 128, 128), (8192, 452, 128)])
def test_weight_gradient_gemm_exact_on_integer_operands(rows, k, n):
    """One linear layer with integer data and rows * n a power of two: every
    value of dY = 2 (Y - T) / (rows n) is exact in BF16 and every sum exact in
    FP32, so dW = X^T dY and db = sum_rows dY must match bit for bit (the
    transposed-operand GEMM of the backward pass, split over K)."""
    print("dW gemm exact", rows, k, n, flush=True)
    rng = np.random.default_rng(rows + 3 * k + n)
    X = rng.integers(-2, 3, size=(rows, k)).astype(np.float32)
    W = rng.integers(-1, 2, size=(k, n)).astype(np.float32)
    b = rng.integers(-4, 5, size=n).astype(np.float32)
    T = rng.integers(-4, 5, size=(rows, n)).astype(np.float32)
    net = dg.Network([k, n], rows)
    net.set_params(dg.Network.flatten([W, b]))
    Xd, _ = _x_tensor(X, net.ld)
    _, g = net.loss_grad(Xd, torch.from_numpy(T).cuda(), want_loss=False, want_grads=True)
    dY = 2.0 * (X.astype(np.float64) @ W + b - T) / (rows * n)
    gw, gb = net.unflatten(g)
    assert np.array_equal(gw.astype(np.float64), X.astype(np.float64).T @ dY)
    assert np.array_equal(gb.astype(np.float64), dY.sum(axis=0))
    net.close()


SIZES = [452, 128, 128, 128, 64]


@pytest.mark.parametrize("sizes", [SIZES, [516, 128, 128, 128, 64], [100, 50, 70, 10], [33, 128, 1]],
                         ids=lambda z: "x".join(map(str, z)))
def test_fused_forward_matches_layerwise_and_oracle(sizes):
    """The fused inference kernel against the per-layer GEMMs (same BF16
    weights and activations, another FP32 summation order: a BF16 rounding of
    a hidden activation can flip, so relative L2 <= 5e-3, cosine >= 0.99999)
    and both against the FP64 oracle MLP (the BF16 bar above); ragged rows
    and widths that are not multiples of 16 or 32."""
    rows = 4133
    print("fused forward", sizes, rows, flush=True)
    rng = np.random.default_rng(sum(sizes))
    ps = _he_params(sizes, 5)
    net = dg.Network(sizes, rows)
    net.set_params(dg.Network.flatten(ps))
    Xd, Xv = _x_tensor(rng.standard_normal((rows, sizes[0])), net.ld)
    y_fused = net.forward(Xd).cpu().numpy().astype(np.float64)
    net.set_fused(False)
    y_layer = net.forward(Xd).cpu().numpy().astype(np.float64)
    y_ref, _ = mlp.forward(_round_weights(ps), Xv)
    assert _rel_l2(y_fused, y_layer) <= 5e-3 and _cos(y_fused, y_layer) >= 0.99999
    for y in (y_fused, y_layer):
        assert _rel_l2(y, y_ref) < 2e-2 and _cos(y, y_ref) > 0.999
    net.close()


def test_fused_form_rejected_for_wide_layers():
    """A layer wider than 128 has no fused form: asking for it returns
    DG_ERR_UNSUPPORTED and inference keeps the per-layer GEMMs (still against
    the oracle)."""
    rows, sizes = 300, [40, 200, 16]
    rng = np.random.default_rng(4)
    ps = _he_params(sizes, 6)
    net = dg.Network(sizes, rows)
    net.set_params(dg.Network.flatten(ps))
    with pytest.raises(dg.DGError) as ex:
        net.set_fused(True)
    assert ex.value.status == dg.DG_ERR_UNSUPPORTED
    Xd, Xv = _x_tensor(rng.standard_normal((rows, sizes[0])), net.ld)
    y = net.forward(Xd).cpu().numpy().astype(np.float64)
    y_ref, _ = mlp.forward(_round_weights(ps), Xv)
    assert _rel_l2(y, y_ref) < 2e-2
    net.close()


def test_fused_forward_follows_parameter_updates():
    """The transposed weights of the fused kernel are refreshed after
    set_params and after AdamW steps: the fused and per-layer forms agree
    again after each update."""
    rows = 500
    sizes = [40, 32, 16]
    rng = np.random.default_rng(9)
    net = dg.Network(sizes, rows)
    net.set_params(dg.Network.flatten(_he_params(sizes, 1)))
    Xd, _ = _x_tensor(rng.standard_normal((rows, sizes[0])), net.ld)
    Td = torch.from_numpy(rng.standard_normal((rows, sizes[-1])).astype(np.float32)).cuda()

    def both():
        net.set_fused(True)
        a = net.forward(Xd).cpu().numpy().astype(np.float64)
        net.set_fused(False)
        b = net.forward(Xd).cpu().numpy().astype(np.float64)
        net.set_fused(True)
        return a, b

    a0, b0 = both()
    assert _rel_l2(a0, b0) <= 5e-3
    net.set_params(dg.Network.flatten(_he_params(sizes, 2)))
    a1, b1 = both()
    assert _rel_l2(a1, b1) <= 5e-3 and _rel_l2(a1, a0) > 0.1
    for _ in range(3):
        net.loss_grad(Xd, Td, want_loss=False, want_grads=True)
        net.adamw(1e-2, 0.0)
    a2, b2 = both()
    assert _rel_l2(a2, b2) <= 5e-3 and _rel_l2(a2, a1) > 1e-3
    net.close()


def test_forward_and_gradients_match_oracle():
    rows = 4133
    print("forward/grad", SIZES, rows, flush=True)
    rng = np.random.default_rng(7)
    ps = _he_params(SIZES, 11)
    net = dg.Network(SIZES, rows)
    net.set_params(dg.Network.flatten(ps))
    Xd, Xv = _x_tensor(rng.standard_normal((rows, SIZES[0])), net.ld)
    T = (rng.standard_normal((rows, SIZES[-1])) * 0.5).astype(np.float32)
    Td = torch.from_numpy(T).cuda()
    pr = _round_weights(ps)
    y_ref, cache = mlp.forward(pr, Xv)
    y = net.forward(Xd).cpu().numpy().astype(np.float64)
    assert _rel_l2(y, y_ref) < 2e-2
    assert _cos(y, y_ref) > 0.999
    loss, g = net.loss_grad(Xd, Td, want_loss=True, want_grads=True)
    loss_ref = mlp.mse(y_ref, T.astype(np.float64))
    assert abs(loss - loss_ref) < 2e-2 * loss_ref
    g_ref, _ = mlp.backward(pr, cache, y_ref, T.astype(np.float64))
    for i, (gg, gr) in enumerate(zip(net.unflatten(g), g_ref)):
        assert _rel_l2(gg, gr) < 2e-2, (i, _rel_l2(gg, gr))
        assert _cos(gg, gr) > 0.999, (i, _cos(gg, gr))
    net.close()


def test_adamw_matches_oracle_step():
    rows = 300
    sizes = [40, 32, 16]
    rng = np.random.default_rng(3)
    ps = _he_params(sizes, 5)
    net = dg.Network(sizes, rows)
    flat = dg.Network.flatten(ps)
    net.set_params(flat)
    Xd, _ = _x_tensor(rng.standard_normal((rows, sizes[0])), net.ld)
    Td = torch.from_numpy(rng.standard_normal((rows, sizes[-1])).astype(np.float32)).cuda()
    params = [p.astype(np.float64) for p in net.unflatten(flat.astype(np.float64))]
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    for t in (1, 2):
        _, g = net.loss_grad(Xd, Td, want_loss=False, want_grads=True)
        net.adamw(1e-3, 0.01)
        params = mlp.adamw_step(params, [x.astype(np.float64) for x in net.unflatten(g)], m, v, t,
                                lr=1e-3, wd=0.01)
        got = net.unflatten(net.get_params())
        for a, b in zip(got, params):
            assert np.max(np.abs(a - b)) < 1e-6
        # continue from the device parameters so that both sides use the same gradients
        params = [x.astype(np.float64) for x in got]
    net.close()


def test_training_reduces_loss_on_a_teacher_network():
    rows = 2048
    sizes = [64, 48, 48, 16]
    rng = np.random.default_rng(21)
    X = rng.standard_normal((rows, sizes[0]))
    teacher = _he_params(sizes, 99)
    T, _ = mlp.forward(teacher, X)
    net = dg.Network(sizes, rows)
    net.set_params(dg.Network.flatten(_he_params(sizes, 1)))
    Xd, _ = _x_tensor(X, net.ld)
    Td = torch.from_numpy(T.astype(np.float32)).cuda()
    l0, _ = net.loss_grad(Xd, Td)
    for _ in range(150):
        net.loss_grad(Xd, Td, want_loss=False)
        net.adamw(3e-3)
    l1, _ = net.loss_grad(Xd, Td)
    assert l1 < 0.2 * l0, (l0, l1)
    net.close()


PROJ_CASES = [
    # nv, (n_f, n_c), fine nelem, coarse nelem
    (2, (8, 4), [4, 4, 4], [2, 2, 2]),
    (2, (5, 3), [6, 4, 6], [3, 2, 2]),
    (1, (6, 4), [8, 12], [4, 4]),
    (2, (4, 4), [2, 3, 2], [2, 3, 1]),
    (2, (4, 4), [3, 4, 8], [3, 2, 2]),
    (1, (5, 5), [4, 6], [4, 6]),
]


@pytest.mark.parametrize("case", PROJ_CASES, ids=lambda c: "nv%d_%d_%d_%s" % (c[0], c[1][0], c[1][1], "x".join(map(str, c[2]))))
def test_projection_matches_oracle(case):
    nv, (nf, nc), nef, nec = case
    print("projection", case, flush=True)
    lo = [0.0, -5.0, -4.0][: 1 + nv]
    hi = [3.0, 5.0, 4.0][: 1 + nv]
    sf = dg.Solver(nv, nf, nef, lo, hi, 1.0 if nv == 2 else 0.0)
    sc = dg.Solver(nv, nc, nec, lo, hi, 1.0 if nv == 2 else 0.0)
    f = inputs.random_nodal(sf.shape, 5 + nf)
    fd = torch.from_numpy(f).float().cuda()
    out = torch.empty(sc.shape, dtype=torch.float32, device="cuda")
    dg.dg_project(sf.ctx, sc.ctx, fd, out)
    fh = fd.cpu().numpy().astype(np.float64)
    ref = fh
    naxes = 1 + nv
    # the oracle's projection assumes one refinement ratio; apply axis by axis
    for a in range(naxes):
        r = nef[a] // nec[a]
        P = projection.projection_matrix(nc, nf, r)
        shp = list(ref.shape)
        x = ref.reshape(shp[:2 * a] + [nec[a], r * nf] + shp[2 * a + 2:])
        ref = np.moveaxis(np.tensordot(x, P, axes=([2 * a + 1], [1])), -1, 2 * a + 1)
    got = out.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - ref)) <= 1e-6 * np.max(np.abs(ref))
    if len(set(nef[a] // nec[a] for a in range(naxes))) == 1:
        ref2 = projection.project(fh, nv, nc, nf, nef[0] // nec[0])
        assert np.max(np.abs(got - ref2)) <= 1e-6 * np.max(np.abs(ref2))


@pytest.mark.parametrize("fine_st,coarse_st", [("f64", "f64"), ("f64", "f32"), ("f32", "f64")])
def test_projection_precisions(fine_st, coarse_st):
    """FP64 states in and out: the projection is FP64 arithmetic throughout."""
    lo, hi = [0.0, -5.0, -4.0], [3.0, 5.0, 4.0]
    sf = dg.Solver(2, 8, [4, 4, 6], lo, hi, 1.0, storage=fine_st)
    sc = dg.Solver(2, 4, [2, 2, 3], lo, hi, 1.0, storage=coarse_st)
    f = inputs.random_nodal(sf.shape, 9)
    fd = torch.from_numpy(f).to(device="cuda", dtype=sf.dtype)
    out = torch.empty(sc.shape, dtype=sc.dtype, device="cuda")
    dg.dg_project(sf.ctx, sc.ctx, fd, out)
    ref = projection.project(fd.cpu().numpy().astype(np.float64), 2, 4, 8, 2)
    tol = 1e-13 if coarse_st == "f64" else 1e-6
    assert np.max(np.abs(out.cpu().numpy().astype(np.float64) - ref)) <= tol * np.max(np.abs(ref))
    # FP64 targets: element-major FP32 copy of (x - sub) minus its x average
    if coarse_st == "f64":
        x2 = torch.from_numpy(inputs.random_nodal(sc.shape, 10)).cuda()
        el = torch.empty((2 * 2 * 3, 64), dtype=torch.float32, device="cuda")
        dg.dg_nn_to_elements(sc.ctx, out, x2, 3.0, el, True)
        d = out.cpu().numpy() - x2.cpu().numpy()
        d = 3.0 * (d - _xmean_np(d, 4))
        want = d.transpose(0, 2, 4, 1, 3, 5).reshape(12, 64)
        assert np.max(np.abs(el.cpu().numpy() - want)) <= 1e-6 * np.max(np.abs(want))


def test_projection_full_size_learned_grids_sampled():
    """Fine 32^3 n=8 -> coarse 16^3 n=4 (the training grids), checked on 64
    sampled coarse elements computed one by one from the fine values."""
    lo, hi = [0.0, -8.0, -8.0], [4 * math.pi, 8.0, 8.0]
    sf = dg.Solver(2, 8, [32, 32, 32], lo, hi, 1.0)
    sc = dg.Solver(2, 4, [16, 16, 16], lo, hi, 1.0)
    g = torch.Generator(device="cuda").manual_seed(4)
    fd = torch.rand(sf.shape, generator=g, device="cuda", dtype=torch.float32)
    out = torch.empty(sc.shape, dtype=torch.float32, device="cuda")
    dg.dg_project(sf.ctx, sc.ctx, fd, out)
    P = projection.projection_matrix(4, 8, 2)
    fh = fd.cpu().numpy().astype(np.float64)
    got = out.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(0)
    for _ in range(64):
        ix, iu, iv = rng.integers(0, 16, size=3)
        blk = fh[2 * ix:2 * ix + 2, :, 2 * iu:2 * iu + 2, :, 2 * iv:2 * iv + 2, :].reshape(16, 16, 16)
        ref = np.einsum("ia,jb,kc,abc->ijk", P, P, P, blk)
        assert np.max(np.abs(got[ix, :, iu, :, iv, :] - ref)) <= 1e-6 * np.max(np.abs(ref))


def _xmean_np(f, n):
    """LGL-weighted average over x (all x elements and nodes) per (u, v) node."""
    w = lgl.lgl_nodes_weights(n)[1]
    Nx = f.shape[0]
    wx = np.tile(w, Nx).reshape(Nx, n, 1, 1, 1, 1)
    return (f * wx).sum(axis=(0, 1), keepdims=True) / wx.sum()


def _features_np(f, E, n, fluct=False):
    """Feature rows by definition: own block, x-1, x+1, u-1, u+1, v-1, v+1
    neighbour blocks (periodic), then E at the element's x nodes; the
    fluctuation form uses f minus its x average in the blocks and appends the
    own block of the x average."""
    Nx, Nu, Nv = f.shape[0], f.shape[2], f.shape[4]
    m = _xmean_np(f, n) if fluct else None
    g = f - m if fluct else f
    B = g.transpose(0, 2, 4, 1, 3, 5).reshape(Nx, Nu, Nv, n ** 3)
    parts = [B, np.roll(B, 1, 0), np.roll(B, -1, 0), np.roll(B, 1, 1), np.roll(B, -1, 1),
             np.roll(B, 1, 2), np.roll(B, -1, 2),
             np.broadcast_to(E.reshape(Nx, 1, 1, n), (Nx, Nu, Nv, n))]
    if fluct:
        M = np.broadcast_to(m, f.shape).transpose(0, 2, 4, 1, 3, 5).reshape(Nx, Nu, Nv, n ** 3)
        parts.append(M)
    return np.concatenate(parts, axis=3).reshape(Nx * Nu * Nv, -1)


def test_features_raw_normalised_and_elements_exact():
    n, nelem = 4, [5, 3, 4]
    s = dg.Solver(2, n, nelem, [0.0, -6.0, -6.0], [6.0, 6.0, 6.0], 1.0)
    ne = 5 * 3 * 4
    nfeat = 7 * n ** 3 + n
    net = dg.Network([nfeat, 16, n ** 3], ne)
    fd = torch.from_numpy(inputs.random_nodal(s.shape, 3)).float().cuda()
    Ed = torch.from_numpy(inputs.random_field(nelem[0] * n, 3)).cuda()
    raw = torch.empty((ne, nfeat), dtype=torch.float32, device="cuda")
    dg.dg_nn_features_raw(s.ctx, fd, Ed, raw, False)
    ref = _features_np(fd.cpu().numpy(), Ed.cpu().numpy().astype(np.float32), n)
    assert np.array_equal(raw.cpu().numpy(), ref)
    rng = np.random.default_rng(1)
    mean = rng.standard_normal(nfeat).astype(np.float32)
    inv = rng.uniform(0.5, 2.0, nfeat).astype(np.float32)
    X = torch.empty((ne, net.ld), dtype=torch.int16, device="cuda")
    dg.dg_nn_features(s.ctx, net.nn, fd, Ed, torch.from_numpy(mean).cuda(), torch.from_numpy(inv).cuda(), X)
    z = (ref - mean) * inv                    # FP32 arithmetic, as on the device
    want = np.zeros((ne, net.ld), dtype=np.uint16)
    want[:, :nfeat] = bf16_bits(z)
    assert np.array_equal(X.cpu().numpy().view(np.uint16), want)
    # element-major reordering and target difference
    f2 = torch.from_numpy(inputs.random_nodal(s.shape, 4)).float().cuda()
    el = torch.empty((ne, n ** 3), dtype=torch.float32, device="cuda")
    dg.dg_nn_to_elements(s.ctx, fd, f2, 1.0, el, False)
    d = (fd - f2).cpu().numpy()
    assert np.array_equal(el.cpu().numpy(), d.transpose(0, 2, 4, 1, 3, 5).reshape(ne, n ** 3))
    # column statistics (FP64 sums)
    su, sq = net.column_stats(raw)
    r64 = ref.astype(np.float64)
    assert np.allclose(su, r64.sum(0), rtol=1e-12, atol=1e-9)
    assert np.allclose(sq, (r64 * r64).sum(0), rtol=1e-12, atol=1e-9)
    net.close()


def test_fluctuation_features_and_targets_match_definition():
    n, nelem = 4, [5, 3, 4]
    s = dg.Solver(2, n, nelem, [0.0, -6.0, -6.0], [6.0, 6.0, 6.0], 1.0)
    ne = 5 * 3 * 4
    nfeat = 8 * n ** 3 + n
    fd = torch.from_numpy(inputs.random_nodal(s.shape, 5)).float().cuda()
    Ed = torch.from_numpy(inputs.random_field(nelem[0] * n, 5)).cuda()
    raw = torch.empty((ne, nfeat), dtype=torch.float32, device="cuda")
    dg.dg_nn_features_raw(s.ctx, fd, Ed, raw, True)
    fh = fd.cpu().numpy().astype(np.float64)
    ref = _features_np(fh, Ed.cpu().numpy(), n, fluct=True)
    got = raw.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - ref)) <= 1e-6 * np.max(np.abs(ref))
    f2 = torch.from_numpy(inputs.random_nodal(s.shape, 6)).float().cuda()
    el = torch.empty((ne, n ** 3), dtype=torch.float32, device="cuda")
    dg.dg_nn_to_elements(s.ctx, fd, f2, 2.0, el, True)
    d = fh - f2.cpu().numpy().astype(np.float64)
    d = 2.0 * (d - _xmean_np(d, n))
    want = d.transpose(0, 2, 4, 1, 3, 5).reshape(ne, n ** 3)
    assert np.max(np.abs(el.cpu().numpy() - want)) <= 1e-6 * np.max(np.abs(want))
    # the targets have zero x average
    back = el.cpu().numpy().astype(np.float64).reshape(5, 3, 4, n, n, n).transpose(0, 3, 1, 4, 2, 5)
    assert np.max(np.abs(_xmean_np(back, n))) <= 1e-6 * np.max(np.abs(want))


def _oracle_corrected_rhs(g, ops, u, params, mean, inv, scale, n, fluct=False):
    E = rk.field(g, u)
    Lu = rhs.rhs(g, ops, u, E)
    Xf = (_features_np(u, E, n, fluct) - mean) * inv
    y, _ = mlp.forward(params, Xf)
    Nx, Nu, Nv = u.shape[0], u.shape[2], u.shape[4]
    if not fluct:   # mass-neutral per element
        w = lgl.lgl_nodes_weights(n)[1]
        W = (w[:, None, None] * w[None, :, None] * w[None, None, :]).ravel()
        y = y - (y @ W / W.sum())[:, None]
    corr = y.reshape(Nx, Nu, Nv, n, n, n).transpose(0, 3, 1, 4, 2, 5)
    if fluct:       # x average removed
        corr = corr - _xmean_np(corr, n)
    return Lu + scale * corr


@pytest.mark.parametrize("fluct", [False, True])
@pytest.mark.parametrize("scale", [0.0, 1.0])
def test_corrected_step_matches_oracle(scale, fluct):
    n, nelem = 4, [4, 3, 5]
    lo, hi = [0.0, -6.0, -6.0], [4 * math.pi, 6.0, 6.0]
    print("corrected step", scale, fluct, flush=True)
    s = dg.Solver(2, n, nelem, lo, hi, 1.0)
    g = grid.PhaseGrid(2, n, nelem, lo, hi, 1.0)
    ops = lgl.operators(n)
    c = g.coords()
    f0 = inputs.mixture(c[0], c[1], c[2], 0.5, 1.0, 0.5, 0.05, 3.0)
    fd = torch.from_numpy(f0).float().cuda()
    fh = fd.cpu().numpy().astype(np.float64)
    ne = 4 * 3 * 5
    nfeat = (8 if fluct else 7) * n ** 3 + n
    sizes = [nfeat, 32, 32, n ** 3]
    net = dg.Network(sizes, ne)
    ps = _he_params(sizes, 8)
    # scale the last layer so that the correction is comparable to L(f)
    ps[-2] = ps[-2] * 0.01
    ps[-1] = ps[-1] * 0.01
    net.set_params(dg.Network.flatten(ps))
    Eh = rk.field(g, fh)
    feats = _features_np(fh, Eh, n, fluct)
    mean = feats.mean(0).astype(np.float32)
    inv = (1.0 / (feats.std(0) + 1e-3)).astype(np.float32)
    E0 = s.poisson(fd)
    dt = 0.5 * s.dt_max(float(E0.abs().max()))
    dg.dg_nn_rk_step(s.ctx, net.nn, torch.from_numpy(mean).cuda(), torch.from_numpy(inv).cuda(), scale, fd, dt, 1)
    pr = _round_weights(ps)

    def Lc(u):
        return _oracle_corrected_rhs(g, ops, u, pr, mean.astype(np.float64), inv.astype(np.float64), scale, n, fluct)

    u1 = fh + dt * Lc(fh)
    u2 = 0.75 * fh + 0.25 * (u1 + dt * Lc(u1))
    ref = fh / 3.0 + 2.0 / 3.0 * (u2 + dt * Lc(u2))
    got = fd.cpu().numpy().astype(np.float64)
    if scale == 0.0:
        assert _rel_l2(got, ref) < 1e-5
    else:
        inc, inc_ref = got - fh, ref - fh
        # the correction is a sizeable part of the increment
        plain = rk.ssprk3_step(g, ops, fh, dt)
        assert np.linalg.norm(ref - plain) > 0.1 * np.linalg.norm(inc_ref)
        assert _rel_l2(inc, inc_ref) < 2e-2
        # mass neutrality of the correction: total mass unchanged to FP32 level
        wts = g.weights()
        assert abs(np.sum(wts * got) - np.sum(wts * fh)) < 1e-5 * np.sum(wts * fh)
    net.close()


@pytest.mark.parametrize("fluct", [False, True])
def test_corrected_step_fused_equals_layerwise(fluct):
    """One corrected step with the fused network against one GEMM launch per
    layer: the same features, the network summed in another order (BF16
    activations can flip), so the two increments agree to relative L2 5e-3."""
    n, nelem = 4, [5, 4, 6]
    lo, hi = [0.0, -6.0, -6.0], [4 * math.pi, 6.0, 6.0]
    s = dg.Solver(2, n, nelem, lo, hi, 1.0)
    g = grid.PhaseGrid(2, n, nelem, lo, hi, 1.0)
    c = g.coords()
    f0 = torch.from_numpy(inputs.mixture(c[0], c[1], c[2], 0.5, 1.0, 0.5, 0.05, 3.0)).float().cuda()
    nfeat = (8 if fluct else 7) * n ** 3 + n
    sizes = [nfeat, 128, 128, 128, n ** 3]
    net = dg.Network(sizes, 5 * 4 * 6)
    ps = _he_params(sizes, 12)
    ps[-2] = ps[-2] * 0.01
    ps[-1] = ps[-1] * 0.01
    net.set_params(dg.Network.flatten(ps))
    mean = torch.zeros(nfeat, device="cuda")
    inv = torch.full((nfeat,), 3.0, device="cuda")
    dt = 0.5 * s.dt_max(float(s.poisson(f0).abs().max()))
    out = {}
    for fused in (True, False):
        net.set_fused(fused)
        f = f0.clone()
        dg.dg_nn_rk_step(s.ctx, net.nn, mean, inv, 1.0, f, dt, 1)
        out[fused] = (f - f0).cpu().numpy().astype(np.float64)
    assert _rel_l2(out[True], out[False]) < 5e-3
    net.close()


def test_corrected_step_graph_replays_match_separate_calls():
    """The corrected step is replayed from a captured graph: three replays in
    one call must equal three one-step calls (each with its own eager field
    solve in between) bit for bit."""
    n, nelem = 4, [4, 3, 5]
    lo, hi = [0.0, -6.0, -6.0], [4 * math.pi, 6.0, 6.0]
    s = dg.Solver(2, n, nelem, lo, hi, 1.0)
    g = grid.PhaseGrid(2, n, nelem, lo, hi, 1.0)
    c = g.coords()
    f0 = torch.from_numpy(inputs.mixture(c[0], c[1], c[2], 0.5, 1.0, 0.5, 0.05, 3.0)).float().cuda()
    ne, nfeat = 60, 7 * n ** 3 + n
    sizes = [nfeat, 32, 32, n ** 3]
    net = dg.Network(sizes, ne)
    ps = _he_params(sizes, 4)
    ps[-2] = ps[-2] * 0.01
    net.set_params(dg.Network.flatten(ps))
    mean = torch.zeros(nfeat, device="cuda")
    inv = torch.full((nfeat,), 2.0, device="cuda")
    dt = 0.5 * s.dt_max(float(s.poisson(f0).abs().max()))
    a, b = f0.clone(), f0.clone()
    recs = dg.dg_nn_rk_step(s.ctx, net.nn, mean, inv, 0.5, a, dt, 3, diag=True)
    for _ in range(3):
        dg.dg_nn_rk_step(s.ctx, net.nn, mean, inv, 0.5, b, dt, 1)
        torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert len(recs) == 3 and all(r["finite"] for r in recs)
    net.close()
