"""Connection-tensor tools on the GPU against the oracle (Sec. 5.3).

* dg_fourier: coefficients of arbitrary nodal data, pmax up to 3 x Nx,
  against the oracle's quadrature tensor (1e-13 of the largest coefficient).
* The errors-figure study (elliptic cosine, 20 elements, n = 2..9) through
  the GPU transform: the same aliasing points as the oracle's, even modes at
  the rounding level.
* dg_filter_x: the global x filter of whole states (1D1V and 1D2V, dense and
  padded rows) against oracle.spectral.filter_x: FP64 1e-12 of the largest
  value, FP32 relative L2 1e-5.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import grid, poisson, spectral  # noqa: E402
from paper_2202_13532_amd import dg, inputs  # noqa: E402
from tests.test_oracle_spectral import N_ELEM, SQRT_M, aliasing_point, cn_study  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,N,L,pmax", [(4, 16, 4 * math.pi, 16), (8, 10, 3.0, 30), (9, 64, 20 * math.pi, 64),
                                        (3, 7, 1.0, 21)])
def test_fourier_matches_oracle(n, N, L, pmax):
    s = dg.Solver(1, n, [N, 3], [0.0, -1.0], [L, 1.0], 0.0, pmax, "f64")
    g = inputs.random_field(N * n, 31 + n, 1.0)
    c = s.fourier(torch.from_numpy(g).cuda())
    co, ps, _ = poisson.fourier_coefficients(grid.Axis(0.0, L, N, n), g, pmax)
    ref = co[pmax + 1:]
    assert np.max(np.abs(c - ref)) <= 1e-13 * np.max(np.abs(ref))
    s.close()


@pytest.mark.parametrize("n", range(2, 10))
def test_errors_figure_study_on_the_gpu(n):
    pmax = 60
    s = dg.Solver(1, n, [N_ELEM, 2], [-0.5, -1.0], [0.5, 1.0], 0.0, pmax, "f64")
    x = s.nodes(0)
    vals = inputs.elliptic_cosine(x, SQRT_M).reshape(-1)
    c = s.fourier(torch.from_numpy(np.ascontiguousarray(vals)).cuda())
    err_o, odd, even_o, cp_o = cn_study(n, pmax)
    assert np.max(np.abs(c - cp_o)) <= 1e-13 * np.max(np.abs(cp_o))
    from tests.test_oracle_spectral import cn_coefficients
    ce = cn_coefficients(pmax)[1:]
    err = np.abs(c[odd - 1] - ce[odd - 1]) / np.abs(ce[odd - 1])
    assert aliasing_point(err, odd) == aliasing_point(err_o, odd)
    assert np.max(np.abs(c[1::2])) < 1e-14 * np.max(np.abs(ce))
    s.close()


CASES = [
    # nv, n, nelem, lo, hi, wc, storage, layout, pmax
    (1, 6, [9, 13], [0.0, -5.0], [4.0, 5.0], 0.0, "f64", "dense", 9),
    (2, 9, [6, 3, 10], [0.0, -6.0, -6.0], [8.0, 6.0, 6.0], 1.0, "f32", "vpad", 12),
    (2, 5, [7, 2, 13], [0.0, -5.0, -5.0], [5.0, 5.0, 5.0], 1.0, "f64", "vpad", 7),
    (2, 8, [4, 3, 9], [0.0, -6.0, -6.0], [6.0, 6.0, 6.0], 0.5, "f32", "dense", 4),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "nv%d_n%d_%s_%s" % (c[0], c[1], c[6], c[7]))
def test_filter_x_matches_oracle(case):
    nv, n, nelem, lo, hi, wc, storage, layout, pmax = case
    s = dg.Solver(nv, n, nelem, lo, hi, wc, pmax, storage, layout=layout)
    dense = inputs.random_nodal(s.dense_shape, 77 + n)
    fd = s.pack(torch.from_numpy(dense).to("cuda", s.dtype))
    fh = s.unpack(fd).double().cpu().numpy()
    sigma = np.exp(-2.0 * (np.arange(1, pmax + 1) / pmax) ** 4)     # exponential filter
    out = s.unpack(s.filter_x(fd, sigma)).double().cpu().numpy()
    ref = spectral.filter_x(grid.Axis(lo[0], hi[0], nelem[0], n), fh, sigma)
    if storage == "f64":
        assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))
    else:
        assert np.linalg.norm(out - ref) <= 1e-5 * np.linalg.norm(ref)
    with pytest.raises(dg.DGError):
        s.filter_x(fd, sigma, out=fd)
    s.close()
