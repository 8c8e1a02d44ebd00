"""The allocation-free entry point dg_rhs_static against dg_rhs (C ABI).

Two calls in a row on one GPU, the second with a smaller configuration, each
compared with dg_rhs through a context on the same input: with the field
given (the same kernels and node tables from the same formulas) and with the
field solved from f (the connection tensor built on the device instead of the
host).  Bars: FP64 storage element-wise 1e-12 of the largest magnitude, FP32
storage relative L2 1e-5 (the stated FP32 bound).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2202_13532_amd import dg, inputs  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [
    # nv, n, nelem, lo, hi, wc, storage, layout
    (2, 9, [6, 5, 11], [0.0, -8.0, -7.0], [20.0, 8.0, 7.0], 1.0, "f64", "dense"),
    (1, 4, [5, 37], [0.0, -6.0], [4 * math.pi, 6.0], 0.0, "f64", "dense"),
    (2, 8, [4, 3, 9], [0.0, -8.0, -8.0], [2 * math.pi, 8.0, 8.0], 1.0, "f32", "vpad"),
    (2, 5, [3, 2, 13], [0.0, -3.0, -3.0], [1.0, 3.0, 3.0], -0.7, "f32", "dense"),
]


def _compare(a, b, storage):
    a = a.double().cpu().numpy()
    b = b.double().cpu().numpy()
    if storage == "f64":
        err = np.max(np.abs(a - b)) / np.max(np.abs(b))
        assert err <= 1e-12, err
    else:
        err = np.linalg.norm(a - b) / np.linalg.norm(b)
        assert err <= 1e-5, err


@pytest.mark.parametrize("pair", [(0, 1), (2, 3)])
def test_rhs_static_matches_rhs_twice_in_a_row(pair):
    for k, case in enumerate(pair):
        nv, n, nelem, lo, hi, wc, storage, layout = CASES[case]
        print("case", case, "call", k, flush=True)
        s = dg.Solver(nv, n, nelem, lo, hi, wc, 0, storage, layout=layout)
        dense = torch.from_numpy(inputs.random_nodal(s.dense_shape, 11 + case)).to("cuda", s.dtype)
        f = s.pack(dense)
        E = torch.from_numpy(inputs.random_field(nelem[0] * n, 5 + case)).cuda()
        stream = torch.cuda.current_stream().cuda_stream
        for Eg in (E, None):
            ref = s.rhs(f, Eg)
            out = torch.full_like(f, float("nan"))
            dg.dg_rhs_static(s.cfg, f, Eg, out, stream)
            torch.cuda.synchronize()
            _compare(out, ref, storage)
        s.close()


def test_rhs_static_rejects_configurations_beyond_its_scratch():
    # 64 x 48 x 48 elements at n = 9 needs more than the 8 MiB of scratch
    cfg = dg.make_config(2, 9, [256, 48, 48], [0.0, -8.0, -8.0], [1.0, 8.0, 8.0], 1.0)
    f = torch.zeros(1, device="cuda")
    with pytest.raises(dg.DGError) as ex:
        dg.dg_rhs_static(cfg, f, None, torch.zeros(1, device="cuda"))
    assert ex.value.status == dg.DG_ERR_OOM
    assert "maximum" in str(ex.value)
