"""Named synthetic workloads (grid sizes, domains, initial-condition recipes).

Pure problem description: no arithmetic of the DG method lives here.  Time
steps are derived from the library's CFL bound by the caller.

  landau_1d1v_n4       1D1V linear Landau damping, x in [0, 4 pi) with 16
                       elements, v in [-8, 8] with 32 elements, n = 4
                       (8192 DOF), FP64 storage, dt = 0.01, 200 steps.
  ring_1d2v_n8         1D2V magnetised ring, x with 32 elements on
                       L = 2 pi / k (k = 0.1 (seed + 1)), vx, vy in [-8, 8]
                       with 32 elements each, n = 8 (16 777 216 DOF),
                       omega_c = 1, FP32 storage, 100 steps at 0.9 dt_max.
  maxwell_1d2v_n9      1D2V Maxwellian with 8 seeded cosine modes, x with 64
                       elements on L = 20 pi (k1 = 0.1), vx, vy with 48
                       elements each, n = 9 (107 495 424 DOF), omega_c = 1,
                       FP32 storage (FP64 for the precision ablation), 50 steps.
  coarse_1d2v_n4 /     learned-correction grids: x, vx, vy with 16 elements
  fine_1d2v_n8         and n = 4 (262 144 DOF) vs 32 elements and n = 8, L = 4 pi.
"""
import math
from dataclasses import dataclass, field
from typing import List, Optional


@dataclass
class Workload:
    name: str
    nv: int
    n: int
    nelem: List[int]
    lo: List[float]
    hi: List[float]
    omega_c: float = 0.0
    storage: str = "f32"
    steps: int = 100
    dt: Optional[float] = None          # fixed dt, else cfl_fraction * dt_max
    cfl_fraction: float = 0.9
    ic: str = "landau"
    ic_args: dict = field(default_factory=dict)

    def dof(self):
        d = 1
        for a in range(1 + self.nv):
            d *= self.nelem[a] * self.n
        return d


def landau_1d1v_n4():
    return Workload("landau_1d1v_n4", 1, 4, [16, 32], [0.0, -8.0], [4 * math.pi, 8.0],
                    0.0, "f64", 200, dt=0.01, ic="landau", ic_args={"k": 0.5, "eps": 0.01})


def ring_1d2v_n8(seed=4):
    k = 0.1 * (seed + 1)
    return Workload("ring_1d2v_n8", 2, 8, [32, 32, 32], [0.0, -8.0, -8.0],
                    [2 * math.pi / k, 8.0, 8.0], 1.0, "f32", 100,
                    ic="ring", ic_args={"k": k, "eps": 1e-3, "r0": 3.0})


def maxwell_1d2v_n9(seed=0, storage="f32"):
    return Workload("maxwell_1d2v_n9", 2, 9, [64, 48, 48], [0.0, -8.0, -8.0],
                    [20 * math.pi, 8.0, 8.0], 1.0, storage, 50,
                    ic="maxwell_multimode", ic_args={"k1": 0.1, "seed": seed, "eps": 1e-3})


def coarse_1d2v_n4(omega_c=1.0):
    return Workload("coarse_1d2v_n4", 2, 4, [16, 16, 16], [0.0, -8.0, -8.0],
                    [4 * math.pi, 8.0, 8.0], omega_c, "f32", 2000, ic="mixture")


def fine_1d2v_n8(omega_c=1.0):
    return Workload("fine_1d2v_n8", 2, 8, [32, 32, 32], [0.0, -8.0, -8.0],
                    [4 * math.pi, 8.0, 8.0], omega_c, "f32", 2000, ic="mixture")


def initial_state(wl, axes_nodes, xp):
    """Evaluate the workload's initial condition on the node arrays (state layout)."""
    from . import inputs
    c = inputs.broadcast_coords(axes_nodes, xp)
    a = wl.ic_args
    if wl.ic == "landau":
        return inputs.landau(c[0], c[1], a.get("k", 0.5), a.get("eps", 0.01), xp)
    if wl.ic == "ring":
        return inputs.ring_perturbed(c[0], c[1], c[2], a["k"], a.get("eps", 1e-3), a.get("r0", 3.0), xp)
    if wl.ic == "maxwell_multimode":
        return inputs.maxwell_multimode(c[0], c[1], c[2], a["k1"], a["seed"], a.get("eps", 1e-3), 8, xp)
    if wl.ic == "maxwell_1v":
        return inputs.maxwellian_1d(c[1], a["vt"], xp) * (1.0 + a["eps"] * xp.cos(a["k"] * c[0]))
    if wl.ic == "maxwell_2v":
        return inputs.maxwellian_2d(c[1], c[2], a["vt"], xp) * (1.0 + a["eps"] * xp.cos(a["k"] * c[0]))
    if wl.ic == "mixture":
        return inputs.mixture(c[0], c[1], c[2], a.get("a", 0.5), a.get("vt", 1.0),
                              a.get("k1", 0.5), a.get("eps", 1e-3), 3.0, xp)
    raise ValueError(wl.ic)


def uneven_sweep(nruns=64, seed0=1000):
    """Batched uneven sweep: half 1D1V, half 1D2V; per run r a generator seeded
    with seed0 + r draws Nx in {8..64}, Nv in {16..64} elements per velocity
    axis, n in {4..9}, k in [0.1, 0.6], thermal speed in [0.5, 1.5] and (1D2V)
    omega_c in {0, 0.5, 1}; L = 2 pi / k, velocity box +-8 vt, FP32."""
    import numpy as np
    out = []
    for r in range(nruns):
        g = np.random.default_rng(seed0 + r)
        nv = 1 if r < nruns // 2 else 2
        Nx = int(g.integers(8, 65))
        Nv = int(g.integers(16, 65))
        n = int(g.integers(4, 10))
        k = float(g.uniform(0.1, 0.6))
        vt = float(g.uniform(0.5, 1.5))
        wc = float(g.choice([0.0, 0.5, 1.0])) if nv == 2 else 0.0
        V = 8.0 * vt
        if nv == 1:
            wl = Workload("sweep_%d" % r, 1, n, [Nx, Nv], [0.0, -V], [2 * math.pi / k, V], 0.0, "f32", 20,
                          ic="maxwell_1v", ic_args={"k": k, "vt": vt, "eps": 0.01})
        else:
            wl = Workload("sweep_%d" % r, 2, n, [Nx, Nv, Nv], [0.0, -V, -V], [2 * math.pi / k, V, V], wc, "f32", 20,
                          ic="maxwell_2v", ic_args={"k": k, "vt": vt, "eps": 0.01})
        out.append(wl)
    return out
