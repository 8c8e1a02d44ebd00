"""The paper's two cyclotron-harmonic instability runs (Sec. 6.1) on one GPU.

Sec. 4 poses the problem, Sec. 6 the runs:
  * equilibrium: the loss-cone ring of eq. loss_cone, j = 6, alpha = 1;
  * perturbation: the eigenmode of eq. ic (20-term partial sum) for the
    printed roots of the Harris dispersion relation (eq. disp),
      A: (k, omega) = (0.886, 0.349i)          (fastest purely growing mode)
      B: (k, omega) = (1.4, 1.182 + 0.131i),
    k in inverse Larmor radii, omega in cyclotron frequencies;
  * B_ext = omega_c / omega_p = 0.1, domain L = 2 pi / k in Debye lengths
    (k / r_L with r_L = 1 / B_ext), velocity box +-8.5;
  * the perturbation scaled so the density perturbation has amplitude 0.002;
  * (Nx, Nu, Nv) = (25, 50, 50) elements, n = 8 (32 M DOF), SSP-RK3 with the
    spectral Poisson solve at every stage.
In the library's units (time in 1/omega_p) the field energy of the linear
phase grows as exp(2 Im(omega) B_ext t): 0.0698 (A) and 0.0262 (B).  The
paper reports saturation near 6 % (A) and 2.5 % (B) of the thermal energy
(0.25 per unit length, App. B), A saturating around t = 100 and run to 175,
B around t = 175 and run to 200.

The initial state is assembled on the device from two velocity-plane arrays
computed on the host (f0 and the complex mode), so no 32 M-point host array is
needed.  ``python -m paper_2202_13532_amd.case_study --which A`` prints one
JSON line with the field-energy history summary.
"""
import argparse
import json
import math
import sys
import time

import numpy as np

CASES = {
    "A": {"k": 0.886, "omega": 0.349j, "t_end": 175.0},
    "B": {"k": 1.4, "omega": 1.182 + 0.131j, "t_end": 200.0},
}
JRING = 6
B_EXT = 0.1
VMAX = 8.5
NELEM = [25, 50, 50]
N = 8
DENSITY_AMPLITUDE = 0.002


def geometry(which):
    k0 = CASES[which]["k"]
    kx = k0 * B_EXT
    return kx, k0, [0.0, -VMAX, -VMAX], [2.0 * math.pi / kx, VMAX, VMAX]


def mode_density(k0, omega, j=JRING, nmax=20):
    """Zeroth moment of the complex mode of eq. ic at x = 0.

    By the Jacobi-Anger identity the angle integral of e^{i k0 v sin phi}
    e^{-i m phi} is 2 pi J_m(k0 v), so
      int psi (f0'/v) dv = 2 pi sum_{0<|m|<=nmax} m/(m - omega)
                           int_0^inf (f0'(v)/v) J_m(k0 v)^2 v dv,
    with f0'(v)/v = (j - v^2/2) f0 / v^2 for eq. loss_cone (alpha = 1).
    """
    from scipy import integrate, special

    def f0(v):
        s = 0.5 * v * v
        return s ** j * math.exp(-s) / (2.0 * math.pi * math.factorial(j))

    total = 0.0 + 0.0j
    for m in range(-nmax, nmax + 1):
        if m == 0:
            continue
        val, _ = integrate.quad(lambda v: (j - 0.5 * v * v) * f0(v) / v * special.jv(m, k0 * v) ** 2,
                                0.0, 40.0, limit=400, epsabs=1e-15, epsrel=1e-12)
        total += 2.0 * math.pi * m / (m - omega) * val
    return total


def initial_state(solver, which, torch):
    """f0 + eps Re(e^{i kx x} psi(u, v)) on the solver's nodes (dense layout),
    eps such that the density perturbation has amplitude 0.002."""
    from . import inputs
    kx, k0, _, _ = geometry(which)
    omega = CASES[which]["omega"]
    x = solver.nodes(0)
    u = solver.nodes(1).reshape(-1)[:, None]
    v = solver.nodes(2).reshape(-1)[None, :]
    f0 = inputs.loss_cone(u, v, JRING)
    psi = inputs.cyclotron_mode(0.0, u, v, kx, k0, omega, JRING, complex_out=True)
    eps = DENSITY_AMPLITUDE / abs(mode_density(k0, omega))
    dev = solver.device
    shape2 = (1, 1, NELEM[1], N, NELEM[2], N)
    F0 = torch.from_numpy(np.ascontiguousarray(f0)).to(dev).reshape(shape2)
    PR = torch.from_numpy(np.ascontiguousarray(eps * psi.real)).to(dev).reshape(shape2)
    PI = torch.from_numpy(np.ascontiguousarray(eps * psi.imag)).to(dev).reshape(shape2)
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(dev).reshape(NELEM[0], N, 1, 1, 1, 1)
    f = F0 + torch.cos(kx * xt) * PR - torch.sin(kx * xt) * PI
    return f.to(solver.dtype).contiguous(), eps


def thermal_energy(which, j=JRING):
    """Domain-integrated thermal energy of the ring, 1/2 <(v - <v>)^2> L
    (App. B: alpha^2 (j + 1 - (Gamma(j + 3/2) / Gamma(j + 1))^2) per unit length)."""
    per_length = (j + 1) - math.exp(2.0 * (math.lgamma(j + 1.5) - math.lgamma(j + 1.0)))
    return per_length * geometry(which)[3][0]


def growth_rate(t, W, t0, t1):
    """Least-squares slope of log W over t in [t0, t1]."""
    t = np.asarray(t)
    W = np.asarray(W)
    m = (t >= t0) & (t <= t1)
    A = np.stack([t[m], np.ones(int(m.sum()))], axis=1)
    coef, *_ = np.linalg.lstsq(A, np.log(W[m]), rcond=None)
    resid = np.log(W[m]) - A @ coef
    return float(coef[0]), float(np.sqrt(np.mean(resid ** 2)))


def run(which="A", t_end=None, storage="f32", layout="vpad", cfl_fraction=0.9, record_every=10, device="cuda"):
    """Step the case study to t_end; returns a dict with the field-energy history."""
    import torch
    from . import dg
    kx, k0, lo, hi = geometry(which)
    t_end = CASES[which]["t_end"] if t_end is None else t_end
    s = dg.Solver(2, N, NELEM, lo, hi, B_EXT, 0, storage, device=device, layout=layout)
    dense, eps = initial_state(s, which, torch)
    f = s.pack(dense)
    del dense
    d0 = s.diagnostics(f)
    E0 = s.poisson(f)
    # bound |E| generously: the field grows by about a factor 10 before saturation
    dt = cfl_fraction * s.dt_max(max(10.0 * float(E0.abs().max()), 0.5))
    nsteps = int(math.ceil(t_end / dt))
    times, W, mass = [0.0], [d0["field_energy"]], [d0["mass"]]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    done = 0
    while done < nsteps:
        k = min(record_every, nsteps - done)
        recs = s.step(f, dt, k, diag=True)
        done += k
        times.append(done * dt)
        W.append(recs[-1]["field_energy"])
        mass.append(recs[-1]["mass"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    s.close()
    return {"which": which, "dt": dt, "steps": nsteps, "t": times, "field_energy": W, "mass": mass,
            "eps": eps, "wall_s": wall, "dof": (NELEM[0] * N) * (NELEM[1] * N) * (NELEM[2] * N),
            "storage": storage, "layout": layout}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--which", default="A", choices=["A", "B"])
    ap.add_argument("--t-end", type=float, default=None)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--fit", type=float, nargs=2, default=None, help="time window of the growth-rate fit")
    args = ap.parse_args()
    r = run(args.which, args.t_end, args.storage)
    fit = args.fit or ((10.0, 50.0) if args.which == "A" else (20.0, 120.0))
    rate, resid = growth_rate(r["t"], r["field_energy"], *fit)
    expected = 2.0 * CASES[args.which]["omega"].imag * B_EXT
    Wmax = max(r["field_energy"])
    out = {"which": args.which, "storage": r["storage"], "dof": r["dof"], "dt": r["dt"], "steps": r["steps"],
           "t_end": r["t"][-1], "wall_s": r["wall_s"],
           "dof_stage_updates_per_s": r["dof"] * 3 * r["steps"] / r["wall_s"],
           "growth_rate_fit": rate, "fit_window": fit, "fit_rms_log_residual": resid,
           "growth_rate_linear_theory": expected, "rate_ratio": rate / expected,
           "field_energy_max": Wmax, "t_of_max": r["t"][int(np.argmax(r["field_energy"]))],
           "thermal_energy": thermal_energy(args.which),
           "saturation_fraction": Wmax / thermal_energy(args.which),
           "mass_drift": abs(r["mass"][-1] - r["mass"][0]) / abs(r["mass"][0]),
           "history_every_10_steps": {"t": r["t"][::20], "field_energy": r["field_energy"][::20]}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    sys.exit(main())
