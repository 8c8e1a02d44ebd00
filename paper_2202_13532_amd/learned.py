"""Learned coarse-grid correction: data from fine DG runs, training, corrected runs.

Orchestration only.  Every numerical step runs in libdg through the C ABI:
fine and coarse SSP-RK3 steps, the fine -> coarse L2 projection, both RHS
evaluations, the target difference, the feature gather and normalisation,
the BF16-MFMA network forward / backward, AdamW and the corrected coarse
steps.  Host code draws seeds, orders minibatches and turns the per-column
sums returned by the library into normalisation constants.

Setting (1D2V, x in [0, 2 pi / k1), v in [-8, 8]^2):
  fine    32^3 elements, n = 8 (16 777 216 DOF), FP64 storage (the reference)
  coarse  16^3 elements, n = 4 (262 144 DOF, 4096 elements), FP32 storage
  network 452 -> 128 -> 128 -> 128 -> 64 (exact GELU), 99 264 parameters
          (whole-value form, default); 516 -> ... in the fluctuation form
Per run r (seed s): a ~ U[a_range], v_t ~ U[vt_range] from default_rng(s);
f0 = a ring(r0 = 3) + (1 - a) Maxwellian(v_t), times 1 + eps cos(k1 x).
Default (the learned-correction workload): omega_c = 0.05, k1 = 0.5,
eps = 0.4, a in [0, 0.3], v_t in [0.9, 1.1]: strong, nonlinear Landau
damping in a weak field, where the coarse velocity grid cannot follow the
filamentation after the initial damping (weakly perturbed, strongly
magnetised settings are resolved by the coarse grid to < 0.1 %, so a
correction has nothing to recover there).
A training snapshot of fine state f gives the coarse input P f and the target
P RHS_fine(f) - RHS_coarse(P f) (per coarse element, n^3 values).

Fluctuation form (Config.fluct): the closure of the x-averaged distribution
can be far larger than that of the perturbation; in this form the inputs are
the blocks of f minus its x average (plus the own block of that average), the
target is the closure minus its x average, and the correction's x average is
removed when it is applied.
"""
import math
import time
from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import dg, inputs

LO = [0.0, -8.0, -8.0]
HI = [4.0 * math.pi, 8.0, 8.0]
OMEGA_C = 0.05


@dataclass
class Config:
    n_fine: int = 8
    nelem_fine: int = 32
    n_coarse: int = 4
    nelem_coarse: int = 16
    hidden: List[int] = field(default_factory=lambda: [128, 128, 128])
    train_seeds: List[int] = field(default_factory=lambda: list(range(32)))
    snapshots_per_run: int = 64
    snapshot_stride: int = 220         # fine steps between snapshots (64 x 220 spans t = 0..9)
    spinup_steps: int = 0              # fine steps before the first snapshot
    epochs: int = 5
    snapshots_per_step: int = 1        # minibatch = this many whole snapshots (ne rows each)
    lr: float = 1e-3
    weight_decay: float = 1e-4
    init_seed: int = 12345
    cfl_fraction: float = 0.9
    fluct: bool = False                # learn the closure of the fluctuation about the x average
    fp64_data: bool = True             # fine runs, projections and both RHS in FP64 (targets then FP32)
    perturbation: float = 0.4          # density perturbation amplitude of the initial states
    omega_c: float = OMEGA_C           # B = omega_c / omega_p
    k1: float = 0.5                    # wavenumber of the perturbation; x period L = 2 pi / k1
    a_range: tuple = (0.0, 0.3)        # ring fraction of the mixture, drawn uniformly per run
    vt_range: tuple = (0.9, 1.1)       # Maxwellian thermal speed, drawn uniformly per run
    late_window: float = 0.5           # evaluation also reports the history error over the last
                                       # fraction of the run (after the initial transient)


def run_parameters(seed, a_range=(0.0, 1.0), vt_range=(0.7, 1.3)):
    g = np.random.default_rng(seed)
    return {"a": float(g.uniform(*a_range)), "vt": float(g.uniform(*vt_range))}


class LearnedCorrection:
    """Fine and coarse solvers, the network and its normalisation."""

    def __init__(self, cfg=None, device="cuda"):
        import torch
        self.torch = torch
        self.cfg = cfg or Config()
        c = self.cfg
        prec = "f64" if c.fp64_data else "f32"
        hi = [2.0 * math.pi / c.k1, HI[1], HI[2]]
        self.fine = dg.Solver(2, c.n_fine, [c.nelem_fine] * 3, LO, hi, c.omega_c, storage=prec, device=device)
        self.coarse = dg.Solver(2, c.n_coarse, [c.nelem_coarse] * 3, LO, hi, c.omega_c, device=device)
        # targets are assembled on a coarse context of the data precision
        self.coarse_t = (dg.Solver(2, c.n_coarse, [c.nelem_coarse] * 3, LO, hi, c.omega_c, storage="f64", device=device)
                         if c.fp64_data else self.coarse)
        n = c.n_coarse
        self.nb = n ** 3
        self.nfeat = (8 if c.fluct else 7) * self.nb + n
        self.ne = c.nelem_coarse ** 3
        self.sizes = [self.nfeat] + list(c.hidden) + [self.nb]
        self.net = dg.Network(self.sizes, self.ne * max(1, c.snapshots_per_step))
        self.device = self.fine.device
        self.mean = None
        self.inv_std = None
        self.target_scale = 1.0

    # ---------------- states ----------------
    def initial_fine_state(self, seed):
        t = self.torch
        c = self.cfg
        p = run_parameters(seed, c.a_range, c.vt_range)
        nodes = [t.from_numpy(self.fine.nodes(a)).to(self.device) for a in range(3)]
        x, u, v = inputs.broadcast_coords(nodes, t)
        f = inputs.mixture(x, u, v, p["a"], p["vt"], c.k1, c.perturbation, 3.0, t)
        return f.to(self.fine.dtype).contiguous()

    def project(self, f_fine, out=None, coarse=None):
        coarse = self.coarse if coarse is None else coarse
        out = coarse.empty_state() if out is None else out
        dg.dg_project(self.fine.ctx, coarse.ctx, f_fine, out)
        return out

    def fine_dt(self, f):
        E = self.fine.poisson(f)
        return self.cfg.cfl_fraction * self.fine.dt_max(2.0 * float(E.abs().max()))

    def coarse_dt(self, fc):
        E = self.coarse.poisson(fc)
        return self.cfg.cfl_fraction * self.coarse.dt_max(2.0 * float(E.abs().max()))

    # ---------------- data ----------------
    def snapshot(self, f):
        """(coarse state P f, its field, P RHS_f(f), RHS_c(P f)), all coarse state layout."""
        fc = self.project(f)
        rf = self.fine.rhs(f)
        ct = self.coarse_t
        fct = fc if ct is self.coarse else self.project(f, coarse=ct)
        prf = self.project(rf, coarse=ct)
        rc = ct.rhs(fct)
        E = self.coarse.poisson(fc)
        return fc, E, (prf, rc)

    def targets(self, pair, scale=1.0, out=None):
        """Element-major target scale * (P RHS_f(f) - RHS_c(P f))."""
        t = self.torch
        out = t.empty((self.ne, self.nb), dtype=t.float32, device=self.device) if out is None else out
        dg.dg_nn_to_elements(self.coarse_t.ctx, pair[0], pair[1], float(scale), out, self.cfg.fluct)
        return out

    def generate(self, seeds, nsnap=None, stride=None, log=None):
        """Snapshots of fine runs: lists of coarse states, fields and targets."""
        c = self.cfg
        nsnap = c.snapshots_per_run if nsnap is None else nsnap
        stride = c.snapshot_stride if stride is None else stride
        states, fields, targets = [], [], []
        for s in seeds:
            f = self.initial_fine_state(s)
            dt = self.fine_dt(f)
            if c.spinup_steps:
                self.fine.step(f, dt, c.spinup_steps)
            for k in range(nsnap):
                fc, E, tg = self.snapshot(f)
                states.append(fc)
                fields.append(E)
                targets.append(tg)
                if k + 1 < nsnap:
                    self.fine.step(f, dt, stride)
            if log:
                log("run seed %d: %d snapshots, dt_fine %.3e" % (s, nsnap, dt))
        return states, fields, targets

    def fit_normalisation(self, states, fields, targets):
        t = self.torch
        raw = t.empty((self.ne, self.nfeat), dtype=t.float32, device=self.device)
        s1 = np.zeros(self.nfeat)
        s2 = np.zeros(self.nfeat)
        for fc, E in zip(states, fields):
            dg.dg_nn_features_raw(self.coarse.ctx, fc, E, raw, self.cfg.fluct)
            a, b = self.net.column_stats(raw)
            s1 += a
            s2 += b
        cnt = float(self.ne * len(states))
        mean = s1 / cnt
        var = np.maximum(s2 / cnt - mean * mean, 0.0)
        std = np.sqrt(var)
        # features that barely vary (e.g. far velocity tails) are not amplified
        floor = 1e-3 * max(float(np.max(std)), 1e-30)
        self.mean = t.from_numpy(mean.astype(np.float32)).to(self.device)
        self.inv_std = t.from_numpy((1.0 / np.maximum(std, floor)).astype(np.float32)).to(self.device)
        tsq = 0.0
        tg = t.empty((self.ne, self.nb), dtype=t.float32, device=self.device)
        for pair in targets:
            a, b = self.net.column_stats(self.targets(pair, 1.0, tg))
            tsq += float(np.sum(b))
        self.target_scale = math.sqrt(tsq / (cnt * self.nb)) if tsq > 0 else 1.0

    def features(self, fc, E, out=None):
        t = self.torch
        X = t.empty((self.ne, self.net.ld), dtype=t.int16, device=self.device) if out is None else out
        dg.dg_nn_features(self.coarse.ctx, self.net.nn, fc, E, self.mean, self.inv_std, X)
        return X

    def dataset(self, states, fields, targets):
        """Stacked BF16 feature rows and normalised FP32 targets (one block of
        ne rows per snapshot)."""
        t = self.torch
        ns = len(states)
        X = t.empty((ns, self.ne, self.net.ld), dtype=t.int16, device=self.device)
        T = t.empty((ns, self.ne, self.nb), dtype=t.float32, device=self.device)
        for i, (fc, E, pair) in enumerate(zip(states, fields, targets)):
            self.features(fc, E, X[i])
            self.targets(pair, 1.0 / self.target_scale, T[i])
        return X, T

    # ---------------- training ----------------
    def init_params(self, seed=None):
        rng = np.random.default_rng(self.cfg.init_seed if seed is None else seed)
        ps = []
        for a, b in zip(self.sizes[:-1], self.sizes[1:]):
            ps.append(rng.standard_normal((a, b)) * math.sqrt(2.0 / a))
            ps.append(np.zeros(b))
        # the last layer starts small: the untrained correction is near zero
        ps[-2] *= 0.01
        self.net.set_params(dg.Network.flatten(ps))

    def train(self, X, T, epochs=None, lr=None, seed=0, log=None, log_every=200):
        c = self.cfg
        epochs = c.epochs if epochs is None else epochs
        lr0 = c.lr if lr is None else lr
        ns = X.shape[0]
        k = max(1, min(c.snapshots_per_step, ns))
        rng = np.random.default_rng(seed)
        if k > 1:
            # one shuffled copy (device-to-device copies), then groups of k
            # consecutive snapshots form the minibatches, visited in a new
            # random order every epoch
            Xs, Ts = self.torch.empty_like(X), self.torch.empty_like(T)
            for j, i in enumerate(rng.permutation(ns)):
                Xs[j].copy_(X[i])
                Ts[j].copy_(T[i])
            X = Xs.reshape(ns * self.ne, -1)
            T = Ts.reshape(ns * self.ne, -1)
        ngroups = ns // k
        rows = k * self.ne
        total = epochs * ngroups
        history = []
        step = 0
        for ep in range(epochs):
            for i in rng.permutation(ngroups):
                lr_t = 0.5 * lr0 * (1.0 + math.cos(math.pi * step / max(total, 1)))
                want = (step % log_every == 0) or step == total - 1
                if k > 1:
                    loss, _ = self.net.loss_grad(X[i * rows:(i + 1) * rows], T[i * rows:(i + 1) * rows], want_loss=want)
                else:
                    loss, _ = self.net.loss_grad(X[i], T[i], want_loss=want)
                self.net.adamw(lr_t, c.weight_decay)
                if want:
                    history.append((step, loss))
                    if log:
                        log("step %d epoch %d loss %.5f lr %.2e" % (step, ep, loss, lr_t))
                step += 1
        return history

    def relative_error(self, X, T):
        """||T - NN(X)|| / ||T|| over the given snapshots (normalised units)."""
        num = den = 0.0
        for i in range(X.shape[0]):
            Y = self.net.forward(X[i])
            num += float(((Y - T[i]) ** 2).sum())
            den += float((T[i] ** 2).sum())
        return math.sqrt(num / den)

    # ---------------- corrected runs ----------------
    def run_coarse(self, fc, dt, nsteps, corrected):
        if corrected:
            return dg.dg_nn_rk_step(self.coarse.ctx, self.net.nn, self.mean, self.inv_std, self.target_scale, fc,
                                    dt, nsteps, diag=True)
        return self.coarse.step(fc, dt, nsteps, diag=True)

    def evaluate(self, seed, coarse_steps, checkpoints=10, log=None):
        """Fine run, plain coarse run and corrected coarse run from the same
        initial state (the coarse ones from its projection).  The fine step is
        the coarse step divided by an integer m, so both grids meet at every
        coarse step time.  Compared: field-energy histories at the coarse
        times, and at `checkpoints` evenly spaced times the relative L2
        distance of each coarse state from the projected fine state."""
        t = self.torch
        f = self.initial_fine_state(seed)
        fc0 = self.project(f)
        dtc = self.coarse_dt(fc0)
        m = int(math.ceil(dtc / self.fine_dt(f)))
        dtf = dtc / m
        f0_energy = self.fine.diagnostics(f)["field_energy"]
        m0 = self.coarse.diagnostics(fc0)["mass"]
        plain_s, nn_s = fc0.clone(), fc0.clone()
        ck = sorted(set(int(round(coarse_steps * (i + 1) / checkpoints)) for i in range(checkpoints)))
        wf, wp, wc = [], [], []
        err_p, err_c, times = [], [], []
        tim = {"fine": 0.0, "plain_coarse": 0.0, "coarse_nn": 0.0}
        done = 0
        pf = self.coarse.empty_state()
        for k in ck:
            nstep = k - done
            t0 = time.perf_counter()
            fine = self.fine.step(f, dtf, nstep * m, diag=True)
            t.cuda.synchronize()
            t1 = time.perf_counter()
            plain = self.run_coarse(plain_s, dtc, nstep, False)
            t.cuda.synchronize()
            t2 = time.perf_counter()
            corr = self.run_coarse(nn_s, dtc, nstep, True)
            t.cuda.synchronize()
            t3 = time.perf_counter()
            tim["fine"] += t1 - t0
            tim["plain_coarse"] += t2 - t1
            tim["coarse_nn"] += t3 - t2
            wf += [d["field_energy"] for d in fine[m - 1::m]]
            wp += [d["field_energy"] for d in plain]
            wc += [d["field_energy"] for d in corr]
            self.project(f, pf)
            nrm = float(t.linalg.vector_norm(pf.double()))
            err_p.append(float(t.linalg.vector_norm((plain_s - pf).double())) / nrm)
            err_c.append(float(t.linalg.vector_norm((nn_s - pf).double())) / nrm)
            times.append(k * dtc)
            done = k
        ref, wp, wc = np.array(wf), np.array(wp), np.array(wc)

        def rel(w):
            return float(np.linalg.norm(w - ref) / np.linalg.norm(ref))

        late = int(len(ref) * (1.0 - self.cfg.late_window))

        def rel_late(w):
            return float(np.linalg.norm(w[late:] - ref[late:]) / np.linalg.norm(ref[late:]))

        def relmax(w):
            return float(np.max(np.abs(w - ref)) / np.max(np.abs(ref)))

        out = {
            "seed": seed, "coarse_steps": coarse_steps, "dt_coarse": dtc, "fine_steps": coarse_steps * m,
            "dt_fine": dtf, "t_end": coarse_steps * dtc, "field_energy_t0": f0_energy,
            "field_energy_rel_l2": {"plain_coarse": rel(wp), "coarse_nn": rel(wc)},
            "field_energy_rel_l2_late": {"plain_coarse": rel_late(wp), "coarse_nn": rel_late(wc),
                                         "from_t": (late + 1) * dtc},
            "field_energy_max_err_over_max": {"plain_coarse": relmax(wp), "coarse_nn": relmax(wc)},
            "state_rel_l2_vs_projected_fine": {"t": times, "plain_coarse": err_p, "coarse_nn": err_c},
            "mass_drift": {"plain_coarse": abs(plain[-1]["mass"] - m0) / m0, "coarse_nn": abs(corr[-1]["mass"] - m0) / m0},
            "wall_s": tim,
            "dof_updates_per_sim_time": {
                "fine": self.fine_dof() * 3 / dtf,
                "coarse": self.coarse_dof() * 3 / dtc,
            },
            "history": {"t": (np.arange(1, len(ref) + 1) * dtc).tolist(), "fine": ref.tolist(), "plain": wp.tolist(),
                        "nn": wc.tolist()},
        }
        if log:
            log("eval seed %d: field energy rel L2 plain %.4f nn %.4f; state error at end plain %.3e nn %.3e"
                % (seed, out["field_energy_rel_l2"]["plain_coarse"], out["field_energy_rel_l2"]["coarse_nn"],
                   err_p[-1], err_c[-1]))
        return out

    def fine_dof(self):
        return (self.cfg.nelem_fine * self.cfg.n_fine) ** 3

    def coarse_dof(self):
        return (self.cfg.nelem_coarse * self.cfg.n_coarse) ** 3

    def close(self):
        for o in (self.net, self.fine, self.coarse, self.coarse_t):
            o.close()


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="train and evaluate the learned coarse-grid correction")
    ap.add_argument("--runs", type=int, default=32)
    ap.add_argument("--snapshots", type=int, default=64)
    ap.add_argument("--stride", type=int, default=220)
    ap.add_argument("--epochs", type=int, default=5)
    ap.add_argument("--eval-seeds", type=int, nargs="*", default=[1000, 1001])
    ap.add_argument("--coarse-steps", type=int, default=2000)
    ap.add_argument("--out", default=None)
    ap.add_argument("--fluct", action="store_true", help="fluctuation form (inputs and targets about the x average)")
    ap.add_argument("--fp32-data", action="store_true", help="fine runs, projections and right-hand sides in FP32")
    d = Config()
    ap.add_argument("--perturbation", type=float, default=d.perturbation, help="density perturbation amplitude")
    ap.add_argument("--omega-c", type=float, default=d.omega_c)
    ap.add_argument("--k1", type=float, default=d.k1)
    ap.add_argument("--a-range", type=float, nargs=2, default=list(d.a_range))
    ap.add_argument("--vt-range", type=float, nargs=2, default=list(d.vt_range))
    ap.add_argument("--spinup", type=int, default=0, help="fine steps before the first snapshot")
    a = ap.parse_args(argv)
    cfg = Config(train_seeds=list(range(a.runs)), snapshots_per_run=a.snapshots, snapshot_stride=a.stride,
                 epochs=a.epochs, fluct=a.fluct, fp64_data=not a.fp32_data, perturbation=a.perturbation,
                 omega_c=a.omega_c, k1=a.k1, a_range=tuple(a.a_range), vt_range=tuple(a.vt_range),
                 spinup_steps=a.spinup)
    log = lambda m: print(m, flush=True)  # noqa: E731
    lc = LearnedCorrection(cfg)
    t0 = time.perf_counter()
    st, fl, tg = lc.generate(cfg.train_seeds, log=log)
    t_gen = time.perf_counter() - t0
    lc.fit_normalisation(st, fl, tg)
    X, T = lc.dataset(st, fl, tg)
    del st, fl, tg
    nval = max(1, X.shape[0] // 16)
    lc.init_params()
    err0 = lc.relative_error(X[-nval:], T[-nval:])
    t0 = time.perf_counter()
    hist = lc.train(X[:-nval], T[:-nval], log=log)
    lc.torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    err1 = lc.relative_error(X[-nval:], T[-nval:])
    # held-out runs: one-step closure error and field-energy histories
    hs, hf, ht = lc.generate(a.eval_seeds, nsnap=16, stride=4 * a.stride)
    Xh, Th = lc.dataset(hs, hf, ht)
    err_h = lc.relative_error(Xh, Th)
    evals = [lc.evaluate(s, a.coarse_steps, log=log) for s in a.eval_seeds]
    rep = {
        "training": {"runs": a.runs, "snapshots": int(X.shape[0]), "rows": int(X.shape[0] * lc.ne),
                     "generate_s": t_gen, "train_s": t_train, "loss_history": hist,
                     "target_scale": lc.target_scale,
                     "val_rel_err_untrained": err0, "val_rel_err_trained": err1,
                     "heldout_rel_err_trained": err_h},
        "evaluation": [{k: v for k, v in e.items() if k != "history"} for e in evals],
    }
    print(json.dumps(rep), flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump({"report": rep, "histories": [e["history"] for e in evals]}, fh)
    lc.close()


if __name__ == "__main__":
    main()
