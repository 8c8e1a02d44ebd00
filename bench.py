"""Benchmark of the DG Vlasov-Poisson hot path on one MI355X.

A step is one SSP-RK3 step: three fused stage kernels, each followed by the
FP64 density reduction + spectral Poisson solve, replayed from a HIP graph.
The metric is phase-space DOF updates per second per RK stage
(DOF x 3 x steps / elapsed), inputs resident in HBM before timing starts.

Default workload: 1D2V magnetised Maxwellian with 8 seeded modes, x 64 / vx 48 /
vy 48 elements, n = 9 (107 495 424 DOF, 430 MB per FP32 state buffer, three
buffers), omega_c = 1, dt = 0.9 dt_max.

The JSON line also carries
  roofline      -- the fused stage kernel's algorithmic HBM bytes per launch
                   (8 B/DOF for stage 1, 12 B/DOF for stages 2-3 in FP32) over
                   its mean duration from HIP events on the library stream
                   (dg_profile_step), against 8 TB/s; traffic from the committed
                   rocprofv3 counter summary when it matches the kernel source.
  cpu_baseline  -- the FP64 NumPy oracle timed on the host on a bounded sample
                   (one RK stage on a 1/8 x-subdomain with halo), plus one RHS
                   and one RK3 step on the 1D1V Landau and 16.8 M DOF ring
                   workloads and the CPU model.
  fp64_storage  -- the same workload in FP64 storage (--no-fp64 skips it).
  sweep         -- the batched 64-run uneven sweep under the tuner's choice,
                   against its solo runs (--no-sweep skips it).
--pattern-copy prints the copy references instead (streaming and tile-pattern
copies of one state buffer next to the stage kernels, and the time of one
empty dependent launch next to the field solve's); --nn-step times the
learned correction's corrected coarse step (fused and per-layer network);
--write-traffic summarises two rocprofv3 counter runs into the traffic file.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# the stage kernels' source: the tile code with the kernel templates, and the
# operator tables they are built with
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2202_13532_amd", "csrc", f)
                  for f in ("stage_tiles.h", "dg_ops_constexpr.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stage_kernel_traffic.json")


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload):
    """Counter-derived HBM bytes per stage launch, if taken on this kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    rec = t.get(workload)
    if not rec or rec.get("kernel_sha256_16") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def workload_by_name(name):
    from paper_2202_13532_amd import workloads as W
    table = {"maxwell_1d2v_n9": W.maxwell_1d2v_n9, "ring_1d2v_n8": W.ring_1d2v_n8,
             "landau_1d1v_n4": W.landau_1d1v_n4}
    return table[name]()


def make_state(torch, solver, wl):
    from paper_2202_13532_amd import workloads as W
    nodes = [torch.from_numpy(solver.nodes(a)).cuda() for a in range(1 + wl.nv)]
    f = W.initial_state(wl, nodes, torch)
    return solver.pack(f.to(solver.dtype).contiguous())   # into the solver's state layout


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_config_timings():
    """The oracle's one RHS and one full SSP-RK3 step (Poisson at every stage)
    on the 1D1V Landau workload (8192 DOF, FP64) and the 1D2V ring workload
    (16.8 M DOF), timed once each."""
    import numpy as np
    from oracle import grid, lgl, rhs, rk
    from paper_2202_13532_amd import workloads as W
    out = []
    for wl in (W.landau_1d1v_n4(), W.ring_1d2v_n8()):
        g = grid.PhaseGrid(wl.nv, wl.n, wl.nelem, wl.lo, wl.hi, wl.omega_c)
        f = np.broadcast_to(np.asarray(W.initial_state(wl, [ax.nodes for ax in g.axes], np), dtype=np.float64),
                            g.shape).copy()
        ops = lgl.operators(wl.n)
        E = np.zeros((wl.nelem[0], wl.n))
        t0 = time.perf_counter()
        rhs.rhs(g, ops, f, E)
        t_rhs = time.perf_counter() - t0
        t0 = time.perf_counter()
        rk.ssprk3_step(g, ops, f, 1e-4)
        t_step = time.perf_counter() - t0
        dof = g.dof()
        out.append({"workload": wl.name, "dof": int(dof), "rhs_s": t_rhs, "rk3_step_s": t_step,
                    "dof_stage_updates_per_s_rk3": 3 * dof / t_step})
        del f
    return out


def cpu_baseline(wl, budget_s=12.0):
    """FP64 oracle, one RK stage on x elements [0, Nx/8) plus a 1-element halo."""
    import numpy as np
    from oracle import grid, lgl, rhs
    from paper_2202_13532_amd import inputs, workloads as W
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count()
    nx_sub = max(1, wl.nelem[0] // 8)
    dxe = (wl.hi[0] - wl.lo[0]) / wl.nelem[0]
    lo = [wl.lo[0] - dxe] + list(wl.lo[1:])
    hi = [wl.lo[0] + (nx_sub + 1) * dxe] + list(wl.hi[1:])
    nel = [nx_sub + 2] + list(wl.nelem[1:])
    g = grid.PhaseGrid(wl.nv, wl.n, nel, lo, hi, wl.omega_c)
    f = np.asarray(W.initial_state(wl, [ax.nodes for ax in g.axes], np), dtype=np.float64)
    f = np.broadcast_to(f, g.shape).copy()
    E = 1e-3 * np.cos(0.1 * g.axes[0].nodes)
    ops = lgl.operators(wl.n)
    t0 = time.perf_counter()
    reps = 0
    dt = 1e-4
    while True:
        f = f + dt * rhs.rhs(g, ops, f, E)          # one SSP-RK3 first stage
        reps += 1
        if time.perf_counter() - t0 > budget_s or reps >= 30:
            break
    el = time.perf_counter() - t0
    dof_inner = g.dof() * nx_sub // (nx_sub + 2)
    return {"value": dof_inner * reps / el, "unit": "DOF-updates/s per RK stage", "cores": int(cores),
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": "%d RK stage(s) of the FP64 NumPy oracle on x elements [0,%d) of %d (+1-element halo), %d DOF each, %.1f s"
                      % (reps, nx_sub, wl.nelem[0], dof_inner, el),
            "oracle_configs": oracle_config_timings()}


def sweep_record(steps, warmup, layout=None, bw_single=None):
    """Uneven batch of 64 runs (32 x 1D1V, 32 x 1D2V, n 4..9): persistent
    stage launches (one per kind of run and RK stage) under the tuner's
    choices, against the same runs stepped one after another with their own
    graphs.  bw_single: algorithmic GB/s of the single-run stage kernels, to
    express the sweep's step time against its algorithmic-byte time."""
    import torch
    from paper_2202_13532_amd import dg
    from paper_2202_13532_amd import workloads as W
    wls = W.uneven_sweep(64)
    lay = [(layout or "vpad") if w.nv == 2 else "dense" for w in wls]   # padded v rows for 1D2V runs
    cfgs = [dg.make_config(w.nv, w.n, w.nelem, w.lo, w.hi, w.omega_c, layout=l) for w, l in zip(wls, lay)]
    solos = [dg.Solver(w.nv, w.n, w.nelem, w.lo, w.hi, w.omega_c, layout=l) for w, l in zip(wls, lay)]
    states, dts = [], []
    for w, so in zip(wls, solos):
        f = make_state(torch, so, w)
        E0 = so.poisson(f)
        dts.append(w.cfl_fraction * so.dt_max(max(float(E0.abs().max()), 0.05)))
        states.append(f)
    dof = sum(w.dof() for w in wls)
    print("[bench] sweep: %d runs, %d DOF" % (len(wls), dof), file=sys.stderr, flush=True)
    b = dg.Batch(cfgs)
    t0 = time.perf_counter()
    tuned_ms = b.tune(states, dts, 3)
    t_tune = time.perf_counter() - t0
    if warmup > 0:
        b.step(states, dts, warmup)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    b.step(states, dts, steps)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    # the same runs one after another (each with its own captured step graph)
    for so, f, dt in zip(solos, states, dts):
        so.step(f, dt, max(1, min(warmup, 10)))
    torch.cuda.synchronize()
    start.record()
    for so, f, dt in zip(solos, states, dts):
        so.step(f, dt, steps)
    end.record()
    torch.cuda.synchronize()
    ms_solo = start.elapsed_time(end)
    alg_bytes = 32 * dof   # FP32: 8 + 12 + 12 bytes per DOF per step
    rec = {
        "workload": "uneven_sweep_64", "runs": len(wls), "dof": dof, "steps": steps, "warmup": warmup,
        "ms_per_step": ms / steps, "value": dof * 3 * steps / (ms / 1e3), "unit": "DOF-updates/s per RK stage",
        "hbm_effective_frac_whole_step": alg_bytes * steps / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
        "solo_sequential": {"ms_per_step": ms_solo / steps, "value": dof * 3 * steps / (ms_solo / 1e3)},
        "batch_speedup_vs_solo": ms_solo / ms,
        "tune": {"seconds": t_tune, "best_ms_per_step": tuned_ms, "grid": b.grid, "choice": b.choice},
    }
    if bw_single:
        rec["step_time_over_algorithmic_time_at_single_run_bw"] = (ms / steps) / (alg_bytes / (bw_single * 1e9) * 1e3)
    b.close()
    for so in solos:
        so.close()
    return rec


def fp64_record(torch, dg, wl, layout, steps, warmup=10):
    """The same workload in FP64 storage (the precision of the paper's code):
    graph-replayed steps and the stage kernels' HIP-event durations."""
    s = dg.Solver(wl.nv, wl.n, wl.nelem, wl.lo, wl.hi, wl.omega_c, 0, "f64", layout=layout)
    f = make_state(torch, s, wl)
    E0 = s.poisson(f)
    dt = wl.cfl_fraction * s.dt_max(max(float(E0.abs().max()), 0.05))
    s.step(f, dt, warmup)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    s.step(f, dt, steps)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    prof = s.profile_step(f, dt, 2)
    st_ms = prof[:, [0, 2, 4]].mean(axis=0)
    dof = wl.dof()
    byts = [16 * dof, 24 * dof, 24 * dof]
    achieved = sum(byts) / (st_ms.sum() / 1e3) / 1e9
    s.close()
    return {"steps": steps, "warmup": warmup, "ms_per_step": ms / steps,
            "value": dof * 3 * steps / (ms / 1e3), "unit": "DOF-updates/s per RK stage",
            "stage_ms_mean": [float(x) for x in st_ms], "algorithmic_GBs": achieved,
            "frac": achieved / HBM_PEAK_GBS}


def bench_sweep(args):
    rec = sweep_record(args.steps, args.warmup, args.layout)
    line = {
        "metric": "phase-space DOF-updates/sec per RK stage (FP32) + % peak HBM BW",
        "value": rec["value"], "unit": "DOF-updates/s per RK stage", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": rec["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "uneven_sweep_64", "runs": rec["runs"], "dof": rec["dof"], "storage": "f32",
                   "layout_1d2v": args.layout or "vpad", "reductions": "f64",
                   "parallelism": "single GPU, persistent launches per kind and stage"},
        "sweep": rec,
    }
    print(json.dumps(line), flush=True)


def bench_nn_step(args):
    """The learned correction's coarse step (coarse_1d2v_n4: 16^3 elements,
    n = 4, omega_c = 0.05 as in the learned setting) with a random-init
    network of the learned shape [7 n^3 + n, 128, 128, 128, n^3]: ms per
    corrected SSP-RK3 step with the fused inference kernel and with one GEMM
    launch per layer, next to the plain coarse step."""
    import numpy as np
    import torch
    from paper_2202_13532_amd import dg
    from paper_2202_13532_amd import workloads as W
    wl = W.coarse_1d2v_n4(0.05)
    s = dg.Solver(wl.nv, wl.n, wl.nelem, wl.lo, wl.hi, wl.omega_c)
    f = make_state(torch, s, wl)
    nfeat, nout = 7 * wl.n ** 3 + wl.n, wl.n ** 3
    sizes = [nfeat, 128, 128, 128, nout]
    rows = wl.nelem[0] * wl.nelem[1] * wl.nelem[2]
    net = dg.Network(sizes, rows)
    rng = np.random.default_rng(3)
    ps = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        ps += [rng.standard_normal((a, b)) * math.sqrt(2.0 / a) * 0.1, rng.standard_normal(b) * 0.01]
    net.set_params(dg.Network.flatten(ps))
    mean = torch.zeros(nfeat, device="cuda")
    inv = torch.ones(nfeat, device="cuda")
    dt = wl.cfl_fraction * s.dt_max(max(float(s.poisson(f).abs().max()), 0.05))
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn(args.warmup)
        torch.cuda.synchronize()
        start.record()
        fn(args.steps)
        end.record()
        torch.cuda.synchronize()
        return start.elapsed_time(end) / args.steps

    rec = {}
    for fused in (True, False):
        net.set_fused(fused)
        g = f.clone()
        rec["corrected_ms_" + ("fused" if fused else "layerwise")] = timed(
            lambda k: dg.dg_nn_rk_step(s.ctx, net.nn, mean, inv, 1e-3, g, dt, k))
    g = f.clone()
    rec["plain_ms"] = timed(lambda k: s.step(g, dt, k))
    dof = wl.dof()
    line = {"metric": "corrected coarse SSP-RK3 step (learned correction)", "value": rec["corrected_ms_fused"],
            "unit": "ms per step", "higher_is_better": False, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "dtype": "f32 state, bf16 network", "data": "synthetic, random-init network",
            "config": {"workload": wl.name, "dof": dof, "network": sizes, "rows": rows, "omega_c": wl.omega_c},
            "nn_step": rec}
    net.close()
    s.close()
    print(json.dumps(line), flush=True)


def write_traffic(fetch_dir, write_dir, workload="maxwell_1d2v_n9"):
    """Summarise two rocprofv3 counter runs of `bench.py --copy-calibration`
    (one with FETCH_SIZE, one with WRITE_SIZE; their output directories) into
    the per-launch HBM bytes of the FP32 stage kernels, each counter scaled by
    what it reads for the plain device copies of one state buffer, and store
    them with the kernel-source hash in the traffic file."""
    import collections
    import csv

    def per_kernel(d):
        acc = collections.defaultdict(list)
        with open(os.path.join(d, "run_counter_collection.csv")) as fh:
            for r in csv.DictReader(fh):
                acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return acc

    import re

    def find(acc, key):
        ks = [k for k in acc if re.search(key, k)]
        if len(ks) != 1:
            raise SystemExit("expected one kernel matching %r, found %s" % (key, ks))
        return acc[ks[0]]

    wl = workload_by_name(workload)
    dof = wl.dof()
    F, W = per_kernel(fetch_dir), per_kernel(write_dir)
    n = wl.n
    # the plain stage kernels (template arguments T, n, UN, BG[, CORR])
    k1 = r"stage2v_kernel<float, %d, false, false(, false)*>" % n
    k23 = r"stage2v_kernel<float, %d, true, false(, false)?(, (true|false))?>" % n
    s1f, s23f = find(F, k1), find(F, k23)
    s1w, s23w = find(W, k1), find(W, k23)
    # the calibration copies: the large copyBuffer dispatches
    cf = [v for v in find(F, "copyBuffer") if v > 1e5]
    cw = [v for v in find(W, "copyBuffer") if v > 1e5]
    from paper_2202_13532_amd import dg
    cfg = dg.make_config(wl.nv, wl.n, wl.nelem, wl.lo, wl.hi, wl.omega_c, 0, "f32", layout="vpad")
    state_bytes = math.prod(dg.state_shape(cfg)) * 4
    mean = lambda x: sum(x) / len(x)
    ff = mean(cf) * 1024 / state_bytes
    fw = mean(cw) * 1024 / state_bytes
    b1 = mean(s1f) * 1024 / ff + mean(s1w) * 1024 / fw
    b23 = mean(s23f) * 1024 / ff + mean(s23w) * 1024 / fw
    alg = [8 * dof, 12 * dof, 12 * dof]
    rec = {workload + "_f32_vpad": {
        "layout": "vpad", "kernel_sha256_16": kernel_source_hash(),
        "bytes_per_launch": [b1, b23, b23], "algorithmic_bytes_per_launch": alg,
        "fetch_kib_per_launch": [mean(s1f), mean(s23f)], "write_kib_per_launch": [mean(s1w), mean(s23w)],
        "copy_calibration": {"bytes_each_way": state_bytes, "fetch_kib": mean(cf), "write_kib": mean(cw),
                             "fetch_factor": ff, "write_factor": fw},
        "launches_counted": {"stage1": len(s1f), "stage23": len(s23f)}}}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps({"traffic_over_algorithmic": [b1 / alg[0], b23 / alg[1]], "fetch_factor": ff,
                      "write_factor": fw, "copies": [len(cf), len(cw)]}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="maxwell_1d2v_n9")
    ap.add_argument("--storage", default=None, help="override storage (f32/f64)")
    ap.add_argument("--layout", default=None, help="state layout: dense or vpad (1D2V only; the 1D2V default is vpad)")
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the batched 64-run sweep sub-record")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-storage sub-record")
    ap.add_argument("--fp64-steps", type=int, default=20)
    ap.add_argument("--sweep-steps", type=int, default=20)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run two plain device copies of one state buffer (reference for HBM byte counters)")
    ap.add_argument("--pattern-copy", action="store_true",
                    help="print the bandwidth of a streaming copy and of a copy with the stage kernel's tile "
                         "access pattern (no halos, no arithmetic) next to the stage kernels'")
    ap.add_argument("--nn-step", action="store_true",
                    help="time the learned correction's corrected coarse step (fused and per-layer network)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"), default=None,
                    help="summarise two rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE) into the traffic file; "
                         "runs nothing on the GPU")
    args = ap.parse_args()
    if args.write_traffic:
        return write_traffic(*args.write_traffic, workload=args.workload)
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the x-slab sharding is a design note); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.workload == "uneven_sweep_64":
        return bench_sweep(args)
    if args.nn_step:
        return bench_nn_step(args)

    import torch
    from paper_2202_13532_amd import dg

    wl = workload_by_name(args.workload)
    if args.storage:
        wl.storage = args.storage
    print("[bench] workload %s storage %s dof %d" % (wl.name, wl.storage, wl.dof()), file=sys.stderr, flush=True)
    # padded v rows (64-value aligned chunks) are the native 1D2V layout
    layout = args.layout or ("vpad" if wl.nv == 2 else "dense")
    s = dg.Solver(wl.nv, wl.n, wl.nelem, wl.lo, wl.hi, wl.omega_c, 0, wl.storage, layout=layout)
    f = make_state(torch, s, wl)
    E0 = s.poisson(f)
    maxE = float(E0.abs().max())
    dt = wl.dt if wl.dt else wl.cfl_fraction * s.dt_max(max(maxE, 0.05))
    torch.cuda.synchronize()
    if args.warmup > 0:
        s.step(f, dt, args.warmup)
    torch.cuda.synchronize()
    print("[bench] warmup done, timing %d steps" % args.steps, file=sys.stderr, flush=True)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    start.record()
    s.step(f, dt, args.steps)
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = start.elapsed_time(end)
    dof = wl.dof()
    value = dof * 3 * args.steps / (ms / 1e3)

    # per-kernel durations on the library stream (eager launches, HIP events)
    prof = s.profile_step(f, dt, max(1, args.profile_steps))
    esize = 8 if wl.storage == "f64" else 4
    st_ms = prof[:, [0, 2, 4]]
    fld_ms = prof[:, [1, 3, 5]]
    bytes_per_launch = [2 * esize * dof, 3 * esize * dof, 3 * esize * dof]
    tot_bytes = sum(bytes_per_launch) * prof.shape[0]
    achieved = tot_bytes / (st_ms.sum() / 1e3) / 1e9
    traffic_stages = load_traffic(wl.name + "_" + wl.storage + ("_vpad" if layout == "vpad" else ""))
    # per launch, averaged over the three stage launches like `achieved`
    traffic = sum(traffic_stages) / len(traffic_stages) if traffic_stages else None
    if args.copy_calibration:
        buf = torch.empty_like(f)
        for _ in range(2):
            buf.copy_(f)
        torch.cuda.synchronize()
        del buf
    if args.pattern_copy:
        state_bytes = f.numel() * f.element_size()
        ms_lin = s.profile_copy(f, 0, 20)
        ms_pat = s.profile_copy(f, 1, 20)
        ms_launch = s.profile_copy(f, 2, 200)
        ms_pat_res = s.profile_copy(f, 3, 20)
        rec = {"metric": "copy references (GB/s, read + write)", "workload": wl.name, "storage": wl.storage,
               "layout": layout, "state_bytes": state_bytes,
               "linear_copy": {"ms": ms_lin, "GBs": 2 * state_bytes / (ms_lin / 1e3) / 1e9},
               "tile_pattern_copy": {"ms": ms_pat, "GBs": 2 * state_bytes / (ms_pat / 1e3) / 1e9},
               # the same copy with no more work-groups resident per CU than the stage-1 kernel
               "tile_pattern_copy_stage_residency": {"ms": ms_pat_res,
                                                     "GBs": 2 * state_bytes / (ms_pat_res / 1e3) / 1e9},
               "stage_kernels_GBs_algorithmic": [b / (t / 1e3) / 1e9 for b, t in
                                                 zip(bytes_per_launch, st_ms.mean(axis=0))],
               "peak_GBs": HBM_PEAK_GBS,
               # the field solve is two dependent launches per stage: its floor
               "dependent_empty_launch_us": ms_launch * 1e3,
               "field_pair_us": [float(x) * 1e3 for x in fld_ms.mean(axis=0)],
               "step_ms": ms / args.steps, "stage_ms_sum": float(st_ms.mean(axis=0).sum())}
        print(json.dumps(rec), flush=True)
        s.close()
        return
    diag = s.diagnostics(f)
    line = {
        "metric": "phase-space DOF-updates/sec per RK stage (FP32) + % peak HBM BW",
        "value": value,
        "unit": "DOF-updates/s per RK stage",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if wl.storage == "f32" else "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "dims": "1D%dV" % wl.nv, "n": wl.n, "nelem": wl.nelem,
                   "dof": dof, "omega_c": wl.omega_c, "dt": dt, "storage": wl.storage, "layout": layout,
                   "reductions": "f64", "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_per_stage_launch": traffic_stages,
                     "algorithmic_bytes_mean_per_launch": sum(bytes_per_launch) / 3.0,
                     "kernel": "stage%dv_kernel<%s,%d>" % (wl.nv, "float" if esize == 4 else "double", wl.n),
                     "stage_ms_mean": [float(x) for x in st_ms.mean(axis=0)],
                     "field_ms_mean": [float(x) for x in fld_ms.mean(axis=0)],
                     "algorithmic_bytes_per_launch": bytes_per_launch},
        "wall_s_timed": wall,
        "hbm_effective_frac_whole_step": (sum(bytes_per_launch) * args.steps / (ms / 1e3) / 1e9) / HBM_PEAK_GBS,
        "final_mass": diag["mass"],
        "final_field_energy": diag["field_energy"],
    }
    s.close()
    if not args.no_fp64 and wl.name == "maxwell_1d2v_n9" and wl.storage == "f32":
        print("[bench] FP64 storage, same workload", file=sys.stderr, flush=True)
        line["fp64_storage"] = fp64_record(torch, dg, wl, layout, args.fp64_steps)
    if not args.no_sweep and wl.name == "maxwell_1d2v_n9":
        print("[bench] batched sweep", file=sys.stderr, flush=True)
        line["sweep"] = sweep_record(args.sweep_steps, 10, None, achieved)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
