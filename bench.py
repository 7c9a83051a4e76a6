"""Benchmark of the MPR prediction path on one MI355X.

A step is one whole prediction of the workload through the C ABI, with the inputs already in
HBM: load (validation, data map, sample energy, initial state), temperature inference
(n_equil sweeps), averaging (n_avg sweeps) and the predictions.  `value` is site updates per
second over the whole step: one site update = one hybrid (over-relaxation + Metropolis) update
of one prediction site in one sweep of one chain.

The default workload is the batch of 256 grids (sides 64 ... 1024, four chains each) with FP16
angle storage and FP32 functions and arithmetic: the reduced-precision batched path (its FP32
storage, FP64 and 1024^2 setups follow in `setups`).

Also printed in the same JSON line:
  roofline      the inference sweep kernel (its average launch time from HIP events on the
                library's stream over the timed steps) against the vector-ALU roof that bounds
                it: the method's VALU issue units per site update (OPS_PER_UPDATE) times the
                site updates of one launch, over the launch time, against two VALU
                instructions per quad-cycle per SIMD; beside it (`hbm`) the algorithmic HBM
                bytes of one launch ((N + 2P) s per chain, s = bytes per angle) against the
                8 TB/s HBM roof and against a measured device copy, and `traffic`, the HBM
                bytes per launch rocprofv3 counted for the same kernel source (null when the
                kernel changed since the counters were taken)
  cpu_baseline  the FP64 CPU oracle timed on a bounded sample of the same workload, on every
                host core and on one
  setups        the same measurements for the other precision setups / workloads, and
                `fp64_factor`: the primary setup's rate over the FP64 setup's on the same
                workload
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1910_08448_amd import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
# VALU issue roof, in lane-operations per second: 256 CUs x 4 SIMDs x 64 lanes x 2.4 GHz / 4
# cycles per wave64 instruction = 39.3 T at one instruction per quad-cycle; gfx950 issues a
# second VALU instruction in the same quad-cycle for some instruction pairs (counter
# SQ_ACTIVE_INST_VALU2), so two per quad-cycle, 78.6 T, is the roof (the published 157.3
# TFLOP/s FP32 figure with an FMA counted as two operations)
ALU_PEAK_TOPS = 256 * 4 * 64 * 2.4e9 / 4 * 2 / 1e12
ALU_SINGLE_ISSUE_TOPS = ALU_PEAK_TOPS / 2
# The method's arithmetic per site update in VALU issue units (transcendentals count two, as in
# SQ_ACTIVE_INST_VALU): the compiled single-precision site code -- field sums of four
# neighbours, half a Philox4x32-10 call, the hybrid update (atan2, two sin/cos pairs, exp,
# uniforms, tests and selects) and the fixed-point energy term -- issues about 110 per update
OPS_PER_UPDATE = 110
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
PREC = {"fp64": 0, "fp32": 1, "fp16": 2, "fix16": 3}
BYTES = {"fp64": 8, "fp32": 4, "fp16": 2, "fix16": 2}
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16": "f32", "fix16": "f32"}   # arithmetic type of the sweep
SWEEPS = {"grid64": (256, 100), "grid1024": (1000, 100), "grid4096": (1000, 100),
          "grid16384": (500, 50), "batch256": (1000, 100)}
CHAINS = {"batch256": 4}
# secondary setups of a default run (besides the primary workload's other precisions), and the
# larger single grids of --extended
SETUPS = [("grid1024", "fp32")]
EXTENDED = [("grid4096", "fp16"), ("grid16384", "fp16"), ("grid16384", "fp32"),
            ("grid16384", "fp64")]
T_MIN, T_MAX = 1e-6, 10.0            # the library's default temperature clamp


def kernel_source_sha():
    """Digest of the sources the sweep kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for f in ("mpr_device.hpp", "mpr_sparse.hpp", "mpr_tiled.hpp", "mpr.hip"):
        with open(os.path.join(ROOT, "paper_1910_08448_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, precision):
    """HBM bytes per launch of the inference sweep kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by its reading for a copy of known size),
    or None when there is none for this workload or the kernel source changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get("entries", {}).get("%s/%s" % (workload, precision))
    if e is None or t.get("kernel_source_sha") != kernel_source_sha():
        return None
    return int(e["bytes_per_launch"])


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_inputs(name, p_missing):
    t = time.time()
    if name == "batch256":
        grids = synth.batch_workload(256, 64, 1024, seed=1)
        inp = {"grids": grids, "mc_seed": 2001}
    else:
        w = synth.workload(name, seed=1, p_missing=p_missing)
        inp = {"grids": [w], "mc_seed": w["mc_seed"]}
    log("inputs %s generated in %.1f s" % (name, time.time() - t))
    return inp


class Inputs:
    """Synthetic inputs of one workload, resident in HBM."""

    def __init__(self, name, p_missing, torch):
        self.name = name
        self.p_missing = p_missing
        inp = make_inputs(name, p_missing)
        self.grids = inp["grids"]
        self.mc_seed = inp["mc_seed"]
        self.shapes = [g["z"].shape for g in self.grids]
        self.z = torch.as_tensor(np.concatenate([g["z"].ravel() for g in self.grids])).cuda()
        self.m = torch.as_tensor(np.concatenate([g["mask"].ravel() for g in self.grids])).cuda()
        self.n_sites = [h * w for h, w in self.shapes]
        self.n_pred = [int((g["mask"] == 0).sum()) for g in self.grids]


GOLDEN = os.path.join(ROOT, "tests", "golden")


def oracle_reference(name, p_missing):
    """The oracle's stored run of this workload (tests/golden, written by a script that calls
    only the oracle), or None."""
    key = {"grid1024": "grid1024_p%.2f" % (0.33 if p_missing is None else p_missing),
           "grid4096": "grid4096", "grid16384": "grid16384",
           "batch256": "batch256_sub16"}.get(name)
    if key is None or (p_missing is not None and name != "grid1024"):
        return None
    path = os.path.join(GOLDEN, "oracle_reference.json")
    try:
        return json.load(open(path)).get(key)
    except (OSError, ValueError):
        return None


def oracle_subset(name):
    """Grids of the batch the oracle's stored run covers (all grids of a single-grid workload)."""
    if name != "batch256":
        return None
    try:
        return json.load(open(os.path.join(GOLDEN, "oracle_zhat_batch256_sub16.json")))["grids"]
    except (OSError, ValueError, KeyError):
        return None


SWEEP_MODE = {"auto": 0, "fused": 1, "sparse": 2, "tiled": 3}


def measure(inp, precision, steps, warmup, kernel_launches, torch, M, sweep_mode="auto", autotune=True):
    chains = CHAINS.get(inp.name, 1)
    n_equil, n_avg = SWEEPS[inp.name]
    P = sum(inp.n_pred) * chains
    updates_per_step = P * (n_equil + n_avg)
    stream = torch.cuda.Stream()
    # tile_rows = -1: the library's autotuner picks the sweep path, the fused path's rows per work
    # item, the tiled path's block shape and the sweeps per captured graph at the first load (a
    # warm-up step); later loads of the same shapes take the remembered choice
    ctx = M.Context(shapes=inp.shapes, stream=stream, precision=PREC[precision], n_chains=chains,
                    seed=inp.mc_seed, sweep_mode=SWEEP_MODE[sweep_mode],
                    tile_rows=-1 if autotune else 0)
    zhat = torch.empty(sum(inp.n_sites), dtype=torch.float64, device="cuda")
    # set-up (not a step): a first load, where the autotuner times its candidates once
    with torch.cuda.stream(stream):
        ctx.batch_load(inp.z, inp.m)
    torch.cuda.synchronize()

    # HIP events on the library's stream around each timed step's inference sweeps: the
    # inference sweep kernel's average duration over the timed region
    marks = []

    def step(timed=False):
        with torch.cuda.stream(stream):
            ctx.batch_load(inp.z, inp.m)
            if timed:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            ctx.infer_temperature(n_equil, want_T=False)
            if timed:
                e1.record(stream)
                marks.append((e0, e1))
            ctx.run(n_avg)
            ctx.predictions(out=zhat)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(timed=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / steps
    value = updates_per_step * steps / elapsed
    lattice_rate = sum(inp.n_sites) * chains * (n_equil + n_avg) * steps / elapsed
    log("%d steps of %s/%s: %.3f ms/step, %.4g site-updates/s"
        % (steps, inp.name, precision, ms_per_step, value))

    # prediction error against the synthetic truth, over every grid and over the grids of the
    # oracle's stored run (the paper's Delta MAAE: MAE relative to the FP64 oracle's, Sec. 3)
    zh = zhat.cpu().numpy()
    sub = oracle_subset(inp.name)
    sub = set(sub) if sub is not None else None
    abs_all, sq_all, n_all, abs_sub, n_sub, off = 0.0, 0.0, 0, 0.0, 0, 0
    for gi, (g, n) in enumerate(zip(inp.grids, inp.n_sites)):
        m = (g["mask"] == 0).ravel()
        err = zh[off:off + n][m] - g["truth"].ravel()[m]
        off += n
        abs_all += float(np.abs(err).sum())
        sq_all += float((err ** 2).sum())
        n_all += err.size
        if sub is None or gi in sub:
            abs_sub += float(np.abs(err).sum())
            n_sub += err.size
    mae, rmse = abs_all / n_all, float(np.sqrt(sq_all / n_all))
    phases = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in ctx.timings().items()}
    stats = ctx.stats()
    T_hat = [s["T"] for s in stats]
    clamped = sum(1 for t in T_hat if t <= T_MIN * (1 + 1e-12) or t >= T_MAX * (1 - 1e-12))

    # per inference sweep over the timed region (graph-captured launches, in-sweep control)
    kernel_ms = sum(a.elapsed_time(b) for a, b in marks) / (len(marks) * n_equil) if marks else None
    # and the sweep kernel launched back to back outside it, without graphs or control
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        ctx.bench_sweeps(2)
        ev0.record(stream)
        ctx.bench_sweeps(kernel_launches)
        ev1.record(stream)
    ev1.synchronize()
    kernel_ms_b2b = ev0.elapsed_time(ev1) / kernel_launches
    if kernel_ms is None:
        kernel_ms = kernel_ms_b2b
    tun = ctx.tuning()
    path = {M.SWEEP_SPARSE: "sparse", M.SWEEP_TILED: "tiled"}.get(tun[0], "fused")
    tuning = {"autotuned": autotune, "path": path, "rows_per_item": tun[1],
              "tile_shape": ["w4_base", "w8_tall", "w4_tall", "w8_base"][tun[2]] if tun[2] >= 0 else None,
              "graph_sweeps": tun[3]}
    kernel_name = {"sparse": "k_sparse<colour 0> + k_sparse<colour 1> (inference variant, one sweep)",
                   "tiled": "k_tiled (inference variant)"}.get(path, "k_sweep (inference variant)")
    s = BYTES[precision]
    alg_bytes = sum((n + 2 * p) * s for n, p in zip(inp.n_sites, inp.n_pred)) * chains
    gbs = alg_bytes / (kernel_ms * 1e-3) / 1e9
    ops = OPS_PER_UPDATE * P
    tops = ops / (kernel_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(tops, 3), "peak": round(ALU_PEAK_TOPS, 2),
                "unit": "T VALU lane-ops/s", "frac": round(tops / ALU_PEAK_TOPS, 4),
                "traffic": measured_traffic(inp.name, precision),
                "frac_single_issue": round(tops / ALU_SINGLE_ISSUE_TOPS, 4),
                "kernel": kernel_name, "kernel_ms": round(kernel_ms, 5),
                "kernel_ms_back_to_back": round(kernel_ms_b2b, 5),
                "ops_per_launch": ops, "ops_per_site_update": OPS_PER_UPDATE,
                "site_updates_per_launch": P,
                "hbm": {"achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_launch": alg_bytes}}
    ctx.close()
    out = {"workload": inp.name, "precision": precision, "value": value,
           "unit": "site-updates/s", "ms_per_step": ms_per_step, "steps": steps,
           "grids": len(inp.shapes), "sites": sum(inp.n_sites), "prediction_sites": sum(inp.n_pred),
           "chains": chains, "sweep_path": path, "tuning": tuning, "n_equil": n_equil, "n_avg": n_avg,
           "lattice_site_rate": lattice_rate, "mae": mae, "rmse": rmse,
           "T_hat": T_hat[:4], "T_hat_clamped": clamped, "phase_ms_last_step": phases,
           "roofline": roofline}
    ref = oracle_reference(inp.name, inp.p_missing)
    if ref is not None and chains == ref["chains"]:
        out["oracle_mae"] = ref["mae"]
        out["mae_oracle_grids"] = abs_sub / n_sub
        out["mae_vs_oracle"] = (abs_sub / n_sub) / ref["mae"] - 1.0
    return out


def streaming_copy_gbs(torch, mib=1024, reps=5):
    """Achieved HBM bandwidth of a device-to-device copy (bytes read + written per second)."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    gbs = 2.0 * n * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    log("streaming copy: %.0f GB/s" % gbs)
    return gbs


def _oracle_rate(O, grid, seed, chains, grid_id, threads, seconds):
    """Inference sweeps of the oracle on one grid: as many as fit in about `seconds` (calibrated
    on 2 sweeps); returns (site-updates/s, sweeps)."""
    n_pred = int((grid["mask"] == 0).sum())
    o = O.Oracle(seed=seed, n_chains=chains, grid_id=grid_id, n_threads=threads)
    o.load(grid["z"], grid["mask"])
    t = time.perf_counter()
    o.infer_temperature(2)
    per = (time.perf_counter() - t) / 2
    o.close()
    n = int(max(2, min(2000, seconds / max(per, 1e-9))))
    o = O.Oracle(seed=seed, n_chains=chains, grid_id=grid_id, n_threads=threads)
    o.load(grid["z"], grid["mask"])
    t = time.perf_counter()
    o.infer_temperature(n)
    dt = time.perf_counter() - t
    o.close()
    return n_pred * chains * n / dt, n


def cpu_baseline(inp, seconds):
    """The FP64 oracle on the host: the first inference sweeps of one grid of the workload with
    the workload's chains (for the batch, its grid whose side is nearest 512, with the batch's
    Philox chain words), timed on every core the process may use and on one core."""
    from oracle import oracle as O
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    chains = CHAINS.get(inp.name, 1)
    if inp.name == "batch256":
        gi = int(np.argmin([abs(g["mask"].shape[0] - 512) for g in inp.grids]))
    else:
        gi = 0
    grid = inp.grids[gi]
    rate, n = _oracle_rate(O, grid, inp.mc_seed, chains, gi, cores, seconds)
    rate1, n1 = _oracle_rate(O, grid, inp.mc_seed, chains, gi, 1, seconds)
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    H, W = grid["mask"].shape
    what = "grid %d of the workload (%dx%d, %d prediction sites), %d chain(s), FP64" % (
        gi, H, W, int((grid["mask"] == 0).sum()), chains)
    log("oracle: %.3g site-updates/s on %d cores, %.3g on one" % (rate, cores, rate1))
    return {"value": rate, "unit": "site-updates/s", "cores": cores, "kind": "oracle",
            "nproc": os.cpu_count(), "cpu_model": model,
            "sample": "first %d inference sweeps of %s" % (n, what),
            "single_thread": {"value": rate1, "cores": 1,
                              "sample": "first %d inference sweeps of %s" % (n1, what)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batch256", choices=sorted(SWEEPS))
    ap.add_argument("--precision", default="fp16", choices=sorted(PREC))
    ap.add_argument("--p-missing", type=float, default=None)
    ap.add_argument("--sweep-mode", default="auto", choices=sorted(SWEEP_MODE),
                    help="sweep path: automatic choice, fused row blocks, compacted site lists, or LDS tiles")
    ap.add_argument("--kernel-launches", type=int, default=20)
    ap.add_argument("--no-autotune", action="store_true",
                    help="the library's automatic rule instead of its autotuner")
    ap.add_argument("--setup-steps", type=int, default=3, help="timed steps of each secondary setup")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="oracle time per CPU-baseline run (all cores, then one core)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-setups", action="store_true", help="only the primary setup")
    ap.add_argument("--extended", action="store_true",
                    help="also the 4096^2 and 16384^2 single-grid workloads")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="copy a buffer of this many MiB once (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs the method on a single MI355X "
              "(--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1910_08448_amd import mpr as M

    torch.cuda.set_device(0)
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy probe: %d MiB read + %d MiB written" % (args.copy_probe_mib, args.copy_probe_mib))
        del a, b
    # (a counter run with a copy probe skips it: its copies would mix with the probe's counts)
    copy_gbs = streaming_copy_gbs(torch) if args.copy_probe_mib <= 0 else None
    inputs = {args.workload: Inputs(args.workload, args.p_missing, torch)}
    prim = measure(inputs[args.workload], args.precision, args.steps, args.warmup,
                   args.kernel_launches, torch, M, args.sweep_mode, not args.no_autotune)

    setups = []
    if not args.no_setups:
        todo = [(args.workload, p) for p in ("fp16", "fp32", "fp64") if p != args.precision]
        todo += [t for t in SETUPS if t[0] != args.workload]
        if args.extended:
            todo += EXTENDED
        for wl, prec in todo:
            if wl not in inputs:
                for k in list(inputs):
                    if k != args.workload:
                        del inputs[k]
                torch.cuda.empty_cache()
                inputs[wl] = Inputs(wl, None, torch)
            steps = max(1, min(args.steps, args.setup_steps))
            setups.append(measure(inputs[wl], prec, steps, 1, args.kernel_launches, torch, M,
                                  args.sweep_mode, not args.no_autotune))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(inputs[args.workload], args.cpu_seconds)

    fp64 = next((u for u in setups if u["workload"] == args.workload and u["precision"] == "fp64"), None)
    out = {
        "metric": "site-updates/s per precision setup (FP64/FP32/FP16) and prediction MAE vs FP64",
        "value": prim["value"], "unit": "site-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": prim["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": args.workload, "precision": args.precision,
                   "grids": prim["grids"], "sites": prim["sites"],
                   "prediction_sites": prim["prediction_sites"], "chains": prim["chains"],
                   "n_equil": prim["n_equil"], "n_avg": prim["n_avg"],
                   "sweep_path": prim["sweep_path"], "tuning": prim["tuning"]},
        "fp64_factor": (prim["value"] / fp64["value"]) if fp64 else None,
        "mae": prim["mae"], "rmse": prim["rmse"], "T_hat": prim["T_hat"],
        "T_hat_clamped": prim["T_hat_clamped"], "phase_ms_last_step": prim["phase_ms_last_step"],
        "roofline": prim["roofline"],
        "cpu_baseline": cpu,
        "setups": setups,
    }
    for k in ("oracle_mae", "mae_oracle_grids", "mae_vs_oracle", "lattice_site_rate"):
        if k in prim:
            out[k] = prim[k]
    # the second HBM denominator: what a plain device-to-device copy achieves on this GPU
    for r in [prim["roofline"]] + [u["roofline"] for u in setups]:
        h = r["hbm"]
        h["copy_gbs"] = round(copy_gbs, 1) if copy_gbs else None
        h["frac_of_copy"] = round(h["achieved"] / copy_gbs, 4) if copy_gbs else None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
