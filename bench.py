"""Benchmark of the MPR prediction path on one MI355X.

A step is one whole prediction of the workload through the C ABI, with the inputs already in
HBM: load (validation, data map, sample energy, initial state), temperature inference
(n_equil sweeps), averaging (n_avg sweeps) and the predictions.  `value` is site updates per
second over the whole step: one site update = one hybrid (over-relaxation + Metropolis) update
of one prediction site in one sweep of one chain.

Also printed in the same JSON line:
  roofline      the sweep kernel against the vector-ALU roof it is bound by: the method's
                arithmetic per site update (OPS_PER_UPDATE FP32-rate issue slots, see below)
                times the site updates of one launch, over the kernel's average launch time
                (HIP events on the library's stream); its algorithmic HBM bytes ((N + 2P) s per
                chain, s = bytes per angle) against the 8 TB/s HBM roof are reported beside it,
                and `traffic` is the HBM bytes per launch that rocprofv3 counted for the same
                kernel source (null when the kernel changed since the counters were taken)
  cpu_baseline  the FP64 CPU oracle timed on a bounded sample of the same workload
  setups        the same measurements for the other precision setups / workloads
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
# FP32 vector issue slots per second: 157.3 TFLOP/s counts a fused multiply-add as 2 flops
ALU_PEAK_TOPS = 157.3 / 2
# The method's arithmetic per site update, in FP32-rate issue slots (a transcendental and a
# 32 x 32 -> 64-bit multiply count 4, at a quarter of the rate): field sums 6, over-relaxation
# (atan2 16, reflection and range test 5) 21, (cos, sin) of the current angle 9, half a
# Philox4x32-10 call (10 rounds of two 4-slot multiplies and two xors) 50, Metropolis (two
# uniforms, proposal and range test, its (cos, sin), the energy change, exp, accept and
# select) 30, energy and acceptance sums 3.
OPS_PER_UPDATE = 119
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
PREC = {"fp64": 0, "fp32": 1, "fp16": 2, "fix16": 3}
BYTES = {"fp64": 8, "fp32": 4, "fp16": 2, "fix16": 2}
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16": "f32", "fix16": "f32"}   # arithmetic type of the sweep
SWEEPS = {"grid64": (256, 100), "grid1024": (1000, 100), "grid4096": (1000, 100),
          "grid16384": (500, 50), "batch256": (1000, 100)}
CHAINS = {"batch256": 4}
EXTENDED = [("grid4096", "fp16"), ("grid16384", "fp16"), ("grid16384", "fp32"),
            ("grid16384", "fp64"), ("batch256", "fp16"), ("batch256", "fp32")]


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


def oracle_reference(name, p_missing):
    path = os.path.join(ROOT, "tests", "golden", "oracle_reference.json")
    if name != "grid1024" or not os.path.exists(path):
        return None
    key = "grid1024_p%.2f" % (0.33 if p_missing is None else p_missing)
    return json.load(open(path)).get(key)


SWEEP_MODE = {"auto": 0, "fused": 1, "sparse": 2, "tiled": 3}


def measure(inp, precision, steps, warmup, kernel_launches, torch, M, sweep_mode="auto"):
    chains = CHAINS.get(inp.name, 1)
    n_equil, n_avg = SWEEPS[inp.name]
    P = sum(inp.n_pred) * chains
    updates_per_step = P * (n_equil + n_avg)
    stream = torch.cuda.Stream()
    ctx = M.Context(shapes=inp.shapes, stream=stream, precision=PREC[precision], n_chains=chains,
                    seed=inp.mc_seed, sweep_mode=SWEEP_MODE[sweep_mode])
    zhat = torch.empty(sum(inp.n_sites), dtype=torch.float64, device="cuda")
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

    zh = zhat.cpu().numpy()
    errs, off = [], 0
    for g, n in zip(inp.grids, inp.n_sites):
        m = (g["mask"] == 0).ravel()
        errs.append(zh[off:off + n][m] - g["truth"].ravel()[m])
        off += n
    err = np.concatenate(errs)
    mae, rmse = float(np.abs(err).mean()), float(np.sqrt((err ** 2).mean()))
    T_hat = [s["T"] for s in ctx.stats()]

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
    path = {M.SWEEP_SPARSE: "sparse", M.SWEEP_TILED: "tiled"}.get(ctx.sweep_mode(), "fused")
    kernel_name = {"sparse": "k_sparse<colour 0> + k_sparse<colour 1> (inference variant, one sweep)",
                   "tiled": "k_tiled (inference variant)"}.get(path, "k_sweep (inference variant)")
    s = BYTES[precision]
    alg_bytes = sum((n + 2 * p) * s for n, p in zip(inp.n_sites, inp.n_pred)) * chains
    gbs = alg_bytes / (kernel_ms * 1e-3) / 1e9
    ops = OPS_PER_UPDATE * P
    tops = ops / (kernel_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(tops, 3), "peak": ALU_PEAK_TOPS,
                "unit": "TOP/s", "frac": round(tops / ALU_PEAK_TOPS, 4),
                "traffic": measured_traffic(inp.name, precision),
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
           "chains": chains, "sweep_path": path, "n_equil": n_equil, "n_avg": n_avg,
           "lattice_site_rate": lattice_rate, "mae": mae, "rmse": rmse,
           "T_hat": T_hat[:4], "roofline": roofline}
    ref = oracle_reference(inp.name, inp.p_missing)
    if ref is not None and chains == ref["chains"]:
        out["oracle_mae"] = ref["mae"]
        out["mae_vs_oracle"] = mae / ref["mae"] - 1.0
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


def cpu_baseline(grid, seed, seconds):
    """The FP64 oracle on the host cores: inference sweeps of the same grid, as many as fit in
    about `seconds` (calibrated on 3 sweeps)."""
    from oracle import oracle as O
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    cores = max(1, min(cores, 16))
    n_pred = int((grid["mask"] == 0).sum())
    o = O.Oracle(seed=seed, n_threads=cores)
    o.load(grid["z"], grid["mask"])
    t = time.perf_counter()
    o.infer_temperature(3)
    per = (time.perf_counter() - t) / 3
    n = int(max(3, min(2000, seconds / max(per, 1e-9))))
    o2 = O.Oracle(seed=seed, n_threads=cores)
    o2.load(grid["z"], grid["mask"])
    t = time.perf_counter()
    o2.infer_temperature(n)
    dt = time.perf_counter() - t
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    return {"value": n_pred * n / dt, "unit": "site-updates/s", "cores": cores, "kind": "oracle",
            "cpu_model": model,
            "sample": "first %d inference sweeps of grid 0 (%dx%d, %d prediction sites), 1 chain, FP64"
                      % (n, grid["z"].shape[0], grid["z"].shape[1], n_pred)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="grid1024", choices=sorted(SWEEPS))
    ap.add_argument("--precision", default="fp32", choices=sorted(PREC))
    ap.add_argument("--p-missing", type=float, default=None)
    ap.add_argument("--sweep-mode", default="auto", choices=sorted(SWEEP_MODE),
                    help="sweep path: automatic choice, fused row blocks, compacted site lists, or LDS tiles")
    ap.add_argument("--kernel-launches", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-setups", action="store_true", help="only the primary setup")
    ap.add_argument("--extended", action="store_true",
                    help="also the 4096^2, 16384^2 and 256-grid batched workloads")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="copy a buffer of this many MiB once (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs the method on a single MI355X "
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
                   args.kernel_launches, torch, M, args.sweep_mode)

    setups = []
    if not args.no_setups:
        todo = [(args.workload, p) for p in ("fp64", "fp32", "fp16") if p != args.precision]
        if args.extended:
            todo += EXTENDED
        for wl, prec in todo:
            if wl not in inputs:
                for k in list(inputs):
                    if k != args.workload:
                        del inputs[k]
                torch.cuda.empty_cache()
                inputs[wl] = Inputs(wl, None, torch)
            steps = max(1, min(args.steps, 3)) if wl != args.workload else args.steps
            setups.append(measure(inputs[wl], prec, steps, 1, args.kernel_launches, torch, M,
                                  args.sweep_mode))

    cpu = None
    if not args.no_cpu_baseline:
        g0 = inputs[args.workload].grids[0]
        cpu = cpu_baseline(g0, inputs[args.workload].mc_seed, args.cpu_seconds)

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
                   "sweep_path": prim["sweep_path"]},
        "mae": prim["mae"], "rmse": prim["rmse"], "T_hat": prim["T_hat"],
        "roofline": prim["roofline"],
        "cpu_baseline": cpu,
        "setups": setups,
    }
    for k in ("oracle_mae", "mae_vs_oracle", "lattice_site_rate"):
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
