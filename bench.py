"""Benchmark of the MPR prediction path on one MI355X.

A step is one whole prediction of the workload through the C ABI, with the inputs already in
HBM: load (validation, data map, sample energy, initial state), temperature inference
(n_equil sweeps), averaging (n_avg sweeps) and the predictions.  `value` is site updates per
second over the whole step: one site update = one hybrid (over-relaxation + Metropolis) update
of one prediction site in one sweep of one chain.

Also printed in the same JSON line:
  roofline      the sweep kernel's algorithmic HBM bytes per launch (other colour read, own
                prediction sites read and written: (N + 2P) s per chain, s = bytes per angle)
                over its average launch time, measured with HIP events on the library's stream
  cpu_baseline  the FP64 CPU oracle timed on a bounded sample of the same workload
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
PREC = {"fp64": 0, "fp32": 1, "fp16": 2}
BYTES = {"fp64": 8, "fp32": 4, "fp16": 2}
SWEEPS = {"grid64": (256, 100), "grid1024": (1000, 100), "grid4096": (1000, 100),
          "grid16384": (500, 50), "batch256": (1000, 100)}


def make_inputs(name, p_missing):
    if name == "batch256":
        grids = synth.batch_workload(256, 64, 1024, seed=1)
        return {"grids": grids, "mc_seed": 2001}
    w = synth.workload(name, seed=1, p_missing=p_missing)
    return {"grids": [w], "mc_seed": w["mc_seed"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="grid1024", choices=sorted(SWEEPS))
    ap.add_argument("--precision", default="fp32", choices=sorted(PREC))
    ap.add_argument("--p-missing", type=float, default=None)
    ap.add_argument("--chains", type=int, default=None)
    ap.add_argument("--kernel-launches", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs the method on a single MI355X "
              "(--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1910_08448_amd import mpr as M

    torch.cuda.set_device(0)
    n_equil, n_avg = SWEEPS[args.workload]
    chains = args.chains or (4 if args.workload == "batch256" else 1)
    inp = make_inputs(args.workload, args.p_missing)
    grids = inp["grids"]
    shapes = [g["z"].shape for g in grids]
    z_d = torch.as_tensor(np.concatenate([g["z"].ravel() for g in grids])).cuda()
    m_d = torch.as_tensor(np.concatenate([g["mask"].ravel() for g in grids])).cuda()
    n_sites = [h * w for h, w in shapes]
    n_pred = [int((g["mask"] == 0).sum()) for g in grids]
    P = sum(n_pred) * chains
    sweeps = n_equil + n_avg
    updates_per_step = P * sweeps

    stream = torch.cuda.Stream()
    ctx = M.Context(shapes=shapes, stream=stream, precision=PREC[args.precision],
                    n_chains=chains, seed=inp["mc_seed"])
    zhat = torch.empty(sum(n_sites), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    def step():
        with torch.cuda.stream(stream):
            ctx.batch_load(z_d, m_d)
            ctx.infer_temperature(n_equil, want_T=False)
            ctx.run(n_avg)
            ctx.predictions(out=zhat)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = updates_per_step * args.steps / elapsed
    print("[bench] %d steps of %s/%s: %.3f ms/step, %.4g site-updates/s"
          % (args.steps, args.workload, args.precision, ms_per_step, value), file=sys.stderr, flush=True)

    # accuracy of the last step against the truth
    zh = zhat.cpu().numpy()
    errs, sq = [], []
    off = 0
    for g, n in zip(grids, n_sites):
        m = (g["mask"] == 0).ravel()
        d = zh[off:off + n][m] - g["truth"].ravel()[m]
        errs.append(np.abs(d))
        off += n
    err = np.concatenate(errs)
    mae = float(err.mean())
    rmse = float(np.sqrt((err ** 2).mean()))
    stats = ctx.stats()
    T_hat = [s["T"] for s in stats]

    # sweep-kernel timing with HIP events on the library's stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    nl = args.kernel_launches
    with torch.cuda.stream(stream):
        ctx.bench_sweeps(2)
        ev0.record(stream)
        ctx.bench_sweeps(nl)
        ev1.record(stream)
    ev1.synchronize()
    kernel_ms = ev0.elapsed_time(ev1) / nl
    s = BYTES[args.precision]
    alg_bytes = sum((n + 2 * p) * s for n, p in zip(n_sites, n_pred)) * chains
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_sweep (inference variant)", "kernel_ms": round(kernel_ms, 5),
                "bytes_per_launch": alg_bytes}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(grids[0], inp["mc_seed"], args.cpu_seconds)

    out = {
        "metric": "site-updates/s per precision setup (FP64/FP32/FP16) and prediction MAE vs FP64",
        "value": value, "unit": "site-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f16"}[args.precision],
        "data": "synthetic",
        "config": {"workload": args.workload, "precision": args.precision,
                   "grids": len(shapes), "sites": sum(n_sites), "prediction_sites": sum(n_pred),
                   "chains": chains, "n_equil": n_equil, "n_avg": n_avg},
        "mae": mae, "rmse": rmse, "T_hat": T_hat[:4],
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


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
    return {"value": n_pred * n / dt, "unit": "site-updates/s", "cores": cores, "kind": "oracle",
            "sample": "first %d inference sweeps of grid 0 (%dx%d, %d prediction sites), 1 chain, FP64"
                      % (n, grid["z"].shape[0], grid["z"].shape[1], n_pred)}


if __name__ == "__main__":
    main()
