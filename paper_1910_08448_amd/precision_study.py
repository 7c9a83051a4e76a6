"""The paper's precision study on MI355X (Sec. 2-3, Fig. 1 and Fig. 2), through the C ABI.

Data as in Sec. 3: Gaussian Z ~ N(50, 10) with the exponential covariance of Eq. (3),
kappa = 0.2 (correlation length 5 sites), 90 % of the sites removed at random.  The eight
settings X_S X_E X_F (spins, energy, functions in double D or single S precision; single-
precision functions are the hardware sin/cos/exp instructions) are run, plus two 16-bit spin
storages.  The paper does not state its sweep counts; 1000 inference + 100 averaging sweeps
are used here, one chain.

  speedup   R_X = t_DDD / t_X for L = 2^k, k = 5 ... 12 (Fig. 1; time of a whole prediction)
  accuracy  Delta MAAE_X = (MAAE_X / MAAE_DDD - 1) * 100 % over M missing-data realisations of
            one field (Fig. 2; MAAE = mean over realisations of the AAE of Eq. (4)), with the
            standard error of the paired difference

Usage: python -m paper_1910_08448_amd.precision_study [--sizes 32,...] [--M 100] [--L-acc 256]
Prints one JSON document.
"""
import argparse
import json
import sys
import time

import numpy as np

from . import synth

SETTINGS = {"DDD": (0, 0, 0), "DSD": (0, 1, 0), "DDS": (0, 0, 1), "SDD": (1, 0, 0),
            "SDS": (1, 0, 1), "DSS": (0, 1, 1), "SSD": (1, 1, 0), "SSS": (1, 1, 1),
            "HDS": (2, 0, 1), "FDS": (3, 0, 1)}


def _field(L, seed):
    return synth.gaussian_field(L, L, 0.5, 5.0, 50.0, 10.0, seed)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="32,64,128,256,512,1024,2048,4096")
    ap.add_argument("--M", type=int, default=100)
    ap.add_argument("--L-acc", type=int, default=256)
    ap.add_argument("--n-equil", type=int, default=1000)
    ap.add_argument("--n-avg", type=int, default=100)
    ap.add_argument("--reps", type=int, default=2)
    args = ap.parse_args()

    import torch
    from . import mpr as M
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()

    def predict(z, mask, setting, seed, ctx_cache):
        key = (z.shape, setting)
        if key not in ctx_cache:
            s, e, f = SETTINGS[setting]
            ctx_cache[key] = M.Context(shapes=[z.shape], stream=stream, precision=s, energy_prec=e,
                                       func_prec=f, seed=seed)
        ctx = ctx_cache[key]
        with torch.cuda.stream(stream):
            ctx.batch_load(z, mask)
            ctx.infer_temperature(args.n_equil, want_T=False)
            ctx.run(args.n_avg)
            zh = ctx.predictions()
        # the caller reads the predictions on its own stream
        torch.cuda.current_stream().wait_stream(stream)
        zh.record_stream(torch.cuda.current_stream())
        return zh

    out = {"n_equil": args.n_equil, "n_avg": args.n_avg, "missing": 0.9, "kappa": 0.2,
           "speedup": {}, "accuracy": {}}
    # ---- Fig. 1: time of a whole prediction per setting and size
    for L in [int(v) for v in args.sizes.split(",")]:
        truth = _field(L, 1)
        mask = synth.random_mask(L, L, 0.9, 1001)
        z = torch.as_tensor(np.where(mask == 1, truth, np.nan)).cuda()
        m = torch.as_tensor(mask).cuda()
        cache, times = {}, {}
        for name in SETTINGS:
            predict(z, m, name, 2001, cache)          # warm-up (allocation, graph capture)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(args.reps):
                predict(z, m, name, 2001, cache)
            torch.cuda.synchronize()
            times[name] = (time.perf_counter() - t) / args.reps
        for c in cache.values():
            c.close()
        out["speedup"][L] = {"t_ms": {k: 1e3 * v for k, v in times.items()},
                             "R": {k: times["DDD"] / v for k, v in times.items()}}
        print("[study] L=%d R_SSS=%.2f R_HDS=%.2f" % (L, times["DDD"] / times["SSS"],
                                                       times["DDD"] / times["HDS"]),
              file=sys.stderr, flush=True)
    # ---- Fig. 2: MAAE over M missing-data realisations of one field
    L = args.L_acc
    truth = _field(L, 7)
    z_true = torch.as_tensor(truth).cuda()
    aae = {k: [] for k in SETTINGS}
    cache = {}
    for r in range(args.M):
        mask = synth.random_mask(L, L, 0.9, 5000 + r)
        m = torch.as_tensor(mask).cuda()
        z = torch.where(m == 1, z_true, torch.full_like(z_true, float("nan")))
        pm = (m == 0).flatten()
        for name in SETTINGS:
            zh = predict(z, m, name, 9000 + r, cache)
            aae[name].append(float((zh[pm] - z_true.flatten()[pm]).abs().mean()))
        if (r + 1) % 10 == 0:
            print("[study] accuracy: %d of %d realisations" % (r + 1, args.M), file=sys.stderr, flush=True)
    for c in cache.values():
        c.close()
    base = np.array(aae["DDD"])
    for name in SETTINGS:
        a = np.array(aae[name])
        rel = (a / base - 1.0) * 100.0
        out["accuracy"][name] = {"MAAE": float(a.mean()),
                                 "dMAAE_pct": float((a.mean() / base.mean() - 1.0) * 100.0),
                                 "dMAAE_paired_se_pct": float(rel.std(ddof=1) / np.sqrt(len(rel)))}
    out["accuracy_L"] = L
    out["M"] = args.M
    print(json.dumps(out))


if __name__ == "__main__":
    main()
