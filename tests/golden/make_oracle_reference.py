"""Writes the FP64 CPU oracle's reference runs of the benchmark workloads into tests/golden/.

For every workload the whole method runs on the host (map, temperature inference, averaging,
predictions) with the benchmark's sweep counts, chains and Monte Carlo seed, and the file
records the prediction error against the synthetic truth (MAE, RMSE: the quantities behind the
paper's Delta MAAE comparison, Sec. 3 and Eq. (4)), the temperature estimate of every chain and
the predictions at a fixed, seeded sample of prediction sites:

  oracle_reference.json            summary of every workload (MAE, RMSE, T_hat, seconds)
  oracle_zhat_<key>.json           the summary plus sampled sites: flat site index and z_hat

Workloads (keys):
  grid1024_p0.33, grid1024_p0.66   1024^2 Gaussian, 33 % / 66 % missing, 1000 + 100 sweeps
  grid4096                         4096^2 lognormal, 50 % missing with 32^2 gaps, 1000 + 100
  batch256_sub16                   16 grids of the 256-grid batch (g = 16 k + (k & 1): both
                                   field kinds), 4 chains each, 1000 + 100; a grid's chains use
                                   the batch's Philox chain words (grid index g), so each grid
                                   equals the same grid inside the whole batch
  grid16384                        16384^2 lognormal, 50 % missing with 256^2 gaps, 500 + 50

Calls only the oracle and the shared input generators.  Usage:
  python tests/golden/make_oracle_reference.py [key ...]     (default: every workload)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O            # noqa: E402
from paper_1910_08448_amd import synth    # noqa: E402

BATCH_SUBSET = [16 * k + (k & 1) for k in range(16)]
SAMPLE_SEED = 4242
N_SAMPLE = 20000          # sampled prediction sites of a single-grid workload
N_SAMPLE_GRID = 1000      # per grid of the batch subset


def sample_sites(mask, n, seed):
    """Sorted flat indices of min(n, P) prediction sites, drawn without replacement."""
    pred = np.flatnonzero(mask.ravel() == 0)
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(pred, size=min(n, pred.size), replace=False))


def run_grid(z, mask, truth, n_equil, n_avg, seed, chains=1, grid_id=0, n_sample=N_SAMPLE,
             sample_seed=SAMPLE_SEED):
    t = time.time()
    o = O.Oracle(seed=seed, n_chains=chains, grid_id=grid_id, n_threads=0)
    o.load(z, mask)
    T = o.infer_temperature(n_equil)
    o.run(n_avg)
    zhat = o.predictions()
    st = o.stats()
    o.close()
    m = mask == 0
    err = zhat[m] - truth[m]
    idx = sample_sites(mask, n_sample, sample_seed)
    return {
        "mae": float(np.abs(err).mean()), "rmse": float(np.sqrt((err ** 2).mean())),
        "abs_err_sum": float(np.abs(err).sum()), "sq_err_sum": float((err ** 2).sum()),
        "n_pred": int(m.sum()), "T_hat": [float(x) for x in T],
        "e_smp": st[0]["e_sample"], "e_sim_last": [s["e_sim"] for s in st],
        "data_range": float(st[0]["zmax"] - st[0]["zmin"]),
        "n_equil": n_equil, "n_avg": n_avg, "chains": chains, "mc_seed": seed, "grid_id": grid_id,
        "seconds": round(time.time() - t, 1),
        "sample_index": [int(i) for i in idx],
        "sample_zhat": [float(v) for v in zhat.ravel()[idx]],
    }


def single(name, p_missing, n_equil, n_avg):
    w = synth.workload(name, seed=1, p_missing=p_missing)
    r = run_grid(w["z"], w["mask"], w["truth"], n_equil, n_avg, w["mc_seed"])
    r["workload"] = name
    r["p_missing"] = p_missing
    return r


def batch_subset():
    grids = synth.batch_workload(256, 64, 1024, seed=1)
    t = time.time()
    per = []
    for g in BATCH_SUBSET:
        w = grids[g]
        r = run_grid(w["z"], w["mask"], w["truth"], 1000, 100, 2001, chains=4, grid_id=g,
                     n_sample=N_SAMPLE_GRID, sample_seed=SAMPLE_SEED + g)
        r["grid"] = g
        r["side"] = int(w["mask"].shape[0])
        per.append(r)
        print("  grid %d (side %d): mae %.6g T %s %.1f s" % (g, r["side"], r["mae"], r["T_hat"],
                                                         r["seconds"]), flush=True)
    n = sum(r["n_pred"] for r in per)
    return {"workload": "batch256", "grids": BATCH_SUBSET, "chains": 4, "n_equil": 1000,
            "n_avg": 100, "mc_seed": 2001, "n_pred": n,
            "mae": sum(r["abs_err_sum"] for r in per) / n,
            "rmse": float(np.sqrt(sum(r["sq_err_sum"] for r in per) / n)),
            "seconds": round(time.time() - t, 1), "per_grid": per}


JOBS = {
    "grid1024_p0.33": lambda: single("grid1024", 0.33, 1000, 100),
    "grid1024_p0.66": lambda: single("grid1024", 0.66, 1000, 100),
    "grid4096": lambda: single("grid4096", None, 1000, 100),
    "batch256_sub16": batch_subset,
    "grid16384": lambda: single("grid16384", None, 500, 50),
}


def main():
    keys = sys.argv[1:] or list(JOBS)
    summary_path = os.path.join(HERE, "oracle_reference.json")
    for key in keys:
        print("running %s" % key, flush=True)
        r = JOBS[key]()
        with open(os.path.join(HERE, "oracle_zhat_%s.json" % key), "w") as f:
            json.dump(r, f, separators=(",", ":"))
        summary = json.load(open(summary_path)) if os.path.exists(summary_path) else {}
        summary[key] = {k: r[k] for k in ("mae", "rmse", "n_equil", "n_avg", "chains", "mc_seed",
                                          "seconds", "n_pred") if k in r}
        summary[key]["T_hat"] = r["T_hat"] if "T_hat" in r else [x for g in r["per_grid"]
                                                                 for x in g["T_hat"]]
        with open(summary_path, "w") as f:
            json.dump(summary, f, indent=1)
        print("%s: mae %.9g rmse %.9g (%.1f s)" % (key, r["mae"], r["rmse"], r["seconds"]), flush=True)


if __name__ == "__main__":
    main()
