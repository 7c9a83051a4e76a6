"""Writes tests/golden/oracle_reference.json: prediction errors of the FP64 CPU oracle on the
1024x1024 workload (33 % and 66 % missing, 1000 inference + 100 averaging sweeps, one chain).

Calls only the oracle and the shared input generators.  The benchmark compares the GPU
setups' MAE against these values (the paper's Delta MAAE, Sec. 3)."""
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


def main():
    out = {}
    for p in (0.33, 0.66):
        w = synth.workload("grid1024", seed=1, p_missing=p)
        t = time.time()
        zhat, T = O.predict(w["z"], w["mask"], 1000, 100, seed=w["mc_seed"], n_threads=0)
        m = w["mask"] == 0
        err = zhat[m] - w["truth"][m]
        out["grid1024_p%.2f" % p] = {
            "mae": float(np.abs(err).mean()), "rmse": float(np.sqrt((err ** 2).mean())),
            "T_hat": float(T[0]), "n_equil": 1000, "n_avg": 100, "chains": 1,
            "mc_seed": w["mc_seed"], "seconds": round(time.time() - t, 1)}
        print(p, out["grid1024_p%.2f" % p], flush=True)
    with open(os.path.join(HERE, "oracle_reference.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
