"""GPU parity at the benchmark's full size, in the configuration bench.py times (the automatic
sweep path, graph-captured sweep loops): the 1024 x 1024 workload with 33 % and 66 % missing,
1000 inference + 100 averaging sweeps, one chain.

* Decisions of whole sweeps from identical states against the FP64 oracle (every site).
(Whole predictions against the oracle's stored runs of every benchmark workload are in
test_gpu_oracle_runs.py.)
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O                      # noqa: E402
from paper_1910_08448_amd import synth              # noqa: E402

TWO_PI = 2.0 * math.pi


@pytest.fixture(scope="module")
def mpr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_08448_amd import mpr as M
    return M


@pytest.fixture(scope="module")
def workloads():
    return {p: synth.workload("grid1024", seed=1, p_missing=p) for p in (0.33, 0.66)}


def _dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _ctx(mpr, w, **cfg):
    ctx = mpr.Context(stream=torch.cuda.Stream(), **cfg)
    ctx.load(_dev(w["z"], torch.float64), _dev(w["mask"], torch.uint8))
    return ctx


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_decisions_match_oracle(mpr, workloads, precision):
    """Two sweeps over all 1.05 M sites from the same random state at T = 0.02: FP64 takes the
    oracle's decisions on >= 99.999 % of the prediction sites with every angle to 1e-9, FP32 on
    >= 99.9 % with 99 % of the angles to 2e-5 (rounding of single-precision functions)."""
    w = workloads[0.33]
    mask = w["mask"]
    ctx = _ctx(mpr, w, seed=w["mc_seed"], precision=precision, alpha0=0.3)
    orc = O.Oracle(seed=w["mc_seed"], alpha0=0.3, n_threads=0)
    orc.load(w["z"], mask)
    u0 = synth.random_state(1, mask, 5)
    ctx.set_state(u=_dev(u0.reshape(-1), torch.float64))
    orc.set_state(phi=TWO_PI * u0)
    ctx.set_temperature(0.02)
    orc.set_temperature(0.02)
    free = mask == 0
    min_agree, tol = (0.99999, 1e-9) if precision == 0 else (0.999, 2e-5)
    for s in (3, 4):
        dg = ctx.debug_sweep(s).cpu().numpy().reshape(mask.shape)
        do = orc.debug_sweep(s).reshape(mask.shape)
        assert not dg[~free].any()
        assert (dg == do)[free].mean() >= min_agree
        ug = ctx.get_state()["u"].cpu().numpy().reshape(mask.shape)
        uo = orc.get_state()["phi"].reshape(mask.shape) / TWO_PI
        same = (dg == do) & free
        assert np.quantile(np.abs(ug - uo)[same], 0.99 if precision else 1.0) <= tol
        ctx.set_state(u=_dev(uo.reshape(-1), torch.float64))   # continue from the oracle's state
