"""The single-precision atan2 of the GPU kernels (Abramowitz & Stegun 4.4.49 polynomial after an
octant reduction) against libm, evaluated on the CPU in float32 with the coefficients read
from the kernel source, so a mistyped coefficient or a wrong octant rule fails here."""
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1910_08448_amd", "csrc", "mpr_device.hpp")


def _kernel_atan2():
    text = open(SRC).read()
    body = text[text.index("static __device__ __forceinline__ float atan2(float y, float x)"):]
    body = body[:body.index("\n    }\n")]
    first = float(re.search(r"float p = ([-0-9.e]+)f;", body).group(1))
    coefs = [float(v) for v in re.findall(r"__builtin_fmaf\(p, t2, ([-0-9.e]+)f\)", body)]
    assert len(coefs) == 7
    f = np.float32

    def atan2(y, x):
        y = y.astype(f)
        x = x.astype(f)
        ax = np.abs(x)
        mx, mn = np.maximum(ax, y), np.minimum(ax, y)
        t = (mn * (f(1) / mx)).astype(f)
        t2 = (t * t).astype(f)
        p = np.full_like(t, f(first))
        for c in coefs:
            p = (p * t2 + f(c)).astype(f)
        r = (t * t2 * p + t).astype(f)
        r = np.where(y > ax, f(np.pi / 2) - r, r).astype(f)
        return np.where(x < 0, f(np.pi) - r, r).astype(f)

    return atan2


def test_fast_atan2_against_libm():
    rng = np.random.default_rng(0)
    y = np.abs(rng.normal(size=200000)) * 10 ** rng.uniform(-3, 1, 200000)
    x = rng.normal(size=200000) * 10 ** rng.uniform(-3, 1, 200000)
    # and the octant boundaries
    y = np.concatenate([y, [1.0, 1.0, 0.0, 0.0, 2.0, 3.0]])
    x = np.concatenate([x, [1.0, -1.0, 1.0, -1.0, 0.0, -3.0]])
    got = _kernel_atan2()(y, x).astype(np.float64)
    ref = np.arctan2(y, x)
    err = np.abs(got - ref)
    assert err.max() < 1e-6, err.max()
    assert np.all((got >= 0) & (got <= np.float32(np.pi)))
