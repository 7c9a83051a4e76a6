"""The sampled-site evaluation used by the full-size GPU tests reproduces the oracle's whole
checkerboard sweep (Sec. 2) site for site, so its sampled comparisons are comparisons with the
oracle itself."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle_sites import oracle_sites
from paper_1910_08448_amd import synth


@pytest.mark.parametrize("H,W,p,T,alpha", [(40, 52, 0.4, 0.02, 0.3), (9, 7, 0.6, 0.5, 1.0), (33, 64, 0.9, 0.1, 0.6)])
def test_sampled_sites_reproduce_the_whole_sweep(H, W, p, T, alpha):
    rng = np.random.default_rng(H * W)
    mask = synth.random_mask(H, W, p, H + W)
    u = synth.random_state(2, mask, 9)
    u = np.where(mask == 1, rng.random((H, W)), u)
    seed, sweep = 2001, 3
    for ch in range(2):
        phi = np.ascontiguousarray(2.0 * math.pi * u[ch])
        dec = np.zeros((H, W), np.uint8)
        O.sweep(phi, mask, T, alpha, seed, sweep, chain=7 + ch, decisions=dec)
        free = np.argwhere(mask == 0)
        sites = [tuple(map(int, s)) for s in free]
        d, new = oracle_sites(u[ch], mask, sites, seed, sweep, 7 + ch, T, alpha)
        assert np.array_equal(d, dec[free[:, 0], free[:, 1]])
        assert np.array_equal(new, phi[free[:, 0], free[:, 1]] / (2.0 * math.pi))
        assert (d & O.DEC_ACCEPT).any() and (d & O.DEC_OR).any()
