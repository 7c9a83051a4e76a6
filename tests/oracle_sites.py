"""Sampled-site evaluation of one oracle sweep (test infrastructure): the oracle's single-site
hybrid update (Sec. 2) of chosen prediction sites, without sweeping the whole grid."""
import math

import numpy as np

from oracle import oracle as O

TWO_PI = 2.0 * math.pi


def oracle_sites(u, mask, sites, seed, sweep, chain_word, T, alpha):
    """Decision bits and new angles (turns) of the given prediction sites (y, x) after one sweep
    with Philox sweep index `sweep` from the state u (turns, H x W), on a 5 x 5 neighbourhood
    (clipped at the open edges): a colour-1 site sees its colour-0 neighbours' new angles, which
    are computed first, each with its own Philox words."""
    H, W = mask.shape
    dec = np.zeros(len(sites), np.uint8)
    new = np.zeros(len(sites))
    for k, (y, x) in enumerate(sites):
        y0, y1, x0, x1 = max(0, y - 2), min(H, y + 3), max(0, x - 2), min(W, x + 3)
        phi = np.ascontiguousarray(TWO_PI * u[y0:y1, x0:x1])
        m = mask[y0:y1, x0:x1]
        cy, cx = y - y0, x - x0
        if (x + y) & 1:
            for dy, dx in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                ny, nx = cy + dy, cx + dx
                if 0 <= ny < phi.shape[0] and 0 <= nx < phi.shape[1] and not m[ny, nx]:
                    wa, wb = O.site_words(seed, W, y + dy, x + dx, sweep, chain_word, 0)
                    O.site_update(phi, ny, nx, T, alpha, wa, wb)
        wa, wb = O.site_words(seed, W, y, x, sweep, chain_word, 0)
        dec[k] = O.site_update(phi, cy, cx, T, alpha, wa, wb)
        new[k] = phi[cy, cx] / TWO_PI
    return dec, new
