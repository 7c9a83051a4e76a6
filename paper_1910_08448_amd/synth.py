"""Seeded synthetic inputs: random fields, missing-data masks and the workloads built on them.

This module holds no arithmetic of the prediction method; it only draws inputs.  Both the
GPU path's tests and benchmark and the CPU oracle's tests take their inputs from here.

Fields follow the paper's synthetic-data setup (Sec. 3: Gaussian data with an exponential
covariance on square grids, a fraction of the sites removed at random), generalised to the
Whittle-Matern family: in two dimensions the spectral density (kappa^2 + |k|^2)^-(nu + 1)
with nu = 1/2 gives the exponential covariance sigma^2 exp(-kappa |h|), kappa = 1/xi.
"""
import os

import numpy as np


def grf(H, W, nu=0.5, xi=8.0, seed=1):
    """Zero-mean, unit-variance stationary Gaussian field on an H x W torus by FFT spectral
    synthesis with the Whittle-Matern density (kappa^2 + |k|^2)^-(nu+1), kappa = 1/xi."""
    import scipy.fft
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((H, W))
    ky = 2.0 * np.pi * np.fft.fftfreq(H)
    kx = 2.0 * np.pi * np.fft.rfftfreq(W)          # half spectrum of a real field
    kappa = 1.0 / xi
    S = (kappa * kappa + ky[:, None] ** 2 + kx[None, :] ** 2) ** (-(nu + 1.0))
    # mean of S over the full spectrum: interior columns of the half spectrum appear twice
    w = np.full(kx.size, 2.0)
    w[0] = 1.0
    if W % 2 == 0:
        w[-1] = 1.0
    S /= (S * w[None, :]).sum() / (H * W)           # unit variance
    workers = min(16, os.cpu_count() or 1)
    spec = scipy.fft.rfft2(noise, workers=workers)
    del noise
    spec *= np.sqrt(S)
    del S
    return scipy.fft.irfft2(spec, s=(H, W), workers=workers)


def gaussian_field(H, W, nu=0.5, xi=8.0, mean=50.0, std=10.0, seed=1):
    return mean + std * grf(H, W, nu, xi, seed)


def lognormal_field(H, W, nu=1.0, xi=64.0, log_std=0.5, seed=1):
    return np.exp(log_std * grf(H, W, nu, xi, seed))


def random_mask(H, W, p_missing, seed):
    """1 = sample (kept), 0 = prediction site; exactly round(p N) sites are removed."""
    N = H * W
    n_miss = int(round(p_missing * N))
    rng = np.random.default_rng(seed)
    mask = np.ones(N, dtype=np.uint8)
    mask[rng.choice(N, size=n_miss, replace=False)] = 0
    return mask.reshape(H, W)


def gap_mask(H, W, p_missing, gap, seed):
    """Square gaps of side `gap` at uniform random corners (clipped, overlaps allowed) until
    at least half of the missing budget is covered, then random sites up to exactly
    round(p N) missing sites."""
    N = H * W
    n_miss = int(round(p_missing * N))
    rng = np.random.default_rng(seed)
    mask = np.ones((H, W), dtype=np.uint8)
    covered = 0
    while covered < n_miss // 2:
        y0 = int(rng.integers(0, H))
        x0 = int(rng.integers(0, W))
        block = mask[y0:y0 + gap, x0:x0 + gap]
        take = int(block.sum())
        if covered + take > n_miss:
            break
        block[...] = 0
        covered += take
    flat = mask.reshape(-1)
    rest = np.flatnonzero(flat)
    need = n_miss - covered
    flat[rng.choice(rest, size=need, replace=False)] = 0
    return mask


def random_state(n_chains, mask, seed):
    """Synthetic spin state in revolutions: uniform on [0, 1] at prediction sites (mask 0),
    0 at sample sites; shape [n_chains, H, W]."""
    rng = np.random.default_rng(seed)
    u = rng.random((n_chains,) + mask.shape)
    u[:, mask == 1] = 0.0
    return u


# ---------------------------------------------------------------- named workloads
def workload(name, seed=1, p_missing=None):
    """Returns dict(z, truth, mask, ...) for the named workloads.

    grid64:     64x64 Gaussian (nu 1/2, xi 8, mean 50, std 10), 33 % missing at random.
    grid1024:   1024x1024 Gaussian (nu 1/2, xi 32), 33 % (or p_missing) missing at random.
    grid4096:   4096x4096 lognormal (nu 1, xi 64, log-std 0.5), 50 % missing, 32x32 gaps.
    grid16384:  16384x16384 lognormal (nu 1, xi 128, log-std 0.5), 50 % missing, 256x256 gaps.
    """
    if name == "grid64":
        truth = gaussian_field(64, 64, 0.5, 8.0, 50.0, 10.0, seed)
        mask = random_mask(64, 64, 0.33 if p_missing is None else p_missing, seed + 1000)
    elif name == "grid1024":
        truth = gaussian_field(1024, 1024, 0.5, 32.0, 50.0, 10.0, seed)
        mask = random_mask(1024, 1024, 0.33 if p_missing is None else p_missing, seed + 1000)
    elif name == "grid4096":
        truth = lognormal_field(4096, 4096, 1.0, 64.0, 0.5, seed)
        mask = gap_mask(4096, 4096, 0.5 if p_missing is None else p_missing, 32, seed + 1000)
    elif name == "grid16384":
        truth = lognormal_field(16384, 16384, 1.0, 128.0, 0.5, seed).astype(np.float64)
        mask = gap_mask(16384, 16384, 0.5 if p_missing is None else p_missing, 256, seed + 1000)
    else:
        raise ValueError("unknown workload %r" % name)
    z = np.where(mask == 1, truth, np.nan)
    return {"name": name, "truth": truth, "z": z, "mask": mask, "mc_seed": seed + 2000}


def batch_workload(n_grids=256, lo=64, hi=1024, seed=1):
    """Many independent square grids: sides uniform in [lo, hi]; even-indexed grids Gaussian
    (nu 1/2, xi = L/32), odd-indexed lognormal (nu 1, xi = L/16, log-std 0.5); missing
    fraction uniform in [0.2, 0.7], random sites."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(lo, hi + 1, size=n_grids)
    fracs = rng.uniform(0.2, 0.7, size=n_grids)
    grids = []
    for g in range(n_grids):
        L = int(sides[g])
        s = seed * 100003 + g
        if g % 2 == 0:
            truth = gaussian_field(L, L, 0.5, L / 32.0, 50.0, 10.0, s)
        else:
            truth = lognormal_field(L, L, 1.0, L / 16.0, 0.5, s)
        mask = random_mask(L, L, float(fracs[g]), s + 1000)
        grids.append({"truth": truth, "z": np.where(mask == 1, truth, np.nan), "mask": mask})
    return grids
