"""Pins of the oracle's sampler, temperature inference and predictions.

Each test compares the oracle with something fixed independently of its code: quadrature of
the exact conditional density of one or two free spins, equipartition at low temperature,
recovery of a known temperature from a configuration drawn at that temperature, the ground
state of Eq. (2) (a linear ramp, and the root of the stationarity equations found by a
library solver) as the low-temperature limit, bitwise resume, thread-count invariance.
"""
import math

import numpy as np
import pytest
import scipy.optimize
import scipy.sparse
import scipy.sparse.linalg

from oracle import oracle as O
from paper_1910_08448_amd import synth

TWO_PI = 2.0 * math.pi


def _gauss_legendre(a, b, n_sub=64, n=24):
    x, w = np.polynomial.legendre.leggauss(n)
    edges = np.linspace(a, b, n_sub + 1)
    xs, ws = [], []
    for lo, hi in zip(edges[:-1], edges[1:]):
        xs.append(0.5 * (hi - lo) * x + 0.5 * (hi + lo))
        ws.append(0.5 * (hi - lo) * w)
    return np.concatenate(xs), np.concatenate(ws)


def _batch_mean_sigma(v, n_batches=50):
    b = v[: len(v) // n_batches * n_batches].reshape(n_batches, -1).mean(axis=1)
    return b.mean(), b.std(ddof=1) / math.sqrt(n_batches)


# ---------------------------------------------------------------- one free spin
CASES_ONE = [
    # T, q, neighbour data in [0, 1], alpha
    (0.1, 0.5, [0.2, 0.3, 0.25, 0.4], 0.2),
    (1.0, 0.5, [0.1, 0.9, 0.5, 0.3], 1.0),
    (0.05, 0.25, [0.02, 0.05, 0.0, 0.1], 0.1),
    (5.0, 0.5, [0.0, 1.0, 0.5, 0.5], 1.0),
    (0.3, 0.4, [0.7, 0.95, 0.8, 0.6], 0.5),
]


@pytest.mark.parametrize("T,q,nb,alpha", CASES_ONE)
def test_single_free_spin_matches_quadrature(T, q, nb, alpha):
    """3x3 open grid, only the centre free: p(phi) ~ exp(J sum_j cos[q(phi - phi_j)] / T) on
    [0, 2 pi].  Mean and second moment of the chain within 3 batch-means sigma."""
    z = np.full((3, 3), 0.5)
    z[0, 0], z[2, 2] = 0.0, 1.0           # fixes the map to phi = 2 pi z
    z[1, 0], z[1, 2], z[0, 1], z[2, 1] = nb
    mask = np.ones((3, 3), np.uint8)
    mask[1, 1] = 0
    o = O.Oracle(q=q, seed=12345, alpha0=alpha, n_threads=1)
    o.load(z, mask)
    o.set_temperature(T)
    o.burn_in(200)
    s = o.run_record(200000, [4])[:, 0]
    phij = TWO_PI * np.array(nb)
    x, w = _gauss_legendre(0.0, TWO_PI)
    logp = np.cos(q * (x[:, None] - phij[None, :])).sum(axis=1) / T
    p = w * np.exp(logp - logp.max())
    p /= p.sum()
    m1, m2 = (p * x).sum(), (p * x * x).sum()
    e1, s1 = _batch_mean_sigma(s)
    e2, s2 = _batch_mean_sigma(s * s)
    assert abs(e1 - m1) < 3 * s1, (e1, m1, s1)
    assert abs(e2 - m2) < 3 * s2, (e2, m2, s2)


def test_single_free_spin_high_temperature_limit():
    """T -> infinity: uniform on [0, 2 pi], mean pi and variance pi^2 / 3."""
    z = np.full((3, 3), 0.5)
    z[0, 0], z[2, 2] = 0.0, 1.0
    mask = np.ones((3, 3), np.uint8)
    mask[1, 1] = 0
    o = O.Oracle(seed=77, alpha0=1.0, n_threads=1, T_max=1e9)
    o.load(z, mask)
    o.set_temperature(1e8)
    s = o.run_record(100000, [4])[:, 0]
    e1, s1 = _batch_mean_sigma(s)
    assert abs(e1 - math.pi) < 3 * s1
    assert abs(s.var() / (math.pi ** 2 / 3) - 1) < 0.02


# ---------------------------------------------------------------- two free spins
@pytest.mark.parametrize("q,J", [(0.5, 1.0), (0.3, 1.7)])
def test_two_free_spins_match_2d_quadrature(q, J):
    """3x4 open grid with (1,1) and (1,2) free: joint density by 2-D quadrature;
    E[phi1], E[phi2] and E[phi1 phi2] within 3 sigma (also for q < 1/2 and J != 1)."""
    T = 0.25
    z = np.full((3, 4), 0.5)
    z[0, 0], z[2, 3] = 0.0, 1.0
    z[1, 0], z[0, 1], z[2, 1] = 0.1, 0.3, 0.2      # fixed neighbours of (1,1)
    z[1, 3], z[0, 2], z[2, 2] = 0.8, 0.6, 0.7      # fixed neighbours of (1,2)
    mask = np.ones((3, 4), np.uint8)
    mask[1, 1] = mask[1, 2] = 0
    o = O.Oracle(q=q, J=J, seed=4242, alpha0=0.5, n_threads=1)
    o.load(z, mask)
    o.set_temperature(T)
    o.burn_in(500)
    s = o.run_record(200000, [5, 6])
    a = TWO_PI * np.array([0.1, 0.3, 0.2])
    b = TWO_PI * np.array([0.8, 0.6, 0.7])
    x, w = _gauss_legendre(0.0, TWO_PI, n_sub=40, n=16)
    la = np.cos(q * (x[:, None] - a[None, :])).sum(axis=1)
    lb = np.cos(q * (x[:, None] - b[None, :])).sum(axis=1)
    L = J * (la[:, None] + lb[None, :] + np.cos(q * (x[:, None] - x[None, :]))) / T
    P = w[:, None] * w[None, :] * np.exp(L - L.max())
    P /= P.sum()
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    for f, exact in [(s[:, 0], (P * X1).sum()), (s[:, 1], (P * X2).sum()),
                     (s[:, 0] * s[:, 1], (P * X1 * X2).sum())]:
        e, sig = _batch_mean_sigma(f)
        assert abs(e - exact) < 3 * sig, (e, exact, sig)


# ---------------------------------------------------------------- temperature
def test_low_temperature_equipartition():
    """Unconditional periodic lattice at T << J: bond energy e + J = T/4 (harmonic spin waves
    of the XY model in theta = q phi), up to O(T) and the missing zero mode."""
    H = W = 64
    T = 0.02
    phi = np.full((H, W), math.pi)
    free = np.zeros((H, W), np.uint8)
    es = []
    for s in range(800):
        O.sweep(phi, free, T, 0.05, seed=5, sweep_index=s, boundary=O.PERIODIC, n_threads=4)
        if s >= 300:
            tot, nb = O.bond_sum(phi, boundary=O.PERIODIC)
            es.append(1.0 - tot / nb)            # e + J with J = 1
    expect = T / 4 * (H * W - 1) / (H * W)
    assert abs(np.mean(es) / expect - 1) < 0.03, (np.mean(es), expect)


@pytest.mark.parametrize("T0", [0.05, 0.3])
def test_temperature_recovery(T0):
    """Draw an equilibrium configuration of Eq. (2) at T0 (two sites pinned at 0 and 2 pi so
    the data map is the identity), remove 33 % of the other sites, infer: T_hat = T0."""
    H = W = 64
    rng = np.random.default_rng(17)
    pins = np.zeros((H, W), np.uint8)
    pins[10, 10] = pins[42, 42] = 1
    phi = np.full((H, W), math.pi)
    phi[10, 10], phi[42, 42] = 0.0, TWO_PI
    for s in range(3000):
        O.sweep(phi, pins, T0, 0.1 if T0 < 0.1 else 0.3, seed=9, sweep_index=s,
                boundary=O.PERIODIC, n_threads=4)
    mask = (rng.random((H, W)) >= 0.33).astype(np.uint8)
    mask[10, 10] = mask[42, 42] = 1
    o = O.Oracle(boundary=O.PERIODIC, seed=31, n_threads=4)
    o.load(phi, mask)
    T = o.infer_temperature(2000)[0]
    assert abs(T / T0 - 1) < 0.05, (T, T0)


def test_window_control_reaches_target_acceptance():
    w = synth.workload("grid64")
    o = O.Oracle(seed=w["mc_seed"], n_threads=2)
    o.load(w["z"], w["mask"])
    o.infer_temperature(300)
    tr = o.trace()
    A = tr[150:, 3]
    alpha = tr[150:, 2]
    assert np.all((alpha > 1e-3) & (alpha < 1.0))
    assert abs(A.mean() - 0.3) < 0.02


# ---------------------------------------------------------------- predictions
def _fixed_T_predict(z, mask, T, n_equil, n_avg, **kw):
    o = O.Oracle(T_min=T, T_max=T, **kw)      # clamped temperature: fixed-T run, alpha adapts
    o.load(z, mask)
    o.infer_temperature(n_equil)
    o.run(n_avg)
    return o.predictions()


def test_ramp_is_reproduced_at_low_temperature():
    """z = x is a ground state of Eq. (2) (every free site sits at the angle of its local
    field); at low T the prediction is the ramp."""
    H, W = 12, 24
    rng = np.random.default_rng(5)
    z = np.tile(np.arange(W, dtype=float), (H, 1))
    mask = (rng.random((H, W)) >= 0.33).astype(np.uint8)
    mask[:, 0] = mask[:, -1] = 1
    zhat = _fixed_T_predict(z, mask, 1e-3, 500, 500, seed=3, n_threads=1)
    err = np.abs(zhat - z)[mask == 0]
    assert err.max() < 0.1 and err.mean() < 0.03, (err.max(), err.mean())
    assert np.array_equal(zhat[mask == 1], z[mask == 1])


def _smooth_field(H, W):
    y, x = np.mgrid[0:H, 0:W]
    return 10 + 3 * np.sin(2 * np.pi * x / (2.3 * W)) * np.cos(2 * np.pi * y / (1.7 * H)) + 0.05 * x


def _neighbours(i, H, W):
    y, x = divmod(i, W)
    out = []
    if x > 0: out.append(i - 1)
    if x < W - 1: out.append(i + 1)
    if y > 0: out.append(i - W)
    if y < H - 1: out.append(i + W)
    return out


def _harmonic(values, mask, H, W):
    """Discrete harmonic interpolation: sum_j (v_i - v_j) = 0 at free sites, samples fixed."""
    free = np.flatnonzero(mask.ravel() == 0)
    pos = {s: k for k, s in enumerate(free)}
    A = scipy.sparse.lil_matrix((free.size, free.size))
    b = np.zeros(free.size)
    for k, i in enumerate(free):
        for j in _neighbours(i, H, W):
            A[k, k] += 1
            if j in pos:
                A[k, pos[j]] -= 1
            else:
                b[k] += values.ravel()[j]
    return free, scipy.sparse.linalg.spsolve(A.tocsr(), b)


def test_low_temperature_limit_is_ground_state():
    """At T -> 0 the mean configuration is the minimum of Eq. (2) with the samples fixed:
    sum_j sin[q(phi_i - phi_j)] = 0 at every free site (solved with scipy from the harmonic
    starting point)."""
    H, W, q = 20, 20, 0.5
    z = _smooth_field(H, W)
    rng = np.random.default_rng(8)
    mask = (rng.random((H, W)) >= 0.33).astype(np.uint8)
    zhat = _fixed_T_predict(z, mask, 1e-5, 1500, 500, seed=4, n_threads=1)
    phi, lo, hi = O.map_data(z, mask)
    free, x0 = _harmonic(phi, mask, H, W)
    base = phi.ravel().copy()
    nb = [_neighbours(i, H, W) for i in free]

    def F(v):
        full = base.copy()
        full[free] = v
        return np.array([sum(math.sin(q * (full[i] - full[j])) for j in n) for i, n in zip(free, nb)])

    sol = scipy.optimize.root(F, x0, tol=1e-13)
    assert sol.success and np.all((sol.x >= 0) & (sol.x <= TWO_PI))
    zg = lo + (hi - lo) * sol.x / TWO_PI
    err = np.abs(zhat.ravel()[free] - zg)
    assert err.max() < 2e-3 * (hi - lo), (err.max(), hi - lo)


def test_low_temperature_limit_near_harmonic_interpolation():
    """For small angle differences the ground state is the discrete harmonic interpolation of
    the samples (sparse Laplace solve), up to O((q dphi)^2)."""
    H, W = 20, 20
    z = _smooth_field(H, W)
    rng = np.random.default_rng(8)
    mask = (rng.random((H, W)) >= 0.33).astype(np.uint8)
    zhat = _fixed_T_predict(z, mask, 1e-5, 1500, 500, seed=4, n_threads=1)
    free, zh = _harmonic(z, mask, H, W)
    rng_z = z[mask == 1].max() - z[mask == 1].min()
    assert np.abs(zhat.ravel()[free] - zh).max() < 0.01 * rng_z


def test_predictions_within_sample_range_and_samples_exact():
    w = synth.workload("grid64")
    zhat, T = O.predict(w["z"], w["mask"], 100, 50, seed=w["mc_seed"], n_threads=2)
    m = w["mask"] == 1
    assert np.array_equal(zhat[m], w["z"][m])
    lo, hi = w["z"][m].min(), w["z"][m].max()
    assert zhat.min() >= lo and zhat.max() <= hi
    # and it predicts: better than the sample mean by a wide margin
    mae = np.abs(zhat - w["truth"])[~m].mean()
    mae_mean = np.abs(w["z"][m].mean() - w["truth"])[~m].mean()
    assert mae < 0.5 * mae_mean


def test_affine_equivariance_of_predictions():
    w = synth.workload("grid64")
    a, _ = O.predict(w["z"], w["mask"], 60, 20, seed=7, n_threads=1)
    b, _ = O.predict(2.5 * w["z"] + 11.0, w["mask"], 60, 20, seed=7, n_threads=1)
    m = w["mask"] == 0
    assert np.allclose(b[m], 2.5 * a[m] + 11.0, rtol=1e-9, atol=1e-9)


# ---------------------------------------------------------------- determinism, resume
def test_resume_is_bitwise():
    w = synth.workload("grid64")
    kw = dict(seed=w["mc_seed"], n_threads=1, n_chains=2)
    A = O.Oracle(**kw); A.load(w["z"], w["mask"]); A.infer_temperature(100); A.run(60)
    B = O.Oracle(**kw); B.load(w["z"], w["mask"]); B.infer_temperature(100); B.run(25)
    st = B.get_state()
    C = O.Oracle(**kw); C.load(w["z"], w["mask"]); C.set_state(**st); C.run(35)
    assert np.array_equal(A.predictions(), C.predictions())
    D = O.Oracle(**kw); D.load(w["z"], w["mask"]); D.infer_temperature(100)
    E = O.Oracle(**kw); E.load(w["z"], w["mask"]); E.set_state(**D.get_state()); E.run(60)
    assert np.array_equal(A.predictions(), E.predictions())


def test_thread_count_does_not_change_results():
    w = synth.workload("grid64", p_missing=0.66)
    a, Ta = O.predict(w["z"], w["mask"], 80, 30, seed=5, n_threads=1)
    b, Tb = O.predict(w["z"], w["mask"], 80, 30, seed=5, n_threads=5)
    assert np.array_equal(a, b) and np.array_equal(Ta, Tb)


def test_chains_average_of_single_chains():
    """Two chains in one context equal two one-chain runs with the matching chain counters."""
    w = synth.workload("grid64")
    two, T2 = O.predict(w["z"], w["mask"], 60, 20, seed=5, n_threads=1, n_chains=2)
    c0, T0 = O.predict(w["z"], w["mask"], 60, 20, seed=5, n_threads=1, n_chains=1, grid_id=0)
    c1, T1 = O.predict(w["z"], w["mask"], 60, 20, seed=5, n_threads=1, n_chains=1, grid_id=1)
    assert T2[0] == T0[0] and T2[1] == T1[0]
    m = w["mask"] == 0
    assert np.allclose(two[m], 0.5 * (c0[m] + c1[m]), rtol=1e-13, atol=1e-12)


# ---------------------------------------------------------------- errors
def _code(fn):
    with pytest.raises(O.OracleError) as e:
        fn()
    return e.value.code


def test_error_codes():
    z = np.arange(16.0).reshape(4, 4)
    m = np.ones((4, 4), np.uint8)
    m[1, 1] = 0
    for kw in [dict(q=0.6), dict(q=0.0), dict(J=0.0), dict(n_chains=0), dict(alpha0=0.0),
               dict(acc_target=1.0), dict(T_min=0.0), dict(T_min=2.0, T_max=1.0)]:
        assert _code(lambda: O.Oracle(**kw)) == O.EINVAL
    o = O.Oracle()
    assert _code(lambda: o.load(np.zeros((1, 4)), np.ones((1, 4), np.uint8))) == O.EINVAL
    assert _code(lambda: o.load(np.ones((4, 4)), m)) == O.ENOSAMPLE
    checker = ((np.add.outer(np.arange(4), np.arange(4)) % 2) == 0).astype(np.uint8)
    assert _code(lambda: o.load(z, checker)) == O.ENOSAMPLE      # no sample-sample bond
    p = O.Oracle(boundary=O.PERIODIC)
    assert _code(lambda: p.load(np.arange(15.0).reshape(3, 5), np.ones((3, 5), np.uint8))) == O.EBIPARTITE
    o.load(z, m)
    assert _code(lambda: o.run(5)) == O.ESTATE
    assert _code(lambda: o.predictions()) == O.ESTATE
    assert _code(lambda: o.infer_temperature(-1)) == O.EINVAL
    o.set_temperature(0.1)
    o.run(0)
    assert _code(lambda: o.predictions()) == O.ESTATE
    o.run(2)
    o.predictions()
