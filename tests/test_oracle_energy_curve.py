"""Pins of the oracle's second temperature reading: the energy-temperature curve of the
data-free model of Eq. (2) and its inversion at the sample energy (Sec. 2 infers T by matching
the sample energy; here the match is made against the unconditional model).

Fixed independently of the oracle's code: the exact mean energy of the 2 x 2 periodic lattice
(a four-cycle with doubled bonds) from a quadrature transfer matrix, the infinite-temperature
limit (independent uniform angles), equipartition of the harmonic limit at low temperature,
the monotonicity of e(T) (its derivative is a variance), and the inversion of curves with a
known inverse.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1910_08448_amd import synth


def _batch_mean_sigma(v, n_batches=50):
    b = v[: len(v) // n_batches * n_batches].reshape(n_batches, -1).mean(axis=1)
    return b.mean(), b.std(ddof=1) / math.sqrt(n_batches)


def _two_by_two_exact(T, q, J, n=160):
    """Mean bond energy of the periodic 2 x 2 lattice: every neighbour pair is joined by two
    bonds, so the weight is a product over the four edges of a cycle of exp(2 J cos(.) / T);
    <cos> of one edge = Tr(Kc K K K) / Tr(K^4) with Gauss-Legendre nodes on [0, 1)."""
    x, w = np.polynomial.legendre.leggauss(n)
    x, w = 0.5 * (x + 1.0), 0.5 * w
    c = np.cos(2.0 * math.pi * q * (x[:, None] - x[None, :]))
    a = 2.0 * J * c / T
    K = np.exp(a - a.max()) * np.sqrt(w[:, None] * w[None, :])
    K2 = K @ K
    return -J * np.trace((c * K) @ K @ K2) / np.trace(K2 @ K2)


@pytest.mark.parametrize("T,q,J", [(0.4, 0.5, 1.0), (1.5, 0.5, 1.0), (0.7, 0.3, 1.7)])
def test_two_by_two_matches_transfer_matrix(T, q, J):
    n_burn, n_meas = 200, 60000
    e, tr = O.energy_curve(2, [T], n_burn, n_meas, with_trace=True, q=q, J=J, seed=91)
    m, s = _batch_mean_sigma(tr[0, n_burn:, 0])
    exact = _two_by_two_exact(T, q, J)
    assert abs(e[0] - m) < 1e-12
    assert abs(m - exact) < 5.0 * s + 1e-4 * J, (m, exact, s)


@pytest.mark.parametrize("q,J", [(0.5, 1.0), (0.3, 1.7)])
def test_infinite_temperature_limit(q, J):
    """Independent uniform angles: E cos(2 pi q d) with d triangular on (-1, 1) equals
    (1 - cos 2 pi q) / (2 pi^2 q^2)."""
    e, tr = O.energy_curve(32, [1e4 * J], 100, 400, with_trace=True, q=q, J=J, seed=7,
                           T_max=1e5 * J)
    m, s = _batch_mean_sigma(tr[0, 100:, 0], 20)
    limit = -J * (1.0 - math.cos(2.0 * math.pi * q)) / (2.0 * math.pi ** 2 * q * q)
    assert abs(m - limit) < 5.0 * s + 2e-4 * J, (m, limit, s)


@pytest.mark.parametrize("q,J", [(0.5, 1.0), (0.3, 1.7)])
def test_low_temperature_equipartition(q, J):
    """Harmonic limit: N - 1 quadratic modes (the uniform shift costs nothing) share
    (N - 1) T / 2 over 2N bonds, so e + J = (T / 4)(1 - 1/N) up to O(T^2)."""
    side, T = 32, 1e-3 * J
    e = O.energy_curve(side, [T], 1000, 500, q=q, J=J, seed=3)
    N = side * side
    assert abs((e[0] + J) / (0.25 * T * (1.0 - 1.0 / N)) - 1.0) < 0.02


def test_curve_is_increasing():
    T = np.array([0.05, 0.15, 0.4, 1.0, 2.5])
    e, tr = O.energy_curve(16, T, 300, 300, with_trace=True, seed=17)
    assert np.all(np.diff(e) > 0)
    # every sweep ran at its chain's temperature
    assert np.array_equal(tr[:, :, 1], np.broadcast_to(T[:, None], tr.shape[:2]))
    assert np.allclose(e, tr[:, 300:, 0].mean(axis=1), rtol=0, atol=1e-15)


def test_curve_chains_are_independent_of_the_other_temperatures():
    """Chain i draws from its own Philox counter word, so its trajectory does not depend on the
    other points of the curve."""
    T = np.array([0.2, 0.6, 1.1])
    e3, tr3 = O.energy_curve(12, T, 20, 30, with_trace=True, seed=5)
    e1, tr1 = O.energy_curve(12, T[:1], 20, 30, with_trace=True, seed=5)
    assert np.array_equal(tr3[0], tr1[0]) and e3[0] == e1[0]


def test_inversion_of_known_curves():
    T = np.array([0.1, 0.2, 0.4, 0.8])
    e = -1.0 + 0.25 * T                                   # linear: exact inverse
    for t in (0.1, 0.13, 0.2, 0.31, 0.55, 0.8):
        assert O.curve_temperature(T, e, -1.0 + 0.25 * t) == pytest.approx(t, rel=1e-14)
    assert O.curve_temperature(T, e, -2.0) == 0.1          # clamped below
    assert O.curve_temperature(T, e, 0.0) == 0.8           # clamped above
    assert O.curve_temperature(T[:1], e[:1], -0.5) == 0.1  # a single point
    # a flat segment returns its low end; with a non-monotone curve the first bracket wins
    assert O.curve_temperature([1.0, 2.0, 3.0], [-1.0, -0.5, -0.5], -0.5) == 2.0
    assert O.curve_temperature([1.0, 2.0, 3.0], [-1.0, -0.2, -0.6], -0.6) == pytest.approx(1.5)


def test_method_with_curve_temperature():
    """Set T from the curve, then equilibrate at that fixed T and average: the temperature
    stays put, the window still adapts, and the predictions land near the data."""
    w = synth.workload("grid64")
    T = np.array([0.005, 0.01, 0.02, 0.05, 0.1, 0.2])
    e = O.energy_curve(32, T, 300, 200, seed=11)
    orc = O.Oracle(seed=w["mc_seed"], n_chains=2, n_threads=2, alpha0=0.5)
    orc.load(w["z"], w["mask"])
    Th = orc.set_temperature_curve(T, e)
    e_smp = orc.stats()[0]["e_sample"]
    assert np.all(Th == O.curve_temperature(T, e, e_smp))
    assert T[0] <= Th[0] <= T[-1]
    Tq = orc.equilibrate(60)
    assert np.array_equal(Tq, Th)
    for ch in range(2):
        tr = orc.trace(ch)
        assert tr.shape == (60, 4)
        assert np.all(tr[:, 1] == Th[ch])
        assert np.all(tr[:, 2] > 0) and tr[-1, 2] != 0.5
    orc.run(20)
    z = orc.predictions()
    m = w["mask"] == 0
    assert np.abs(z - w["truth"])[m].mean() < 0.5 * np.std(w["truth"])


def test_errors():
    with pytest.raises(O.OracleError) as ei:
        O.energy_curve(7, [1.0], 1, 1)
    assert ei.value.code == O.EBIPARTITE
    for bad in (dict(n_meas=0), dict(T=[0.0]), dict(T=[np.nan])):
        kw = dict(side=8, T=[1.0], n_burn=1, n_meas=1)
        kw.update(bad)
        with pytest.raises(O.OracleError) as ei:
            O.energy_curve(**kw)
        assert ei.value.code == O.EINVAL
    w = synth.workload("grid64")
    orc = O.Oracle()
    with pytest.raises(O.OracleError):
        orc.set_temperature_curve([1.0], [-0.5])          # nothing loaded
    orc.load(w["z"], w["mask"])
    with pytest.raises(O.OracleError) as ei:
        orc.equilibrate(5)                                 # no temperature yet
    assert ei.value.code == O.ESTATE
    with pytest.raises(O.OracleError) as ei:
        orc.set_temperature_curve([1.0, 1.0], [-0.9, -0.5])
    assert ei.value.code == O.EINVAL
