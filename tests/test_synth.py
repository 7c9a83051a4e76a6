"""Input generators: the synthetic fields have the covariance they claim, and masks remove
exactly the requested number of sites."""
import numpy as np

from paper_1910_08448_amd import synth


def test_grf_unit_variance_and_exponential_covariance():
    """nu = 1/2 Whittle-Matern in 2-D is the exponential covariance exp(-|h| / xi)
    (the paper's Sec. 3 data model); check lags 1..3 xi along both axes."""
    xi = 8.0
    acc = np.zeros(4)
    var = 0.0
    n = 8
    for s in range(n):
        g = synth.grf(256, 256, nu=0.5, xi=xi, seed=100 + s)
        var += g.var() / n
        for k, lag in enumerate([0, 8, 16, 24]):
            c = 0.5 * ((g * np.roll(g, lag, axis=0)).mean() + (g * np.roll(g, lag, axis=1)).mean())
            acc[k] += c / n
    assert abs(var - 1.0) < 0.05
    # the torus makes the covariance periodic; compare with the exponential within 0.06
    for k, lag in enumerate([0, 8, 16, 24]):
        assert abs(acc[k] - np.exp(-lag / xi)) < 0.06, (lag, acc[k], np.exp(-lag / xi))


def test_masks_exact_counts():
    m = synth.random_mask(50, 70, 0.33, seed=3)
    assert m.dtype == np.uint8 and set(np.unique(m)) <= {0, 1}
    assert (m == 0).sum() == round(0.33 * 50 * 70)
    g = synth.gap_mask(128, 96, 0.5, 8, seed=4)
    assert (g == 0).sum() == round(0.5 * 128 * 96)


def test_workload_hides_truth_at_prediction_sites():
    w = synth.workload("grid64")
    m = w["mask"] == 0
    assert np.all(np.isnan(w["z"][m])) and np.all(np.isfinite(w["z"][~m]))
    assert (m.sum()) == round(0.33 * 4096)
