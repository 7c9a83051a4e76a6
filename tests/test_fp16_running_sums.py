"""The arithmetic behind the 32-bit running sums of FP16 storage (CPU, numpy only).

With FP16 angle storage the averaging sweeps add each prediction site's new value, as a whole
number of 2^-24 units, into a 32-bit word, and the library folds the words into the FP64 running
sums (acc += word * 2^-24, word = 0) after at most 128 sweeps.  That equals adding every sweep's
value in double precision, bit for bit, because:
  * every FP16 value u in [0, 1] is a whole multiple of 2^-24, at most 2^24 of them;
  * 128 sweeps of at most 2^24 units stay below 2^32 (a 32-bit word does not wrap);
  * every partial sum of the double-precision running sum is a multiple of 2^-24 below 2^29
    (for fewer than 2^29 averaging sweeps), so it is exact, and so is the fold.
16-bit fixed point (u = k / 32767) is not a dyadic fraction: its double-precision running sums
round, and they differ from integer sums; that format keeps the FP64 sums.
"""
import numpy as np

UNIT = 2.0 ** -24
FOLD = 128                     # averaging sweeps between two folds, at most


def _fp16_in_unit_interval():
    bits = np.arange(0, 0x8000, dtype=np.uint16)          # sign bit clear (prediction sites)
    v = bits.view(np.float16).astype(np.float64)
    return v[np.isfinite(v) & (v <= 1.0)]


def test_every_fp16_value_in_the_unit_interval_is_a_whole_number_of_units():
    v = _fp16_in_unit_interval()
    units = v / UNIT
    assert np.array_equal(units, np.round(units))
    assert units.max() == 2.0 ** 24 and units.min() == 0.0
    # the smallest subnormal is one unit, the largest value below 1 is 2^24 - 2^13 units
    assert np.float16(2.0 ** -24).astype(np.float64) / UNIT == 1.0
    assert np.nextafter(np.float16(1.0), np.float16(0.0)).astype(np.float64) / UNIT == 2.0 ** 24 - 2.0 ** 13


def test_a_fold_period_of_values_fits_a_32_bit_word():
    assert FOLD * 2 ** 24 <= 2 ** 32 - 1
    assert FOLD * 2 ** 24 <= 2 ** 31          # even as a signed word


def test_folded_word_sums_equal_double_precision_running_sums():
    rng = np.random.default_rng(11)
    v = _fp16_in_unit_interval()
    for n_sweeps, calls in ((133, (130, 3)), (1100, (100, 1000)), (300, (1,) * 300), (257, (257,))):
        seq = rng.choice(v, size=(n_sweeps, 64))            # 64 sites, one value per sweep
        run = np.zeros(64)
        for row in seq:                                     # the FP64 path: one add per sweep
            run = run + row
        acc = np.zeros(64)
        word = np.zeros(64, dtype=np.uint32)
        done = 0
        for n in calls:                                     # one library run call of n sweeps
            for start in range(0, n, FOLD):
                for row in seq[done + start:done + min(start + FOLD, n)]:
                    word = word + (row / UNIT).astype(np.uint32)
                acc = acc + word.astype(np.float64) * UNIT  # the fold
                word[:] = 0
            done += n
        assert done == n_sweeps
        assert np.array_equal(acc, run)


def test_fixed_point_values_would_not_sum_exactly():
    """The premise fails for u = k / 32767: integer sums of k then one division differ from the
    double-precision running sum of the values for some sequences."""
    rng = np.random.default_rng(5)
    k = rng.integers(0, 32768, size=(200, 4096))
    run = np.zeros(4096)
    for row in k:
        run = run + row * (1.0 / 32767.0)
    exact = k.sum(axis=0) * (1.0 / 32767.0)
    assert not np.array_equal(run, exact)
