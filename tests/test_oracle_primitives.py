"""Pins of the FP64 oracle's primitives against values fixed independently of it.

Philox: published known-answer vectors, plus a cross-check against rocRAND's open-source
Philox4x32-10 when hipcc is present.  Energy: closed forms of Eq. (2) for configurations whose
bond sums are known exactly.  Map: exact endpoints and affine equivariance.  Over-relaxation:
closed-form reflection, energy conservation, involution.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TWO_PI = 2.0 * math.pi


# ---------------------------------------------------------------- Philox
def _kat():
    rows = []
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat())
def test_philox_known_answers(ctr, key, expect):
    assert list(O.philox(ctr, key)) == expect


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand(tmp_path):
    """rocRAND's Philox4x32-10 is an independent implementation: compare 256 random counters."""
    rng = np.random.default_rng(7)
    ctrs = rng.integers(0, 2**32, size=(256, 4), dtype=np.uint64)
    keys = rng.integers(0, 2**32, size=(256, 2), dtype=np.uint64)
    src = tmp_path / "r.cpp"
    src.write_text(
        "#include <rocrand/rocrand_philox4x32_10.h>\n#include <cstdio>\n"
        "struct E : rocrand_device::philox4x32_10_engine {\n"
        "  uint4 go(uint4 c, uint2 k) { return ten_rounds(c, k); } };\n"
        "int main() { E e; unsigned a[6];\n"
        "  while (scanf(\"%u %u %u %u %u %u\", a, a+1, a+2, a+3, a+4, a+5) == 6) {\n"
        "    uint4 r = e.go(uint4{a[0], a[1], a[2], a[3]}, uint2{a[4], a[5]});\n"
        "    printf(\"%u %u %u %u\\n\", r.x, r.y, r.z, r.w); } }\n")
    exe = tmp_path / "r"
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-O1", "-o", str(exe), str(src)],
                          stderr=subprocess.DEVNULL)
    inp = "\n".join(" ".join(str(int(v)) for v in list(c) + list(k)) for c, k in zip(ctrs, keys))
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(t) for t in l.split()] for l in out.strip().splitlines()], dtype=np.uint64)
    ours = np.array([O.philox(c, k) for c, k in zip(ctrs, keys)], dtype=np.uint64)
    assert np.array_equal(ours, ref)


def test_uniform_open_interval_and_moments():
    assert O.uniform(0) == 0.5 / 2**32
    assert O.uniform(2**32 - 1) == (2**32 - 0.5) / 2**32
    assert 0.0 < O.uniform(0) and O.uniform(2**32 - 1) < 1.0
    # uniform words from many distinct counters: mean 1/2, variance 1/12
    u = np.array([O.uniform(w) for c in range(4000)
                  for w in O.philox([c, 3, 5, 0], [11, 13])])
    assert abs(u.mean() - 0.5) < 4 * math.sqrt(1 / 12 / u.size)
    assert abs(u.var() - 1 / 12) < 0.005


def test_site_words_pairing_and_uniqueness():
    """Two neighbouring same-colour sites share one Philox call (words 0,1 and 2,3), and every
    (site, sweep, chain, tag) gets its own words."""
    seed, W = 0x1234_5678_9ABC_DEF0, 11
    key = [seed & 0xFFFFFFFF, seed >> 32]
    Wc = (W + 1) // 2
    NP = (Wc + 1) // 2
    seen = set()
    for y in range(5):
        for x in range(W):
            c = (x + y) & 1
            kx = x // 2
            for sweep, chain, tag in [(0, 0, 0), (3, 0, 0), (0, 2, 0), (0, 0, 1)]:
                wa, wb = O.site_words(seed, W, y, x, sweep, chain, tag)
                full = O.philox([y * NP + kx // 2, sweep, chain, (tag << 1) | c], key)
                pair = (full[0], full[1]) if kx % 2 == 0 else (full[2], full[3])
                assert (wa, wb) == pair
                seen.add((wa, wb))
    assert len(seen) == 5 * W * 4


# ---------------------------------------------------------------- energy, Eq. (2)
@pytest.mark.parametrize("H,W", [(4, 6), (6, 4), (8, 8)])
def test_uniform_configuration_energy(H, W):
    """All angles equal: every bond contributes cos 0 = 1.  Open: 2HW - H - W bonds;
    periodic: 2HW bonds, so H = -2 J N."""
    phi = np.full((H, W), 1.234)
    s, nb = O.bond_sum(phi, boundary=O.OPEN)
    assert nb == 2 * H * W - H - W and s == nb
    s, nb = O.bond_sum(phi, boundary=O.PERIODIC)
    assert nb == 2 * H * W and s == nb


def test_staggered_configuration_energy():
    """Checkerboard of 0 and 2 pi at q = 1/2: every bond has cos(pi) = -1."""
    H, W = 6, 8
    y, x = np.mgrid[0:H, 0:W]
    phi = np.where((x + y) % 2 == 0, 0.0, TWO_PI)
    s, nb = O.bond_sum(phi, boundary=O.PERIODIC, q=0.5)
    assert nb == 2 * H * W and s == -nb
    # at q = 1/4 every bond has cos(pi/2) = 0
    s, _ = O.bond_sum(phi, boundary=O.OPEN, q=0.25)
    assert abs(s) < 1e-12


def test_twisted_periodic_energy_closed_form():
    """phi = 2 pi x / W on a periodic H x W grid: vertical bonds give cos 0; horizontal bonds
    give cos(q 2pi/W) except the wrap bond, cos(q 2pi (W-1)/W).  Non-square and q = 0.3
    catch transposed indices and a wrong q."""
    H, W, q = 4, 10, 0.3
    x = np.arange(W)
    phi = np.tile(TWO_PI * x / W, (H, 1))
    s, nb = O.bond_sum(phi, boundary=O.PERIODIC, q=q)
    expect = H * W + H * ((W - 1) * math.cos(q * TWO_PI / W) + math.cos(q * TWO_PI * (W - 1) / W))
    assert nb == 2 * H * W
    assert abs(s - expect) < 1e-12 * abs(expect)


def test_sample_bond_mask():
    """Only bonds with both ends sampled count; a 3x3 open grid with the centre missing keeps
    the 8 perimeter bonds out of 12."""
    phi = np.full((3, 3), 0.7)
    mask = np.ones((3, 3), np.uint8)
    mask[1, 1] = 0
    s, nb = O.bond_sum(phi, mask=mask)
    assert nb == 8 and s == 8.0


def test_local_field_and_site_energy_by_hand():
    """Site (1, 2) of a 3x4 open grid has neighbours (1,1), (1,3), (0,2), (2,2)."""
    phi = np.zeros((3, 4))
    phi[1, 1], phi[1, 3], phi[0, 2], phi[2, 2] = 0.5, 1.0, 2.0, 4.0
    phi[0, 0] = 6.0  # not a neighbour
    q = 0.5
    C, S = O.local_field(phi, 1, 2, q=q)
    nbv = [0.5, 1.0, 2.0, 4.0]
    assert abs(C - sum(math.cos(q * v) for v in nbv)) < 1e-15
    assert abs(S - sum(math.sin(q * v) for v in nbv)) < 1e-15
    e = O.site_energy(phi, 1, 2, 3.0, q=q, J=2.0)
    assert abs(e - (-2.0 * sum(math.cos(q * (3.0 - v)) for v in nbv))) < 1e-14
    # site (2, 3) of a 4x5 grid: neighbours (2,2), (2,4), (1,3), (3,3)
    p45 = np.arange(20.0).reshape(4, 5) * 0.1
    C, S = O.local_field(p45, 2, 3, q=q)
    nbv = [p45[2, 2], p45[2, 4], p45[1, 3], p45[3, 3]]
    assert abs(C - sum(math.cos(q * v) for v in nbv)) < 1e-15
    assert abs(S - sum(math.sin(q * v) for v in nbv)) < 1e-15
    # corner (0, 0) of an open grid has two neighbours
    C, S = O.local_field(phi, 0, 0, q=q)
    assert abs(C - (math.cos(0) + math.cos(0))) < 1e-15 and S == 0.0
    # the same corner on a periodic 4x4 grid has four
    p4 = np.zeros((4, 4))
    p4[0, 3], p4[3, 0] = 1.0, 2.0
    C, S = O.local_field(p4, 0, 0, boundary=O.PERIODIC, q=q)
    assert abs(S - (math.sin(0.5) + math.sin(1.0))) < 1e-15


# ---------------------------------------------------------------- mapping
def test_map_endpoints_and_equivariance():
    rng = np.random.default_rng(3)
    z = rng.normal(50, 10, size=(7, 9))
    mask = (rng.random((7, 9)) > 0.4).astype(np.uint8)
    phi, lo, hi = O.map_data(z, mask)
    zs = z[mask == 1]
    assert lo == zs.min() and hi == zs.max()
    assert phi[mask == 1].min() == 0.0 and phi[mask == 1].max() == TWO_PI
    assert np.all(phi[mask == 0] == 0.0)
    # affine equivariance z -> a z + b (a > 0): identical angles up to rounding
    phi2, lo2, hi2 = O.map_data(3.0 * z - 7.0, mask)
    assert np.allclose(phi2, phi, rtol=0, atol=8 * np.finfo(float).eps * TWO_PI)
    # inverse map recovers the data
    back = lo + (hi - lo) * phi / TWO_PI
    assert np.allclose(back[mask == 1], z[mask == 1], rtol=4 * np.finfo(float).eps, atol=1e-12)


def test_map_errors():
    z = np.ones((3, 3))
    mask = np.ones((3, 3), np.uint8)
    with pytest.raises(O.OracleError) as e:
        O.map_data(z, mask)
    assert e.value.code == O.ENOSAMPLE
    z2 = np.arange(9.0).reshape(3, 3)
    z2[1, 1] = np.nan
    with pytest.raises(O.OracleError) as e:
        O.map_data(z2, mask)
    assert e.value.code == O.EINVAL
    z2[1, 1] = 4.0
    m2 = mask.copy()
    m2[0, 0] = 2
    with pytest.raises(O.OracleError) as e:
        O.map_data(z2, m2)
    assert e.value.code == O.EINVAL
    # NaN at a prediction site is fine
    m3 = mask.copy()
    m3[1, 1] = 0
    z2[1, 1] = np.nan
    O.map_data(z2, m3)


# ---------------------------------------------------------------- over-relaxation
def test_overrelax_closed_form_equal_neighbours():
    """All neighbours at phi0: psi = q phi0, the reflection is phi' = 2 phi0 - phi."""
    for q in (0.5, 0.3, 0.1):
        phi0 = 2.0
        C, S = 4 * math.cos(q * phi0), 4 * math.sin(q * phi0)
        v, applied = O.overrelax(1.5, C, S, q)
        assert applied and abs(v - 2.5) < 1e-13
        # reflection leaving [0, 2 pi] is refused
        v, applied = O.overrelax(5.0, C, S, q)
        assert not applied and v == 5.0


def test_overrelax_conserves_energy_and_is_involution():
    rng = np.random.default_rng(11)
    n_applied = 0
    for trial in range(500):
        q = [0.5, 0.4, 0.25][trial % 3]
        phi = rng.uniform(0, TWO_PI, size=(3, 3))
        C, S = O.local_field(phi, 1, 1, q=q)
        v, applied = O.overrelax(phi[1, 1], C, S, q)
        if not applied:
            assert v == phi[1, 1]
            continue
        n_applied += 1
        e0 = O.site_energy(phi, 1, 1, phi[1, 1], q=q)
        e1 = O.site_energy(phi, 1, 1, v, q=q)
        assert abs(e1 - e0) <= 1e-12 * max(1.0, abs(e0))
        w, again = O.overrelax(v, C, S, q)
        assert again and abs(w - phi[1, 1]) < 1e-12
    assert n_applied > 100


def test_overrelax_degenerate_field():
    v, applied = O.overrelax(1.0, 0.0, 0.0, 0.5)
    assert not applied and v == 1.0


def test_site_update_decisions():
    """Out-of-range proposals are rejected; downhill proposals are always accepted."""
    p4 = np.full((3, 3), 4.0)
    # word giving U_a - 1/2 = +0.4999...: proposal 4.0 + 2pi * 1.0 * 0.5 > 2 pi
    dec = O.site_update(p4, 1, 1, T=1.0, alpha=1.0, wa=2**32 - 1, wb=0)
    assert dec & O.DEC_OUTSIDE and not dec & O.DEC_ACCEPT and p4[1, 1] == 4.0
    # all neighbours at 4.0, site at 4.0: OR reflects 4.0 onto itself
    assert dec & O.DEC_OR
    phi = np.full((3, 3), 3.0)
    # site off the minimum, proposal towards it: accepted whatever U_b is
    phi[1, 1] = 4.0
    wa = int((0.5 - 0.5 / TWO_PI / 0.5) * 2**32)  # step of about -0.5 rad at alpha 0.5
    dec = O.site_update(phi, 1, 1, T=1e-3, alpha=0.5, wa=wa, wb=2**32 - 1)
    # OR first moves 4.0 -> 2.0 (reflection about 3.0), then the step goes to about 1.5:
    # uphill, so at T = 1e-3 it is rejected
    assert dec & O.DEC_OR and not dec & O.DEC_ACCEPT and abs(phi[1, 1] - 2.0) < 1e-12
    phi[1, 1] = 2.5
    wa_up = int((0.5 + 0.5 / TWO_PI / 0.5) * 2**32)  # step of about +0.5 rad
    dec = O.site_update(phi, 1, 1, T=1e-3, alpha=0.5, wa=wa_up, wb=2**32 - 1)
    # OR: 2.5 -> 3.5; step +0.5 -> 4.0: uphill, rejected; state stays 3.5
    assert abs(phi[1, 1] - 3.5) < 1e-12 and not dec & O.DEC_ACCEPT
    phi[1, 1] = 3.5
    dec = O.site_update(phi, 1, 1, T=1e-3, alpha=0.5, wa=wa_up, wb=2**32 - 1)
    # OR: 3.5 -> 2.5; step +0.5 -> 3.0 is downhill (to the minimum): accepted
    assert dec & O.DEC_ACCEPT and abs(phi[1, 1] - 3.0) < 1e-6


def test_init_uniform_and_samples_untouched():
    H, W = 64, 64
    mask = np.zeros((H, W), np.uint8)
    mask[::3, ::2] = 1
    phi = np.full((H, W), -1.0)
    O.init_chain(phi, mask, seed=99, chain=0)
    assert np.all(phi[mask == 1] == -1.0)
    v = phi[mask == 0]
    assert v.min() > 0 and v.max() < TWO_PI
    n = v.size
    assert abs(v.mean() - math.pi) < 4 * TWO_PI / math.sqrt(12 * n)
    assert abs(v.var() / (TWO_PI ** 2 / 12) - 1) < 0.05
    phi2 = np.full((H, W), -1.0)
    O.init_chain(phi2, mask, seed=99, chain=1)
    assert not np.array_equal(phi, phi2)
