"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle.

FP64 setups must reproduce the oracle's per-site decisions (over-relaxation applied,
Metropolis accepted) on >= 99.999 % of sites from an identical state, its new angles to
1e-9, its per-sweep energy / temperature / window trace, and its predictions to
MAE <= 1e-3 of the data range.  FP32 and FP16 setups are compared statistically: decisions
from an identical state, and prediction MAE against the truth within 1 % of the oracle's.
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


def _dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _field(H, W, seed, p=0.33):
    truth = synth.gaussian_field(H, W, 0.5, 8.0, 50.0, 10.0, seed)
    mask = synth.random_mask(H, W, p, seed + 1000)
    z = np.where(mask == 1, truth, np.nan)
    return truth, z, mask


def _gpu_ctx(mpr, z, mask, **cfg):
    ctx = mpr.Context(stream=torch.cuda.Stream(), **cfg)
    ctx.load(_dev(z, torch.float64), _dev(mask, torch.uint8))
    return ctx


def _decisions_case(mpr, H, W, boundary, n_chains, precision, seed, T=0.08, alpha=0.4, sweeps=3,
                    mode=1, p=0.33, **gpu_cfg):
    truth, z, mask = _field(H, W, seed, p=p)
    kw = dict(boundary=boundary, n_chains=n_chains, seed=seed + 5, alpha0=alpha)
    ctx = _gpu_ctx(mpr, z, mask, precision=precision, sweep_mode=mode, **kw, **gpu_cfg)
    orc = O.Oracle(n_threads=2, **kw)
    orc.load(z, mask)
    u0 = synth.random_state(n_chains, mask, seed + 7)
    ctx.set_state(u=_dev(u0.reshape(-1), torch.float64))
    orc.set_state(phi=TWO_PI * u0)
    ctx.set_temperature(T)
    orc.set_temperature(T)
    out = []
    before = (orc.get_state()["phi"] / TWO_PI).reshape(n_chains, H, W)   # samples included
    for s in range(sweeps):
        dg = ctx.debug_sweep(11 + s).cpu().numpy().reshape(n_chains, H, W)
        do = orc.debug_sweep(11 + s)
        ug = ctx.get_state()["u"].cpu().numpy().reshape(n_chains, H, W)
        uo = orc.get_state()["phi"] / TWO_PI
        out.append((dg, do, ug, uo))
        _LAST_BEFORE.append(before)
        before = uo.reshape(n_chains, H, W)
        # continue both from the oracle's state so each sweep is compared from identical input
        ctx.set_state(u=_dev(uo.reshape(-1), torch.float64))
    return mask, out


@pytest.mark.parametrize("H,W,boundary,chains", [
    (64, 64, 0, 1), (37, 53, 0, 2), (70, 130, 0, 1), (16, 24, 1, 1), (130, 244, 0, 1)])
def test_fp64_decisions_and_angles_match_oracle(mpr, H, W, boundary, chains):
    mask, rounds = _decisions_case(mpr, H, W, boundary, chains, mpr.FP64, seed=H * 31 + W)
    free = np.broadcast_to(mask == 0, rounds[0][0].shape)
    for dg, do, ug, uo in rounds:
        assert np.array_equal(dg[~free], do[~free]) and not dg[~free].any()
        same = (dg == do)[free]
        assert same.mean() >= 0.99999, same.mean()
        assert (dg[free] & mpr.DEC_ACCEPT).any() and (dg[free] & mpr.DEC_OR).any()
        agree = free & (dg == do)
        assert np.abs(ug - uo)[agree].max() <= 1e-9
        assert np.array_equal(ug[~free] * 0, uo[~free] * 0)


_LAST_BEFORE = []


def _degenerate_sites(mask, before, after, boundary):
    """Free sites whose local field vanishes up to rounding (|C| + |S| < 1e-12), and the colour-1
    sites next to a degenerate colour-0 site.  The field of neighbours at exactly half a turn
    apart (the extreme samples map to 0 and 1) is exactly zero in turns, where the device
    evaluates it, but sin of the radian angle fl(pi) is 1.2e-16, so the two sides may take
    different (each valid) over-relaxation decisions there; elsewhere they must agree."""
    C, H, W = before.shape
    bad = np.zeros((C, H, W), bool)
    for ch in range(C):
        for y in range(H):
            for x in range(W):
                if mask[y, x]:
                    continue
                phi = TWO_PI * (before[ch] if (x + y) % 2 == 0 else after[ch])
                c, s = O.local_field(np.ascontiguousarray(phi), y, x, boundary=boundary)
                if abs(c) + abs(s) < 1e-12:
                    bad[ch, y, x] = True
        for y in range(H):
            for x in range(W):
                if bad[ch, y, x] and (x + y) % 2 == 0:
                    for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
                        yy, xx = y + dy, x + dx
                        if boundary:
                            yy, xx = yy % H, xx % W
                        if 0 <= yy < H and 0 <= xx < W:
                            bad[ch, yy, xx] = True
    return bad


@pytest.mark.parametrize("mode", [1, 2, 3])
@pytest.mark.parametrize("H,W,boundary,chains", [
    (2, 2, 0, 1), (3, 2, 0, 1), (2, 3, 0, 2), (5, 7, 0, 1), (2, 4, 1, 1), (4, 8, 1, 2),
    (6, 4, 1, 1), (1 + 2 * 60, 9, 0, 1), (3, 4 * 60 + 3, 0, 1)])
def test_fp64_tiny_and_ragged_grids_match_oracle(mpr, H, W, boundary, chains, mode):
    """Degenerate shapes: the smallest grids (open and periodic, where the row window wraps
    onto itself), one-pair-wide and one-work-item-tall strips, and sides one past a work
    item's 60 lane pairs.  Every decision and angle agrees except where the local field
    vanishes (see _degenerate_sites)."""
    _LAST_BEFORE.clear()
    mask, rounds = _decisions_case(mpr, H, W, boundary, chains, mpr.FP64, seed=H * 7 + W + 100,
                                   mode=mode)
    free = np.broadcast_to(mask == 0, rounds[0][0].shape)
    n_checked = 0
    for (dg, do, ug, uo), before in zip(rounds, _LAST_BEFORE):
        uo = uo.reshape(dg.shape)
        assert np.array_equal(dg[~free], do[~free]) and not dg[~free].any()
        ok = free & ~_degenerate_sites(mask, before, uo, boundary)
        assert np.array_equal(dg[ok], do[ok])
        assert np.allclose(ug[ok], uo[ok], rtol=0, atol=1e-9)
        n_checked += int(ok.sum())
    assert n_checked > 0



@pytest.mark.parametrize("H,W,boundary,rows", [
    (12, 40, 0, 2), (13, 280, 0, 2), (19, 112, 0, 4), (11, 113, 0, 2), (16, 112, 1, 2),
    (24, 280, 1, 4), (13, 40, 0, 3), (10, 40, 1, 2), (9, 40, 0, 2)])
def test_fp64_two_half_items_match_oracle(mpr, H, W, boundary, rows):
    """Fused sweeps whose last column strip (at most 28 lane pairs) is swept by half waves, two
    inner row blocks per wave (blocks 1, 2 | 3, 4 | ... while both halves' halo rows lie in the
    grid): one strip (W = 40), a last strip after a full one (W = 280), exactly 28 pairs
    (W = 112), 29 pairs (W = 113, one item per block), an odd row count (rows = 3, one item per
    block), too few rows for a pair (9 x 40), ragged last row blocks, periodic grids.  Every
    decision and angle agrees with the oracle except where the local field vanishes (see
    _degenerate_sites)."""
    _LAST_BEFORE.clear()
    mask, rounds = _decisions_case(mpr, H, W, boundary, 2, mpr.FP64, seed=H * 11 + W + rows,
                                   mode=1, tile_rows=rows)
    free = np.broadcast_to(mask == 0, rounds[0][0].shape)
    n_checked = 0
    for (dg, do, ug, uo), before in zip(rounds, _LAST_BEFORE):
        uo = uo.reshape(dg.shape)
        assert np.array_equal(dg[~free], do[~free]) and not dg[~free].any()
        ok = free & ~_degenerate_sites(mask, before, uo, boundary)
        assert np.array_equal(dg[ok], do[ok])
        assert np.allclose(ug[ok], uo[ok], rtol=0, atol=1e-9)
        n_checked += int(ok.sum())
    assert n_checked > 0

def test_fp64_trace_matches_oracle(mpr):
    """Per-sweep (e_sim, T, alpha, acceptance) of the temperature inference."""
    truth, z, mask = _field(64, 64, 1)
    kw = dict(seed=2001, n_chains=2)
    ctx = _gpu_ctx(mpr, z, mask, **kw)
    orc = O.Oracle(n_threads=2, **kw)
    orc.load(z, mask)
    Tg = ctx.infer_temperature(64)
    To = orc.infer_temperature(64)
    assert np.allclose(Tg, To, rtol=1e-10, atol=0)
    for ch in range(2):
        tg, to = ctx.trace(ch), orc.trace(ch)
        assert tg.shape == to.shape == (64, 4)
        assert np.allclose(tg, to, rtol=1e-10, atol=1e-13), np.abs(tg - to).max(axis=0)
    sg, so = ctx.stats(), orc.stats()
    for a, b in zip(sg, so):
        assert abs(a["e_sample"] - b["e_sample"]) <= 1e-13
        assert a["n_pred"] == b["n_pred"] and a["n_bonds"] == b["n_bonds"]
        assert a["n_sample_bonds"] == b["n_sample_bonds"]
        assert a["zmin"] == b["zmin"] and a["zmax"] == b["zmax"]


@pytest.mark.parametrize("p", [0.33, 0.66])
def test_fp64_predictions_match_oracle_grid64(mpr, p):
    """The 64x64 workload: 256 inference + 100 averaging sweeps; MAE <= 1e-3 of the range."""
    w = synth.workload("grid64", p_missing=p)
    zo, To = O.predict(w["z"], w["mask"], 256, 100, seed=w["mc_seed"], n_threads=2)
    ctx = _gpu_ctx(mpr, w["z"], w["mask"], seed=w["mc_seed"])
    Tg = ctx.infer_temperature(256)
    ctx.run(100)
    zg = ctx.predictions().cpu().numpy().reshape(64, 64)
    m = w["mask"] == 0
    rng = np.ptp(w["z"][~m])
    assert abs(Tg[0] / To[0] - 1) < 1e-9
    assert np.abs(zg - zo)[m].mean() <= 1e-3 * rng
    assert np.array_equal(zg[~m], w["z"][~m])


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_predictions_invariant_to_tiles_and_graphs(mpr, mode):
    w = synth.workload("grid64")
    res = []
    # graphs of 6 and 64 sweeps leave remainders (odd ones: 41 = 6 * 6 + 5) that run as graphs
    # of their own length
    for tile_rows, graph in [(16, 0), (64, 0), (16, -1), (8, 4), (8, 6), (8, 64)]:
        ctx = _gpu_ctx(mpr, w["z"], w["mask"], seed=3, precision=mpr.FP32, tile_rows=tile_rows,
                       graph_sweeps=graph, n_chains=2, sweep_mode=mode)
        ctx.infer_temperature(41)
        ctx.run(11)
        res.append(ctx.predictions().cpu().numpy())
    for r in res[1:]:
        assert np.array_equal(r, res[0])


def test_batch_equals_single_grids(mpr):
    """Every grid of a batch is bit-identical to the same grid run alone with the same global
    grid index (the Philox counters carry it)."""
    rng = np.random.default_rng(4)
    grids = []
    for g in range(5):
        H, W = int(rng.integers(9, 140)), int(rng.integers(9, 140))
        truth, z, mask = _field(H, W, 50 + g, p=float(rng.uniform(0.2, 0.7)))
        grids.append((z, mask))
    kw = dict(seed=77, n_chains=2, precision=mpr.FP32, sweep_mode=mpr.SWEEP_FUSED)
    b = mpr.Context(shapes=[z.shape for z, _ in grids], stream=torch.cuda.Stream(), **kw)
    b.batch_load(_dev(np.concatenate([z.ravel() for z, _ in grids]), torch.float64),
                 _dev(np.concatenate([m.ravel() for _, m in grids]), torch.uint8))
    Tb = b.infer_temperature(30)
    b.run(8)
    zb = b.predictions().cpu().numpy()
    off = 0
    for g, (z, mask) in enumerate(grids):
        s = _gpu_ctx(mpr, z, mask, grid_offset=g, **kw)
        Ts = s.infer_temperature(30)
        s.run(8)
        assert np.array_equal(Ts, Tb[2 * g: 2 * g + 2])
        assert np.array_equal(s.predictions().cpu().numpy(), zb[off: off + z.size])
        off += z.size


def test_batch_fp64_matches_oracle_per_grid(mpr):
    rng = np.random.default_rng(5)
    grids = []
    for g in range(4):
        H, W = int(rng.integers(9, 90)), int(rng.integers(9, 90))
        truth, z, mask = _field(H, W, 70 + g, p=float(rng.uniform(0.2, 0.7)))
        grids.append((z, mask))
    kw = dict(seed=78, n_chains=2)
    b = mpr.Context(shapes=[z.shape for z, _ in grids], stream=torch.cuda.Stream(), **kw)
    b.batch_load(_dev(np.concatenate([z.ravel() for z, _ in grids]), torch.float64),
                 _dev(np.concatenate([m.ravel() for _, m in grids]), torch.uint8))
    Tb = b.infer_temperature(40)
    b.run(20)
    zb = b.predictions().cpu().numpy()
    off = 0
    for g, (z, mask) in enumerate(grids):
        zo, To = O.predict(z, mask, 40, 20, grid_id=g, n_threads=2, **kw)
        assert np.allclose(Tb[2 * g: 2 * g + 2], To, rtol=1e-9)
        m = mask == 0
        zz = zb[off: off + z.size].reshape(z.shape)
        assert np.abs(zz - zo)[m].mean() <= 1e-3 * np.ptp(z[~m])
        assert np.array_equal(zz[~m], z[~m])
        off += z.size


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_resume_is_bitwise_on_gpu(mpr, mode):
    w = synth.workload("grid64")
    kw = dict(seed=9, n_chains=2, precision=mpr.FP16, sweep_mode=mode)
    A = _gpu_ctx(mpr, w["z"], w["mask"], **kw)
    A.infer_temperature(50)
    A.run(30)
    B = _gpu_ctx(mpr, w["z"], w["mask"], **kw)
    B.infer_temperature(50)
    B.run(11)
    st = B.get_state()
    C = _gpu_ctx(mpr, w["z"], w["mask"], **kw)
    C.set_state(**st)
    C.run(19)
    assert np.array_equal(A.predictions().cpu().numpy(), C.predictions().cpu().numpy())


@pytest.mark.parametrize("precision,min_agree,tol", [(1, 0.999, 2e-5), (2, 0.99, 2e-3)])
def test_reduced_precision_decisions(mpr, precision, min_agree, tol):
    mask, rounds = _decisions_case(mpr, 64, 96, 0, 1, precision, seed=21)
    free = np.broadcast_to(mask == 0, rounds[0][0].shape)
    for dg, do, ug, uo in rounds:
        same = (dg == do)[free]
        assert same.mean() >= min_agree, same.mean()
        agree = free & (dg == do)
        assert np.quantile(np.abs(ug - uo)[agree], 0.99) <= tol


@pytest.mark.parametrize("precision", [1, 2])
def test_reduced_precision_mae_within_one_percent(mpr, precision):
    """MAE against the truth of FP32 / FP16 setups within 1 % of the FP64 oracle's (the
    paper's Delta MAAE, Sec. 3), on the 64x64 workload with 4 chains."""
    w = synth.workload("grid64")
    m = w["mask"] == 0
    kw = dict(seed=w["mc_seed"], n_chains=4)
    zo, _ = O.predict(w["z"], w["mask"], 256, 100, n_threads=4, **kw)
    ctx = _gpu_ctx(mpr, w["z"], w["mask"], precision=precision, **kw)
    ctx.infer_temperature(256)
    ctx.run(100)
    zg = ctx.predictions().cpu().numpy().reshape(64, 64)
    mae_o = np.abs(zo - w["truth"])[m].mean()
    mae_g = np.abs(zg - w["truth"])[m].mean()
    assert abs(mae_g / mae_o - 1) <= 0.01, (mae_g, mae_o)


def test_gpu_error_codes(mpr):
    z = np.arange(16.0).reshape(4, 4)
    m = np.ones((4, 4), np.uint8)
    m[1, 1] = 0
    for kw in [dict(q=0.6), dict(J=-1.0), dict(n_chains=0), dict(precision=7),
               dict(precision=2, func_prec=0), dict(group_waves=-1), dict(group_waves=33)]:
        with pytest.raises(mpr.MprError) as e:
            mpr.Context(**kw)
        assert e.value.code == mpr.EINVAL
    ctx = mpr.Context()
    with pytest.raises(mpr.MprError) as e:
        ctx.load(_dev(np.ones((4, 4)), torch.float64), _dev(m, torch.uint8))
    assert e.value.code == mpr.ENOSAMPLE
    checker = ((np.add.outer(np.arange(4), np.arange(4)) % 2) == 0).astype(np.uint8)
    with pytest.raises(mpr.MprError) as e:
        ctx.load(_dev(z, torch.float64), _dev(checker, torch.uint8))
    assert e.value.code == mpr.ENOSAMPLE
    bad = m.copy()
    bad[0, 0] = 3
    with pytest.raises(mpr.MprError) as e:
        ctx.load(_dev(z, torch.float64), _dev(bad, torch.uint8))
    assert e.value.code == mpr.EINVAL
    zn = z.copy()
    zn[0, 0] = np.inf
    with pytest.raises(mpr.MprError) as e:
        ctx.load(_dev(zn, torch.float64), _dev(m, torch.uint8))
    assert e.value.code == mpr.EINVAL
    per = mpr.Context(boundary=mpr.PERIODIC)
    with pytest.raises(mpr.MprError) as e:
        per.load(_dev(np.arange(15.0).reshape(3, 5), torch.float64), _dev(np.ones((3, 5), np.uint8), torch.uint8))
    assert e.value.code == mpr.EBIPARTITE
    ctx.load(_dev(z, torch.float64), _dev(m, torch.uint8))
    with pytest.raises(mpr.MprError) as e:
        ctx.run(3)
    assert e.value.code == mpr.ESTATE
    with pytest.raises(mpr.MprError) as e:
        ctx.predictions()
    assert e.value.code == mpr.ESTATE
    with pytest.raises(mpr.MprError) as e:
        ctx.set_state(u=_dev(np.full(16, 1.5), torch.float64))
    assert e.value.code == mpr.EINVAL
    ctx.set_temperature(0.1)
    ctx.run(2)
    out = ctx.predictions().cpu().numpy().reshape(4, 4)
    assert np.array_equal(out[m == 1], z[m == 1])


def test_autotune_keeps_results(mpr):
    """The autotuner only changes the work decomposition: the tuned context reproduces the
    untuned one bit for bit."""
    w = synth.workload("grid64")
    res = []
    for tune in (False, True):
        ctx = _gpu_ctx(mpr, w["z"], w["mask"], seed=5, precision=mpr.FP32, n_chains=2,
                       sweep_mode=mpr.SWEEP_FUSED)
        if tune:
            rows = ctx.autotune(4)
            assert rows >= 2
        ctx.infer_temperature(30)
        ctx.run(10)
        res.append(ctx.predictions().cpu().numpy())
    assert np.array_equal(res[0], res[1])


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_large_grid_trace_matches_oracle(mpr, mode):
    """Inference trace on a 512 x 1000 grid: several column strips and row blocks per chain
    (fused path), several thousand waves per colour (compacted path), 32 x 4 tiles with a
    ragged last column of tiles (tiled path)."""
    truth, z, mask = _field(512, 1000, 9)
    kw = dict(seed=31, n_chains=1)
    ctx = _gpu_ctx(mpr, z, mask, sweep_mode=mode, **kw)
    orc = O.Oracle(n_threads=8, **kw)
    orc.load(z, mask)
    Tg = ctx.infer_temperature(24)
    To = orc.infer_temperature(24)
    tg, to = ctx.trace(0), orc.trace(0)
    assert np.allclose(tg, to, rtol=1e-9, atol=1e-13), np.abs(tg - to).max(axis=0)
    assert np.allclose(Tg, To, rtol=1e-9)


SETTINGS = {  # the paper's X_S X_E X_F (Sec. 2): spins, energy, functions in D(ouble) or S(ingle)
    "DDD": (0, 0, 0), "DSD": (0, 1, 0), "DDS": (0, 0, 1), "SDD": (1, 0, 0),
    "SDS": (1, 0, 1), "DSS": (0, 1, 1), "SSD": (1, 1, 0), "SSS": (1, 1, 1),
    "H-DS (FP16 spins)": (2, 0, 1), "F-DS (16-bit fixed-point spins)": (3, 0, 1),
}


@pytest.mark.parametrize("name", sorted(SETTINGS))
def test_precision_settings(mpr, name):
    """Every precision setting: decisions from an identical state agree with the FP64 oracle
    (>= 99.99 % with double functions, >= 99 % otherwise) and the prediction MAE against the
    truth stays within 1 % of the oracle's (the paper finds Delta MAAE ~ 1e-4 %, Sec. 3)."""
    prec, eprec, fprec = SETTINGS[name]
    kw = dict(precision=prec, energy_prec=eprec, func_prec=fprec)
    # decisions
    truth, z, mask = _field(48, 80, 123)
    ctx = _gpu_ctx(mpr, z, mask, seed=7, alpha0=0.4, **kw)
    orc = O.Oracle(n_threads=2, seed=7, alpha0=0.4)
    orc.load(z, mask)
    u0 = synth.random_state(1, mask, 8)
    ctx.set_state(u=_dev(u0.reshape(-1), torch.float64))
    orc.set_state(phi=TWO_PI * u0)
    ctx.set_temperature(0.08)
    orc.set_temperature(0.08)
    dg = ctx.debug_sweep(3).cpu().numpy().reshape(1, 48, 80)
    do = orc.debug_sweep(3)
    free = np.broadcast_to(mask == 0, dg.shape)
    agree = (dg == do)[free].mean()
    assert agree >= (0.9999 if fprec == 0 else 0.99), agree
    # predictions
    w = synth.workload("grid64")
    m = w["mask"] == 0
    kwo = dict(seed=w["mc_seed"], n_chains=4)
    zo, _ = O.predict(w["z"], w["mask"], 256, 100, n_threads=4, **kwo)
    ctx = _gpu_ctx(mpr, w["z"], w["mask"], **kwo, **kw)
    ctx.infer_temperature(256)
    ctx.run(100)
    zg = ctx.predictions().cpu().numpy().reshape(64, 64)
    mae_o = np.abs(zo - w["truth"])[m].mean()
    mae_g = np.abs(zg - w["truth"])[m].mean()
    assert abs(mae_g / mae_o - 1) <= 0.01, (mae_g, mae_o)


# ---------------------------------------------------------------- compacted (sparse) sweep path
@pytest.mark.parametrize("mode", [2, 3])
@pytest.mark.parametrize("H,W,boundary,chains", [
    (64, 64, 0, 1), (37, 53, 0, 2), (16, 24, 1, 1), (2, 2, 0, 1), (2, 4, 1, 1), (3, 243, 0, 1),
    (130, 244, 0, 1), (40, 300, 1, 2)])
def test_sparse_fp64_decisions_and_angles_match_oracle(mpr, H, W, boundary, chains, mode):
    """The compacted and tiled paths take the oracle's decisions from identical states."""
    mask, rounds = _decisions_case(mpr, H, W, boundary, chains, mpr.FP64, seed=H * 13 + W,
                                   mode=mode)
    free = np.broadcast_to(mask == 0, rounds[0][0].shape)
    for dg, do, ug, uo in rounds:
        assert np.array_equal(dg[~free], do[~free]) and not dg[~free].any()
        assert (dg == do)[free].mean() >= 0.99999
        assert np.allclose(ug, uo, rtol=0, atol=1e-9)


@pytest.mark.parametrize("precision", [0, 1, 2, 3])
def test_sparse_and_fused_decisions_are_identical(mpr, precision):
    """Same field arithmetic, functions and counters: bitwise-equal decisions and angles from
    identical states, in every storage precision."""
    H, W = 45, 70
    truth, z, mask = _field(H, W, 99)
    u0 = synth.random_state(2, mask, 5)
    out = []
    for mode in (mpr.SWEEP_FUSED, mpr.SWEEP_SPARSE, mpr.SWEEP_TILED):
        ctx = _gpu_ctx(mpr, z, mask, precision=precision, sweep_mode=mode, n_chains=2, seed=3,
                       alpha0=0.5)
        assert ctx.sweep_mode() == mode
        ctx.set_state(u=_dev(u0.reshape(-1), torch.float64))
        ctx.set_temperature(0.05)
        decs = [ctx.debug_sweep(s).cpu().numpy() for s in (4, 5, 6)]
        out.append((decs, ctx.get_state()["u"].cpu().numpy()))
    for other in out[1:]:
        for a, b in zip(out[0][0], other[0]):
            assert np.array_equal(a, b)
        assert np.array_equal(out[0][1], other[1])


@pytest.mark.parametrize("mode", [2, 3])
def test_sparse_trace_matches_oracle(mpr, mode):
    truth, z, mask = _field(48, 64, 17)
    kw = dict(seed=21, n_chains=2)
    ctx = _gpu_ctx(mpr, z, mask, sweep_mode=mode, **kw)
    orc = O.Oracle(n_threads=4, **kw)
    orc.load(z, mask)
    Tg = ctx.infer_temperature(40)
    To = orc.infer_temperature(40)
    for ch in range(2):
        tg, to = ctx.trace(ch), orc.trace(ch)
        assert np.allclose(tg, to, rtol=1e-9, atol=1e-13), np.abs(tg - to).max(axis=0)
    assert np.allclose(Tg, To, rtol=1e-9)


@pytest.mark.parametrize("mode", [2, 3])
@pytest.mark.parametrize("p", [0.33, 0.66])
def test_sparse_predictions_match_oracle_grid64(mpr, p, mode):
    w = synth.workload("grid64", p_missing=p)
    kw = dict(seed=w["mc_seed"], n_chains=2)
    zo, To = O.predict(w["z"], w["mask"], 256, 100, n_threads=4, **kw)
    ctx = _gpu_ctx(mpr, w["z"], w["mask"], sweep_mode=mode, **kw)
    Tg = ctx.infer_temperature(256)
    ctx.run(100)
    zg = ctx.predictions().cpu().numpy().reshape(64, 64)
    rng = np.nanmax(w["z"]) - np.nanmin(w["z"])
    assert np.allclose(Tg, To, rtol=1e-8)
    assert np.abs(zg - zo).mean() <= 1e-3 * rng


@pytest.mark.parametrize("mode", [2, 3])
def test_sparse_batch_equals_single_grids(mpr, mode):
    shapes = [(40, 56), (33, 17), (64, 64), (20, 300)]
    fields = [_field(h, w, 300 + i) for i, (h, w) in enumerate(shapes)]
    kw = dict(seed=8, n_chains=2, sweep_mode=mode)
    bctx = mpr.Context(shapes=shapes, stream=torch.cuda.Stream(), **kw)
    bctx.batch_load(_dev(np.concatenate([f[1].ravel() for f in fields]), torch.float64),
                    _dev(np.concatenate([f[2].ravel() for f in fields]), torch.uint8))
    bctx.infer_temperature(30)
    bctx.run(10)
    zb = bctx.predictions().cpu().numpy()
    off = 0
    for i, (h, w) in enumerate(shapes):
        ctx = _gpu_ctx(mpr, fields[i][1], fields[i][2], grid_offset=i, **kw)
        ctx.infer_temperature(30)
        ctx.run(10)
        zs = ctx.predictions().cpu().numpy()
        assert np.array_equal(zs, zb[off:off + h * w])
        off += h * w


def test_automatic_path_choice(mpr):
    """AUTO takes the tiled path for small grids with single-precision functions or with
    double-precision functions and mostly prediction sites, the compacted path with fewer
    prediction sites (at any size with double-precision functions or 16-bit storage, on small
    grids with FP32 storage), when the energy is summed in double precision; the fused path
    otherwise."""
    for p, prec, esingle, want in [(0.33, mpr.FP32, False, mpr.SWEEP_TILED),
                                   (0.5, mpr.FP16, False, mpr.SWEEP_TILED),
                                   (0.5, mpr.FP64, False, mpr.SWEEP_SPARSE),
                                   (0.9, mpr.FP64, False, mpr.SWEEP_TILED),
                                   (0.33, mpr.FP32, True, mpr.SWEEP_FUSED)]:
        truth, z, mask = _field(64, 64, 5, p=p)
        ctx = _gpu_ctx(mpr, z, mask, precision=prec,
                       energy_prec=mpr.PREC_SINGLE if esingle else mpr.PREC_DEFAULT)
        assert ctx.sweep_mode() == want, (p, prec, esingle)
    # the tiled limit (1.5 * 2^20 sites x chains), then compacted up to 2^23 sites with few
    # prediction sites, else fused
    rng = np.random.default_rng(3)
    for side, p, want in [(1254, 0.33, mpr.SWEEP_TILED), (1255, 0.33, mpr.SWEEP_SPARSE),
                          (1536, 0.33, mpr.SWEEP_SPARSE), (2896, 0.33, mpr.SWEEP_SPARSE),
                          (2048, 0.5, mpr.SWEEP_FUSED), (4096, 0.33, mpr.SWEEP_FUSED)]:
        mask = (rng.random((side, side)) >= p).astype(np.uint8)
        z = np.where(mask == 1, rng.standard_normal((side, side)), np.nan)
        assert _gpu_ctx(mpr, z, mask, precision=mpr.FP32).sweep_mode() == want, (side, p)
    # double-precision functions past the tiled limit: compacted up to 60 % prediction sites at
    # any size and up to 70 % with 2^23 sites, else fused
    for side, p, want in [(2048, 0.66, mpr.SWEEP_SPARSE), (2048, 0.9, mpr.SWEEP_FUSED),
                          (4096, 0.66, mpr.SWEEP_FUSED), (4096, 0.5, mpr.SWEEP_SPARSE)]:
        mask = (rng.random((side, side)) >= p).astype(np.uint8)
        z = np.where(mask == 1, rng.standard_normal((side, side)), np.nan)
        assert _gpu_ctx(mpr, z, mask, precision=mpr.FP64).sweep_mode() == want, (side, p)
    # 16-bit storage past the tiled limit: compacted up to 50 % prediction sites at any size
    for side, p, prec, want in [(2048, 0.45, mpr.FP16, mpr.SWEEP_SPARSE),
                                (4096, 0.45, mpr.FIX16, mpr.SWEEP_SPARSE),
                                (2048, 0.6, mpr.FP16, mpr.SWEEP_FUSED)]:
        mask = (rng.random((side, side)) >= p).astype(np.uint8)
        z = np.where(mask == 1, rng.standard_normal((side, side)), np.nan)
        assert _gpu_ctx(mpr, z, mask, precision=prec).sweep_mode() == want, (side, p, prec)
    truth, z, mask = _field(64, 64, 5)
    for mode in (mpr.SWEEP_SPARSE, mpr.SWEEP_TILED):
        with pytest.raises(mpr.MprError):
            _gpu_ctx(mpr, z, mask, precision=mpr.FP32, energy_prec=mpr.PREC_SINGLE, sweep_mode=mode)


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_other_q_and_J_match_oracle(mpr, mode):
    """q < 1/2 and J != 1 (Eq. (2)): decisions from identical states and the inference trace."""
    truth, z, mask = _field(40, 52, 61)
    kw = dict(q=0.3, J=1.7, seed=12, n_chains=1)
    ctx = _gpu_ctx(mpr, z, mask, sweep_mode=mode, alpha0=0.5, **kw)
    orc = O.Oracle(n_threads=2, alpha0=0.5, **kw)
    orc.load(z, mask)
    u0 = synth.random_state(1, mask, 3)
    ctx.set_state(u=_dev(u0.reshape(-1), torch.float64))
    orc.set_state(phi=TWO_PI * u0)
    ctx.set_temperature(0.1)
    orc.set_temperature(0.1)
    dg = ctx.debug_sweep(2).cpu().numpy().reshape(1, 40, 52)
    do = orc.debug_sweep(2)
    free = np.broadcast_to(mask == 0, dg.shape)
    assert (dg == do)[free].mean() >= 0.99999
    ctx = _gpu_ctx(mpr, z, mask, sweep_mode=mode, **kw)
    orc = O.Oracle(n_threads=2, **kw)
    orc.load(z, mask)
    Tg = ctx.infer_temperature(30)
    To = orc.infer_temperature(30)
    assert np.allclose(ctx.trace(0), orc.trace(0), rtol=1e-9, atol=1e-13)
    assert np.allclose(Tg, To, rtol=1e-9)


def test_sparse_colour_without_prediction_sites(mpr):
    """A grid whose colour-0 sites are all samples: that colour's list is one padding wave, and
    the compacted path still matches the oracle's trace and the fused path's decisions."""
    H, W = 30, 44
    truth = synth.gaussian_field(H, W, 0.5, 8.0, 50.0, 10.0, 71)
    yy, xx = np.mgrid[0:H, 0:W]
    rng = np.random.default_rng(3)
    mask = np.ones((H, W), np.uint8)
    odd = (yy + xx) % 2 == 1
    mask[odd & (rng.random((H, W)) < 0.5)] = 0          # only colour-1 sites are missing
    z = np.where(mask == 1, truth, np.nan)
    kw = dict(seed=5, n_chains=2)
    ctx = _gpu_ctx(mpr, z, mask, sweep_mode=mpr.SWEEP_SPARSE, **kw)
    orc = O.Oracle(n_threads=2, **kw)
    orc.load(z, mask)
    Tg = ctx.infer_temperature(20)
    To = orc.infer_temperature(20)
    for ch in range(2):
        assert np.allclose(ctx.trace(ch), orc.trace(ch), rtol=1e-9, atol=1e-13)
    assert np.allclose(Tg, To, rtol=1e-9)
    ctx.run(5)
    zs = ctx.predictions().cpu().numpy()
    f = _gpu_ctx(mpr, z, mask, sweep_mode=mpr.SWEEP_FUSED, **kw)
    f.infer_temperature(20)
    f.run(5)
    zf = f.predictions().cpu().numpy()
    m = (mask == 0).ravel()
    rng_z = np.nanmax(z) - np.nanmin(z)
    assert np.abs(zs - zf)[m].mean() <= 1e-6 * rng_z


@pytest.mark.parametrize("precision,func_prec,p", [(0, -1, 0.33), (1, -1, 0.33), (2, -1, 0.33),
                                                   (3, -1, 0.33), (1, 0, 0.33), (1, 0, 0.9)])
def test_tiled_equals_sparse_bitwise(mpr, precision, func_prec, p):
    """The tiled path sums the energy by the same bond kinds and per-site terms as the compacted
    path, so whole runs (temperature trajectories, estimates, predictions) agree bit for bit;
    a batch of uneven grids with two chains each, open and periodic; every storage precision
    with its default functions, and FP32 storage with double-precision functions (the paper's
    SDD setting, whose tiled kernel stages 16-row tiles) at 33 % and at the paper's 90 %
    missing."""
    for boundary, shapes in ((0, [(45, 70), (17, 300), (2, 3), (64, 64)]),
                             (1, [(16, 24), (34, 264), (2, 4)])):
        if p > 0.5:     # grids too small to keep two distinct sample values at 90 % missing
            shapes = [(h, w) for h, w in shapes if h * w >= 256]
        fields = [_field(h, w, 500 + i, p=p) for i, (h, w) in enumerate(shapes)]
        z = np.concatenate([f[1].ravel() for f in fields])
        m = np.concatenate([f[2].ravel() for f in fields])
        res = []
        for mode in (mpr.SWEEP_SPARSE, mpr.SWEEP_TILED):
            ctx = mpr.Context(shapes=shapes, stream=torch.cuda.Stream(), seed=4, n_chains=2,
                              precision=precision, func_prec=func_prec, boundary=boundary,
                              sweep_mode=mode)
            ctx.batch_load(_dev(z, torch.float64), _dev(m, torch.uint8))
            assert ctx.sweep_mode() == mode
            T = ctx.infer_temperature(24)
            tr = [ctx.trace(i) for i in range(2 * len(shapes))]
            ctx.run(6)
            res.append((T, tr, ctx.predictions().cpu().numpy()))
        assert np.array_equal(res[0][0], res[1][0])
        for a, b in zip(res[0][1], res[1][1]):
            assert np.array_equal(a, b)
        assert np.array_equal(res[0][2], res[1][2])



@pytest.mark.parametrize("precision", [0, 1, 2])
def test_sparse_group_sizes_are_bitwise_equal(mpr, precision):
    """A compacted-path wave sweeps a group of up to group_waves list waves of one (grid, chain):
    whole runs (temperature trajectories, estimates, predictions, the averaging sweeps' running
    sums) agree bit for bit with one list wave per group, for groups of 2, 3, 7 and 32 list
    waves (uneven tails and (grid, chain)s with fewer list waves than a group), and the
    decisions of a single sweep too; a batch of uneven open grids with two chains, a periodic
    batch, and one grid."""
    cases = [([(45, 70), (17, 300), (2, 3), (130, 244), (64, 64)], 2, 0),
             ([(16, 24), (34, 264), (96, 128)], 2, 1), ([(200, 340)], 1, 0)]
    for shapes, chains, boundary in cases:
        fields = [_field(h, w, 700 + i) for i, (h, w) in enumerate(shapes)]
        z = np.concatenate([f[1].ravel() for f in fields])
        m = np.concatenate([f[2].ravel() for f in fields])
        res = []
        for gw in (1, 2, 3, 7, 32):
            ctx = mpr.Context(shapes=shapes, stream=torch.cuda.Stream(), seed=5, n_chains=chains,
                              precision=precision, sweep_mode=mpr.SWEEP_SPARSE, group_waves=gw,
                              boundary=boundary)
            ctx.batch_load(_dev(z, torch.float64), _dev(m, torch.uint8))
            T = ctx.infer_temperature(20)
            tr = [ctx.trace(i) for i in range(chains * len(shapes))]
            ctx.run(5)
            pred = ctx.predictions().cpu().numpy()
            st = ctx.get_state()
            dec = ctx.debug_sweep(77).cpu().numpy()
            res.append((T, tr, pred, st["u"].cpu().numpy(), st["acc"].cpu().numpy(), dec))
        for r in res[1:]:
            assert np.array_equal(res[0][0], r[0])
            for a, b in zip(res[0][1], r[1]):
                assert np.array_equal(a, b)
            for i in (2, 3, 4, 5):
                assert np.array_equal(res[0][i], r[i])
        assert (res[0][5] & mpr.DEC_ACCEPT).any()

@pytest.mark.parametrize("mode", [1, 2, 3])
@pytest.mark.parametrize("p_first,p_second", [(0.3, 0.6), (0.6, 0.3)])
def test_reload_with_the_same_shape_matches_a_fresh_context(mpr, mode, p_first, p_second):
    """A second load with the same shape keeps the buffers and may keep the captured sweep
    graphs; the new data's mask-dependent quantities (prediction-site count, site lists, sample
    energy) must still take effect: the run equals a fresh context's bit for bit, whether the
    second mask has more or fewer prediction sites."""
    a = _field(96, 136, 21, p=p_first)
    b = _field(96, 136, 22, p=p_second)
    kw = dict(seed=6, n_chains=2, precision=mpr.FP32, sweep_mode=mode, graph_sweeps=4)
    ctx = _gpu_ctx(mpr, a[1], a[2], **kw)
    ctx.infer_temperature(16)
    ctx.run(8)
    ctx.load(_dev(b[1], torch.float64), _dev(b[2], torch.uint8))
    Tr = ctx.infer_temperature(16)
    ctx.run(8)
    fresh = _gpu_ctx(mpr, b[1], b[2], **kw)
    Tf = fresh.infer_temperature(16)
    fresh.run(8)
    assert np.array_equal(Tr, Tf)
    for ch in range(2):
        assert np.array_equal(ctx.trace(ch), fresh.trace(ch))
    assert np.array_equal(ctx.predictions().cpu().numpy(), fresh.predictions().cpu().numpy())


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_autotuned_path_reproduces_the_chosen_path(mpr, precision):
    """With sweep_mode AUTO and tile_rows = -1 the tuner times every possible sweep path at
    load and keeps the fastest; the state it timed from is restored, so the tuned context
    reproduces a fresh context forced onto the chosen path bit for bit, and a second load of
    the same data takes the remembered choice."""
    w = synth.workload("grid64", p_missing=0.5)
    kw = dict(seed=5, precision=precision, n_chains=2)
    tuned = _gpu_ctx(mpr, w["z"], w["mask"], tile_rows=-1, **kw)
    mode = tuned.sweep_mode()
    path, rows, shape, gk = tuned.tuning()
    assert mode == path and mode in (mpr.SWEEP_FUSED, mpr.SWEEP_SPARSE, mpr.SWEEP_TILED)
    assert gk in (16, 32, 64)
    assert (shape in range(4)) == (mode == mpr.SWEEP_TILED)
    Tt = tuned.infer_temperature(30)
    tuned.run(10)
    # the same configuration forced: path, rows per work item, tile shape, graph length
    forced = _gpu_ctx(mpr, w["z"], w["mask"], sweep_mode=mode, tile_rows=rows, graph_sweeps=gk,
                      tile_shape=shape + 1 if shape >= 0 else 0, **kw)
    assert forced.tuning() == (path, rows, shape, gk)
    Tf = forced.infer_temperature(30)
    forced.run(10)
    assert np.array_equal(Tt, Tf)
    assert np.array_equal(tuned.predictions().cpu().numpy(), forced.predictions().cpu().numpy())
    again = _gpu_ctx(mpr, w["z"], w["mask"], tile_rows=-1, **kw)
    assert again.tuning() == (path, rows, shape, gk)


@pytest.mark.parametrize("precision", [1, 2])
def test_tiled_four_wave_blocks_equal_sparse(mpr, precision):
    """From 2048 tiles on, the tiled kernel runs four-wave blocks (eight below): on a
    2048 x 2048 grid (2048 tiles) the run still equals the compacted path's bit for bit."""
    H = W = 2048
    rng = np.random.default_rng(12)
    z = rng.normal(50.0, 10.0, (H, W))
    mask = (rng.random((H, W)) >= 0.4).astype(np.uint8)
    z = np.where(mask == 1, z, np.nan)
    res = []
    for mode in (mpr.SWEEP_SPARSE, mpr.SWEEP_TILED):
        ctx = _gpu_ctx(mpr, z, mask, precision=precision, sweep_mode=mode, seed=17)
        T = ctx.infer_temperature(12)
        ctx.run(4)
        res.append((T, ctx.trace(0), ctx.predictions().cpu().numpy()))
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1], res[1][1])
    assert np.array_equal(res[0][2], res[1][2])


def test_contexts_on_two_host_threads(mpr):
    """Two contexts driven from two host threads at once, both autotuning at load (the tuner's
    table is shared by the process), give the results each gives alone."""
    import threading
    fields = [_field(52, 76, 5), _field(44, 90, 6)]      # shapes no other test tunes

    def run(i, out):
        truth, z, mask = fields[i]
        ctx = _gpu_ctx(mpr, z, mask, precision=mpr.FP32, sweep_mode=mpr.SWEEP_FUSED, tile_rows=-1,
                       seed=9 + i)
        ctx.infer_temperature(20)
        ctx.run(5)
        out[i] = ctx.predictions().cpu().numpy()

    both = [None, None]
    threads = [threading.Thread(target=run, args=(i, both)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads)
    alone = [None, None]
    for i in range(2):
        run(i, alone)
    for i in range(2):
        assert both[i] is not None and np.array_equal(both[i], alone[i])


@pytest.mark.parametrize("mode", [1, 2, 3])
@pytest.mark.parametrize("p", [0.33, 0.9])
def test_fp32_storage_double_functions_match_oracle(mpr, mode, p):
    """FP32 storage with double-precision functions (the paper's SDD setting) on every sweep
    path, at 33 % and at the paper's 90 % missing: from identical states (rounded to FP32 on
    the device) the decisions equal the oracle's on >= 99.9 % of the prediction sites and the
    equal ones agree to a few FP32 roundings of the stored angles (1e-6 turns, 99.9 %)."""
    mask, rounds = _decisions_case(mpr, 70, 130, 0, 2, mpr.FP32, seed=77, mode=mode, p=p,
                                   func_prec=mpr.PREC_DOUBLE)
    free = np.broadcast_to(mask == 0, rounds[0][0].shape)
    for dg, do, ug, uo in rounds:
        assert not dg[~free].any()
        assert (dg == do)[free].mean() >= 0.999
        agree = free & (dg == do)
        assert np.quantile(np.abs(ug - uo)[agree], 0.999) <= 1e-6


def test_automatic_path_choice_double_functions_at_90_percent(mpr):
    """AUTO takes the tiled path for a small grid with FP32 storage, double-precision functions
    and 90 % prediction sites, and its run equals the compacted path's bit for bit."""
    truth, z, mask = _field(96, 136, 8, p=0.9)
    res = []
    for mode in (mpr.SWEEP_AUTO, mpr.SWEEP_SPARSE):
        ctx = _gpu_ctx(mpr, z, mask, precision=mpr.FP32, func_prec=mpr.PREC_DOUBLE, seed=3,
                       n_chains=2, sweep_mode=mode)
        if mode == mpr.SWEEP_AUTO:
            assert ctx.sweep_mode() == mpr.SWEEP_TILED
        T = ctx.infer_temperature(20)
        ctx.run(6)
        res.append((T, ctx.trace(0), ctx.predictions().cpu().numpy()))
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1], res[1][1])
    assert np.array_equal(res[0][2], res[1][2])


def test_binding_refuses_buffers_the_kernels_cannot_use(mpr):
    """The binding checks every device buffer it hands to the library (type, dtype, contiguity,
    element count) before the call, so a host array or a short tensor never reaches a kernel."""
    truth, z, mask = _field(12, 16, 4)
    ctx = _gpu_ctx(mpr, z, mask, precision=mpr.FP32)
    n = 12 * 16
    with pytest.raises(TypeError):
        ctx.set_state(u=np.zeros(n))
    with pytest.raises(TypeError):
        ctx.set_state(u=torch.zeros(n, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        ctx.set_state(u=torch.zeros(n - 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        ctx.set_state(acc=torch.zeros(2 * n, dtype=torch.float64, device="cuda")[::2])
    ctx.set_temperature(0.1)
    ctx.run(2)
    with pytest.raises(ValueError):
        ctx.predictions(out=torch.empty(n - 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(TypeError):
        ctx.predictions(out=torch.empty(n, dtype=torch.float64))
    with pytest.raises(TypeError):
        ctx.load(_dev(z, torch.float32), _dev(mask, torch.uint8))
    out = ctx.predictions(out=torch.empty(n, dtype=torch.float64, device="cuda"))
    assert np.isfinite(out.cpu().numpy()).all()


@pytest.mark.parametrize("precision", [1, 2])
def test_every_tile_shape_equals_sparse(mpr, precision):
    """The tiled path's four block shapes (four or eight waves, base or double tile height) run
    a batch of uneven grids with two chains bit for bit like the compacted path; with
    double-precision functions only the four-wave base shape exists."""
    shapes = [(45, 70), (130, 300), (66, 264), (2, 3)]
    fields = [_field(h, w, 700 + i) for i, (h, w) in enumerate(shapes)]
    z = np.concatenate([f[1].ravel() for f in fields])
    m = np.concatenate([f[2].ravel() for f in fields])

    def run(**cfg):
        ctx = mpr.Context(shapes=shapes, stream=torch.cuda.Stream(), seed=8, n_chains=2,
                          precision=precision, **cfg)
        ctx.batch_load(_dev(z, torch.float64), _dev(m, torch.uint8))
        T = ctx.infer_temperature(20)
        tr = ctx.trace(3)
        ctx.run(6)
        return ctx.tuning(), T, tr, ctx.predictions().cpu().numpy()

    ref = run(sweep_mode=mpr.SWEEP_SPARSE)
    for shape in range(4):
        tun, T, tr, zh = run(sweep_mode=mpr.SWEEP_TILED, tile_shape=shape + 1)
        assert tun[0] == mpr.SWEEP_TILED and tun[2] == shape
        assert np.array_equal(T, ref[1]) and np.array_equal(tr, ref[2]) and np.array_equal(zh, ref[3])
    with pytest.raises(mpr.MprError):
        mpr.Context(precision=mpr.FP32, func_prec=mpr.PREC_DOUBLE, tile_shape=mpr.TILE_W8_TALL + 1)


def test_timings_report_each_phase(mpr):
    """mpr_get_timings: stream time of the last load, inference, averaging run and predictions,
    and their sweep counts; -1 for phases not run yet."""
    truth, z, mask = _field(40, 56, 9)
    ctx = mpr.Context(stream=torch.cuda.Stream(), precision=mpr.FP32)
    ctx.load(_dev(z, torch.float64), _dev(mask, torch.uint8))
    t = ctx.timings()
    assert t["load_ms"] > 0.0 and t["infer_ms"] == -1.0 and t["run_ms"] == -1.0
    ctx.infer_temperature(33)
    ctx.run(7)
    ctx.predictions()
    t = ctx.timings()
    assert t["infer_ms"] > 0.0 and t["run_ms"] > 0.0 and t["predict_ms"] > 0.0
    assert t["infer_sweeps"] == 33 and t["run_sweeps"] == 7


def _far_rows_field(seed):
    """300 x 1024 grid whose prediction sites lie in a few rows up to 150 apart (five random
    sites and the last two columns of each); every other site is a sample."""
    H, W = 300, 1024
    truth = synth.gaussian_field(H, W, 0.5, 32.0, 50.0, 10.0, seed)
    rng = np.random.default_rng(seed)
    mask = np.ones((H, W), np.uint8)
    for y in (0, 1, 126, 127, 128, 140, 290, 299):
        mask[y, rng.choice(W - 2, 5, replace=False)] = 0
        mask[y, W - 2:] = 0
    return truth, np.where(mask == 1, truth, np.nan), mask


def test_sparse_far_rows_and_wide_grids(mpr):
    """Compacted-path list waves whose sites lie in rows far apart (a 300 x 1024 grid with
    prediction sites in eight rows up to 150 apart) and plane rows of thousands of sites (a
    6 x 40000 grid): from identical states the decisions and angles equal the fused path's bit
    for bit (FP64, FP16), and whole runs of a batch of both grids equal the tiled path's."""
    wide = _field(6, 40000, 41)
    far = _far_rows_field(43)
    for truth, z, mask in (wide, far):
        H, W = mask.shape
        u0 = synth.random_state(2, mask, 9)
        for precision in (mpr.FP64, mpr.FP16):
            out = []
            for mode in (mpr.SWEEP_FUSED, mpr.SWEEP_SPARSE):
                ctx = _gpu_ctx(mpr, z, mask, precision=precision, sweep_mode=mode, n_chains=2,
                               seed=3, alpha0=0.5)
                assert ctx.sweep_mode() == mode
                ctx.set_state(u=_dev(u0.reshape(-1), torch.float64))
                ctx.set_temperature(0.05)
                decs = [ctx.debug_sweep(s).cpu().numpy() for s in (4, 5, 6)]
                out.append((decs, ctx.get_state()["u"].cpu().numpy()))
            for a, b in zip(out[0][0], out[1][0]):
                assert np.array_equal(a, b)
            assert np.array_equal(out[0][1], out[1][1])
            free = np.broadcast_to(mask == 0, (2, H, W)).reshape(-1)
            assert (out[1][0][0] != 0)[free].mean() > 0.5
    shapes = [(6, 40000), (300, 1024), (45, 70)]
    fields = [wide, far, _field(45, 70, 47)]
    zb = np.concatenate([f[1].ravel() for f in fields])
    mb = np.concatenate([f[2].ravel() for f in fields])
    res = []
    for mode in (mpr.SWEEP_SPARSE, mpr.SWEEP_TILED):
        ctx = mpr.Context(shapes=shapes, stream=torch.cuda.Stream(), seed=4, n_chains=2,
                          precision=mpr.FP16, sweep_mode=mode)
        ctx.batch_load(_dev(zb, torch.float64), _dev(mb, torch.uint8))
        T = ctx.infer_temperature(16)
        tr = [ctx.trace(i) for i in range(2 * len(shapes))]
        ctx.run(4)
        res.append((T, tr, ctx.predictions().cpu().numpy()))
    assert np.array_equal(res[0][0], res[1][0])
    for a, b in zip(res[0][1], res[1][1]):
        assert np.array_equal(a, b)
    assert np.array_equal(res[0][2], res[1][2])


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_fp16_running_sums_over_many_sweeps(mpr, mode):
    """With FP16 storage the averaging sweeps sum into 32-bit words of 2^-24 units, folded into
    the FP64 sums after at most 128 sweeps.  On every sweep path, the running sums after runs of
    130 and then 3 averaging sweeps (two folds in one call, then another call) equal bit for bit
    the double-precision sum of the angles read back after each of 133 one-sweep runs of a
    second context, and the two contexts' sums and predictions are equal; a batch of uneven open
    grids with two chains."""
    shapes = [(45, 70), (17, 300), (64, 64)]
    chains = 2
    fields = [_field(h, w, 900 + i) for i, (h, w) in enumerate(shapes)]
    z = np.concatenate([f[1].ravel() for f in fields])
    m = np.concatenate([f[2].ravel() for f in fields])
    # state layout: grid, then chain, then the grid's sites row-major
    free = np.concatenate([np.tile((f[2] == 0).ravel(), chains) for f in fields])

    def tempered():
        ctx = mpr.Context(shapes=shapes, stream=torch.cuda.Stream(), seed=6, n_chains=chains,
                          precision=mpr.FP16, sweep_mode=mode)
        ctx.batch_load(_dev(z, torch.float64), _dev(m, torch.uint8))
        assert ctx.sweep_mode() == mode
        ctx.infer_temperature(12)
        return ctx

    a = tempered()
    a.run(130)
    acc130 = a.get_state()["acc"].cpu().numpy()
    a.run(3)
    acc_a = a.get_state()["acc"].cpu().numpy()
    b = tempered()
    host = np.zeros_like(acc_a)
    for _ in range(133):
        b.run(1)
        host += b.get_state()["u"].cpu().numpy()
    acc_b = b.get_state()["acc"].cpu().numpy()
    assert np.array_equal(acc_a[free], host[free])
    assert np.array_equal(acc_a, acc_b)
    assert np.array_equal(a.predictions().cpu().numpy(), b.predictions().cpu().numpy())
    assert acc_a[free].max() > 20.0 and (acc_a[free] > acc130[free]).any()
