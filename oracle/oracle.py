"""ctypes wrapper of the FP64 CPU oracle (oracle/mpr_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the benchmark's
CPU-baseline leg.  The GPU library and its Python binding never import this module.
Angles here are in radians (phi in [0, 2 pi]), as in the paper's Eq. (2).
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mpr_oracle.c")
# MPR_ORACLE_LIB points the wrapper at another build of the oracle (the planted-mistake test
# uses it to check that the pins fail on a broken oracle)
_OVERRIDE = os.environ.get("MPR_ORACLE_LIB")
LIB_PATH = _OVERRIDE or os.path.join(HERE, "liboracle.so")

OK, EINVAL, ENOSAMPLE, EBIPARTITE, ESTATE, ENOMEM = range(6)
OPEN, PERIODIC = 0, 1
DEC_OR, DEC_ACCEPT, DEC_OUTSIDE = 1, 2, 4


def build(force=False):
    """Compile the oracle with gcc (plain IEEE double arithmetic, no FMA contraction)."""
    if _OVERRIDE:
        return LIB_PATH
    if not force and os.path.exists(LIB_PATH) and os.path.getmtime(LIB_PATH) >= max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "mpr_oracle.h"))):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
                           "-fno-fast-math", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Config(ctypes.Structure):
    _fields_ = [("q", ctypes.c_double), ("J", ctypes.c_double),
                ("boundary", ctypes.c_int32), ("n_chains", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("alpha0", ctypes.c_double),
                ("acc_target", ctypes.c_double), ("T_min", ctypes.c_double),
                ("T_max", ctypes.c_double), ("grid_id", ctypes.c_int32),
                ("n_threads", ctypes.c_int32)]


class ChainStats(ctypes.Structure):
    _fields_ = [("T", ctypes.c_double), ("alpha", ctypes.c_double),
                ("e_sample", ctypes.c_double), ("e_sim", ctypes.c_double),
                ("acc_rate", ctypes.c_double), ("n_pred", ctypes.c_int64),
                ("n_bonds", ctypes.c_int64), ("n_sample_bonds", ctypes.c_int64),
                ("zmin", ctypes.c_double), ("zmax", ctypes.c_double)]


_lib = None
_P = ctypes.POINTER
_d, _i64, _i32, _u32, _u64 = ctypes.c_double, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
_vp = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "orc_philox4x32_10": (None, [_vp, _vp, _vp]),
            "orc_uniform": (_d, [_u32]),
            "orc_site_words": (None, [_u64, _i64, _i64, _i64, _u32, _u32, _u32, _vp, _vp]),
            "orc_map": (ctypes.c_int, [_i64, _vp, _vp, _vp, _vp, _vp]),
            "orc_bond_sum": (_d, [_i64, _i64, _vp, _vp, _i32, _d, _vp, _i32]),
            "orc_local_field": (None, [_i64, _i64, _vp, _i32, _d, _i64, _i64, _vp, _vp]),
            "orc_site_energy": (_d, [_i64, _i64, _vp, _i32, _d, _d, _i64, _i64, _d]),
            "orc_overrelax": (_d, [_d, _d, _d, _d, _vp]),
            "orc_site_update": (_i32, [_i64, _i64, _vp, _i32, _d, _d, _d, _d, _i64, _i64, _u32, _u32]),
            "orc_sweep": (_i64, [_i64, _i64, _vp, _vp, _i32, _d, _d, _d, _d, _u64, _u32, _u32, _i32, _vp]),
            "orc_init_chain": (None, [_i64, _i64, _vp, _vp, _u64, _u32]),
            "orc_create": (ctypes.c_int, [_vp, _vp]),
            "orc_destroy": (None, [_vp]),
            "orc_load": (ctypes.c_int, [_vp, _i64, _i64, _vp, _vp]),
            "orc_infer_temperature": (ctypes.c_int, [_vp, _i32, _vp]),
            "orc_set_temperature": (ctypes.c_int, [_vp, _d]),
            "orc_run": (ctypes.c_int, [_vp, _i32]),
            "orc_get_predictions": (ctypes.c_int, [_vp, _vp]),
            "orc_get_stats": (ctypes.c_int, [_vp, _vp]),
            "orc_get_trace": (ctypes.c_int, [_vp, _i32, _i32, _vp, _vp]),
            "orc_get_state": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
            "orc_set_state": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
            "orc_debug_sweep": (ctypes.c_int, [_vp, _i32, _vp]),
            "orc_burn_in": (ctypes.c_int, [_vp, _i32]),
            "orc_run_record": (ctypes.c_int, [_vp, _i32, _i32, _vp, _vp]),
            "orc_equilibrate": (ctypes.c_int, [_vp, _i32, _vp]),
            "orc_energy_curve": (ctypes.c_int, [_vp, _i64, _i32, _vp, _i32, _i32, _vp, _vp]),
            "orc_curve_temperature": (_d, [_i32, _vp, _vp, _d]),
            "orc_set_temperature_curve": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s failed with code %d" % (what, code))
        self.code = code


def _chk(rc, what):
    if rc != OK:
        raise OracleError(rc, what)


# ---------------------------------------------------------------- primitives
def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(w):
    return lib().orc_uniform(int(w))


def site_words(seed, W, y, x, sweep, chain, tag):
    wa, wb = ctypes.c_uint32(), ctypes.c_uint32()
    lib().orc_site_words(seed, W, y, x, sweep, chain, tag, ctypes.byref(wa), ctypes.byref(wb))
    return wa.value, wb.value


def map_data(z, mask):
    z = np.ascontiguousarray(z, dtype=np.float64)
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    phi = np.zeros_like(z)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    rc = lib().orc_map(z.size, _ptr(z), _ptr(m), ctypes.byref(lo), ctypes.byref(hi), _ptr(phi))
    _chk(rc, "orc_map")
    return phi, lo.value, hi.value


def bond_sum(phi, mask=None, boundary=OPEN, q=0.5, n_threads=1):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    nb = ctypes.c_int64()
    s = lib().orc_bond_sum(phi.shape[0], phi.shape[1], _ptr(phi), _ptr(m), boundary, q,
                           ctypes.byref(nb), n_threads)
    return s, nb.value


def local_field(phi, y, x, boundary=OPEN, q=0.5):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    C, S = ctypes.c_double(), ctypes.c_double()
    lib().orc_local_field(phi.shape[0], phi.shape[1], _ptr(phi), boundary, q, y, x,
                          ctypes.byref(C), ctypes.byref(S))
    return C.value, S.value


def site_energy(phi, y, x, phi_i, boundary=OPEN, q=0.5, J=1.0):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    return lib().orc_site_energy(phi.shape[0], phi.shape[1], _ptr(phi), boundary, q, J, y, x, phi_i)


def overrelax(phi_i, C, S, q=0.5):
    applied = ctypes.c_int32()
    v = lib().orc_overrelax(phi_i, C, S, q, ctypes.byref(applied))
    return v, bool(applied.value)


def site_update(phi, y, x, T, alpha, wa, wb, boundary=OPEN, q=0.5, J=1.0):
    """Updates phi (a C-contiguous float64 array) in place; returns the decision bits."""
    assert phi.dtype == np.float64 and phi.flags.c_contiguous
    return lib().orc_site_update(phi.shape[0], phi.shape[1], _ptr(phi), boundary, q, J, T,
                                 alpha, y, x, wa, wb)


def sweep(phi, mask, T, alpha, seed, sweep_index, chain=0, boundary=OPEN, q=0.5, J=1.0,
          n_threads=1, decisions=None):
    """One hybrid sweep on a plain array (in place); returns the number of accepted moves."""
    assert phi.dtype == np.float64 and phi.flags.c_contiguous
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    return lib().orc_sweep(phi.shape[0], phi.shape[1], _ptr(phi), _ptr(m), boundary, q, J, T,
                           alpha, seed, sweep_index, chain, n_threads, _ptr(decisions))


def init_chain(phi, mask, seed, chain=0):
    assert phi.dtype == np.float64 and phi.flags.c_contiguous
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    lib().orc_init_chain(phi.shape[0], phi.shape[1], _ptr(phi), _ptr(m), seed, chain)


# ---------------------------------------------------------------- context
def config(q=0.5, J=1.0, boundary=OPEN, n_chains=1, seed=2001, alpha0=1.0, acc_target=0.3,
           T_min=1e-6, T_max=10.0, grid_id=0, n_threads=0):
    return Config(q, J, boundary, n_chains, seed, alpha0, acc_target, T_min, T_max, grid_id,
                  n_threads)


class Oracle:
    """Context verbs of the oracle, mirroring the GPU library's verbs on host arrays."""

    def __init__(self, **kw):
        self.h = None
        self.cfg = config(**kw)
        h = ctypes.c_void_p()
        _chk(lib().orc_create(ctypes.byref(self.cfg), ctypes.byref(h)), "orc_create")
        self.h = h
        self.shape = None

    def close(self):
        if self.h:
            lib().orc_destroy(self.h)
            self.h = None

    __del__ = close

    def load(self, z, mask):
        z = np.ascontiguousarray(z, dtype=np.float64)
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        _chk(lib().orc_load(self.h, z.shape[0], z.shape[1], _ptr(z), _ptr(m)), "orc_load")
        self.shape = z.shape

    def infer_temperature(self, n_equil):
        T = np.zeros(self.cfg.n_chains)
        _chk(lib().orc_infer_temperature(self.h, n_equil, _ptr(T)), "orc_infer_temperature")
        return T

    def set_temperature(self, T):
        _chk(lib().orc_set_temperature(self.h, T), "orc_set_temperature")

    def run(self, n_avg):
        _chk(lib().orc_run(self.h, n_avg), "orc_run")

    def predictions(self):
        out = np.zeros(self.shape)
        _chk(lib().orc_get_predictions(self.h, _ptr(out)), "orc_get_predictions")
        return out

    def stats(self):
        arr = (ChainStats * self.cfg.n_chains)()
        _chk(lib().orc_get_stats(self.h, arr), "orc_get_stats")
        return [{k: getattr(s, k) for k, _ in ChainStats._fields_} for s in arr]

    def trace(self, chain=0, max_entries=1 << 20):
        buf = np.zeros((max_entries, 4))
        n = ctypes.c_int32()
        _chk(lib().orc_get_trace(self.h, chain, max_entries, _ptr(buf), ctypes.byref(n)),
             "orc_get_trace")
        return buf[:n.value]

    def get_state(self):
        C = self.cfg.n_chains
        n = self.shape[0] * self.shape[1]
        phi = np.zeros((C,) + tuple(self.shape))
        acc = np.zeros((C,) + tuple(self.shape))
        ctl = np.zeros((C, 2))
        meta = np.zeros(3, dtype=np.int64)
        _chk(lib().orc_get_state(self.h, _ptr(phi), _ptr(acc), _ptr(ctl), _ptr(meta)),
             "orc_get_state")
        assert phi.size == C * n
        return {"phi": phi, "acc": acc, "ctl": ctl, "meta": meta}

    def set_state(self, phi=None, acc=None, ctl=None, meta=None):
        f = lambda a, dt: None if a is None else np.ascontiguousarray(a, dtype=dt)
        phi, acc, ctl, meta = f(phi, np.float64), f(acc, np.float64), f(ctl, np.float64), f(meta, np.int64)
        _chk(lib().orc_set_state(self.h, _ptr(phi), _ptr(acc), _ptr(ctl), _ptr(meta)),
             "orc_set_state")

    def debug_sweep(self, sweep_index):
        d = np.zeros((self.cfg.n_chains,) + tuple(self.shape), dtype=np.uint8)
        _chk(lib().orc_debug_sweep(self.h, sweep_index, _ptr(d)), "orc_debug_sweep")
        return d

    def burn_in(self, n):
        _chk(lib().orc_burn_in(self.h, n), "orc_burn_in")

    def equilibrate(self, n):
        T = np.zeros(self.cfg.n_chains)
        _chk(lib().orc_equilibrate(self.h, n, _ptr(T)), "orc_equilibrate")
        return T

    def set_temperature_curve(self, T, e):
        T = np.ascontiguousarray(T, dtype=np.float64)
        e = np.ascontiguousarray(e, dtype=np.float64)
        out = np.zeros(self.cfg.n_chains)
        _chk(lib().orc_set_temperature_curve(self.h, T.size, _ptr(T), _ptr(e), _ptr(out)),
             "orc_set_temperature_curve")
        return out

    def run_record(self, n, sites):
        sites = np.ascontiguousarray(np.atleast_1d(sites), dtype=np.int64)
        out = np.zeros((n, sites.size))
        _chk(lib().orc_run_record(self.h, n, sites.size, _ptr(sites), _ptr(out)),
             "orc_run_record")
        return out


def energy_curve(side, T, n_burn, n_meas, with_trace=False, **kw):
    """Unconditional mean bond energy e(T) on a periodic side x side lattice (see the C header);
    returns e (and the per-sweep trace [n_T][n_burn + n_meas][4] if with_trace)."""
    T = np.ascontiguousarray(T, dtype=np.float64)
    cfg = config(**kw)
    e = np.zeros(T.size)
    tr = np.zeros((T.size, n_burn + n_meas, 4)) if with_trace else None
    _chk(lib().orc_energy_curve(ctypes.byref(cfg), side, T.size, _ptr(T), n_burn, n_meas,
                                _ptr(e), _ptr(tr)), "orc_energy_curve")
    return (e, tr) if with_trace else e


def curve_temperature(T, e, e_target):
    T = np.ascontiguousarray(T, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    return lib().orc_curve_temperature(T.size, _ptr(T), _ptr(e), e_target)


def predict(z, mask, n_equil, n_avg, **kw):
    """Whole method on host arrays: returns (zhat, T_hat per chain)."""
    o = Oracle(**kw)
    o.load(z, mask)
    T = o.infer_temperature(n_equil)
    o.run(n_avg)
    return o.predictions(), T
