"""Python binding of libmpr.so (include/mpr.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels; PyTorch provides device memory
(tensors) and the stream.  The functions below carry the C names; `Context` wraps them for
convenience.  If the library is missing, importing this module raises: there is no fallback.
"""
import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmpr.so")

OK, EINVAL, ENOSAMPLE, EBIPARTITE, ESTATE, ENOMEM, EHIP = range(7)
FP64, FP32, FP16, FIX16 = 0, 1, 2, 3
PREC_DEFAULT, PREC_DOUBLE, PREC_SINGLE = -1, 0, 1
OPEN, PERIODIC = 0, 1
DEC_OR, DEC_ACCEPT, DEC_OUTSIDE = 1, 2, 4
SWEEP_AUTO, SWEEP_FUSED, SWEEP_SPARSE, SWEEP_TILED = 0, 1, 2, 3
TILE_W4_BASE, TILE_W8_TALL, TILE_W4_TALL, TILE_W8_BASE = 0, 1, 2, 3

if not os.path.exists(LIB_PATH):
    raise ImportError("libmpr.so is not built (%s); run paper_1910_08448_amd/build.py" % LIB_PATH)
_lib = ctypes.CDLL(LIB_PATH)


class mpr_config(ctypes.Structure):
    _fields_ = [("q", ctypes.c_double), ("J", ctypes.c_double),
                ("precision", ctypes.c_int32), ("energy_prec", ctypes.c_int32),
                ("func_prec", ctypes.c_int32), ("boundary", ctypes.c_int32),
                ("n_chains", ctypes.c_int32), ("grid_offset", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("alpha0", ctypes.c_double),
                ("acc_target", ctypes.c_double), ("T_min", ctypes.c_double),
                ("T_max", ctypes.c_double), ("tile_rows", ctypes.c_int32),
                ("graph_sweeps", ctypes.c_int32), ("sweep_mode", ctypes.c_int32),
                ("tile_shape", ctypes.c_int32), ("group_waves", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 3)]


class mpr_timings(ctypes.Structure):
    _fields_ = [("load_ms", ctypes.c_double), ("infer_ms", ctypes.c_double),
                ("run_ms", ctypes.c_double), ("predict_ms", ctypes.c_double),
                ("infer_sweeps", ctypes.c_int64), ("run_sweeps", ctypes.c_int64)]


class mpr_chain_stats(ctypes.Structure):
    _fields_ = [("T", ctypes.c_double), ("alpha", ctypes.c_double),
                ("e_sample", ctypes.c_double), ("e_sim", ctypes.c_double),
                ("acc_rate", ctypes.c_double), ("n_pred", ctypes.c_int64),
                ("n_bonds", ctypes.c_int64), ("n_sample_bonds", ctypes.c_int64),
                ("zmin", ctypes.c_double), ("zmax", ctypes.c_double)]


_vp, _i32, _i64, _d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_SIG = {
    "mpr_config_default": (None, [_vp]),
    "mpr_create": (ctypes.c_int, [_vp, _vp, _vp]),
    "mpr_batch_create": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp, _vp]),
    "mpr_destroy": (None, [_vp]),
    "mpr_load": (ctypes.c_int, [_vp, _i64, _i64, _vp, _vp]),
    "mpr_batch_load": (ctypes.c_int, [_vp, _vp, _vp]),
    "mpr_infer_temperature": (ctypes.c_int, [_vp, _i32, _vp]),
    "mpr_set_temperature": (ctypes.c_int, [_vp, _d]),
    "mpr_equilibrate": (ctypes.c_int, [_vp, _i32, _vp]),
    "mpr_energy_curve": (ctypes.c_int, [_vp, _vp, _i32, _i32, _vp, _i32, _i32, _vp, _vp]),
    "mpr_set_temperature_curve": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp]),
    "mpr_set_temperature_curve_noalloc": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp]),
    "mpr_burn_in": (ctypes.c_int, [_vp, _i32]),
    "mpr_run": (ctypes.c_int, [_vp, _i32]),
    "mpr_get_predictions": (ctypes.c_int, [_vp, _vp]),
    "mpr_get_stats": (ctypes.c_int, [_vp, _vp]),
    "mpr_get_trace": (ctypes.c_int, [_vp, _i32, _i32, _vp, _vp]),
    "mpr_get_state": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "mpr_set_state": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "mpr_debug_sweep": (ctypes.c_int, [_vp, _i32, _vp]),
    "mpr_bench_sweeps": (ctypes.c_int, [_vp, _i32]),
    "mpr_autotune": (ctypes.c_int, [_vp, _i32, _vp]),
    "mpr_get_shape": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "mpr_get_sweep_mode": (ctypes.c_int, [_vp, _vp]),
    "mpr_get_tuning": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "mpr_get_timings": (ctypes.c_int, [_vp, _vp]),
    "mpr_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "mpr_last_error": (ctypes.c_char_p, [_vp]),
}
EXPORTS = tuple(_SIG)
for _name, (_res, _args) in _SIG.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f


class MprError(RuntimeError):
    def __init__(self, code, what, detail=""):
        super().__init__("%s: %s (%d) %s" % (what, _lib.mpr_strerror(code).decode(), code, detail))
        self.code = code


def _ptr(t):
    """Device pointer of a torch tensor (or host pointer of a numpy array); None -> NULL."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return ctypes.c_void_p(t.data_ptr())
    return t.ctypes.data_as(ctypes.c_void_p)


def _check_dev(t, dtype, numel, what):
    """A device buffer handed to the library: a contiguous CUDA tensor of the given dtype and
    element count (the kernels read or write exactly that many elements, so anything else --
    a host array, another dtype, a short tensor -- is refused here instead of reaching them)."""
    if not hasattr(t, "data_ptr") or not getattr(t, "is_cuda", False):
        raise TypeError("%s must be a CUDA tensor" % what)
    if t.dtype != dtype:
        raise TypeError("%s must have dtype %s, not %s" % (what, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must hold %d elements, not %d" % (what, numel, t.numel()))


def default_config(**kw):
    cfg = mpr_config()
    _lib.mpr_config_default(ctypes.byref(cfg))
    for k, v in kw.items():
        if not hasattr(cfg, k):
            raise TypeError("unknown config field %r" % k)
        setattr(cfg, k, v)
    return cfg


class Context:
    """One library context on torch's current device.  `stream` is a torch.cuda.Stream (or None
    for torch's current stream)."""

    def __init__(self, shapes=None, stream=None, **cfg):
        import torch
        self.torch = torch
        self.cfg = default_config(**cfg)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        sp = ctypes.c_void_p(self.stream.cuda_stream)
        if shapes is None:
            rc = _lib.mpr_create(ctypes.byref(self.cfg), sp, ctypes.byref(h))
            self.shapes = None
        else:
            Hs = np.ascontiguousarray([s[0] for s in shapes], dtype=np.int64)
            Ws = np.ascontiguousarray([s[1] for s in shapes], dtype=np.int64)
            rc = _lib.mpr_batch_create(ctypes.byref(self.cfg), sp, len(shapes), _ptr(Hs), _ptr(Ws),
                                       ctypes.byref(h))
            self.shapes = [(int(a), int(b)) for a, b in zip(Hs, Ws)]
        if rc != OK:
            raise MprError(rc, "mpr_create")
        self.h = h

    def _chk(self, rc, what):
        if rc != OK:
            raise MprError(rc, what, _lib.mpr_last_error(self.h).decode())

    def _call(self, what, fn, *args):
        """Stream-ordered call: the library's stream waits for torch's current stream (inputs
        written there), and torch's current stream then waits for the library (outputs)."""
        cur = self.torch.cuda.current_stream()
        other = cur.cuda_stream != self.stream.cuda_stream
        if other:
            self.stream.wait_stream(cur)
        rc = fn(self.h, *args)
        if other:
            cur.wait_stream(self.stream)
        self._chk(rc, what)

    def close(self):
        if getattr(self, "h", None):
            _lib.mpr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- verbs
    @property
    def n_chains(self):
        return self.cfg.n_chains

    @property
    def n_grids(self):
        return 1 if self.shapes is None else len(self.shapes)

    def n_sites(self):
        return sum(h * w for h, w in self.shapes)

    def sweep_mode(self):
        """The sweep path chosen at the last load: SWEEP_FUSED, SWEEP_SPARSE or SWEEP_TILED."""
        m = ctypes.c_int32()
        self._chk(_lib.mpr_get_sweep_mode(self.h, ctypes.byref(m)), "mpr_get_sweep_mode")
        return m.value

    def timings(self):
        """Stream time (ms) of the last load, inference, averaging run and predictions, and the
        sweeps of the last inference and run."""
        t = mpr_timings()
        self._chk(_lib.mpr_get_timings(self.h, ctypes.byref(t)), "mpr_get_timings")
        return {k: getattr(t, k) for k, _ in mpr_timings._fields_}

    def tuning(self):
        """(sweep path, fused rows per work item, tiled block shape or -1, sweeps per graph or -1)
        the context sweeps with."""
        v = [ctypes.c_int32() for _ in range(4)]
        self._chk(_lib.mpr_get_tuning(self.h, *[ctypes.byref(x) for x in v]), "mpr_get_tuning")
        return tuple(x.value for x in v)

    def load(self, z, mask):
        """z: float64 CUDA tensor [H, W]; mask: uint8 CUDA tensor [H, W]."""
        if z.dim() != 2 or tuple(mask.shape) != tuple(z.shape):
            raise ValueError("z and mask must be [H, W] tensors of the same shape")
        _check_dev(z, self.torch.float64, None, "z")
        _check_dev(mask, self.torch.uint8, None, "mask")
        self._call("mpr_load", _lib.mpr_load, z.shape[0], z.shape[1], _ptr(z), _ptr(mask))
        self.shapes = [(int(z.shape[0]), int(z.shape[1]))]

    def batch_load(self, z_packed, mask_packed):
        _check_dev(z_packed, self.torch.float64, self.n_sites(), "z_packed")
        _check_dev(mask_packed, self.torch.uint8, self.n_sites(), "mask_packed")
        self._call("mpr_batch_load", _lib.mpr_batch_load, _ptr(z_packed), _ptr(mask_packed))

    def infer_temperature(self, n_equil, want_T=True):
        T = np.zeros(self.n_grids * self.n_chains) if want_T else None
        self._call("mpr_infer_temperature", _lib.mpr_infer_temperature, n_equil, _ptr(T))
        return T

    def set_temperature(self, T):
        self._call("mpr_set_temperature", _lib.mpr_set_temperature, T)

    def equilibrate(self, n, want_T=True):
        T = np.zeros(self.n_grids * self.n_chains) if want_T else None
        self._call("mpr_equilibrate", _lib.mpr_equilibrate, n, _ptr(T))
        return T

    def set_temperature_curve(self, T, e):
        T = np.ascontiguousarray(T, dtype=np.float64)
        e = np.ascontiguousarray(e, dtype=np.float64)
        out = np.zeros(self.n_grids * self.n_chains)
        self._call("mpr_set_temperature_curve", _lib.mpr_set_temperature_curve, T.size, _ptr(T),
                   _ptr(e), _ptr(out))
        return out

    def burn_in(self, n):
        self._call("mpr_burn_in", _lib.mpr_burn_in, n)

    def autotune(self, n_sweeps=8):
        rows = ctypes.c_int32()
        self._call("mpr_autotune", _lib.mpr_autotune, n_sweeps, ctypes.byref(rows))
        return rows.value

    def bench_sweeps(self, n):
        self._call("mpr_bench_sweeps", _lib.mpr_bench_sweeps, n)

    def run(self, n_avg):
        self._call("mpr_run", _lib.mpr_run, n_avg)

    def predictions(self, out=None):
        t = self.torch
        if out is None:
            out = t.empty(self.n_sites(), dtype=t.float64, device="cuda")
        _check_dev(out, t.float64, self.n_sites(), "out")
        self._call("mpr_get_predictions", _lib.mpr_get_predictions, _ptr(out))
        return out

    def stats(self):
        arr = (mpr_chain_stats * (self.n_grids * self.n_chains))()
        self._call("mpr_get_stats", _lib.mpr_get_stats, arr)
        return [{k: getattr(s, k) for k, _ in mpr_chain_stats._fields_} for s in arr]

    def trace(self, grid_chain=0, max_entries=1 << 20):
        n_out = ctypes.c_int32()
        buf = np.zeros((max_entries, 4))
        self._call("mpr_get_trace", _lib.mpr_get_trace, grid_chain, max_entries, _ptr(buf), ctypes.byref(n_out))
        return buf[: n_out.value]

    def get_state(self):
        t = self.torch
        n = self.n_sites() * self.n_chains
        u = t.empty(n, dtype=t.float64, device="cuda")
        acc = t.empty(n, dtype=t.float64, device="cuda")
        ctl = np.zeros((self.n_grids * self.n_chains, 2))
        meta = np.zeros(3, dtype=np.int64)
        self._call("mpr_get_state", _lib.mpr_get_state, _ptr(u), _ptr(acc), _ptr(ctl), _ptr(meta))
        return {"u": u, "acc": acc, "ctl": ctl, "meta": meta}

    def set_state(self, u=None, acc=None, ctl=None, meta=None):
        n = self.n_sites() * self.n_chains
        for name, a in (("u", u), ("acc", acc)):
            if a is not None:
                _check_dev(a, self.torch.float64, n, name)
        ctl = None if ctl is None else np.ascontiguousarray(ctl, dtype=np.float64)
        meta = None if meta is None else np.ascontiguousarray(meta, dtype=np.int64)
        if ctl is not None and ctl.size != 2 * self.n_grids * self.n_chains:
            raise ValueError("ctl must hold (T, alpha) for each of the %d chains" % (self.n_grids * self.n_chains))
        if meta is not None and meta.size != 3:
            raise ValueError("meta must hold 3 values")
        self._call("mpr_set_state", _lib.mpr_set_state, _ptr(u), _ptr(acc), _ptr(ctl), _ptr(meta))

    def debug_sweep(self, sweep):
        t = self.torch
        d = t.empty(self.n_sites() * self.n_chains, dtype=t.uint8, device="cuda")
        self._call("mpr_debug_sweep", _lib.mpr_debug_sweep, sweep, _ptr(d))
        return d


def energy_curve(side, T, n_burn, n_meas, with_trace=False, stream=None, **cfg):
    """Mean bond energy e(T) of the data-free model on a periodic side x side lattice at each
    temperature of T (host array); returns a numpy array (and the per-sweep trace
    [n_T][n_burn + n_meas][4] if with_trace).  Runs on `stream` (torch's current stream if
    None) and synchronises."""
    import torch
    T = np.ascontiguousarray(T, dtype=np.float64)
    e = np.zeros(T.size)
    tr = np.zeros((T.size, n_burn + n_meas, 4)) if with_trace else None
    st = stream if stream is not None else torch.cuda.current_stream()
    c = default_config(**cfg)
    rc = _lib.mpr_energy_curve(ctypes.byref(c), ctypes.c_void_p(st.cuda_stream), side, T.size,
                               _ptr(T), n_burn, n_meas, _ptr(e), _ptr(tr))
    if rc != OK:
        raise MprError(rc, "mpr_energy_curve")
    return (e, tr) if with_trace else e


def predict(z, mask, n_equil, n_avg, stream=None, **cfg):
    """Whole method on one grid (torch CUDA tensors in, float64 CUDA tensor out)."""
    ctx = Context(stream=stream, **cfg)
    ctx.load(z, mask)
    T = ctx.infer_temperature(n_equil)
    ctx.run(n_avg)
    out = ctx.predictions().view(z.shape[0], z.shape[1])
    ctx.close()
    return out, T
