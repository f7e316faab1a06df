"""ctypes binding of include/ipt.h.  Argument marshalling only: every step of a
solve runs in the HIP kernels of libipt.so.  Tensors must be CUDA (ROCm) tensors
on the handle's device; the library writes the outputs in place on the current
torch stream."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libipt.so")

IPT_OK, IPT_EINVAL, IPT_EDEGENERATE, IPT_ENOTCONV, IPT_EHIP, IPT_ENOMEM, IPT_EGUARD = range(7)
CONVERGED, NOT_CONVERGED, DIVERGED = 0, 1, 2
PREC_FP64, PREC_LADDER = 0, 1
LOW_BF16, LOW_FP16, LOW_NONE = 0, 1, 2
SWEEP_NAMES = {0: "exact-first", 1: "low", 2: "fp32", 3: "fp64"}
IPT_HIST = 128
FLAG_NO_NORM = 1
FLAG_TIME_KERNELS = 2
FLAG_NO_GRAPH = 4
FLAG_ACX = 8
FLAG_MID_FP32 = 16
FLAG_CHOOSE_D = 32
PAIR_TAU = 0.05
CERTIFY_SLACK = 2.0
TILE_BUCKETS = 64  # batched tile table: bucket q holds 64 q < n <= 64 (q + 1)


class Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("precision", C.c_int32), ("low_type", C.c_int32),
                ("sync_every", C.c_int32), ("tau_low", C.c_double), ("tau_32", C.c_double),
                ("div_norm", C.c_double), ("div_growth", C.c_int32), ("flags", C.c_int32),
                ("cont_alpha", C.c_double), ("homotopy_q", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("converged", C.c_int32), ("not_converged", C.c_int32),
                ("diverged", C.c_int32), ("matvecs", C.c_int64), ("max_step", C.c_double), ("norm1", C.c_double),
                ("max_resid", C.c_double), ("time_ms", C.c_float), ("hist_len", C.c_int32),
                ("sweep_prec", C.c_int32 * IPT_HIST), ("sweep_active", C.c_int32 * IPT_HIST),
                ("sweep_max_step", C.c_double * IPT_HIST), ("prec_ms", C.c_float * 4),
                ("prec_sweeps", C.c_int32 * 4), ("sweep_ms", C.c_float * IPT_HIST)]

    def as_dict(self):
        h = self.hist_len
        return {"sweeps": self.sweeps, "converged": self.converged, "not_converged": self.not_converged,
                "diverged": self.diverged, "matvecs": self.matvecs, "max_step": self.max_step,
                "norm1": self.norm1, "max_resid": self.max_resid, "time_ms": self.time_ms,
                "sweep_prec": [SWEEP_NAMES[p] for p in self.sweep_prec[:h]],
                "sweep_active": list(self.sweep_active[:h]), "sweep_max_step": list(self.sweep_max_step[:h]),
                "prec_ms": {SWEEP_NAMES[q]: self.prec_ms[q] for q in range(4)},
                "prec_sweeps": {SWEEP_NAMES[q]: self.prec_sweeps[q] for q in range(4)},
                "sweep_ms": list(self.sweep_ms[:h])}


class ColInfo(C.Structure):
    _fields_ = [("sweeps", C.c_void_p), ("step", C.c_void_p), ("resid", C.c_void_p)]


class IPTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%s)" % (msg, status))
        self.status = status


_lib = None


def library_path() -> str:
    return _LIB


def _hip_runtimes():
    try:
        maps = open("/proc/self/maps").read().splitlines()
    except OSError:
        return []
    return sorted({ln.split()[-1] for ln in maps if "libamdhip64" in ln})


def load_library():
    """Load libipt.so; raises if it has not been built (there is no fallback).

    torch is imported first so that its HIP runtime is the one in the process:
    libipt.so then binds to it by soname and the streams and device pointers that
    torch hands over belong to the same runtime.  Two HIP runtimes in one process
    are refused."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        raise ImportError("libipt.so is not built: run __graft_entry__.build() (hipcc --offload-arch=gfx950)")
    import torch  # noqa: F401  (loads the HIP runtime the tensors live in)
    lib = C.CDLL(_LIB)
    runtimes = _hip_runtimes()
    if len(runtimes) > 1:
        raise ImportError("two HIP runtimes are loaded (%s); import torch before loading libipt.so" % runtimes)
    p, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
    lib.ipt_opts_default.argtypes = [C.POINTER(Opts)]
    lib.ipt_opts_default.restype = None
    lib.ipt_create.argtypes = [C.POINTER(p), p]
    lib.ipt_destroy.argtypes = [p]
    lib.ipt_set_stream.argtypes = [p, p]
    lib.ipt_solve_dense.argtypes = [p, i64, p, p, i64, i64, p, p, i64, C.POINTER(Opts), p, i64, p, p,
                                    C.POINTER(Info), C.POINTER(ColInfo)]
    lib.ipt_solve_dense_noalloc.argtypes = [p, i64, p, p, i64, i64, p, p, i64, C.POINTER(Opts), p, i64, p, p,
                                            C.POINTER(Info), C.POINTER(ColInfo)]
    lib.ipt_solve_dense_z.argtypes = [p, i64, p, p, i64, i64, p, p, i64, C.POINTER(Opts), p, i64, p, p,
                                    C.POINTER(Info), C.POINTER(ColInfo)]
    lib.ipt_solve_csr.argtypes = [p, i64, p, p, p, p, i64, i64, p, p, i64, C.POINTER(Opts), p, i64, p, p,
                                  C.POINTER(Info), C.POINTER(ColInfo)]
    lib.ipt_solve_csr_z.argtypes = lib.ipt_solve_csr.argtypes
    lib.ipt_solve_batched.argtypes = [p, i32, p, p, p, p, p, p, C.POINTER(Opts), p, p, p, C.POINTER(Info)]
    lib.ipt_batched_tune.argtypes = [p, i32, p, p, p, p, p, p, p, p, p, p]
    lib.ipt_batched_get_tiles.argtypes = [p, p]
    lib.ipt_batched_set_tiles.argtypes = [p, p]
    lib.ipt_status_string.argtypes = [C.c_int]
    lib.ipt_status_string.restype = C.c_char_p
    lib.ipt_last_error.argtypes = [p]
    lib.ipt_last_error.restype = C.c_char_p
    for fn in ("ipt_create", "ipt_destroy", "ipt_set_stream", "ipt_solve_dense", "ipt_solve_dense_noalloc",
               "ipt_solve_dense_z", "ipt_solve_csr", "ipt_solve_csr_z",
               "ipt_solve_batched", "ipt_batched_tune", "ipt_batched_get_tiles", "ipt_batched_set_tiles"):
        getattr(lib, fn).restype = C.c_int
    _lib = lib
    return lib


def default_opts(**kw) -> Opts:
    o = Opts()
    load_library().ipt_opts_default(C.byref(o))
    for key, val in kw.items():
        if not hasattr(o, key):
            raise TypeError("unknown option " + key)
        setattr(o, key, val)
    return o


class Handle:
    """An ipt_handle bound to the current device and torch stream."""

    def __init__(self, stream=None):
        import torch
        lib = load_library()
        s = stream if stream is not None else torch.cuda.current_stream()
        self._h = C.c_void_p()
        st = lib.ipt_create(C.byref(self._h), C.c_void_p(s.cuda_stream))
        if st != IPT_OK:
            raise IPTError(st, "ipt_create failed")
        self._stream = s

    def set_stream(self, stream):
        load_library().ipt_set_stream(self._h, C.c_void_p(stream.cuda_stream))
        self._stream = stream

    @property
    def ptr(self):
        return self._h

    def last_error(self) -> str:
        return load_library().ipt_last_error(self._h).decode()

    def close(self):
        if self._h:
            load_library().ipt_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_handles = {}


def _handle(h):
    if h is not None:
        return h
    import torch
    key = (torch.cuda.current_device(), torch.cuda.current_stream().cuda_stream)
    if key not in _default_handles:
        _default_handles[key] = Handle()
    return _default_handles[key]


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check(t, dtype, name, cuda=True):
    import torch
    if t is None:
        return
    if cuda and not t.is_cuda:
        raise ValueError(name + " must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError("%s must be %s" % (name, dtype))


def _opts(opts, kw):
    if opts is None:
        return default_opts(**kw)
    for key, val in kw.items():
        setattr(opts, key, val)
    return opts


class Result(dict):
    __getattr__ = dict.__getitem__


def _colinfo(k, want):
    import torch
    if not want:
        return None, None
    dev = torch.cuda.current_device()
    sw = torch.empty(k, dtype=torch.int32, device=dev)
    stp = torch.empty(k, dtype=torch.float64, device=dev)
    res = torch.empty(k, dtype=torch.float64, device=dev)
    ci = ColInfo(sw.data_ptr(), stp.data_ptr(), res.data_ptr())
    return ci, (sw, stp, res)


def _finish(lib, h, st, z, lam, status, info, extra, raise_on=(IPT_EINVAL, IPT_EDEGENERATE, IPT_EHIP, IPT_ENOMEM, IPT_EGUARD)):
    if st in raise_on:
        raise IPTError(st, h.last_error())
    r = Result(z=z, lam=lam, status=status, info=info.as_dict(), code=st)
    if extra is not None:
        r["sweeps"], r["step"], r["resid"] = extra
    return r


def ipt_solve_dense(theta, delta, idx=None, z0=None, opts=None, handle=None, colinfo=True, z_out=None, **kw):
    """Dense IPT solve (ipt_solve_dense).  theta [n] f64, delta [n, n] f64 (row-major,
    row stride = lda), idx [k] int32 or None, z0 [n, k] f64 or None.  Returns a Result
    with z [n, k], lam [k], status [k] and info (a dict of ipt_info)."""
    return _solve_dense("ipt_solve_dense", theta, delta, idx, z0, opts, handle, colinfo, z_out, None, None, kw)


def ipt_solve_dense_noalloc(theta, delta, idx=None, z0=None, opts=None, handle=None, colinfo=True, z_out=None,
                            lam_out=None, status_out=None, **kw):
    """ipt_solve_dense_noalloc: the dense solve on the library's fixed per-device
    workspace (no allocation inside the call; the outputs are the caller's, allocated
    here when not given).  Same arguments and Result as ipt_solve_dense."""
    return _solve_dense("ipt_solve_dense_noalloc", theta, delta, idx, z0, opts, handle, colinfo, z_out, lam_out,
                        status_out, kw)


def _solve_dense(entry, theta, delta, idx, z0, opts, handle, colinfo, z_out, lam, status, kw):
    import torch
    lib = load_library()
    h = _handle(handle)
    _check(theta, torch.float64, "theta")
    _check(delta, torch.float64, "delta")
    _check(idx, torch.int32, "idx")
    _check(z0, torch.float64, "z0")
    n = theta.shape[0]
    if delta.dim() != 2 or delta.shape[0] != n or delta.shape[1] != n or delta.stride(1) != 1:
        raise ValueError("delta must be n x n with unit column stride")
    k = n if idx is None else idx.shape[0]
    if z0 is not None and (z0.dim() != 2 or z0.shape[0] != n or z0.shape[1] != k or z0.stride(1) != 1):
        raise ValueError("z0 must be n x k with unit column stride")
    dev = theta.device
    if z_out is None:
        z_out = torch.empty((n, k), dtype=torch.float64, device=dev)
    if lam is None:
        lam = torch.empty(k, dtype=torch.float64, device=dev)
    if status is None:
        status = torch.empty(k, dtype=torch.int32, device=dev)
    _check(lam, torch.float64, "lam_out")
    _check(status, torch.int32, "status_out")
    if z_out.dim() != 2 or z_out.shape[0] != n or z_out.shape[1] != k or z_out.stride(1) != 1 or lam.numel() < k \
            or status.numel() < k:
        raise ValueError("outputs must be z_out [n, k] with unit column stride, lam_out [k], status_out [k]")
    o = _opts(opts, kw)
    info = Info()
    ci, extra = _colinfo(k, colinfo)
    st = getattr(lib, entry)(h.ptr, n, _ptr(theta), _ptr(delta), delta.stride(0), k, _ptr(idx), _ptr(z0),
                             z0.stride(0) if z0 is not None else 0, C.byref(o), _ptr(z_out), z_out.stride(0),
                             _ptr(lam), _ptr(status), C.byref(info), C.byref(ci) if ci is not None else None)
    return _finish(lib, h, st, z_out, lam, status, info, extra)


def ipt_solve_dense_z(theta, delta, idx=None, z0=None, opts=None, handle=None, colinfo=True, z_out=None, **kw):
    """Dense IPT over C^n (ipt_solve_dense_z).  theta [n], delta [n, n] (row-major,
    row stride = lda) and z0 [n, k] complex128; idx [k] int32 or None.  Returns a
    Result with z [n, k] and lam [k] complex128, status [k] and info."""
    import torch
    lib = load_library()
    h = _handle(handle)
    _check(theta, torch.complex128, "theta")
    _check(delta, torch.complex128, "delta")
    _check(idx, torch.int32, "idx")
    _check(z0, torch.complex128, "z0")
    n = theta.shape[0]
    if theta.dim() != 1 or theta.stride(0) != 1:
        raise ValueError("theta must be a contiguous vector")
    if delta.dim() != 2 or delta.shape[0] != n or delta.shape[1] != n or delta.stride(1) != 1:
        raise ValueError("delta must be n x n with unit column stride")
    k = n if idx is None else idx.shape[0]
    if z0 is not None and (z0.dim() != 2 or z0.shape[0] != n or z0.shape[1] != k or z0.stride(1) != 1):
        raise ValueError("z0 must be n x k with unit column stride")
    dev = theta.device
    if z_out is None:
        z_out = torch.empty((n, k), dtype=torch.complex128, device=dev)
    lam = torch.empty(k, dtype=torch.complex128, device=dev)
    status = torch.empty(k, dtype=torch.int32, device=dev)
    o = _opts(opts, kw)
    info = Info()
    ci, extra = _colinfo(k, colinfo)
    st = lib.ipt_solve_dense_z(h.ptr, n, _ptr(theta), _ptr(delta), delta.stride(0), k, _ptr(idx), _ptr(z0),
                               z0.stride(0) if z0 is not None else 0, C.byref(o), _ptr(z_out), z_out.stride(0),
                               _ptr(lam), _ptr(status), C.byref(info), C.byref(ci) if ci is not None else None)
    return _finish(lib, h, st, z_out, lam, status, info, extra)


def ipt_solve_csr(theta, row_ptr, col, val, idx, z0=None, opts=None, handle=None, colinfo=True, **kw):
    """Sparse IPT solve (ipt_solve_csr) with Delta in CSR form (int32 row_ptr/col,
    f64 val) for the requested columns idx [k] int32."""
    import torch
    lib = load_library()
    h = _handle(handle)
    _check(theta, torch.float64, "theta")
    _check(row_ptr, torch.int32, "row_ptr")
    _check(col, torch.int32, "col")
    _check(val, torch.float64, "val")
    _check(idx, torch.int32, "idx")
    _check(z0, torch.float64, "z0")
    n = theta.shape[0]
    k = idx.shape[0]
    dev = theta.device
    z = torch.empty((n, k), dtype=torch.float64, device=dev)
    lam = torch.empty(k, dtype=torch.float64, device=dev)
    status = torch.empty(k, dtype=torch.int32, device=dev)
    o = _opts(opts, kw)
    info = Info()
    ci, extra = _colinfo(k, colinfo)
    st = lib.ipt_solve_csr(h.ptr, n, _ptr(theta), _ptr(row_ptr), _ptr(col), _ptr(val), val.shape[0], k, _ptr(idx),
                           _ptr(z0), z0.stride(0) if z0 is not None else 0, C.byref(o), _ptr(z), z.stride(0),
                           _ptr(lam), _ptr(status), C.byref(info), C.byref(ci) if ci is not None else None)
    return _finish(lib, h, st, z, lam, status, info, extra)


def ipt_solve_csr_z(theta, row_ptr, col, val, idx, z0=None, opts=None, handle=None, colinfo=True, **kw):
    """Sparse IPT over C^n (ipt_solve_csr_z): theta [n] and val [nnz] complex128, int32
    row_ptr / col, requested columns idx [k] int32, optional warm start z0 [n, k]
    complex128.  Returns a Result with z [n, k] and lam [k] complex128."""
    import torch
    lib = load_library()
    h = _handle(handle)
    _check(theta, torch.complex128, "theta")
    _check(row_ptr, torch.int32, "row_ptr")
    _check(col, torch.int32, "col")
    _check(val, torch.complex128, "val")
    _check(idx, torch.int32, "idx")
    _check(z0, torch.complex128, "z0")
    n = theta.shape[0]
    k = idx.shape[0]
    dev = theta.device
    z = torch.empty((n, k), dtype=torch.complex128, device=dev)
    lam = torch.empty(k, dtype=torch.complex128, device=dev)
    status = torch.empty(k, dtype=torch.int32, device=dev)
    o = _opts(opts, kw)
    info = Info()
    ci, extra = _colinfo(k, colinfo)
    st = lib.ipt_solve_csr_z(h.ptr, n, _ptr(theta), _ptr(row_ptr), _ptr(col), _ptr(val), val.shape[0], k, _ptr(idx),
                             _ptr(z0), z0.stride(0) if z0 is not None else 0, C.byref(o), _ptr(z), z.stride(0),
                             _ptr(lam), _ptr(status), C.byref(info), C.byref(ci) if ci is not None else None)
    return _finish(lib, h, st, z, lam, status, info, extra)


def _batch_layout(ns, theta_off, delta_off):
    ns = np.ascontiguousarray(np.asarray(ns, dtype=np.int32))
    if theta_off is None:
        theta_off = np.concatenate([[0], np.cumsum(ns.astype(np.int64))[:-1]]).astype(np.int64)
    if delta_off is None:
        delta_off = np.concatenate([[0], np.cumsum(ns.astype(np.int64) ** 2)[:-1]]).astype(np.int64)
    return (ns, np.ascontiguousarray(theta_off, dtype=np.int64), np.ascontiguousarray(delta_off, dtype=np.int64))


def ipt_solve_batched(ns, theta_pool, delta_pool, theta_off=None, delta_off=None, opts=None, handle=None,
                      z_out=None, lam_out=None, status_out=None, **kw):
    """Batched full-spectrum IPT (ipt_solve_batched).  ns: host int sequence of sizes;
    pools are GPU f64 tensors; offsets default to the packed layout.  Returns z_pool
    (same layout as delta_pool), lam_pool and status_pool (same layout as theta_pool);
    z_out / lam_out / status_out may be given to reuse output tensors."""
    import torch
    lib = load_library()
    h = _handle(handle)
    ns, theta_off, delta_off = _batch_layout(ns, theta_off, delta_off)
    _check(theta_pool, torch.float64, "theta_pool")
    _check(delta_pool, torch.float64, "delta_pool")
    z = torch.empty_like(delta_pool) if z_out is None else z_out
    lam = torch.empty_like(theta_pool) if lam_out is None else lam_out
    status = (torch.empty(theta_pool.shape[0], dtype=torch.int32, device=theta_pool.device)
              if status_out is None else status_out)
    _check(z, torch.float64, "z_out")
    _check(lam, torch.float64, "lam_out")
    _check(status, torch.int32, "status_out")
    if z.numel() < delta_pool.numel() or lam.numel() < theta_pool.numel() or status.numel() < theta_pool.numel():
        raise ValueError("output tensors smaller than the pools")
    o = _opts(opts, kw)
    info = Info()
    hp = lambda a: a.ctypes.data_as(C.c_void_p)
    st = lib.ipt_solve_batched(h.ptr, ns.shape[0], hp(ns), hp(theta_off), hp(delta_off), hp(delta_off),
                               _ptr(theta_pool), _ptr(delta_pool), C.byref(o), _ptr(z), _ptr(lam), _ptr(status),
                               C.byref(info))
    return _finish(lib, h, st, z, lam, status, info, None)


def ipt_batched_tune(ns, theta_pool, delta_pool, theta_off=None, delta_off=None, handle=None):
    """Autotune the handle's batched tile table on this batch (ipt_batched_tune);
    returns the table (TILE_BUCKETS tile sizes)."""
    import torch
    lib = load_library()
    h = _handle(handle)
    ns, theta_off, delta_off = _batch_layout(ns, theta_off, delta_off)
    _check(theta_pool, torch.float64, "theta_pool")
    _check(delta_pool, torch.float64, "delta_pool")
    z = torch.empty_like(delta_pool)
    lam = torch.empty_like(theta_pool)
    status = torch.empty(theta_pool.shape[0], dtype=torch.int32, device=theta_pool.device)
    tiles = np.zeros(TILE_BUCKETS, dtype=np.int32)
    hp = lambda a: a.ctypes.data_as(C.c_void_p)
    st = lib.ipt_batched_tune(h.ptr, ns.shape[0], hp(ns), hp(theta_off), hp(delta_off), hp(delta_off),
                              _ptr(theta_pool), _ptr(delta_pool), _ptr(z), _ptr(lam), _ptr(status), hp(tiles))
    if st != IPT_OK:
        raise IPTError(st, h.last_error())
    return [int(t) for t in tiles]


def ipt_batched_get_tiles(handle=None):
    """The handle's batched tile table (ipt_batched_get_tiles)."""
    lib = load_library()
    h = _handle(handle)
    tiles = np.zeros(TILE_BUCKETS, dtype=np.int32)
    st = lib.ipt_batched_get_tiles(h.ptr, tiles.ctypes.data_as(C.c_void_p))
    if st != IPT_OK:
        raise IPTError(st, h.last_error())
    return [int(t) for t in tiles]


def ipt_batched_set_tiles(tiles, handle=None):
    """Replace the handle's batched tile table (ipt_batched_set_tiles), e.g. with a
    table tuned earlier and stored as JSON."""
    lib = load_library()
    h = _handle(handle)
    arr = np.ascontiguousarray(np.asarray(tiles, dtype=np.int32))
    if arr.shape != (TILE_BUCKETS,):
        raise ValueError("tile table must have %d entries" % TILE_BUCKETS)
    st = lib.ipt_batched_set_tiles(h.ptr, arr.ctypes.data_as(C.c_void_p))
    if st != IPT_OK:
        raise IPTError(st, h.last_error())


# ------------------------------------------------------------------ learned warm start
_mlp_bound = False


def _bind_mlp(lib):
    global _mlp_bound
    if _mlp_bound:
        return
    p, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    lib.ipt_mlp_create.argtypes = [p, i32, i32, i32, i32, C.c_uint64, C.POINTER(p)]
    lib.ipt_mlp_destroy.argtypes = [p]
    lib.ipt_mlp_num_params.argtypes = [p]
    lib.ipt_mlp_num_params.restype = i64
    lib.ipt_mlp_get_params.argtypes = [p, p]
    lib.ipt_mlp_set_params.argtypes = [p, p]
    lib.ipt_mlp_forward.argtypes = [p, p, i32, p]
    lib.ipt_mlp_loss_grad.argtypes = [p, p, p, p, i32, C.POINTER(C.c_float), p]
    lib.ipt_mlp_train.argtypes = [p, p, p, p, i32, i32, C.c_float, C.POINTER(C.c_float)]
    lib.ipt_mlp_predict_z0.argtypes = [p, p, i32, p, p, p, i32, p, i64, i64, p, p, i64, i64]
    lib.ipt_mlp_targets.argtypes = [p, p, i32, i64, i64, i64, i64, p, p, i32, p, p, p, p, p]
    lib.ipt_rs_terms.argtypes = [p, i64, p, p, i64, i64, p, i32, p]
    lib.ipt_rs_start.argtypes = [p, p, i32, i32, p, i64, i64, p, p, i64, i64]
    for fn in ("ipt_mlp_create", "ipt_mlp_destroy", "ipt_mlp_get_params", "ipt_mlp_set_params", "ipt_mlp_forward",
               "ipt_mlp_loss_grad", "ipt_mlp_train", "ipt_mlp_predict_z0", "ipt_mlp_targets", "ipt_rs_terms",
               "ipt_rs_start"):
        getattr(lib, fn).restype = C.c_int
    _mlp_bound = True


class MLP:
    """ipt_mlp: x -> [Linear -> tanh] x depth -> Linear -> y with BF16 weights and FP32
    accumulation, trained by the library's own kernels (ipt_mlp_train)."""

    def __init__(self, in_dim, hidden, depth, out_dim, seed=0, handle=None):
        lib = load_library()
        _bind_mlp(lib)
        self._lib = lib
        self._handle = _handle(handle)
        self._m = C.c_void_p()
        st = lib.ipt_mlp_create(self._handle.ptr, in_dim, hidden, depth, out_dim, seed, C.byref(self._m))
        if st != IPT_OK:
            raise IPTError(st, "ipt_mlp_create: " + self._handle.last_error())
        self.in_dim, self.hidden, self.depth, self.out_dim = in_dim, hidden, depth, out_dim

    def _chk(self, st, what):
        if st != IPT_OK:
            raise IPTError(st, what + ": " + self._handle.last_error())

    @property
    def num_params(self):
        return int(self._lib.ipt_mlp_num_params(self._m))

    def get_params(self):
        import torch
        out = torch.empty(self.num_params, dtype=torch.float32, device="cuda")
        self._chk(self._lib.ipt_mlp_get_params(self._m, _ptr(out)), "ipt_mlp_get_params")
        return out

    def set_params(self, params):
        _check(params, __import__("torch").float32, "params")
        self._chk(self._lib.ipt_mlp_set_params(self._m, _ptr(params.contiguous())), "ipt_mlp_set_params")

    def forward(self, x):
        import torch
        x = x.contiguous()
        y = torch.empty((x.shape[0], self.out_dim), dtype=torch.float32, device=x.device)
        self._chk(self._lib.ipt_mlp_forward(self._m, _ptr(x), x.shape[0], _ptr(y)), "ipt_mlp_forward")
        return y

    def loss_grad(self, x, targets, weights=None):
        """Loss and gradient; weights: optional FP32 [batch] per-example loss weights."""
        import torch
        g = torch.empty(self.num_params, dtype=torch.float32, device=x.device)
        loss = C.c_float()
        _check(weights, torch.float32, "weights")
        self._chk(self._lib.ipt_mlp_loss_grad(self._m, _ptr(x.contiguous()), _ptr(targets.contiguous()),
                                              None if weights is None else _ptr(weights.contiguous()), x.shape[0],
                                              C.byref(loss), _ptr(g)), "ipt_mlp_loss_grad")
        return float(loss.value), g

    def train(self, x, targets, steps, lr=1e-3, weights=None):
        import torch
        loss = C.c_float()
        _check(weights, torch.float32, "weights")
        self._chk(self._lib.ipt_mlp_train(self._m, _ptr(x.contiguous()), _ptr(targets.contiguous()),
                                          None if weights is None else _ptr(weights.contiguous()), x.shape[0],
                                          int(steps), float(lr), C.byref(loss)), "ipt_mlp_train")
        return float(loss.value)

    def predict_z0(self, x, mu, sigma, eps, n, k, idx, terms=None, z0=None):
        """Warm starts Z0 [batch, n, k] (FP64) for the inputs x [batch, in_dim] of family
        members eps [batch] (FP64): E + sum_l eps^l T_l + eps^(order+1) (mu + sigma y),
        with T = terms [order, n, k] (ipt_rs_terms) or no terms."""
        import torch
        b = x.shape[0]
        if z0 is None:
            z0 = torch.empty((b, n, k), dtype=torch.float64, device=x.device)
        order = 0 if terms is None else terms.shape[0]
        self._chk(self._lib.ipt_mlp_predict_z0(self._m, _ptr(x.contiguous()), b, _ptr(mu.contiguous()),
                                               _ptr(sigma.contiguous()), _ptr(eps.contiguous()), order,
                                               None if terms is None else _ptr(terms.contiguous()), n, k,
                                               _ptr(idx.contiguous()), _ptr(z0), k, n * k), "ipt_mlp_predict_z0")
        return z0

    def close(self):
        if self._m:
            self._lib.ipt_mlp_destroy(self._m)
            self._m = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ipt_mlp_targets(z, idx, eps, terms=None, weights=None, handle=None):
    """Standardised targets (ipt_mlp_targets) from solutions z [batch, n, k] (FP64) of
    family members eps [batch] (FP64), as remainders after E + sum_l eps^l T_l (terms
    [order, n, k] or None): returns (targets [batch, n k], mu [n k], sigma [n k]) as FP32
    GPU tensors."""
    import torch
    lib = load_library()
    _bind_mlp(lib)
    h = _handle(handle)
    z = z.contiguous()
    b, n, k = z.shape
    tg = torch.empty((b, n * k), dtype=torch.float32, device=z.device)
    mu = torch.empty(n * k, dtype=torch.float32, device=z.device)
    sd = torch.empty(n * k, dtype=torch.float32, device=z.device)
    order = 0 if terms is None else terms.shape[0]
    st = lib.ipt_mlp_targets(h.ptr, _ptr(z), b, n, k, k, n * k, _ptr(idx.contiguous()), _ptr(eps.contiguous()), order,
                             None if terms is None else _ptr(terms.contiguous()),
                             None if weights is None else _ptr(weights.contiguous()), _ptr(tg), _ptr(mu), _ptr(sd))
    if st != IPT_OK:
        raise IPTError(st, "ipt_mlp_targets: " + h.last_error())
    return tg, mu, sd


def ipt_rs_terms(theta, delta, idx, order, handle=None):
    """Rayleigh-Schroedinger terms Z^[1..order] of D + Delta on the columns idx
    (ipt_rs_terms): returns terms [order, n, k] (FP64 GPU tensor)."""
    import torch
    lib = load_library()
    _bind_mlp(lib)
    h = _handle(handle)
    _check(theta, torch.float64, "theta")
    _check(delta, torch.float64, "delta")
    _check(idx, torch.int32, "idx")
    n, k = theta.shape[0], idx.shape[0]
    if delta.dim() != 2 or delta.shape[0] != n or delta.shape[1] != n or delta.stride(1) != 1:
        raise ValueError("delta must be n x n with unit column stride")
    terms = torch.empty((order, n, k), dtype=torch.float64, device=theta.device)
    st = lib.ipt_rs_terms(h.ptr, n, _ptr(theta), _ptr(delta), delta.stride(0), k, _ptr(idx.contiguous()), order,
                          _ptr(terms))
    if st != IPT_OK:
        raise IPTError(st, "ipt_rs_terms: " + h.last_error())
    return terms


def ipt_rs_start(terms, eps, idx, handle=None):
    """Series warm starts (ipt_rs_start): Z0 [batch, n, k] = E + sum_l eps^l T_l for the
    family members eps [batch] (FP64 GPU tensor), terms [order, n, k] from ipt_rs_terms."""
    import torch
    lib = load_library()
    _bind_mlp(lib)
    h = _handle(handle)
    order, n, k = terms.shape
    b = eps.shape[0]
    z0 = torch.empty((b, n, k), dtype=torch.float64, device=terms.device)
    st = lib.ipt_rs_start(h.ptr, _ptr(eps.contiguous()), b, order, _ptr(terms.contiguous()), n, k,
                          _ptr(idx.contiguous()), _ptr(z0), k, n * k)
    if st != IPT_OK:
        raise IPTError(st, "ipt_rs_start: " + h.last_error())
    return z0
