"""Thin Python binding of libsdd.so (the C ABI in include/sdd.h).

Argument marshalling only: every step of the walk and the reduction runs in
the library's HIP kernels.  PyTorch provides the device workspace and the
stream.  If the library has not been built this module raises on use -- there
is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsdd.so")

SDD_OK, SDD_E_INVALID, SDD_E_NOMEM, SDD_E_DEVICE = 0, -1, -2, -3
SDD_E_BUSY, SDD_E_NOTFOUND, SDD_E_TIMEOUT, SDD_E_CANCELLED = -4, -5, -6, -7
SDD_FP64, SDD_FP32_MIXED = 0, 1
SDD_FLAG_NO_SIGMA_GRID = 1
SDD_FLAG_EXIT_NAIVE = 2
SDD_FLAG_NO_LDS_GRID = 4
SDD_MAX_REGIONS = 16
SDD_DIAG_DT_UNRESOLVED = 1
SDD_NOALLOC_SCRATCH_BYTES = 64 << 20


class SddError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"sdd status {status}: {msg}")
        self.status = status


class sdd_region(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("v", C.c_double * 6), ("sigma", C.c_double)]


class sdd_model_desc(C.Structure):
    _fields_ = [("y_lo", C.c_double), ("y_hi", C.c_double), ("z_lo", C.c_double), ("z_hi", C.c_double),
                ("length_unit_m", C.c_double), ("sigma_background", C.c_double),
                ("n_regions", C.c_uint32), ("regions", C.POINTER(sdd_region))]


class sdd_request(C.Structure):
    _fields_ = [("model", C.c_uint32), ("precision", C.c_int32), ("freq_hz", C.c_double),
                ("alpha_direct", C.c_double), ("g_tables", C.POINTER(C.c_double)), ("g_samples", C.c_uint32),
                ("n_nodes", C.c_uint32), ("nodes_yz", C.POINTER(C.c_double)),
                ("path_begin", C.POINTER(C.c_uint32)), ("path_count", C.POINTER(C.c_uint32)),
                ("paths_uniform", C.c_uint32), ("dt", C.c_double), ("seed", C.c_uint64),
                ("stream", C.c_uint32), ("max_steps", C.c_uint32), ("flags", C.c_uint32),
                ("reserved", C.c_uint32), ("target_rel_se", C.c_double)]


class sdd_kappa_request(C.Structure):
    _fields_ = [("y_lo", C.c_double), ("y_hi", C.c_double), ("z_lo", C.c_double), ("z_hi", C.c_double),
                ("y_if", C.c_double), ("kappa", C.c_double * 2), ("lambda_re", C.c_double * 2),
                ("lambda_im", C.c_double * 2), ("g_tables", C.POINTER(C.c_double)), ("g_samples", C.c_uint32),
                ("n_nodes", C.c_uint32), ("nodes_yz", C.POINTER(C.c_double)),
                ("path_begin", C.POINTER(C.c_uint32)), ("path_count", C.POINTER(C.c_uint32)),
                ("paths_uniform", C.c_uint32), ("max_steps", C.c_uint32), ("dt", C.c_double),
                ("seed", C.c_uint64), ("stream", C.c_uint32), ("precision", C.c_uint32)]


class sdd_path_record(C.Structure):
    _fields_ = [("w_re", C.c_double), ("w_im", C.c_double), ("tau", C.c_double),
                ("steps", C.c_uint32), ("wall", C.c_int32)]


PATH_RECORD_DTYPE = np.dtype([("w_re", "<f8"), ("w_im", "<f8"), ("tau", "<f8"), ("steps", "<u4"), ("wall", "<i4")])
assert PATH_RECORD_DTYPE.itemsize == C.sizeof(sdd_path_record) == 32


class sdd_diag(C.Structure):
    _fields_ = [("rho_dt", C.c_double), ("flags", C.c_uint32), ("reserved", C.c_uint32), ("g_norm", C.c_double),
                ("se_over_gnorm", C.c_double)]


class sdd_result(C.Structure):
    _fields_ = [("mean", C.POINTER(C.c_double)), ("var", C.POINTER(C.c_double)), ("se", C.POINTER(C.c_double)),
                ("paths_done", C.POINTER(C.c_uint64)), ("steps", C.POINTER(C.c_uint64)),
                ("unfinished", C.POINTER(C.c_uint64)), ("mean_exit_time", C.POINTER(C.c_double)),
                ("path_records", C.c_void_p), ("diag", C.POINTER(sdd_diag))]


class sdd_tuning(C.Structure):
    _fields_ = [("block_threads", C.c_uint32), ("blocks_per_cu", C.c_uint32), ("tile_paths", C.c_uint32),
                ("slice_iters", C.c_uint32), ("refill_every", C.c_uint32)]


class sdd_tune_trial(C.Structure):
    _fields_ = [("tuning", sdd_tuning), ("walk_ms", C.c_double), ("walk_steps_per_s", C.c_double)]


class sdd_stats(C.Structure):
    _fields_ = [("last_walk_ms", C.c_double), ("last_reduce_ms", C.c_double), ("last_walk_steps", C.c_uint64),
                ("last_walk_paths", C.c_uint64), ("last_blocks", C.c_uint32), ("last_threads", C.c_uint32),
                ("launches", C.c_uint64), ("served_in_flight_max", C.c_uint32), ("served_waits", C.c_uint32),
                ("served_requeues", C.c_uint32), ("reserved", C.c_uint32), ("served_walk_ms", C.c_double),
                ("served_slices", C.c_uint64)]


# (name, restype, argtypes) of every entry point in include/sdd.h
_PROTOS = [
    ("sdd_create", C.c_int, [C.c_int, C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    ("sdd_destroy", C.c_int, [C.c_void_p]),
    ("sdd_model_create", C.c_int, [C.c_void_p, C.POINTER(sdd_model_desc), C.POINTER(C.c_uint32)]),
    ("sdd_model_destroy", C.c_int, [C.c_void_p, C.c_uint32]),
    ("sdd_solve", C.c_int, [C.c_void_p, C.POINTER(sdd_request), C.POINTER(sdd_result)]),
    ("sdd_solve_batch", C.c_int, [C.c_void_p, C.c_uint32, C.POINTER(sdd_request), C.POINTER(sdd_result)]),
    ("sdd_solve_plain", C.c_int, [C.c_void_p, C.POINTER(sdd_request), C.POINTER(sdd_result)]),
    ("sdd_solve_noalloc", C.c_int, [C.c_void_p, C.POINTER(sdd_request), C.POINTER(sdd_result)]),
    ("sdd_mt_te_response", C.c_int, [C.c_uint32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), C.c_double, C.c_double, C.c_double,
                                     C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("sdd_mt_te_response_jump", C.c_int, [C.c_uint32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                          C.POINTER(C.c_double), C.c_double, C.c_double, C.c_double, C.c_double,
                                          C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("sdd_rbffd_solve", C.c_int, [C.c_uint32, C.c_uint32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.c_double, C.c_double, C.POINTER(C.c_double)]),
    ("sdd_rbffd_weights", C.c_int, [C.c_uint32, C.c_uint32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                    C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("sdd_solve_multi_freq", C.c_int, [C.c_void_p, C.POINTER(sdd_request), C.c_uint32, C.POINTER(C.c_double),
                                       C.POINTER(C.POINTER(C.c_double)), C.POINTER(sdd_result)]),
    ("sdd_solve_kappa", C.c_int, [C.c_void_p, C.POINTER(sdd_kappa_request), C.POINTER(sdd_result)]),
    ("sdd_submit", C.c_int, [C.c_void_p, C.POINTER(sdd_request), C.POINTER(sdd_result), C.POINTER(C.c_uint64)]),
    ("sdd_poll", C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_int)]),
    ("sdd_wait", C.c_int, [C.c_void_p, C.c_uint64, C.c_int64]),
    ("sdd_cancel", C.c_int, [C.c_void_p, C.c_uint64]),
    ("sdd_set_tuning", C.c_int, [C.c_void_p, C.POINTER(sdd_tuning)]),
    ("sdd_get_tuning", C.c_int, [C.c_void_p, C.POINTER(sdd_tuning)]),
    ("sdd_autotune", C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.POINTER(sdd_tuning),
                               C.POINTER(sdd_tune_trial), C.c_uint32, C.POINTER(C.c_uint32)]),
    ("sdd_get_stats", C.c_int, [C.c_void_p, C.POINTER(sdd_stats)]),
    ("sdd_request_footprint", C.c_int, [C.c_void_p, C.POINTER(sdd_request), C.POINTER(C.c_uint64)]),
    ("sdd_batch_create", C.c_int, [C.c_void_p, C.c_uint32, C.POINTER(sdd_request), C.POINTER(C.c_void_p)]),
    ("sdd_batch_run", C.c_int, [C.c_void_p, C.POINTER(sdd_result)]),
    ("sdd_batch_destroy", C.c_int, [C.c_void_p]),
    ("sdd_status_string", C.c_char_p, [C.c_int]),
    ("sdd_last_error", C.c_char_p, []),
]
EXPORTED = [p[0] for p in _PROTOS]

_lib = None


def lib():
    """The loaded libsdd.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -m paper_1603_09311_amd.build)")
        # torch first: the library then binds to the HIP runtime torch has
        # loaded (same sonames).  Loaded the other way round, the process
        # holds two HIP runtimes and the library's sees no device once torch
        # has opened it.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, res, args in _PROTOS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st: int):
    if st != SDD_OK:
        raise SddError(st, lib().sdd_last_error().decode(errors="replace"))


def _ptr(a: Optional[np.ndarray], ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else C.POINTER(ct)()


# ---------------------------------------------------------------------------
# Marshalling of workloads.Problem objects
# ---------------------------------------------------------------------------

def model_desc(p):
    regs = (sdd_region * max(1, len(p.regions)))()
    for i, r in enumerate(p.regions):
        regs[i].kind = r.kind
        regs[i].reserved = 0
        for k, v in enumerate(r.param6()):
            regs[i].v[k] = v
        regs[i].sigma = r.sigma
    d = sdd_model_desc(p.y_lo, p.y_hi, p.z_lo, p.z_hi, p.length_unit_m, p.sigma_background,
                       len(p.regions), C.cast(regs, C.POINTER(sdd_region)))
    return d, regs


def model_key(p):
    return (p.y_lo, p.y_hi, p.z_lo, p.z_hi, p.length_unit_m, p.sigma_background,
            tuple((r.kind, tuple(r.param6()), r.sigma) for r in p.regions))


class _Req:
    """An sdd_request and the numpy buffers it points into."""

    def __init__(self, p, model: int, precision: Optional[int] = None, target_rel_se: float = 0.0, flags: int = 0):
        self.g = np.ascontiguousarray(np.stack([p.g.real, p.g.imag], axis=-1).reshape(-1), dtype=np.float64)
        self.nodes = np.ascontiguousarray(p.nodes, dtype=np.float64).reshape(-1)
        self.pb = np.ascontiguousarray(p.path_begin, dtype=np.uint32)
        self.pc = np.ascontiguousarray(p.path_count, dtype=np.uint32)
        prec = p.precision if precision is None else precision
        self.s = sdd_request(model, prec, p.freq_hz, p.alpha_direct, _ptr(self.g, C.c_double),
                             p.g.shape[1], p.n_nodes, _ptr(self.nodes, C.c_double), _ptr(self.pb, C.c_uint32),
                             _ptr(self.pc, C.c_uint32), 0, p.dt, p.seed, p.stream,
                             min(int(p.max_steps), 0xFFFFFFFF),
                             flags | (SDD_FLAG_EXIT_NAIVE if getattr(p, "naive_exit", False) else 0), 0,
                             target_rel_se)
        self.n = p.n_nodes
        self.total = int(self.pc.astype(np.uint64).sum())


class _KReq:
    """An sdd_kappa_request (discontinuous kappa) and the numpy buffers it points into."""

    def __init__(self, p, precision: int = 0):
        self.g = np.ascontiguousarray(np.stack([p.g.real, p.g.imag], axis=-1).reshape(-1), dtype=np.float64)
        self.nodes = np.ascontiguousarray(p.nodes, dtype=np.float64).reshape(-1)
        self.pb = np.ascontiguousarray(p.path_begin, dtype=np.uint32)
        self.pc = np.ascontiguousarray(p.path_count, dtype=np.uint32)
        lam = [complex(x) for x in p.lam]
        d2 = C.c_double * 2
        self.s = sdd_kappa_request(p.y_lo, p.y_hi, p.z_lo, p.z_hi, p.y_if, d2(*p.kappa),
                                   d2(*[x.real for x in lam]), d2(*[x.imag for x in lam]),
                                   _ptr(self.g, C.c_double), p.g.shape[1], p.n_nodes, _ptr(self.nodes, C.c_double),
                                   _ptr(self.pb, C.c_uint32), _ptr(self.pc, C.c_uint32), 0,
                                   min(int(p.max_steps), 0xFFFFFFFF), p.dt, p.seed, p.stream, precision)
        self.n = p.n_nodes
        self.total = int(self.pc.astype(np.uint64).sum())


class _Res:
    def __init__(self, n: int, records: int = 0):
        self.mean = np.zeros((max(n, 1), 2))
        self.var = np.zeros((max(n, 1), 3))
        self.se = np.zeros((max(n, 1), 3))
        self.paths_done = np.zeros(max(n, 1), np.uint64)
        self.steps = np.zeros(max(n, 1), np.uint64)
        self.unfinished = np.zeros(max(n, 1), np.uint64)
        self.mean_exit_time = np.zeros(max(n, 1))
        self.records = np.zeros(records, PATH_RECORD_DTYPE) if records else None
        self.diag = sdd_diag()
        self.n = n
        self.s = sdd_result(_ptr(self.mean, C.c_double), _ptr(self.var, C.c_double), _ptr(self.se, C.c_double),
                            _ptr(self.paths_done, C.c_uint64), _ptr(self.steps, C.c_uint64),
                            _ptr(self.unfinished, C.c_uint64), _ptr(self.mean_exit_time, C.c_double),
                            self.records.ctypes.data if self.records is not None and records else None,
                            C.pointer(self.diag))

    def as_dict(self) -> Dict[str, np.ndarray]:
        n = self.n
        d = dict(mean=self.mean[:n, 0] + 1j * self.mean[:n, 1], var_re=self.var[:n, 0], var_im=self.var[:n, 1],
                 cov=self.var[:n, 2], se_re=self.se[:n, 0], se_im=self.se[:n, 1], se=self.se[:n, 2],
                 paths_done=self.paths_done[:n].copy(), steps=self.steps[:n].copy(),
                 unfinished=self.unfinished[:n].copy(), mean_exit_time=self.mean_exit_time[:n].copy())
        if self.records is not None:
            d["records"] = self.records
        d["diag"] = {"rho_dt": self.diag.rho_dt, "dt_unresolved": bool(self.diag.flags & SDD_DIAG_DT_UNRESOLVED),
                     "g_norm": self.diag.g_norm, "se_over_gnorm": self.diag.se_over_gnorm}
        return d


def mt_te_response(e_minus, e_mid, e_plus, h: float, length_unit_m: float, freq_hz: float,
                   sigma_jump: float = 0.0):
    """TE apparent resistivity (ohm m) and phase (degrees) per site from the
    complex field at z - h, z, z + h (sdd_mt_te_response); with sigma_jump
    (S/m, the conductivity below the site less the one above) the
    first-order term of a jump between the points is removed
    (sdd_mt_te_response_jump)."""
    arrs = [np.ascontiguousarray(np.stack([np.asarray(e).real, np.asarray(e).imag], axis=-1), dtype=np.float64)
            for e in (e_minus, e_mid, e_plus)]
    n = arrs[0].shape[0]
    if any(a.shape != (n, 2) for a in arrs):
        raise ValueError("three arrays of the same length")
    rho = np.zeros(max(n, 1))
    phi = np.zeros(max(n, 1))
    ptrs = [_ptr(a, C.c_double) for a in arrs]
    if sigma_jump == 0.0:
        _check(lib().sdd_mt_te_response(n, *ptrs, h, length_unit_m, freq_hz,
                                        _ptr(rho, C.c_double), _ptr(phi, C.c_double)))
    else:
        _check(lib().sdd_mt_te_response_jump(n, *ptrs, h, length_unit_m, freq_hz, sigma_jump,
                                             _ptr(rho, C.c_double), _ptr(phi, C.c_double)))
    return rho[:n], phi[:n]


def rbffd_solve(y, z, alpha: float, eps: float, field):
    """RBF-FD sub-domain solve (sdd_rbffd_solve): `field` is a complex
    (nz, ny) array whose boundary rows and columns hold the Dirichlet values;
    returns a copy with the interior solved."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    f = np.asarray(field, dtype=np.complex128)
    if f.shape != (z.size, y.size):
        raise ValueError(f"field of shape {f.shape}, the grid is {(z.size, y.size)}")
    buf = np.ascontiguousarray(np.stack([f.real, f.imag], axis=-1), dtype=np.float64)
    _check(lib().sdd_rbffd_solve(y.size, z.size, _ptr(y, C.c_double), _ptr(z, C.c_double), alpha, eps,
                                 _ptr(buf, C.c_double)))
    return buf[..., 0] + 1j * buf[..., 1]


def rbffd_weights(y, z, eps: float):
    """Stencil weights (sdd_rbffd_weights): two ((nz-2)(ny-2), 9) arrays."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    n = max(0, (y.size - 2) * (z.size - 2))
    wy = np.zeros((max(n, 1), 9))
    wz = np.zeros((max(n, 1), 9))
    _check(lib().sdd_rbffd_weights(y.size, z.size, _ptr(y, C.c_double), _ptr(z, C.c_double), eps,
                                   _ptr(wy, C.c_double), _ptr(wz, C.c_double)))
    return wy[:n], wz[:n]


class Context:
    """A library context on cuda:`device` whose workspace is a torch tensor."""

    def __init__(self, device: int = 0, workspace_bytes: int = 8 << 30, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the sdd library needs an MI355X")
        L = lib()
        self.device = device
        self.ws = torch.empty(workspace_bytes, dtype=torch.uint8, device=f"cuda:{device}")
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        _check(L.sdd_create(device, self.ws.data_ptr(), workspace_bytes, C.c_void_p(self.stream.cuda_stream),
                            C.byref(h)))
        self.h = h
        self._models: Dict[tuple, int] = {}
        self._keep = {}

    def close(self):
        if getattr(self, "h", None):
            lib().sdd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # models ---------------------------------------------------------------
    def model(self, p) -> int:
        key = model_key(p)
        if key not in self._models:
            d, regs = model_desc(p)
            mid = C.c_uint32()
            _check(lib().sdd_model_create(self.h, C.byref(d), C.byref(mid)))
            self._models[key] = mid.value
        return self._models[key]

    def drop_model(self, p):
        key = model_key(p)
        if key in self._models:
            _check(lib().sdd_model_destroy(self.h, self._models.pop(key)))

    # tuning -----------------------------------------------------------------
    def autotune(self, p, sample_paths: int = 0, precision: Optional[int] = None):
        """Time the walker on a sample of problem p under candidate tunings,
        keep the fastest on this context; returns (chosen tuning dict, list of
        trial dicts)."""
        q = _Req(p, self.model(p), precision)
        chosen = sdd_tuning()
        trials = (sdd_tune_trial * 32)()
        n = C.c_uint32()
        _check(lib().sdd_autotune(self.h, C.byref(q.s), sample_paths, C.byref(chosen), trials, 32, C.byref(n)))
        tdict = lambda t: {f: getattr(t, f) for f, _ in sdd_tuning._fields_}  # noqa: E731
        return tdict(chosen), [dict(tdict(trials[i].tuning), walk_ms=trials[i].walk_ms,
                                    walk_steps_per_s=trials[i].walk_steps_per_s) for i in range(n.value)]

    def set_tuning(self, block_threads=0, blocks_per_cu=0, tile_paths=0, slice_iters=0, refill_every=0):
        t = sdd_tuning(block_threads, blocks_per_cu, tile_paths, slice_iters, refill_every)
        _check(lib().sdd_set_tuning(self.h, C.byref(t)))

    def stats(self) -> dict:
        t = sdd_stats()
        _check(lib().sdd_get_stats(self.h, C.byref(t)))
        return {k: getattr(t, k) for k, _ in sdd_stats._fields_}

    def get_tuning(self) -> dict:
        t = sdd_tuning()
        _check(lib().sdd_get_tuning(self.h, C.byref(t)))
        return {k: getattr(t, k) for k, _ in sdd_tuning._fields_}

    # solves -----------------------------------------------------------------
    def footprint(self, p, target_rel_se: float = 0.0) -> int:
        q = _Req(p, self.model(p), target_rel_se=target_rel_se)
        b = C.c_uint64()
        _check(lib().sdd_request_footprint(self.h, C.byref(q.s), C.byref(b)))
        return b.value

    def solve(self, p, precision: Optional[int] = None, records: bool = False, target_rel_se: float = 0.0,
              flags: int = 0):
        q = _Req(p, self.model(p), precision, target_rel_se, flags)
        r = _Res(q.n, q.total if records else 0)
        _check(lib().sdd_solve(self.h, C.byref(q.s), C.byref(r.s)))
        return r.as_dict()

    def solve_noalloc(self, p, precision: Optional[int] = None, records: bool = False, flags: int = 0):
        """sdd_solve with every device buffer in the library's static scratch
        (sdd_solve_noalloc): no allocation during the call, bitwise the result
        of solve()."""
        q = _Req(p, self.model(p), precision, 0.0, flags)
        r = _Res(q.n, q.total if records else 0)
        _check(lib().sdd_solve_noalloc(self.h, C.byref(q.s), C.byref(r.s)))
        return r.as_dict()

    def solve_multi_freq(self, p, freqs: Sequence[float], g_tables: Sequence[np.ndarray],
                         precision: Optional[int] = None) -> List[dict]:
        """One walk of problem p (its own frequency sets the phase scale),
        weighted for every frequency in freqs with that frequency's (4, M+1)
        complex boundary tables; one result dict per frequency."""
        if len(freqs) != len(g_tables):
            raise ValueError("one table set per frequency")
        q = _Req(p, self.model(p), precision)
        fr = np.ascontiguousarray(freqs, dtype=np.float64)
        tabs = []
        for g in g_tables:
            g = np.asarray(g)
            if g.shape != p.g.shape:
                raise ValueError(f"tables of shape {g.shape}, the request has {p.g.shape}")
            tabs.append(np.ascontiguousarray(np.stack([g.real, g.imag], axis=-1).reshape(-1), dtype=np.float64))
        ptrs = (C.POINTER(C.c_double) * max(1, len(tabs)))(*[_ptr(t, C.c_double) for t in tabs])
        rs = [_Res(q.n) for _ in tabs]
        ress = (sdd_result * max(1, len(rs)))(*[r.s for r in rs])
        _check(lib().sdd_solve_multi_freq(self.h, C.byref(q.s), len(tabs), _ptr(fr, C.c_double), ptrs, ress))
        return [r.as_dict() for r in rs]

    def solve_kappa(self, p, records: bool = False, precision: int = 0):
        """The discontinuous-kappa walk of a workloads.KappaProblem (one
        vertical interface; Secs. 2.2 and 3.1): SDD_FP64 (default) or
        SDD_FP32_MIXED."""
        q = _KReq(p, precision)
        r = _Res(q.n, q.total if records else 0)
        _check(lib().sdd_solve_kappa(self.h, C.byref(q.s), C.byref(r.s)))
        return r.as_dict()

    def solve_plain(self, p, records: bool = False):
        q = _Req(p, self.model(p), SDD_FP64)
        r = _Res(q.n, q.total if records else 0)
        _check(lib().sdd_solve_plain(self.h, C.byref(q.s), C.byref(r.s)))
        return r.as_dict()

    def solve_batch(self, ps: Sequence, records: bool = False, target_rel_se: float = 0.0) -> List[dict]:
        qs = [_Req(p, self.model(p), None, target_rel_se) for p in ps]
        rs = [_Res(q.n, q.total if records else 0) for q in qs]
        reqs = (sdd_request * max(1, len(qs)))(*[q.s for q in qs])
        ress = (sdd_result * max(1, len(rs)))(*[r.s for r in rs])
        _check(lib().sdd_solve_batch(self.h, len(qs), reqs, ress))
        return [r.as_dict() for r in rs]

    def batch(self, ps: Sequence, records: bool = False) -> "Batch":
        """A prepared batch replayed as a HIP graph (see Batch)."""
        return Batch(self, ps, records)

    # served mode --------------------------------------------------------------
    def submit(self, p, precision: Optional[int] = None, records: bool = False, target_rel_se: float = 0.0):
        q = _Req(p, self.model(p), precision, target_rel_se)
        r = _Res(q.n, q.total if records else 0)
        t = C.c_uint64()
        _check(lib().sdd_submit(self.h, C.byref(q.s), C.byref(r.s), C.byref(t)))
        self._keep[t.value] = (q, r)
        return t.value

    def poll(self, ticket: int):
        """None while running; the result dict when done (raises on failure
        or cancellation)."""
        done = C.c_int()
        st = lib().sdd_poll(self.h, ticket, C.byref(done))
        if st == SDD_OK and not done.value:
            return None
        if st in (SDD_E_NOTFOUND, SDD_E_INVALID):
            _check(st)
        q, r = self._keep.pop(ticket)
        _check(st)
        return r.as_dict()

    def wait(self, ticket: int, timeout_s: Optional[float] = None):
        ns = -1 if timeout_s is None else int(timeout_s * 1e9)
        st = lib().sdd_wait(self.h, ticket, ns)
        if st in (SDD_E_TIMEOUT, SDD_E_NOTFOUND, SDD_E_INVALID):
            _check(st)
        q, r = self._keep.pop(ticket)
        _check(st)
        return r.as_dict()

    def cancel(self, ticket: int) -> int:
        """SDD_OK if cancelled, SDD_E_BUSY if it had already finished."""
        return lib().sdd_cancel(self.h, ticket)


class Batch:
    """Requests kept resident with their launch sequence captured as a HIP
    graph; run() replays it and returns one result dict per request."""

    def __init__(self, ctx: Context, ps: Sequence, records: bool = False):
        self.ctx = ctx
        self.qs = [_Req(p, ctx.model(p)) for p in ps]
        self.records = records
        reqs = (sdd_request * max(1, len(self.qs)))(*[q.s for q in self.qs])
        h = C.c_void_p()
        _check(lib().sdd_batch_create(ctx.h, len(self.qs), reqs, C.byref(h)))
        self.h = h

    def run(self) -> List[dict]:
        rs = [_Res(q.n, q.total if self.records else 0) for q in self.qs]
        ress = (sdd_result * max(1, len(rs)))(*[r.s for r in rs])
        _check(lib().sdd_batch_run(self.h, ress))
        return [r.as_dict() for r in rs]

    def close(self):
        if getattr(self, "h", None):
            lib().sdd_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
