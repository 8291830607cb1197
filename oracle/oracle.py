"""ctypes binding of the FP64 CPU oracle (sdd_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the library's product path.
It marshals a ``workloads.Problem`` into the oracle's own C structs.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sdd_oracle.c")
LIB = os.environ.get("SDD_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so."""
    if os.environ.get("SDD_ORACLE_LIB"):
        return LIB
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm", "-lpthread"])
        os.replace(tmp, LIB)
    return LIB


class Problem_C(C.Structure):
    _fields_ = [
        ("y_lo", C.c_double), ("y_hi", C.c_double), ("z_lo", C.c_double), ("z_hi", C.c_double),
        ("n_regions", C.c_int32),
        ("region_kind", C.POINTER(C.c_int32)),
        ("region_param", C.POINTER(C.c_double)),
        ("region_sigma", C.POINTER(C.c_double)),
        ("sigma_background", C.c_double),
        ("length_unit_m", C.c_double),
        ("freq_hz", C.c_double),
        ("alpha_direct", C.c_double),
        ("g_samples", C.c_int32),
        ("g", C.POINTER(C.c_double)),
        ("n_nodes", C.c_int32),
        ("nodes", C.POINTER(C.c_double)),
        ("path_begin", C.POINTER(C.c_uint32)),
        ("path_count", C.POINTER(C.c_uint32)),
        ("dt", C.c_double),
        ("seed", C.c_uint64),
        ("stream", C.c_uint32),
        ("max_steps", C.c_uint32),
        ("naive_exit", C.c_int32),
    ]


class Path_C(C.Structure):
    _fields_ = [("w_re", C.c_double), ("w_im", C.c_double), ("S", C.c_double),
                ("tau", C.c_double), ("exit_t", C.c_double),
                ("steps", C.c_uint32), ("wall", C.c_int32)]


class Node_C(C.Structure):
    _fields_ = [("mean_re", C.c_double), ("mean_im", C.c_double),
                ("var_re", C.c_double), ("var_im", C.c_double), ("cov", C.c_double),
                ("se_re", C.c_double), ("se_im", C.c_double), ("se", C.c_double),
                ("mean_exit_time", C.c_double),
                ("paths_done", C.c_uint64), ("steps", C.c_uint64), ("unfinished", C.c_uint64)]


PATH_DTYPE = np.dtype([("w_re", "<f8"), ("w_im", "<f8"), ("S", "<f8"), ("tau", "<f8"),
                       ("exit_t", "<f8"), ("steps", "<u4"), ("wall", "<i4")])
NODE_DTYPE = np.dtype([("mean_re", "<f8"), ("mean_im", "<f8"), ("var_re", "<f8"),
                       ("var_im", "<f8"), ("cov", "<f8"), ("se_re", "<f8"), ("se_im", "<f8"),
                       ("se", "<f8"), ("mean_exit_time", "<f8"), ("paths_done", "<u8"),
                       ("steps", "<u8"), ("unfinished", "<u8")])
assert PATH_DTYPE.itemsize == C.sizeof(Path_C)
assert NODE_DTYPE.itemsize == C.sizeof(Node_C)

class KProblem_C(C.Structure):
    _fields_ = [
        ("y_lo", C.c_double), ("y_hi", C.c_double), ("z_lo", C.c_double), ("z_hi", C.c_double),
        ("y_if", C.c_double), ("kappa", C.c_double * 2),
        ("lambda_re", C.c_double * 2), ("lambda_im", C.c_double * 2),
        ("g_samples", C.c_int32), ("g", C.POINTER(C.c_double)),
        ("n_nodes", C.c_int32), ("nodes", C.POINTER(C.c_double)),
        ("path_begin", C.POINTER(C.c_uint32)), ("path_count", C.POINTER(C.c_uint32)),
        ("dt", C.c_double), ("seed", C.c_uint64), ("stream", C.c_uint32), ("max_steps", C.c_uint32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        L.orc_solve.argtypes = [C.POINTER(Problem_C), C.c_int, C.c_void_p, C.c_void_p]
        L.orc_solve.restype = C.c_int
        L.orc_validate.argtypes = [C.POINTER(Problem_C)]
        L.orc_validate.restype = C.c_int
        L.orc_walk_path.argtypes = [C.POINTER(Problem_C), C.c_int, C.c_uint32, C.POINTER(Path_C)]
        L.orc_walk_path.restype = C.c_int
        L.orc_region.argtypes = [C.POINTER(Problem_C), C.c_double, C.c_double]
        L.orc_region.restype = C.c_int
        L.orc_table_g.argtypes = [C.POINTER(Problem_C), C.c_int, C.c_double, C.POINTER(C.c_double)]
        L.orc_table_g.restype = None
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_philox4x32_10.restype = None
        L.orc_u01.argtypes = [C.c_uint32]
        L.orc_u01.restype = C.c_double
        L.orc_box_muller.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_double)]
        L.orc_box_muller.restype = None
        L.orc_node_stats.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(Node_C)]
        L.orc_node_stats.restype = C.c_int
        L.orc_ksolve.argtypes = [C.POINTER(KProblem_C), C.c_int, C.c_void_p, C.c_void_p]
        L.orc_ksolve.restype = C.c_int
        L.orc_kwalk_path.argtypes = [C.POINTER(KProblem_C), C.c_int, C.c_uint32, C.POINTER(Path_C)]
        L.orc_kwalk_path.restype = C.c_int
        L.orc_kvalidate.argtypes = [C.POINTER(KProblem_C)]
        L.orc_kvalidate.restype = C.c_int
        _lib = L
    return _lib


class _Marshalled:
    """Keeps the numpy buffers alive while the C struct points into them."""

    def __init__(self, p):
        self.kinds = np.array([r.kind for r in p.regions] or [0], dtype=np.int32)
        self.params = np.array([r.param6() for r in p.regions] or [[0.0] * 6], dtype=np.float64).reshape(-1)
        self.sigmas = np.array([r.sigma for r in p.regions] or [0.0], dtype=np.float64)
        self.g = np.ascontiguousarray(np.stack([p.g.real, p.g.imag], axis=-1), dtype=np.float64).reshape(-1)
        self.nodes = np.ascontiguousarray(p.nodes, dtype=np.float64).reshape(-1)
        if self.nodes.size == 0:
            self.nodes = np.zeros(2)
        self.pb = np.ascontiguousarray(p.path_begin, dtype=np.uint32)
        self.pc = np.ascontiguousarray(p.path_count, dtype=np.uint32)
        if self.pb.size == 0:
            self.pb = np.zeros(1, np.uint32)
            self.pc = np.ones(1, np.uint32)
        dp = C.POINTER(C.c_double)
        self.s = Problem_C(
            p.y_lo, p.y_hi, p.z_lo, p.z_hi, len(p.regions),
            self.kinds.ctypes.data_as(C.POINTER(C.c_int32)), self.params.ctypes.data_as(dp),
            self.sigmas.ctypes.data_as(dp), p.sigma_background, p.length_unit_m, p.freq_hz,
            p.alpha_direct, p.g.shape[1], self.g.ctypes.data_as(dp), p.n_nodes,
            self.nodes.ctypes.data_as(dp), self.pb.ctypes.data_as(C.POINTER(C.c_uint32)),
            self.pc.ctypes.data_as(C.POINTER(C.c_uint32)), p.dt, p.seed, p.stream,
            min(int(p.max_steps), 0xFFFFFFFF), 1 if getattr(p, "naive_exit", False) else 0)


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


def solve(p, threads: Optional[int] = None, records: bool = False):
    """Run the oracle.  Returns (nodes structured array, path records or None).
    Path records are node-major: node j's paths at offsets cumsum(path_count)."""
    m = _Marshalled(p)
    n = p.n_nodes
    out = np.zeros(max(n, 1), dtype=NODE_DTYPE)
    recs = np.zeros(p.total_paths, dtype=PATH_DTYPE) if records else None
    rc = lib().orc_solve(C.byref(m.s), threads or default_threads(), out.ctypes.data,
                         recs.ctypes.data if recs is not None and recs.size else None)
    if rc != 0:
        raise ValueError(f"oracle rejected the problem (code {rc})")
    return out[:n], recs


def validate(p) -> int:
    m = _Marshalled(p)
    return int(lib().orc_validate(C.byref(m.s)))


def walk_path(p, node: int, path: int):
    m = _Marshalled(p)
    rec = Path_C()
    rc = lib().orc_walk_path(C.byref(m.s), node, path, C.byref(rec))
    if rc != 0:
        raise ValueError(rc)
    return {k: getattr(rec, k) for k, _ in Path_C._fields_}


def region(p, y: float, z: float) -> int:
    m = _Marshalled(p)
    return int(lib().orc_region(C.byref(m.s), y, z))


def table_g(p, wall: int, t: float) -> complex:
    m = _Marshalled(p)
    o = (C.c_double * 2)()
    lib().orc_table_g(C.byref(m.s), wall, t, o)
    return complex(o[0], o[1])


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return tuple(int(x) for x in o)


def u01(w: int) -> float:
    return float(lib().orc_u01(int(w) & 0xFFFFFFFF))


def box_muller(ua: float, ub: float):
    o = (C.c_double * 2)()
    lib().orc_box_muller(ua, ub, o)
    return o[0], o[1]


def node_stats(recs: np.ndarray):
    recs = np.ascontiguousarray(recs, dtype=PATH_DTYPE)
    out = Node_C()
    lib().orc_node_stats(recs.ctypes.data, recs.size, C.byref(out))
    return {k: getattr(out, k) for k, _ in Node_C._fields_}


class _KMarshalled:
    """The discontinuous-kappa problem as the oracle's C struct."""

    def __init__(self, p):
        self.g = np.ascontiguousarray(np.stack([p.g.real, p.g.imag], axis=-1), dtype=np.float64).reshape(-1)
        self.nodes = np.ascontiguousarray(p.nodes, dtype=np.float64).reshape(-1)
        if self.nodes.size == 0:
            self.nodes = np.zeros(2)
        self.pb = np.ascontiguousarray(p.path_begin, dtype=np.uint32)
        self.pc = np.ascontiguousarray(p.path_count, dtype=np.uint32)
        if self.pb.size == 0:
            self.pb = np.zeros(1, np.uint32)
            self.pc = np.ones(1, np.uint32)
        dp = C.POINTER(C.c_double)
        lam = [complex(x) for x in p.lam]
        self.s = KProblem_C(p.y_lo, p.y_hi, p.z_lo, p.z_hi, p.y_if, (C.c_double * 2)(*p.kappa),
                            (C.c_double * 2)(*[x.real for x in lam]), (C.c_double * 2)(*[x.imag for x in lam]),
                            p.g.shape[1], self.g.ctypes.data_as(dp), p.n_nodes, self.nodes.ctypes.data_as(dp),
                            self.pb.ctypes.data_as(C.POINTER(C.c_uint32)),
                            self.pc.ctypes.data_as(C.POINTER(C.c_uint32)), p.dt, p.seed, p.stream,
                            min(int(p.max_steps), 0xFFFFFFFF))


def ksolve(p, threads: Optional[int] = None, records: bool = False):
    """The discontinuous-kappa walk (interface scheme of Secs. 2.2, 3.1)."""
    m = _KMarshalled(p)
    n = p.n_nodes
    out = np.zeros(max(n, 1), dtype=NODE_DTYPE)
    recs = np.zeros(p.total_paths, dtype=PATH_DTYPE) if records else None
    rc = lib().orc_ksolve(C.byref(m.s), threads or default_threads(), out.ctypes.data,
                          recs.ctypes.data if recs is not None and recs.size else None)
    if rc != 0:
        raise ValueError(f"oracle rejected the problem (code {rc})")
    return out[:n], recs


def kwalk_path(p, node: int, path: int):
    m = _KMarshalled(p)
    rec = Path_C()
    rc = lib().orc_kwalk_path(C.byref(m.s), node, path, C.byref(rec))
    if rc != 0:
        raise ValueError(rc)
    return {k: getattr(rec, k) for k, _ in Path_C._fields_}


def kwalk_nodes(p, node_idx):
    """Records of every path of the chosen nodes of p, walked with their own
    node indices (the same realisations as in a solve of all of p)."""
    m = _KMarshalled(p)
    if lib().orc_kvalidate(C.byref(m.s)) != 0:
        raise ValueError("oracle rejected the problem")
    out = []
    rec = Path_C()
    for j in node_idx:
        b, c = int(p.path_begin[j]), int(p.path_count[j])
        r = np.zeros(c, dtype=PATH_DTYPE)
        for k in range(c):
            lib().orc_kwalk_path(C.byref(m.s), int(j), b + k, C.byref(rec))
            r[k] = tuple(getattr(rec, f) for f, _ in Path_C._fields_)
        out.append(r)
    return out


def kvalidate(p) -> int:
    m = _KMarshalled(p)
    return int(lib().orc_kvalidate(C.byref(m.s)))
