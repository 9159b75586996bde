"""Python binding of libhmat.so, the MI355X H-matrix library for the Lame
single-layer operator (Kelvin kernel, collocation, ACA, H-matrix product).

Argument marshalling only: every step runs in the HIP library through its C
ABI (``include/hmat.h``). Device vectors are torch tensors on the ROCm device;
torch supplies device memory and the current stream. There is no CPU fallback:
if the library has not been built, loading it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = ["lib", "HMatrix", "Server", "plan", "amvm", "release_memory", "HmatError", "LIB_PATH"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhmat.so")

HMAT_OK, HMAT_EINVAL, HMAT_ENOMEM, HMAT_EDEVICE, HMAT_ENOCONV, HMAT_ENOTSUP, HMAT_ECANCELED = range(7)
_STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENOCONV", 5: "ENOTSUP", 6: "ECANCELED"}


class HmatError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hmat {_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Mesh(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("n_triangles", C.c_int32),
                ("vertices", C.c_void_p), ("triangles", C.c_void_p)]


class _Stats(C.Structure):
    _fields_ = [("n_dof", C.c_int64), ("n_triangles", C.c_int32), ("n_clusters", C.c_int32),
                ("depth", C.c_int32), ("n_blocks", C.c_int32), ("n_far", C.c_int32),
                ("n_near", C.c_int32), ("c_sp", C.c_int32), ("rank_min", C.c_int32),
                ("rank_max", C.c_int32), ("rank_mean", C.c_double), ("far_scalars", C.c_int64),
                ("near_scalars", C.c_int64), ("compression", C.c_double),
                ("n_rank_full", C.c_int32), ("n_near_threshold", C.c_int32),
                ("aca_passes", C.c_int32), ("n_exact", C.c_int32), ("t_plan_ms", C.c_double),
                ("t_near_ms", C.c_double), ("t_aca_ms", C.c_double), ("t_build_ms", C.c_double),
                ("device_bytes", C.c_int64), ("far_u_scalars", C.c_int64),
                ("far_v_scalars", C.c_int64), ("t_aca_kernel_ms", C.c_double),
                ("t_layout_ms", C.c_double), ("aca_groups", C.c_int32), ("n_bodies", C.c_int32),
                ("precision", C.c_int32), ("aca_fp32", C.c_int32)]


class _SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("restarts", C.c_int32), ("relres", C.c_double),
                ("time_ms", C.c_double), ("refinements", C.c_int32), ("reserved", C.c_int32)]


class _TuneInfo(C.Structure):
    _fields_ = [("nrhs", C.c_int32), ("n_candidates", C.c_int32), ("chunk_kb", C.c_int32 * 8),
                ("unroll", C.c_int32 * 8), ("ms", C.c_double * 8), ("best", C.c_int32),
                ("reserved", C.c_int32), ("best_ms", C.c_double)]


class _AmvmInfo(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("exhausted", C.c_int32), ("aca_steps", C.c_int64),
                ("marked_total", C.c_int64), ("gamma", C.c_double), ("time_ms", C.c_double)]


class _Opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("aca_small_tri", C.c_int32), ("aca_stop_factor", C.c_double),
                ("aca_wide", C.c_int32), ("reserved", C.c_int32)]


class _AcaTuneInfo(C.Structure):
    _fields_ = [("n_candidates", C.c_int32), ("best", C.c_int32), ("small_tri", C.c_int32 * 8),
                ("wide", C.c_int32 * 8), ("aca_ms", C.c_double * 8), ("best_ms", C.c_double)]


class _Request(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nvec", C.c_int32), ("precision", C.c_int32),
                ("restart", C.c_int32), ("E", C.c_double), ("nu", C.c_double), ("eps", C.c_double),
                ("tol", C.c_double)]


class _Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("refinements", C.c_int32),
                ("reserved", C.c_int32), ("relres", C.c_double), ("t_submit_ms", C.c_double),
                ("t_admit_ms", C.c_double), ("t_done_ms", C.c_double), ("build_ms", C.c_double),
                ("device_bytes", C.c_int64)]


EXPORTS = ["hmat_build", "hmat_build_ex", "hmat_tune_aca", "hmat_build_batch", "hmat_bodies", "hmat_matvec", "hmat_matvec_ex",
           "hmat_solve", "hmat_solve_noalloc", "hmat_solve_ir", "hmat_set_precision", "hmat_info", "hmat_free",
           "hmat_last_error", "hmat_plan", "hmat_block", "hmat_entries", "hmat_set_factors",
           "hmat_profile", "hmat_tune", "hmat_matvec_graph", "hmat_amvm", "hmat_server_create", "hmat_server_submit", "hmat_server_wait", "hmat_server_cancel", "hmat_server_status",
           "hmat_server_destroy", "hmat_server_last_error", "hmat_release_memory",
           "hmat_set_mem_budget", "hmat_mem_held"]

_lib = None


def lib():
    """Load libhmat.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "or python paper_2205_04752_amd/build.py")
    # torch first: the library then binds to the HIP runtime torch has loaded
    # (same soname), so torch's streams and device pointers are valid in it.
    # Loaded on its own, it binds to the system runtime instead.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.hmat_build.argtypes = [C.POINTER(_Mesh), dbl, dbl, dbl, i32, dbl, vp, C.POINTER(vp)]
    L.hmat_build_ex.argtypes = [C.POINTER(_Mesh), dbl, dbl, dbl, i32, dbl, C.POINTER(_Opts), vp, C.POINTER(vp)]
    L.hmat_tune_aca.argtypes = [C.POINTER(_Mesh), dbl, dbl, dbl, i32, dbl, C.POINTER(_Opts), i32, vp,
                                C.POINTER(_AcaTuneInfo)]
    L.hmat_build_batch.argtypes = [i32, vp, vp, vp, vp, dbl, i32, vp, C.POINTER(vp)]
    L.hmat_bodies.argtypes = [vp, C.POINTER(i32), vp]
    L.hmat_matvec.argtypes = [vp, i32, vp, i64, vp, i64, vp]
    L.hmat_solve.argtypes = [vp, vp, vp, dbl, i32, i32, vp, C.POINTER(_SolveInfo)]
    L.hmat_solve_noalloc.argtypes = [vp, vp, vp, dbl, i32, i32, vp, C.POINTER(_SolveInfo)]
    L.hmat_solve_ir.argtypes = [vp, vp, vp, dbl, i32, i32, i32, dbl, vp, C.POINTER(_SolveInfo)]
    L.hmat_set_precision.argtypes = [vp, i32, vp]
    L.hmat_matvec_ex.argtypes = [vp, i32, i32, vp, i64, vp, i64, vp]
    L.hmat_info.argtypes = [vp, C.POINTER(_Stats)]
    L.hmat_free.argtypes = [vp]
    L.hmat_release_memory.argtypes = [vp]
    L.hmat_set_mem_budget.argtypes = [i64]
    L.hmat_mem_held.argtypes = [C.POINTER(i64), C.POINTER(i64)]
    L.hmat_last_error.restype = C.c_char_p
    L.hmat_plan.argtypes = [C.POINTER(_Mesh), dbl, i32, vp, C.POINTER(i32), vp]
    L.hmat_block.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    L.hmat_entries.argtypes = [vp, i64, vp, vp, vp, vp]
    L.hmat_set_factors.argtypes = [vp, vp, vp, vp, vp]
    L.hmat_profile.argtypes = [vp, i32, vp, C.POINTER(i64)]
    L.hmat_tune.argtypes = [vp, i32, i32, vp, C.POINTER(_TuneInfo)]
    L.hmat_matvec_graph.argtypes = [vp, i32, i32, vp, i64, vp, i64, vp]
    L.hmat_amvm.argtypes = [C.POINTER(_Mesh), dbl, dbl, dbl, i32, vp, vp, dbl, dbl, i32, i32, vp,
                            vp, C.POINTER(_AmvmInfo)]
    L.hmat_server_create.argtypes = [i32, i64, dbl, i32, C.POINTER(vp)]
    L.hmat_server_submit.argtypes = [vp, C.POINTER(_Mesh), C.POINTER(_Request), vp, C.POINTER(i64)]
    L.hmat_server_wait.argtypes = [vp, i64, vp, C.POINTER(_Result)]
    L.hmat_server_cancel.argtypes = [vp, i64]
    L.hmat_server_status.argtypes = [vp, C.POINTER(i64), C.POINTER(i32), C.POINTER(i32)]
    L.hmat_server_destroy.argtypes = [vp]
    L.hmat_server_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("hmat_last_error", "hmat_server_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(st: int) -> None:
    if st != HMAT_OK:
        raise HmatError(st, lib().hmat_last_error().decode())


def _mesh(vertices, triangles):
    V = np.ascontiguousarray(vertices, dtype=np.float64)
    T = np.ascontiguousarray(triangles, dtype=np.int32)
    if V.ndim != 2 or V.shape[1] != 3 or T.ndim != 2 or T.shape[1] != 3:
        raise ValueError("vertices must be [nv, 3] and triangles [nt, 3]")
    m = _Mesh(V.shape[0], T.shape[0], V.ctypes.data, T.ctypes.data)
    return m, (V, T)


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(getattr(stream, "cuda_stream", stream)))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, n_dof, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 tensor on the GPU")
    if t.dim() == 1:
        t = t.unsqueeze(0)
    if t.dim() != 2 or t.shape[1] != n_dof or t.stride(1) != 1:
        raise ValueError(f"{name} must be [nrhs, {n_dof}] with unit column stride")
    return t, t.data_ptr(), t.stride(0)


def release_memory(stream=None) -> None:
    """Hand the device memory the library keeps for reuse back to the device
    (hmat_release_memory); live handles keep theirs."""
    _check(lib().hmat_release_memory(_stream(stream)))


def set_mem_budget(nbytes: int) -> None:
    """Cap on the device memory the library holds (0: none); see hmat_set_mem_budget."""
    _check(lib().hmat_set_mem_budget(int(nbytes)))


def mem_held() -> tuple[int, int]:
    """(bytes of device memory the library holds on the current device, the
    most it held since the previous call)."""
    v, pk = C.c_int64(0), C.c_int64(0)
    _check(lib().hmat_mem_held(C.byref(v), C.byref(pk)))
    return v.value, pk.value


def plan(vertices, triangles, eta: float = 2.0, leaf: int = 32):
    """Host-only partition: (order [nt], blocks [nb, 5]: row_off, row_len, col_off, col_len, far)."""
    m, keep = _mesh(vertices, triangles)
    nb = C.c_int32(0)
    order = np.zeros(m.n_triangles, dtype=np.int32)
    _check(lib().hmat_plan(C.byref(m), float(eta), int(leaf), order.ctypes.data, C.byref(nb), None))
    blocks = np.zeros((nb.value, 5), dtype=np.int32)
    _check(lib().hmat_plan(C.byref(m), float(eta), int(leaf), None, C.byref(nb), blocks.ctypes.data))
    return order, blocks


def tune_aca(vertices, triangles, E=1.0, nu=0.3, eta=2.0, leaf=32, eps=1e-4, reps=2, precision=0,
             aca_stop_factor=1.0, stream=None) -> dict:
    """Time the ACA launch schedules on this mesh (hmat_tune_aca); returns the
    candidates and the best as an aca_schedule for HMatrix."""
    m, keep = _mesh(vertices, triangles)
    o = _Opts(int(precision), 0, float(aca_stop_factor), 0, 0)
    t = _AcaTuneInfo()
    _check(lib().hmat_tune_aca(C.byref(m), float(E), float(nu), float(eta), int(leaf), float(eps), C.byref(o),
                               int(reps), _stream(stream), C.byref(t)))
    n = t.n_candidates
    cands = [(t.small_tri[c], t.wide[c], t.aca_ms[c]) for c in range(n)]
    return dict(candidates=cands, best=t.best, best_ms=t.best_ms,
                aca_schedule=(t.small_tri[t.best], t.wide[t.best]))


def amvm(vertices, triangles, x, E=1.0, nu=0.3, eta=2.0, leaf=32, theta=0.5, tol=1e-6,
         max_rounds=1000, kmax=128, stream=None):
    """Adaptive matrix-vector multiplication (hmat_amvm): returns (y, info, ranks)
    with y on the device, ranks per block in canonical order (-1: dense)."""
    import torch
    m, keep = _mesh(vertices, triangles)
    N = 3 * m.n_triangles
    x2, xp, _ = _dev_ptr(x, N, "x")
    y = torch.empty_like(x2[0])
    info = _AmvmInfo()
    nb = C.c_int32(0)
    lib().hmat_plan(C.byref(m), float(eta), int(leaf), None, C.byref(nb), None)
    ranks = np.zeros(max(nb.value, 1), dtype=np.int32)
    _check(lib().hmat_amvm(C.byref(m), float(E), float(nu), float(eta), int(leaf), xp, y.data_ptr(),
                           float(theta), float(tol), int(max_rounds), int(kmax), _stream(stream),
                           ranks.ctypes.data, C.byref(info)))
    return y, {k: getattr(info, k) for k, _ in _AmvmInfo._fields_}, ranks[:nb.value]


class HMatrix:
    """Device-resident H-matrix of the Kelvin single-layer collocation matrix."""

    def __init__(self, vertices, triangles, E=1.0, nu=0.3, eta=2.0, leaf=32, eps=1e-4,
                 stream=None, precision: int = 0, aca_stop_factor: float = 1.0, aca_schedule=None):
        """precision 1 stores the entries in FP32 only (hmat_build_ex);
        aca_stop_factor is the constant of the ACA stop test; aca_schedule is
        (aca_small_tri, aca_wide), e.g. from tune_aca."""
        m, keep = _mesh(vertices, triangles)
        h = C.c_void_p()
        small, wide = aca_schedule if aca_schedule is not None else (0, 0)
        if precision == 0 and aca_stop_factor == 1.0 and aca_schedule is None:
            _check(lib().hmat_build(C.byref(m), float(E), float(nu), float(eta), int(leaf),
                                    float(eps), _stream(stream), C.byref(h)))
        else:
            o = _Opts(int(precision), int(small), float(aca_stop_factor), int(wide), 0)
            _check(lib().hmat_build_ex(C.byref(m), float(E), float(nu), float(eta), int(leaf),
                                       float(eps), C.byref(o), _stream(stream), C.byref(h)))
        self._h = h
        self.n_triangles = m.n_triangles
        self.n_dof = 3 * m.n_triangles

    @classmethod
    def batch(cls, bodies, eta=2.0, leaf=32, stream=None):
        """One handle for several independent bodies (block-diagonal operator).
        bodies: sequence of dicts with vertices, triangles, E, nu, eps. Vectors
        are the bodies' DOF vectors concatenated (offsets: bodies())."""
        nb = len(bodies)
        arr = (_Mesh * nb)()
        keep = []
        for i, b in enumerate(bodies):
            m, k = _mesh(b["vertices"], b["triangles"])
            arr[i] = m
            keep.append(k)
        E = np.ascontiguousarray([float(b["E"]) for b in bodies])
        nu = np.ascontiguousarray([float(b["nu"]) for b in bodies])
        eps = np.ascontiguousarray([float(b["eps"]) for b in bodies])
        h = C.c_void_p()
        _check(lib().hmat_build_batch(nb, C.cast(arr, C.c_void_p), E.ctypes.data, nu.ctypes.data,
                                      eps.ctypes.data, float(eta), int(leaf), _stream(stream),
                                      C.byref(h)))
        self = cls.__new__(cls)
        self._h = h
        self.n_triangles = int(sum(int(np.asarray(b["triangles"]).shape[0]) for b in bodies))
        self.n_dof = 3 * self.n_triangles
        return self

    def bodies(self) -> np.ndarray:
        """DOF offsets of the bodies: [n_bodies + 1], last entry n_dof."""
        n = C.c_int32(0)
        _check(lib().hmat_bodies(self._h, C.byref(n), None))
        off = np.zeros(n.value + 1, dtype=np.int64)
        _check(lib().hmat_bodies(self._h, C.byref(n), off.ctypes.data))
        return off

    def close(self):
        if getattr(self, "_h", None):
            lib().hmat_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def matvec(self, x, y=None, stream=None, precision: int = 0, graph: bool = False):
        """y = A_H x for x of shape [nrhs, n_dof] (or [n_dof]); float64 on the GPU.
        precision 1 reads the FP32 copies of the entries (set_precision(1));
        graph replays a captured HIP graph for this (x, y) pair."""
        import torch
        squeeze = x.dim() == 1
        x2, xp, ldx = _dev_ptr(x, self.n_dof, "x")
        if y is None:
            y = torch.empty_like(x2)
        y2, yp, ldy = _dev_ptr(y, self.n_dof, "y")
        if y2.shape[0] != x2.shape[0]:
            raise ValueError("x and y must hold the same number of vectors")
        if graph:
            _check(lib().hmat_matvec_graph(self._h, int(precision), x2.shape[0], xp, ldx, yp, ldy,
                                           _stream(stream)))
        elif precision == 0:
            _check(lib().hmat_matvec(self._h, x2.shape[0], xp, ldx, yp, ldy, _stream(stream)))
        else:
            _check(lib().hmat_matvec_ex(self._h, int(precision), x2.shape[0], xp, ldx, yp, ldy,
                                        _stream(stream)))
        return y2[0] if squeeze else y2

    def tune(self, nrhs: int = 1, reps: int = 5, stream=None) -> dict:
        """Autotune the product schedule for nrhs vectors (hmat_tune)."""
        t = _TuneInfo()
        _check(lib().hmat_tune(self._h, int(nrhs), int(reps), _stream(stream), C.byref(t)))
        n = t.n_candidates
        return dict(nrhs=t.nrhs, candidates=[(t.chunk_kb[c], t.unroll[c], t.ms[c]) for c in range(n)],
                    best=t.best, best_ms=t.best_ms, chunk_kb=t.chunk_kb[t.best], unroll=t.unroll[t.best])

    def set_precision(self, precision: int, stream=None) -> None:
        """1: make FP32 copies of the stored entries; 0: free them."""
        _check(lib().hmat_set_precision(self._h, int(precision), _stream(stream)))

    def solve_ir(self, b, x=None, tol=1e-8, restart=50, maxit=10000, inner_precision=1,
                 inner_tol=1e-6, stream=None, check=True):
        """Iterative refinement: FP64 residuals, inner GMRES on the entries stored
        in inner_precision; returns (x, info dict)."""
        import torch
        b2, bp, _ = _dev_ptr(b, self.n_dof, "b")
        if x is None:
            x = torch.empty_like(b2[0])
        x2, xp, _ = _dev_ptr(x, self.n_dof, "x")
        info = _SolveInfo()
        st = lib().hmat_solve_ir(self._h, bp, xp, float(tol), int(restart), int(maxit),
                                 int(inner_precision), float(inner_tol), _stream(stream),
                                 C.byref(info))
        if st not in (HMAT_OK, HMAT_ENOCONV) or (check and st != HMAT_OK):
            _check(st)
        return x2[0], dict(status=st, iterations=info.iterations, restarts=info.restarts,
                           relres=info.relres, time_ms=info.time_ms,
                           refinements=info.refinements)

    def solve(self, b, x=None, tol=1e-8, restart=50, maxit=10000, stream=None, check=True,
              noalloc=False):
        """GMRES(restart) for A_H x = b; returns (x, info dict). noalloc=True calls
        hmat_solve_noalloc (fixed per-device workspace; x must then be given
        to avoid an allocation here)."""
        import torch
        b2, bp, _ = _dev_ptr(b, self.n_dof, "b")
        if x is None:
            x = torch.empty_like(b2[0])
        x2, xp, _ = _dev_ptr(x, self.n_dof, "x")
        info = _SolveInfo()
        fn = lib().hmat_solve_noalloc if noalloc else lib().hmat_solve
        st = fn(self._h, bp, xp, float(tol), int(restart), int(maxit), _stream(stream), C.byref(info))
        if st not in (HMAT_OK, HMAT_ENOCONV) or (check and st != HMAT_OK):
            _check(st)
        return x2[0], dict(status=st, iterations=info.iterations, restarts=info.restarts,
                           relres=info.relres, time_ms=info.time_ms)

    def info(self) -> dict:
        s = _Stats()
        _check(lib().hmat_info(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in _Stats._fields_}

    def block(self, b: int) -> dict:
        """Host copy of block b (canonical order): info, dense D or factors U, V, pivots."""
        info = np.zeros(8, dtype=np.int32)
        _check(lib().hmat_block(self._h, int(b), info.ctypes.data, None, None, None, None))
        m, n, k = 3 * int(info[1]), 3 * int(info[3]), int(info[5])
        out = dict(row_off=int(info[0]), row_len=int(info[1]), col_off=int(info[2]),
                   col_len=int(info[3]), far=int(info[4]), rank=k, stop=int(info[6]))
        if info[4]:
            U = np.zeros(m * k)
            V = np.zeros(n * k)
            pr = np.zeros(k, dtype=np.int32)
            pc = np.zeros(k, dtype=np.int32)
            _check(lib().hmat_block(self._h, int(b), info.ctypes.data, U.ctypes.data,
                                    V.ctypes.data, pr.ctypes.data, pc.ctypes.data))
            out.update(U=U.reshape(k, m).T.copy(), V=V.reshape(k, n).T.copy(), rows=pr, cols=pc)
        else:
            D = np.zeros(m * n)
            _check(lib().hmat_block(self._h, int(b), info.ctypes.data, D.ctypes.data, None,
                                    None, None))
            out.update(D=D.reshape(n, m).T.copy())
        return out

    def entries(self, rows, cols, stream=None) -> np.ndarray:
        r = np.ascontiguousarray(rows, dtype=np.int64)
        c = np.ascontiguousarray(cols, dtype=np.int64)
        out = np.zeros(r.shape[0])
        _check(lib().hmat_entries(self._h, r.shape[0], r.ctypes.data, c.ctypes.data,
                                  out.ctypes.data, _stream(stream)))
        return out

    def profile(self, enable: bool):
        """Start (True, resets) or stop (False) per-phase product timing; returns the
        accumulated (phase_ms[4], calls) so far: gather, V^T x, U z + D x, reduce."""
        ms = np.zeros(4)
        calls = C.c_int64(0)
        _check(lib().hmat_profile(self._h, 1 if enable else 0, ms.ctypes.data, C.byref(calls)))
        return ms, calls.value

    def set_factors(self, ranks, U_cat, V_cat, stream=None) -> None:
        rk = np.ascontiguousarray(ranks, dtype=np.int32)
        U = np.ascontiguousarray(U_cat, dtype=np.float64)
        V = np.ascontiguousarray(V_cat, dtype=np.float64)
        _check(lib().hmat_set_factors(self._h, rk.ctypes.data, U.ctypes.data, V.ctypes.data,
                                      _stream(stream)))


REQ_MATVEC, REQ_SOLVE = 0, 1


class Server:
    """Request server (hmat_server_*): `slots` workers with their own streams
    admit queued requests under a device-memory budget; inputs and outputs are
    host arrays (NumPy)."""

    def __init__(self, slots: int = 4, hbm_budget: int = 0, eta: float = 2.0, leaf: int = 32):
        h = C.c_void_p()
        st = lib().hmat_server_create(int(slots), int(hbm_budget), float(eta), int(leaf), C.byref(h))
        if st != HMAT_OK:
            raise HmatError(st, lib().hmat_server_last_error().decode())
        self._s = h
        self._n = {}

    def submit(self, vertices, triangles, x, kind: int = REQ_MATVEC, E: float = 1.0,
               nu: float = 0.3, eps: float = 1e-5, precision: int = 0, tol: float = 1e-8,
               restart: int = 50) -> int:
        """x: [nvec, n_dof] vectors (products) or [n_dof] right-hand side (solve)."""
        m, keep = _mesh(vertices, triangles)
        X = np.ascontiguousarray(x, dtype=np.float64)
        N = 3 * m.n_triangles
        nvec = 1 if (kind == REQ_SOLVE or X.ndim == 1) else X.shape[0]
        if X.size != nvec * N:
            raise ValueError("x must hold nvec x n_dof values")
        q = _Request(int(kind), int(nvec), int(precision), int(restart), float(E), float(nu),
                     float(eps), float(tol))
        rid = C.c_int64(0)
        st = lib().hmat_server_submit(self._s, C.byref(m), C.byref(q), X.ctypes.data, C.byref(rid))
        if st != HMAT_OK:
            raise HmatError(st, lib().hmat_server_last_error().decode())
        self._n[rid.value] = (nvec, N, kind)
        return rid.value

    def wait(self, rid: int, check: bool = True):
        """(output array, result dict) of request rid; output None on failure."""
        nvec, N, kind = self._n.pop(rid)
        out = np.zeros(N if kind == REQ_SOLVE else (nvec, N))
        res = _Result()
        st = lib().hmat_server_wait(self._s, int(rid), out.ctypes.data, C.byref(res))
        info = {k: getattr(res, k) for k, _ in _Result._fields_}
        if st != HMAT_OK:
            if check:
                raise HmatError(st, lib().hmat_server_last_error().decode())
            return None, info
        return out, info

    def cancel(self, rid: int) -> None:
        """Stop request rid if it has not finished (its wait then reports ECANCELED)."""
        st = lib().hmat_server_cancel(self._s, int(rid))
        if st != HMAT_OK:
            raise HmatError(st, lib().hmat_server_last_error().decode())

    def status(self) -> dict:
        """Bytes reserved by running requests, queued and running counts."""
        u, q, r = C.c_int64(0), C.c_int32(0), C.c_int32(0)
        st = lib().hmat_server_status(self._s, C.byref(u), C.byref(q), C.byref(r))
        if st != HMAT_OK:
            raise HmatError(st, lib().hmat_server_last_error().decode())
        return dict(in_use=u.value, queued=q.value, running=r.value)

    def close(self):
        if getattr(self, "_s", None):
            lib().hmat_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
