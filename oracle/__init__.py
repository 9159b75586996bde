"""ctypes binding of the FP64 CPU oracle (``hmat_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``. The HIP path never imports it, and it
imports nothing from the HIP path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def lib():
    """Load the oracle library, compiling it first if it is missing or stale."""
    global _lib
    if _lib is not None:
        return _lib
    path = _build.build(force=False)
    L = C.CDLL(path)
    vp = C.c_void_p
    L.or_version.restype = C.c_int
    L.or_num_threads.restype = C.c_int
    L.or_set_threads.argtypes = [C.c_int]
    L.or_kelvin.argtypes = [_dp, C.c_double, C.c_double, _dp]
    L.or_rule_radon7.argtypes = [_dp, _dp]
    L.or_gauss_legendre.argtypes = [C.c_int, _dp, _dp]
    L.or_ctx_new.restype = vp
    L.or_ctx_new.argtypes = [C.c_int, C.c_int, _dp, _ip, C.c_double, C.c_double]
    L.or_ctx_free.argtypes = [vp]
    L.or_ctx_set_self_order.argtypes = [vp, C.c_int]
    L.or_ctx_geometry.argtypes = [vp, _dp, _dp, _dp, _dp]
    L.or_entry_block.argtypes = [vp, C.c_int, C.c_int, _dp]
    L.or_entries.argtypes = [vp, C.c_int, _lp, _lp, _dp]
    L.or_dense.argtypes = [vp, _dp]
    L.or_brute_matvec_rows.argtypes = [vp, C.c_int, vp, C.c_int, _dp, _dp]
    L.or_aca_dense.restype = C.c_int
    L.or_aca_dense.argtypes = [C.c_int, C.c_int, _dp, C.c_double, _dp, _dp, _ip, _ip,
                               C.POINTER(C.c_int), C.POINTER(C.c_double)]
    L.or_aca_dense_steps.restype = C.c_int
    L.or_aca_dense_steps.argtypes = [C.c_int, C.c_int, _dp, C.c_int, C.c_int, _dp, _dp, _ip, _ip,
                                     C.POINTER(C.c_int)]
    L.or_h_plan.restype = vp
    L.or_h_plan.argtypes = [vp, C.c_double, C.c_int]
    L.or_h_fill.restype = C.c_int
    L.or_h_fill.argtypes = [vp, C.c_double]
    L.or_h_fill_steps.restype = C.c_int
    L.or_h_fill_steps.argtypes = [vp, C.c_int]
    L.or_h_free.argtypes = [vp]
    L.or_h_nclusters.restype = C.c_int
    L.or_h_nclusters.argtypes = [vp]
    L.or_h_cluster.argtypes = [vp, C.c_int, _ip, _dp]
    L.or_h_order.argtypes = [vp, _ip]
    L.or_h_nblocks.restype = C.c_int
    L.or_h_nblocks.argtypes = [vp]
    L.or_h_block.argtypes = [vp, C.c_int, _ip, C.POINTER(C.c_double)]
    L.or_h_csp.restype = C.c_int
    L.or_h_csp.argtypes = [vp]
    L.or_h_times.argtypes = [vp, _dp]
    L.or_h_factors.argtypes = [vp, C.c_int, vp, vp, vp, vp]
    L.or_h_dense_block.argtypes = [vp, C.c_int, _dp]
    L.or_h_stored.restype = C.c_int64
    L.or_h_stored.argtypes = [vp]
    L.or_h_matvec.argtypes = [vp, C.c_int, _dp, _dp]
    L.or_h_gmres.restype = C.c_int
    L.or_h_gmres.argtypes = [vp, _dp, _dp, C.c_double, C.c_int, C.c_int,
                             C.POINTER(C.c_int), C.POINTER(C.c_double)]
    L.or_dense_gmres.restype = C.c_int
    L.or_dense_gmres.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_double, C.c_int, C.c_int,
                                 C.POINTER(C.c_int), C.POINTER(C.c_double)]
    _lib = L
    return L


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def num_threads() -> int:
    return int(lib().or_num_threads())


def kelvin(r, E: float = 1.0, nu: float = 0.3) -> np.ndarray:
    """Kelvin tensor S(r) as a 3x3 array."""
    out = np.zeros(9)
    lib().or_kelvin(np.ascontiguousarray(r, dtype=np.float64), float(E), float(nu), out)
    return out.reshape(3, 3)


def radon7():
    """Seven-point rule: (barycentric points [7,3], weights [7])."""
    b = np.zeros(21)
    w = np.zeros(7)
    lib().or_rule_radon7(b, w)
    return b.reshape(7, 3), w


def gauss_legendre(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().or_gauss_legendre(int(n), x, w)
    return x, w


def aca_dense(A: np.ndarray, eps: float):
    """ACA on a dense matrix. Returns dict(U, V, rows, cols, stop, ratio)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    m, n = A.shape
    kmax = min(m, n)
    U = np.zeros(m * kmax)
    V = np.zeros(n * kmax)
    pr = np.zeros(kmax, dtype=np.int32)
    pc = np.zeros(kmax, dtype=np.int32)
    st = C.c_int(0)
    ra = C.c_double(0)
    k = lib().or_aca_dense(m, n, A, float(eps), U, V, pr, pc, C.byref(st), C.byref(ra))
    return dict(U=U[: m * k].reshape(k, m).T.copy(), V=V[: n * k].reshape(k, n).T.copy(),
                rows=pr[:k].copy(), cols=pc[:k].copy(), stop=st.value, ratio=ra.value)


def aca_dense_steps(A: np.ndarray, kcap: int, ncls: int = 3):
    """Step-limited ACA (no accuracy test, class-cycling rows; the adaptive
    multiplication's look-ahead) on a dense matrix whose row i is in class
    i mod ncls. Returns dict(U, V, rows, cols, stop)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    m, n = A.shape
    kmax = min(m, n, kcap)
    U = np.zeros(m * kmax)
    V = np.zeros(n * kmax)
    pr = np.zeros(kmax, dtype=np.int32)
    pc = np.zeros(kmax, dtype=np.int32)
    st = C.c_int(0)
    k = lib().or_aca_dense_steps(m, n, A, int(kcap), int(ncls), U, V, pr, pc, C.byref(st))
    return dict(U=U[: m * k].reshape(k, m).T.copy(), V=V[: n * k].reshape(k, n).T.copy(),
                rows=pr[:k].copy(), cols=pc[:k].copy(), stop=st.value)


class Mesh:
    """Geometry and material of a triangulated surface (owns an ``or_ctx``)."""

    def __init__(self, vertices, triangles, E: float = 1.0, nu: float = 0.3):
        self.V = np.ascontiguousarray(vertices, dtype=np.float64)
        self.T = np.ascontiguousarray(triangles, dtype=np.int32)
        self.E, self.nu = float(E), float(nu)
        self.nt = self.T.shape[0]
        self.N = 3 * self.nt
        self._c = lib().or_ctx_new(self.V.shape[0], self.nt, self.V, self.T, self.E, self.nu)
        if not self._c:
            raise ValueError("oracle: invalid mesh")

    def __del__(self):
        if getattr(self, "_c", None):
            lib().or_ctx_free(self._c)
            self._c = None

    def set_self_order(self, n: int) -> None:
        lib().or_ctx_set_self_order(self._c, int(n))

    def geometry(self):
        nt = self.nt
        cen, area, qn, qw = np.zeros(3 * nt), np.zeros(nt), np.zeros(21 * nt), np.zeros(7 * nt)
        lib().or_ctx_geometry(self._c, cen, area, qn, qw)
        return cen.reshape(nt, 3), area, qn.reshape(nt, 7, 3), qw.reshape(nt, 7)

    def entry_block(self, i: int, j: int) -> np.ndarray:
        out = np.zeros(9)
        lib().or_entry_block(self._c, int(i), int(j), out)
        return out.reshape(3, 3)

    def entries(self, rows, cols) -> np.ndarray:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        out = np.zeros(rows.shape[0])
        lib().or_entries(self._c, rows.shape[0], rows, cols, out)
        return out

    def dense(self) -> np.ndarray:
        A = np.zeros(self.N * self.N)
        lib().or_dense(self._c, A)
        return A.reshape(self.N, self.N)

    def brute_matvec(self, x, tri_rows=None) -> np.ndarray:
        """Matrix-free A x; x is (nrhs, N). With ``tri_rows`` only those triangles' 3 rows each."""
        x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float64)
        nrhs = x.shape[0]
        if tri_rows is None:
            y = np.zeros((nrhs, self.N))
            lib().or_brute_matvec_rows(self._c, 0, None, nrhs, x, y)
        else:
            tr = np.ascontiguousarray(tri_rows, dtype=np.int32)
            y = np.zeros((nrhs, 3 * tr.shape[0]))
            lib().or_brute_matvec_rows(self._c, tr.shape[0], tr.ctypes.data_as(C.c_void_p),
                                       nrhs, x, y)
        return y


class HMatrix:
    """Cluster tree, partition and (after ``fill``) near blocks plus ACA factors."""

    def __init__(self, mesh: Mesh, eta: float = 2.0, leaf: int = 32, eps: float | None = None):
        self.mesh = mesh
        self._h = lib().or_h_plan(mesh._c, float(eta), int(leaf))
        if not self._h:
            raise ValueError("oracle: invalid partition parameters")
        if eps is not None:
            self.fill(eps)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_h_free(self._h)
            self._h = None

    def fill(self, eps: float) -> None:
        if lib().or_h_fill(self._h, float(eps)) != 0:
            raise ValueError("oracle: invalid eps")

    def fill_steps(self, kcap: int) -> None:
        """Dense blocks, and ACA on every admissible block for kcap steps
        without the accuracy test (crosses for the adaptive multiplication)."""
        if lib().or_h_fill_steps(self._h, int(kcap)) != 0:
            raise ValueError("oracle: invalid step count")

    @property
    def order(self) -> np.ndarray:
        o = np.zeros(self.mesh.nt, dtype=np.int32)
        lib().or_h_order(self._h, o)
        return o

    def clusters(self):
        """List of dict(off, len, son0, son1, level, lo, hi)."""
        out = []
        info = np.zeros(5, dtype=np.int32)
        box = np.zeros(6)
        for c in range(lib().or_h_nclusters(self._h)):
            lib().or_h_cluster(self._h, c, info, box)
            out.append(dict(off=int(info[0]), len=int(info[1]), son0=int(info[2]),
                            son1=int(info[3]), level=int(info[4]), lo=box[:3].copy(),
                            hi=box[3:].copy()))
        return out

    def blocks(self) -> np.ndarray:
        """int array [nb, 9]: row_off, row_len, col_off, col_len (triangles), far, rank, stop, t, s."""
        nb = lib().or_h_nblocks(self._h)
        out = np.zeros((nb, 9), dtype=np.int32)
        info = np.zeros(9, dtype=np.int32)
        r = C.c_double(0)
        for b in range(nb):
            lib().or_h_block(self._h, b, info, C.byref(r))
            out[b] = info
        return out

    def stop_ratios(self) -> np.ndarray:
        nb = lib().or_h_nblocks(self._h)
        out = np.zeros(nb)
        info = np.zeros(9, dtype=np.int32)
        r = C.c_double(0)
        for b in range(nb):
            lib().or_h_block(self._h, b, info, C.byref(r))
            out[b] = r.value
        return out

    def csp(self) -> int:
        return int(lib().or_h_csp(self._h))

    def times(self):
        t = np.zeros(3)
        lib().or_h_times(self._h, t)
        return dict(plan=t[0], near=t[1], aca=t[2])

    def factors(self, b: int):
        """(U [m,k], V [n,k], pivot rows [k], pivot cols [k]) of far block b."""
        info = np.zeros(9, dtype=np.int32)
        r = C.c_double(0)
        lib().or_h_block(self._h, b, info, C.byref(r))
        m, n, k = 3 * int(info[1]), 3 * int(info[3]), int(info[5])
        U = np.zeros(m * k)
        V = np.zeros(n * k)
        pr = np.zeros(k, dtype=np.int32)
        pc = np.zeros(k, dtype=np.int32)
        lib().or_h_factors(self._h, b, U.ctypes.data, V.ctypes.data, pr.ctypes.data,
                           pc.ctypes.data)
        return U.reshape(k, m).T.copy(), V.reshape(k, n).T.copy(), pr, pc

    def dense_block(self, b: int) -> np.ndarray:
        info = np.zeros(9, dtype=np.int32)
        r = C.c_double(0)
        lib().or_h_block(self._h, b, info, C.byref(r))
        m, n = 3 * int(info[1]), 3 * int(info[3])
        D = np.zeros(m * n)
        lib().or_h_dense_block(self._h, b, D)
        return D.reshape(n, m).T.copy()

    def stored(self) -> int:
        return int(lib().or_h_stored(self._h))

    def matvec(self, x) -> np.ndarray:
        x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float64)
        y = np.zeros_like(x)
        lib().or_h_matvec(self._h, x.shape[0], x, y)
        return y

    def gmres(self, b, tol: float = 1e-8, restart: int = 50, maxit: int = 10000):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b)
        it = C.c_int(0)
        rr = C.c_double(0)
        st = lib().or_h_gmres(self._h, b, x, float(tol), int(restart), int(maxit), C.byref(it),
                              C.byref(rr))
        return x, dict(status=st, iters=it.value, relres=rr.value)


def dense_gmres(A, b, tol: float = 1e-8, restart: int = 50, maxit: int = 10000):
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    it = C.c_int(0)
    rr = C.c_double(0)
    st = lib().or_dense_gmres(A.shape[0], A, b, x, float(tol), int(restart), int(maxit),
                              C.byref(it), C.byref(rr))
    return x, dict(status=st, iters=it.value, relres=rr.value)
