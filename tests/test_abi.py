"""C ABI checks that need no GPU: the library loads, exports every entry point
that include/hmat.h declares, rejects invalid arguments before any device
work, and its host planner reproduces the oracle's cluster tree order and
block partition (Sec. 2.1) exactly."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
import workloads as W
import paper_2205_04752_amd as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hmat.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hmat_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    names = _declared()
    assert set(names) == set(H.EXPORTS), names
    L = H.lib()
    for n in names:
        assert hasattr(L, n), n


def test_environment_variables_documented():
    """Every environment variable the library reads is documented in the
    header's conventions, and the header documents none it does not read."""
    csrc = os.path.join(ROOT, "paper_2205_04752_amd", "csrc")
    read = set()
    for f in os.listdir(csrc):
        if f.endswith((".cpp", ".hip", ".hpp")):
            read |= set(re.findall(r'getenv\("(HMAT_[A-Z0-9_]+)"', open(os.path.join(csrc, f)).read()))
    hdr = open(os.path.join(ROOT, "include", "hmat.h")).read()
    env = hdr[hdr.index("Environment"):]
    env = env[:env.index("*/")]
    documented = set(re.findall(r"\n \*\s+(HMAT_[A-Z0-9_]+)\s", env))
    assert read, "no environment variables found"
    assert read == documented, (sorted(read), sorted(documented))


def _mesh_struct(V, T):
    m, keep = H._mesh(V, T)
    return m, keep


def test_build_validation_before_device_work():
    V, T = W.icosphere(1)
    L = H.lib()
    m, keep = _mesh_struct(V, T)
    h = C.c_void_p(123)
    bad = [
        (0.0, 0.3, 2.0, 32, 1e-4), (-1.0, 0.3, 2.0, 32, 1e-4), (1.0, 0.0, 2.0, 32, 1e-4),
        (1.0, 0.5, 2.0, 32, 1e-4), (1.0, 0.3, 0.0, 32, 1e-4), (1.0, 0.3, 2.0, 0, 1e-4),
        (1.0, 0.3, 2.0, 32, 0.0), (1.0, 0.3, 2.0, 32, 1.0), (float("nan"), 0.3, 2.0, 32, 1e-4),
    ]
    for args in bad:
        st = L.hmat_build(C.byref(m), *args, None, C.byref(h))
        assert st == H.HMAT_EINVAL, args
        assert h.value is None
        assert L.hmat_last_error().decode()
    # mesh errors
    T2 = T.copy()
    T2[5, 1] = len(V)
    m2, keep2 = _mesh_struct(V, T2)
    assert L.hmat_build(C.byref(m2), 1.0, 0.3, 2.0, 32, 1e-4, None, C.byref(h)) == H.HMAT_EINVAL
    assert "out of range" in L.hmat_last_error().decode()
    T3 = T.copy()
    T3[7] = [T3[7, 0], T3[7, 0], T3[7, 2]]
    m3, keep3 = _mesh_struct(V, T3)
    assert L.hmat_build(C.byref(m3), 1.0, 0.3, 2.0, 32, 1e-4, None, C.byref(h)) == H.HMAT_EINVAL
    assert "zero area" in L.hmat_last_error().decode()
    V4 = V.copy()
    V4[3, 2] = np.inf
    m4, keep4 = _mesh_struct(V4, T)
    assert L.hmat_build(C.byref(m4), 1.0, 0.3, 2.0, 32, 1e-4, None, C.byref(h)) == H.HMAT_EINVAL
    assert L.hmat_build(None, 1.0, 0.3, 2.0, 32, 1e-4, None, C.byref(h)) == H.HMAT_EINVAL
    # options of hmat_build_ex
    for prec, fac, eps in ((2, 1.0, 1e-4), (-1, 1.0, 1e-4), (0, 0.0, 1e-4), (0, -1.0, 1e-4),
                           (1, float("nan"), 1e-4), (0, 2e4, 1e-4)):
        o = H._Opts(prec, 0, fac)
        h = C.c_void_p(123)
        assert L.hmat_build_ex(C.byref(m), 1.0, 0.3, 2.0, 32, eps, C.byref(o), None,
                               C.byref(h)) == H.HMAT_EINVAL, (prec, fac)
        assert h.value is None and L.hmat_last_error().decode()
    o = H._Opts(0, 0, 1.0)
    assert L.hmat_build_ex(C.byref(m), 1.0, 0.5, 2.0, 32, 1e-4, C.byref(o), None, C.byref(h)) == H.HMAT_EINVAL
    # ACA schedule fields
    for small, wide in ((-1, 0), (1025, 0), (64, 2), (64, -1)):
        o = H._Opts(0, small, 1.0, wide, 0)
        assert L.hmat_build_ex(C.byref(m), 1.0, 0.3, 2.0, 32, 1e-4, C.byref(o), None,
                               C.byref(h)) == H.HMAT_EINVAL, (small, wide)
        assert "aca_" in L.hmat_last_error().decode()
    # the schedule autotuner validates before building anything
    t = H._AcaTuneInfo()
    assert L.hmat_tune_aca(C.byref(m), 1.0, 0.3, 2.0, 32, 1e-4, None, 0, None, C.byref(t)) == H.HMAT_EINVAL
    assert L.hmat_tune_aca(C.byref(m), 1.0, 0.3, 2.0, 32, 1e-4, None, 1, None, None) == H.HMAT_EINVAL
    assert L.hmat_tune_aca(None, 1.0, 0.3, 2.0, 32, 1e-4, None, 1, None, C.byref(t)) == H.HMAT_EINVAL
    assert L.hmat_tune_aca(C.byref(m), 1.0, 0.6, 2.0, 32, 1e-4, None, 1, None, C.byref(t)) == H.HMAT_EINVAL
    o = H._Opts(3, 0, 1.0, 0, 0)
    assert L.hmat_tune_aca(C.byref(m), 1.0, 0.3, 2.0, 32, 1e-4, C.byref(o), 1, None, C.byref(t)) == H.HMAT_EINVAL
    assert L.hmat_build(C.byref(m), 1.0, 0.3, 2.0, 32, 1e-4, None, None) == H.HMAT_EINVAL


def test_batch_validation_before_device_work():
    L = H.lib()
    V, T = W.icosphere(1)
    V2, T2 = W.torus(1.0, 0.3, 12, 6)
    arr = (H._Mesh * 2)()
    keep = []
    for i, (v, t) in enumerate([(V, T), (V2, T2)]):
        m, k = _mesh_struct(v, t)
        arr[i] = m
        keep.append(k)
    h = C.c_void_p(123)

    def call(n, E, nu, eps, eta=2.0, leaf=32, meshes=arr):
        E = np.ascontiguousarray(E, dtype=np.float64)
        nu = np.ascontiguousarray(nu, dtype=np.float64)
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        return L.hmat_build_batch(n, C.cast(meshes, C.c_void_p) if meshes is not None else None,
                                  E.ctypes.data, nu.ctypes.data, eps.ctypes.data, eta, leaf, None,
                                  C.byref(h))

    assert call(0, [1.0], [0.3], [1e-4]) == H.HMAT_EINVAL and h.value is None
    assert call(2, [1.0, 1.0], [0.3, 0.6], [1e-4, 1e-4]) == H.HMAT_EINVAL
    assert "body 1" in L.hmat_last_error().decode()
    assert call(2, [1.0, -2.0], [0.3, 0.3], [1e-4, 1e-4]) == H.HMAT_EINVAL
    assert call(2, [1.0, 1.0], [0.3, 0.3], [1e-4, 1.5]) == H.HMAT_EINVAL
    assert call(2, [1.0, 1.0], [0.3, 0.3], [1e-4, 1e-4], eta=0.0) == H.HMAT_EINVAL
    assert call(2, [1.0, 1.0], [0.3, 0.3], [1e-4, 1e-4], meshes=None) == H.HMAT_EINVAL
    T3 = T2.copy()
    T3[0, 0] = len(V2) + 4
    m3, k3 = _mesh_struct(V2, T3)
    arr[1] = m3
    assert call(2, [1.0, 1.0], [0.3, 0.3], [1e-4, 1e-4]) == H.HMAT_EINVAL
    assert "body 1" in L.hmat_last_error().decode()
    assert L.hmat_bodies(None, None, None) == H.HMAT_EINVAL


def test_amvm_validation_before_device_work():
    L = H.lib()
    V, T = W.icosphere(1)
    m, keep = _mesh_struct(V, T)
    buf = np.zeros(3 * len(T))
    x = buf.ctypes.data
    y = np.zeros(3 * len(T)).ctypes.data
    ok = dict(E=1.0, nu=0.3, eta=2.0, leaf=32, theta=0.5, tol=1e-6, rounds=10, kmax=64)

    def call(**kw):
        a = dict(ok, **kw)
        return L.hmat_amvm(C.byref(m), a["E"], a["nu"], a["eta"], a["leaf"], a.get("x", x),
                           a.get("y", y), a["theta"], a["tol"], a["rounds"], a["kmax"], None, None,
                           None)

    for bad in (dict(theta=0.0), dict(theta=1.0), dict(tol=0.0), dict(kmax=1), dict(rounds=-1),
                dict(nu=0.5), dict(E=-1.0), dict(eta=0.0), dict(x=None), dict(y=x)):
        assert call(**bad) == H.HMAT_EINVAL, bad
        assert L.hmat_last_error().decode()


def test_other_entry_points_reject_null_handle():
    L = H.lib()
    assert L.hmat_matvec(None, 1, None, 3, None, 3, None) == H.HMAT_EINVAL
    assert L.hmat_solve(None, None, None, 1e-8, 50, 10, None, None) == H.HMAT_EINVAL
    assert L.hmat_solve_noalloc(None, None, None, 1e-8, 50, 10, None, None) == H.HMAT_EINVAL
    assert L.hmat_build_ex(None, 1.0, 0.3, 2.0, 32, 1e-4, None, None, None) == H.HMAT_EINVAL
    assert L.hmat_info(None, None) == H.HMAT_EINVAL
    assert L.hmat_block(None, 0, None, None, None, None, None) == H.HMAT_EINVAL
    assert L.hmat_entries(None, 0, None, None, None, None) == H.HMAT_EINVAL
    assert L.hmat_set_factors(None, None, None, None, None) == H.HMAT_EINVAL
    assert L.hmat_set_precision(None, 1, None) == H.HMAT_EINVAL
    assert L.hmat_matvec_ex(None, 1, 1, None, 3, None, 3, None) == H.HMAT_EINVAL
    assert L.hmat_solve_ir(None, None, None, 1e-8, 50, 10, 1, 1e-6, None, None) == H.HMAT_EINVAL
    assert L.hmat_free(None) == H.HMAT_OK
    assert L.hmat_set_mem_budget(-1) == H.HMAT_EINVAL
    assert "budget" in L.hmat_last_error().decode()
    assert L.hmat_set_mem_budget(0) == H.HMAT_OK
    assert L.hmat_mem_held(None, None) == H.HMAT_EINVAL
    srv = C.c_void_p(5)
    assert L.hmat_server_create(0, 0, 2.0, 32, C.byref(srv)) == H.HMAT_EINVAL and srv.value is None
    assert L.hmat_server_create(2, -1, 2.0, 32, C.byref(srv)) == H.HMAT_EINVAL
    assert L.hmat_server_create(2, 0, 0.0, 32, C.byref(srv)) == H.HMAT_EINVAL
    assert L.hmat_server_last_error().decode()
    assert L.hmat_server_submit(None, None, None, None, None) == H.HMAT_EINVAL
    assert L.hmat_server_wait(None, 1, None, None) == H.HMAT_EINVAL
    assert L.hmat_server_cancel(None, 1) == H.HMAT_EINVAL
    assert L.hmat_server_status(None, None, None, None) == H.HMAT_EINVAL
    assert L.hmat_server_destroy(None) == H.HMAT_OK


MESHES = {
    "ico3": lambda: W.icosphere(3),
    "ico5": lambda: W.icosphere(5),
    "torus": lambda: W.torus(1.0, 0.3, 60, 20),
    "ellipsoid": lambda: W.ellipsoid(12, [2.0, 1.0, 0.5]),
    "box": lambda: W.box_surface(10.0, 1.0, 1.0, 40, 4, 4),
    "cube": lambda: W.cube_surface(9),
}


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("eta,leaf", [(2.0, 32), (0.8, 15)])
def test_plan_equals_oracle(name, eta, leaf):
    V, T = MESHES[name]()
    order, blocks = H.plan(V, T, eta, leaf)
    h = O.HMatrix(O.Mesh(V, T), eta, leaf)
    assert np.array_equal(order, h.order)
    ob = h.blocks()
    assert np.array_equal(blocks[:, :5], ob[:, :5])


def test_plan_capacity_error():
    V, T = W.icosphere(2)
    m, keep = _mesh_struct(V, T)
    nb = C.c_int32(1)
    buf = np.zeros(5, dtype=np.int32)
    st = H.lib().hmat_plan(C.byref(m), 2.0, 8, None, C.byref(nb), buf.ctypes.data)
    assert st == H.HMAT_EINVAL and nb.value > 1
