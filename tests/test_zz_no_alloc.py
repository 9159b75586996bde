"""hmat_solve_noalloc: GMRES with its workspace in the library's fixed
per-device array, checked against hmat_solve through the C ABI.

Two calls in a row, the second on a smaller system (icosphere level 3, then
level 2); each must give hmat_solve's solution (same kernels in the same
order: the same bits, asserted within 1e-13 relative), iterations and status,
reach the FP64 relative residual 1e-8, and leave the handle's device
memory unchanged (hmat_solve grows the handle by its GMRES workspace). A
request beyond the fixed workspace is refused before any device work.
"""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _solve(L, H, h, b, restart, fn):
    x = torch.zeros_like(b)
    info = H._SolveInfo()
    st = fn(h._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), 1e-8, restart, 10000,
            C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(info))
    torch.cuda.synchronize()
    return st, x, info


def test_noalloc_solve_matches_solve():
    import paper_2205_04752_amd as H
    L = H.lib()
    for level, restart in ((3, 50), (2, 30)):
        print(f"noalloc solve: icosphere level {level}, GMRES({restart})", flush=True)
        V, T = W.icosphere(level)
        g = H.HMatrix(V, T, 1.0, 0.3, 2.0, 32, 1e-6)
        b = torch.from_numpy(W.smooth_rhs(V, T, seed=1)).cuda()
        bytes0 = g.info()["device_bytes"]
        st_n, x_n, inf_n = _solve(L, H, g, b, restart, L.hmat_solve_noalloc)
        assert st_n == H.HMAT_OK, L.hmat_last_error()
        assert g.info()["device_bytes"] == bytes0
        st_s, x_s, inf_s = _solve(L, H, g, b, restart, L.hmat_solve)
        assert st_s == H.HMAT_OK, L.hmat_last_error()
        assert g.info()["device_bytes"] > bytes0  # hmat_solve allocated its basis
        assert inf_n.iterations == inf_s.iterations and inf_n.restarts == inf_s.restarts
        d = float(torch.linalg.norm(x_n - x_s) / torch.linalg.norm(x_s))
        assert d <= 1e-13, d
        r = float(torch.linalg.norm(b - g.matvec(x_n)) / torch.linalg.norm(b))
        assert r <= 1e-8 and abs(inf_n.relres - inf_s.relres) <= 1e-20 + 1e-12 * inf_s.relres
        print(f"  iterations {inf_n.iterations}, relres {r:.2e}, bitwise {bool(torch.equal(x_n, x_s))}",
              flush=True)
        g.close()


def test_noalloc_solve_rejects_oversize():
    import paper_2205_04752_amd as H
    L = H.lib()
    V, T = W.icosphere(5)
    g = H.HMatrix(V, T, 1.0, 0.3, 2.0, 32, 1e-4)
    b = torch.ones(g.n_dof, dtype=torch.float64, device="cuda")
    x = torch.full_like(b, 7.0)
    st = L.hmat_solve_noalloc(g._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), 1e-8, 100,
                              100, None, None)
    assert st == H.HMAT_EINVAL
    assert "fixed workspace" in L.hmat_last_error().decode()
    torch.cuda.synchronize()
    assert bool((x == 7.0).all())  # nothing launched
    # the same handle within the limit: GMRES(50) fits 61440 DOF
    st, x2, info = _solve(L, H, g, b, 50, L.hmat_solve_noalloc)
    assert st == H.HMAT_OK, L.hmat_last_error()
    r = float(torch.linalg.norm(b - g.matvec(x2)) / torch.linalg.norm(b))
    assert r <= 1e-8
    g.close()
