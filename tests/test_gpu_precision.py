"""Reduced-precision storage (FP32 copies of the stored entries, FP64
arithmetic) and GMRES with FP64 iterative refinement, against the oracle.

  * the FP32-storage product equals the product with the oracle's factors and
    dense blocks rounded to FP32 (the operator the kernels apply) within
    1e-9 (the FP64 factors agree to 1e-10, so a few entries may round to the
    neighbouring FP32 value), and the FP64 oracle product within the
    requested eps;
  * several vectors at once give the single-vector results;
  * iterative refinement reaches the FP64 relative residual 1e-8 and the
    FP64 GMRES solution within what the residual bound allows;
  * the FP32 copies can be dropped again, after which precision 1 is refused.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _H():
    import paper_2205_04752_amd as H
    return H


@pytest.fixture(scope="module")
def c0():
    H = _H()
    print("case precision: icosphere level 3, eps 1e-4", flush=True)
    V, T = W.icosphere(3)
    g = H.HMatrix(V, T, 1.0, 0.3, 2.0, 32, 1e-4)
    g.set_precision(1)
    mesh = O.Mesh(V, T, 1.0, 0.3)
    o = O.HMatrix(mesh, 2.0, 32, eps=1e-4)
    return dict(V=V, T=T, g=g, o=o, N=3 * len(T))


def _rounded_product(o, x):
    """Oracle H-matrix product with every stored entry rounded to FP32."""
    ob = o.blocks()
    order = o.order
    N = 3 * len(order)
    perm = (3 * order[:, None] + np.arange(3)).ravel()  # cluster DOF -> caller DOF
    xp = x[:, perm]
    yp = np.zeros_like(xp)
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    for b in range(len(ob)):
        r0, rl, c0_, cl_, far = (int(v) for v in ob[b, :5])
        rs, cs = slice(3 * r0, 3 * (r0 + rl)), slice(3 * c0_, 3 * (c0_ + cl_))
        if far:
            U, V, _, _ = o.factors(b)
            if U.shape[1]:
                yp[:, rs] += (xp[:, cs] @ f32(V)) @ f32(U).T
        else:
            yp[:, rs] += xp[:, cs] @ f32(o.dense_block(b)).T
    y = np.zeros_like(yp)
    y[:, perm] = yp
    return y


def test_f32_product_parity(c0):
    g, o = c0["g"], c0["o"]
    x = W.random_x(c0["N"], 3, seed=11)
    y32 = g.matvec(torch.from_numpy(x).cuda(), precision=1).cpu().numpy()
    y64 = o.matvec(x)
    yr = _rounded_product(o, x)
    for r in range(3):
        # the rounded operator itself
        assert np.linalg.norm(y32[r] - yr[r]) <= 1e-9 * np.linalg.norm(yr[r]), r
        # within the requested accuracy of the FP64 H-matrix, and not FP64 by accident
        d = np.linalg.norm(y32[r] - y64[r]) / np.linalg.norm(y64[r])
        assert 1e-10 < d <= 1e-4, d
    # single vectors agree with the multi-vector pass
    for r in range(3):
        y1 = g.matvec(torch.from_numpy(x[r]).cuda(), precision=1).cpu().numpy()
        assert np.linalg.norm(y1 - y32[r]) <= 1e-13 * np.linalg.norm(y32[r])


def test_iterative_refinement(c0):
    g = c0["g"]
    b = torch.from_numpy(W.smooth_rhs(c0["V"], c0["T"], seed=3)).cuda()
    x, info = g.solve_ir(b, tol=1e-8, restart=50, inner_precision=1, inner_tol=1e-6)
    assert info["status"] == 0 and info["refinements"] >= 1
    rel = float(torch.linalg.norm(b - g.matvec(x)) / torch.linalg.norm(b))
    assert rel <= 1e-8 and abs(rel - info["relres"]) <= 1e-10
    x64, i64 = g.solve(b, tol=1e-8, restart=50)
    assert float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64)) <= 1e-5
    print("ir:", info, "fp64:", i64, flush=True)
    # FP64 inner solves are refinement too (one outer step suffices)
    x2, info2 = g.solve_ir(b, tol=1e-8, restart=50, inner_precision=0, inner_tol=1e-9)
    assert info2["status"] == 0
    assert float(torch.linalg.norm(b - g.matvec(x2)) / torch.linalg.norm(b)) <= 1e-8


def test_precision_switch_and_errors(c0):
    H = _H()
    V, T = c0["V"], c0["T"]
    g = H.HMatrix(V, T, 1.0, 0.3, 2.0, 32, 1e-4)
    x = torch.from_numpy(W.random_x(c0["N"], 1, seed=2)[0]).cuda()
    with pytest.raises(H.HmatError):
        g.matvec(x, precision=1)
    with pytest.raises(H.HmatError):
        g.solve_ir(x, inner_precision=1)
    g.set_precision(1)
    st1 = g.info()["device_bytes"]
    y = g.matvec(x, precision=1)
    g.set_precision(0)
    assert g.info()["device_bytes"] < st1
    with pytest.raises(H.HmatError):
        g.matvec(x, precision=1)
    with pytest.raises(H.HmatError):
        g.set_precision(2)
    g.close()


@pytest.fixture(scope="module")
def f32():
    """FP32 builds (hmat_build_ex precision 1) of icosphere level 3: eps 1e-5
    (ACA in FP32) and 1e-7 (ACA in FP64, factors rounded), beside FP64 builds."""
    H = _H()
    V, T = W.icosphere(3)
    mesh = O.Mesh(V, T, 1.0, 0.3)
    out = {}
    for eps in (1e-5, 1e-7):
        print(f"case precision: FP32 build, icosphere level 3, eps {eps}", flush=True)
        out[eps] = (H.HMatrix(V, T, 1.0, 0.3, 2.0, 32, eps, precision=1),
                    H.HMatrix(V, T, 1.0, 0.3, 2.0, 32, eps))
    return dict(V=V, T=T, mesh=mesh, A=mesh.dense(), out=out, N=3 * len(T))


def test_fp32_build_accuracy_and_memory(f32):
    """The FP32 build's product is within the requested accuracy of the exact
    collocation product (the bound the FP64 build meets, 10 eps, plus FP32
    rounding), within that of the FP64 build's, and the handle holds about
    half the device memory."""
    x = W.random_x(f32["N"], 4, seed=21)
    bt = x @ f32["A"].T
    for eps, (g32, g64) in f32["out"].items():
        st32, st64 = g32.info(), g64.info()
        assert st32["precision"] == 1 and st64["precision"] == 0
        assert st32["aca_fp32"] == (1 if eps >= 1e-5 else 0)
        assert st32["device_bytes"] < 0.62 * st64["device_bytes"], (st32["device_bytes"], st64["device_bytes"])
        xd = torch.from_numpy(x).cuda()
        y32 = g32.matvec(xd).cpu().numpy()
        y64 = g64.matvec(xd).cpu().numpy()
        tol = 10 * max(eps, 1e-7)
        for r in range(4):
            e32 = np.linalg.norm(y32[r] - bt[r]) / np.linalg.norm(bt[r])
            e64 = np.linalg.norm(y64[r] - bt[r]) / np.linalg.norm(bt[r])
            assert e32 <= tol, (eps, r, e32, e64)
            assert np.linalg.norm(y32[r] - y64[r]) <= tol * np.linalg.norm(y64[r])
        print(f"fp32 build eps {eps}: ranks mean {st32['rank_mean']:.1f} (fp64 {st64['rank_mean']:.1f}), "
              f"bytes {st32['device_bytes']} (fp64 {st64['device_bytes']}), product error {e32:.2e} "
              f"(fp64 {e64:.2e})", flush=True)


def test_fp32_build_refinement(f32):
    """Iterative refinement on an FP32 build: the residual uses the stored FP32
    operator in FP64 arithmetic, so the relative residual 1e-8 refers to it;
    the solution differs from the FP64 build's by what the operators' eps
    allows."""
    V, T = f32["V"], f32["T"]
    b = torch.from_numpy(W.smooth_rhs(V, T, seed=5)).cuda()
    for eps, (g32, g64) in f32["out"].items():
        x, info = g32.solve_ir(b, tol=1e-8, restart=50, inner_precision=1, inner_tol=1e-6)
        assert info["status"] == 0
        rel = float(torch.linalg.norm(b - g32.matvec(x)) / torch.linalg.norm(b))
        assert rel <= 1e-8
        x64, _ = g64.solve(b, tol=1e-8, restart=50)
        d = float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64))
        assert d <= 1e3 * max(eps, 1e-7), (eps, d)
        print(f"fp32 build eps {eps}: refinement {info['refinements']} steps, "
              f"{info['iterations']} inner iterations, relres {rel:.2e}, vs FP64 solution {d:.2e}", flush=True)
        xs, _ = g32.solve(b, tol=1e-8, restart=50)  # plain GMRES on the FP32 entries
        assert float(torch.linalg.norm(b - g32.matvec(xs)) / torch.linalg.norm(b)) <= 1e-8


def test_fp32_build_refuses_fp64(f32):
    H = _H()
    g32 = f32["out"][1e-5][0]
    x = torch.from_numpy(W.random_x(f32["N"], 1, seed=2)[0]).cuda()
    with pytest.raises(H.HmatError) as ei:
        g32.set_precision(0)
    assert ei.value.status == H.HMAT_ENOTSUP
    g32.set_precision(1)  # already so
    with pytest.raises(H.HmatError):
        g32.solve_ir(x, inner_precision=0)
    y1 = g32.matvec(x, precision=1)
    y = g32.matvec(x)
    assert torch.equal(y, y1)


def test_aca_stop_factor():
    """hmat_build_ex's stop constant c: ACA stops at |u||v| <= c eps ||S||, so
    (eps, c = 0.5) is the build at eps / 2, bit for bit, and the oracle's
    ranks and pivots at eps / 2."""
    H = _H()
    V, T = W.icosphere(3)
    ga = H.HMatrix(V, T, 1.0, 0.3, 2.0, 32, 1e-4, aca_stop_factor=0.5)
    gb = H.HMatrix(V, T, 1.0, 0.3, 2.0, 32, 5e-5)
    o = O.HMatrix(O.Mesh(V, T, 1.0, 0.3), 2.0, 32, eps=5e-5)
    ob = o.blocks()
    for b in np.nonzero(ob[:, 4] == 1)[0]:
        ba, bb = ga.block(int(b)), gb.block(int(b))
        assert ba["rank"] == bb["rank"] == ob[b, 5]
        assert np.array_equal(ba["U"], bb["U"]) and np.array_equal(ba["V"], bb["V"])
        _, _, pr, pc = o.factors(int(b))
        assert np.array_equal(ba["rows"], pr) and np.array_equal(ba["cols"], pc)
    ga.close()
    gb.close()
