"""Pins of the oracle's H-matrix and its product (Sec. 2, Sec. 2.2) and of its GMRES.

PIN-H1  on small icospheres (dense A affordable): ||A_H x - A x|| <= 3 eps
        ||A_far||_F ||x||, from the blockwise Frobenius target of ACA and
        Cauchy-Schwarz. The blockwise ratio ||A_b - U_b V_b^T||_F/||A_b||_F is
        a heuristic target of partial-pivoting ACA, not a guarantee (its stop
        test only sees the newest cross): its median must be <= 2 eps and its
        95th percentile <= 10 eps; isolated blocks may exceed it.
PIN-H2  with eta -> 0 nothing is admissible: A_H x equals the dense product to
        1e-14, and every dense block equals its sub-block of A (permutation).
PIN-B1  the matrix-free brute-force product equals the dense product.
PIN-G1  GMRES(m): on small dense systems the solution matches LAPACK's
        (numpy.linalg.solve) within cond * 1e-8 and the explicit residual
        is <= 1e-8; an iteration cap yields status 4 with x and relres written.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


@pytest.fixture(scope="module", params=[2, 3])
def small(request):
    V, T = W.icosphere(request.param)
    mesh = O.Mesh(V, T, 1.0, 0.3)
    A = mesh.dense()
    return V, T, mesh, A


def _perm_dofs(order):
    return (3 * order[:, None] + np.arange(3)[None, :]).ravel()


@pytest.mark.parametrize("eps", [1e-3, 1e-6])
@pytest.mark.parametrize("leaf", [8, 32])
def test_hmatvec_error_bound(small, eps, leaf):
    V, T, mesh, A = small
    h = O.HMatrix(mesh, 2.0, leaf, eps=eps)
    B = h.blocks()
    assert B[:, 4].sum() > 0
    order = h.order
    pd = _perm_dofs(order)
    Ap = A[np.ix_(pd, pd)]
    far_f2 = 0.0
    ratios = []
    for b, bl in enumerate(B):
        r0, r1 = 3 * bl[0], 3 * (bl[0] + bl[1])
        c0, c1 = 3 * bl[2], 3 * (bl[2] + bl[3])
        sub = Ap[r0:r1, c0:c1]
        if bl[4] == 1:
            U, Vf, _, _ = h.factors(b)
            ratios.append(np.linalg.norm(sub - U @ Vf.T) / np.linalg.norm(sub))
            far_f2 += np.linalg.norm(sub) ** 2
        else:
            D = h.dense_block(b)
            assert np.array_equal(D, sub)
    ratios = np.array(ratios) / eps
    assert np.median(ratios) <= 2.0 and np.percentile(ratios, 95) <= 10.0, ratios
    x = W.random_x(mesh.N, 3, seed=0)
    y = h.matvec(x)
    yd = x @ A.T
    rnd = 1e-14 * np.linalg.norm(A)  # rounding floor of the two products
    for r in range(3):
        bound = (3 * eps * np.sqrt(far_f2) + rnd) * np.linalg.norm(x[r])
        assert np.linalg.norm(y[r] - yd[r]) <= bound


def test_everything_dense_equals_gemv(small):
    V, T, mesh, A = small
    h = O.HMatrix(mesh, 1e-12, 8, eps=1e-6)
    assert h.blocks()[:, 4].sum() == 0
    x = W.random_x(mesh.N, 2, seed=1)
    y = h.matvec(x)
    yd = x @ A.T
    assert np.abs(y - yd).max() <= 1e-14 * np.abs(yd).max() * 10


def test_brute_equals_dense(small):
    V, T, mesh, A = small
    x = W.random_x(mesh.N, 2, seed=2)
    y = mesh.brute_matvec(x)
    yd = x @ A.T
    assert np.abs(y - yd).max() <= 1e-13 * np.abs(yd).max()
    rows = np.array([0, 5, len(T) - 1], dtype=np.int32)
    ys = mesh.brute_matvec(x, rows)
    sel = _perm_dofs(rows)
    assert np.array_equal(ys, y[:, sel])


def test_storage_counts(small):
    V, T, mesh, A = small
    h = O.HMatrix(mesh, 2.0, 8, eps=1e-4)
    B = h.blocks()
    k = B[:, 5].astype(np.int64)
    m, n = 3 * B[:, 1].astype(np.int64), 3 * B[:, 3].astype(np.int64)
    expect = int(np.sum(np.where(B[:, 4] == 1, k * (m + n), m * n)))
    assert h.stored() == expect


@pytest.mark.parametrize("level", [1, 2])
def test_gmres_dense_matches_lapack(level):
    V, T = W.icosphere(level)
    mesh = O.Mesh(V, T, 1.0, 0.3)
    A = mesh.dense()
    b = W.smooth_rhs(V, T, seed=1)
    x, info = O.dense_gmres(A, b, tol=1e-8, restart=50)
    assert info["status"] == 0
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)
    assert abs(info["relres"] - np.linalg.norm(b - A @ x) / np.linalg.norm(b)) < 1e-12
    xs = np.linalg.solve(A, b)
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(x - xs) <= kappa * 1e-8 * np.linalg.norm(xs)
    # restarted with a short cycle still converges
    x5, info5 = O.dense_gmres(A, b, tol=1e-8, restart=5, maxit=20000)
    assert info5["status"] == 0 and info5["iters"] >= info["iters"]
    # iteration cap: no convergence, but x and relres are written
    xc, infoc = O.dense_gmres(A, b, tol=1e-12, restart=50, maxit=3)
    assert infoc["status"] == 4 and infoc["iters"] == 3
    assert abs(infoc["relres"] - np.linalg.norm(b - A @ xc) / np.linalg.norm(b)) < 1e-12
    assert infoc["relres"] < 1.0


def test_gmres_on_hmatrix():
    V, T = W.icosphere(3)
    mesh = O.Mesh(V, T, 1.0, 0.3)
    h = O.HMatrix(mesh, 2.0, 32, eps=1e-6)
    b = W.smooth_rhs(V, T, seed=1)
    x, info = h.gmres(b, tol=1e-8, restart=50)
    assert info["status"] == 0
    r = b - h.matvec(x)[0]
    assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(b)
