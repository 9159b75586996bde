"""GPU adaptive matrix-vector multiplication (Algorithm 2) against the oracle.

Both sides take the same integer decisions (which blocks are marked in each
round) from FP64 values computed in different orders, so the final ranks of
all admissible blocks and the number of rounds must agree exactly unless a
row error or a block entry lies within rounding of a threshold (not the case
for these inputs); the results agree within 1e-9, and both are within the
estimator's bound of the exact collocation product.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.amvm import amvm as oracle_amvm

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _H():
    import paper_2205_04752_amd as H
    return H


def _point_force_x(V, T, p=(5.0, 5.0, 5.0)):
    c = V[T].mean(axis=1)
    return np.concatenate([O.kelvin(ci - np.asarray(p))[:, 2] for ci in c])


CASES = {
    "ico2-leaf16-pointforce": (lambda: W.icosphere(2), 16, "point", 0.5, 1e-7),
    "ico3-pointforce": (lambda: W.icosphere(3), 32, "point", 0.5, 1e-6),
    "torus-random": (lambda: W.torus(1.0, 0.3, 36, 12), 32, "random", 0.7, 1e-5),
    # coplanar clusters: the in-plane and normal components decouple
    "plate20-pointforce": (lambda: W.plate(20), 32, "point", 0.5, 1e-6),
    "cube12-leaf16-pointforce": (lambda: W.cube_surface(12), 16, "point", 0.5, 1e-6),
}


@pytest.mark.parametrize("name", list(CASES))
def test_amvm_matches_oracle(name):
    H = _H()
    mk, leaf, kind, theta, tol = CASES[name]
    V, T = mk()
    print("case amvm:", name, flush=True)
    x = _point_force_x(V, T) if kind == "point" else W.random_x(3 * len(T), 1, seed=6)[0]
    y, info, ranks = H.amvm(V, T, torch.from_numpy(x).cuda(), 1.0, 0.3, 2.0, leaf, theta, tol,
                            max_rounds=1000, kmax=96)
    mesh = O.Mesh(V, T, 1.0, 0.3)
    yo, hist, hm = oracle_amvm(mesh, x, theta=theta, tol=tol, leaf=leaf, kcap=96, max_iter=1001)
    ob = hm.blocks()
    final = hist[-1]["ranks"]
    far = ob[:, 4] == 1
    assert np.array_equal(ranks[far], final[far]), np.nonzero(ranks[far] != final[far])
    assert info["rounds"] == len(hist) - 1
    yg = y.cpu().numpy()
    assert np.linalg.norm(yg - yo) <= 1e-9 * np.linalg.norm(yo)
    assert abs(info["gamma"] - hist[-1]["gamma"]) <= 1e-6 * max(hist[-1]["gamma"], 1e-300)
    # the result is within a few tolerances of the exact product
    bt = mesh.brute_matvec(x[None, :])[0]
    assert np.linalg.norm(yg - bt) <= 20 * tol * np.linalg.norm(bt)
    print(name, info, flush=True)


def test_amvm_zero_vector():
    H = _H()
    V, T = W.icosphere(2)
    y, info, ranks = H.amvm(V, T, torch.zeros(3 * len(T), dtype=torch.float64, device="cuda"),
                            leaf=16)
    assert float(torch.abs(y).max()) == 0.0 and info["rounds"] == 0
    assert np.all(ranks[ranks >= 0] == 0)


def test_amvm_without_admissible_blocks():
    """A mesh whose partition has no admissible block (one leaf cluster): the
    adaptive product is the dense product after zero rounds."""
    H = _H()
    V, T = W.icosahedron()
    x = W.random_x(3 * len(T), 1, seed=2)[0]
    y, info, ranks = H.amvm(V, T, torch.from_numpy(x).cuda(), leaf=32)
    assert info["rounds"] == 0 and info["gamma"] == 0.0 and np.all(ranks == -1)
    bt = O.Mesh(V, T, 1.0, 0.3).brute_matvec(x[None, :])[0]
    assert np.linalg.norm(y.cpu().numpy() - bt) <= 1e-13 * np.linalg.norm(bt)
