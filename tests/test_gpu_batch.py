"""GPU parity of batched builds (several bodies in one handle) against the
FP64 oracle, body by body, through the C ABI.

A batch is the block-diagonal operator of its bodies: every body has its own
tree, partition, Kelvin constants (E, nu) and ACA accuracy. Checked:
  * DOF offsets and block counts;
  * every admissible block of every body: the oracle's rank and pivots, and
    factors within 1e-10 (relative Frobenius norm of U V^T);
  * dense blocks within 1e-13 of the oracle's;
  * the 8-vector product equals each body's oracle product within 1e-10 and
    the single-body GPU builds within 1e-13 (same blocks, other chunking);
  * a build that runs ACA in many small groups gives the same bits;
  * GMRES on the whole batch reaches the explicit relative residual 1e-8.
"""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _H():
    import paper_2205_04752_amd as H
    return H


def _bodies():
    V0, T0 = W.icosphere(2)
    V1, T1 = W.torus(1.0, 0.3, 30, 12)
    V2, T2 = W.ellipsoid(7, (1.0, 0.6, 0.4))
    V3, T3 = W.icosahedron()
    V4 = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    T4 = np.array([[0, 1, 2]], dtype=np.int32)
    V5, T5 = W.box_surface(3.0, 1.0, 1.0, 12, 4, 4)
    return [dict(vertices=V0, triangles=T0, E=1.0, nu=0.3, eps=1e-6),
            dict(vertices=V1, triangles=T1, E=2.5, nu=0.25, eps=1e-5),
            dict(vertices=V2, triangles=T2, E=0.7, nu=0.42, eps=1e-4),
            dict(vertices=V3, triangles=T3, E=1.0, nu=0.2, eps=1e-6),
            dict(vertices=V4, triangles=T4, E=1.0, nu=0.3, eps=1e-6),
            dict(vertices=V5, triangles=T5, E=1.3, nu=0.35, eps=1e-7)]


@pytest.fixture(scope="module")
def batch():
    H = _H()
    bodies = _bodies()
    print("case batch: 6 bodies (icosphere L2, torus, ellipsoid, icosahedron, one triangle, box)",
          flush=True)
    g = H.HMatrix.batch(bodies, eta=2.0, leaf=32)
    orc = []
    for b in bodies:
        mesh = O.Mesh(b["vertices"], b["triangles"], b["E"], b["nu"])
        orc.append((mesh, O.HMatrix(mesh, 2.0, 32, eps=b["eps"])))
    return dict(bodies=bodies, g=g, orc=orc)


def test_offsets_and_counts(batch):
    g, bodies = batch["g"], batch["bodies"]
    off = g.bodies()
    nts = [len(b["triangles"]) for b in bodies]
    assert list(off) == list(np.concatenate([[0], np.cumsum(3 * np.array(nts))]))
    st = g.info()
    obs = [o.blocks() for _, o in batch["orc"]]
    assert st["n_blocks"] == sum(len(ob) for ob in obs)
    assert st["n_far"] == sum(int(ob[:, 4].sum()) for ob in obs)
    assert st["c_sp"] == max(o.csp() for _, o in batch["orc"])


def test_blocks_match_oracle(batch):
    g = batch["g"]
    base, tri = 0, 0
    worst_lr, worst_d = 0.0, 0.0
    for (mesh, o), body in zip(batch["orc"], batch["bodies"]):
        ob = o.blocks()
        for b in range(len(ob)):
            gb = g.block(base + b)
            assert (gb["row_off"] - tri, gb["row_len"], gb["col_off"] - tri, gb["col_len"],
                    gb["far"]) == tuple(ob[b, :5])
            if ob[b, 4]:
                assert gb["rank"] == ob[b, 5], (base + b, gb["rank"], ob[b, 5])
                Uo, Vo, pr, pc = o.factors(b)
                assert np.array_equal(gb["rows"], pr) and np.array_equal(gb["cols"], pc)
                Ao = Uo @ Vo.T
                if np.linalg.norm(Ao) > 0:
                    worst_lr = max(worst_lr, np.linalg.norm(gb["U"] @ gb["V"].T - Ao) / np.linalg.norm(Ao))
            else:
                Do = o.dense_block(b)
                worst_d = max(worst_d, np.abs(gb["D"] - Do).max() / np.abs(Do).max())
        base += len(ob)
        tri += len(body["triangles"])
    assert worst_lr <= 1e-10, worst_lr
    assert worst_d <= 1e-13, worst_d


def test_product_8_rhs(batch):
    H = _H()
    g, bodies = batch["g"], batch["bodies"]
    off = g.bodies()
    x = W.random_x(g.n_dof, 8, seed=3)
    y = g.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    for i, ((mesh, o), body) in enumerate(zip(batch["orc"], bodies)):
        sl = slice(off[i], off[i + 1])
        yo = o.matvec(x[:, sl])
        rel = np.linalg.norm(y[:, sl] - yo, axis=1) / np.linalg.norm(yo, axis=1)
        assert rel.max() <= 1e-10, (i, rel)
        single = H.HMatrix(body["vertices"], body["triangles"], body["E"], body["nu"], 2.0, 32,
                           body["eps"])
        ys = single.matvec(torch.from_numpy(np.ascontiguousarray(x[:, sl])).cuda()).cpu().numpy()
        rel = np.linalg.norm(y[:, sl] - ys, axis=1) / np.linalg.norm(ys, axis=1)
        assert rel.max() <= 1e-13, (i, rel)
        single.close()
    # one vector at a time (the single-vector chunk list) gives the same vectors
    for r in (0, 5):
        y1 = g.matvec(torch.from_numpy(x[r]).cuda()).cpu().numpy()
        assert np.linalg.norm(y1 - y[r]) <= 1e-13 * np.linalg.norm(y[r])


def test_grouped_aca_same_bits(batch, monkeypatch):
    H = _H()
    monkeypatch.setenv("HMAT_ACA_BUDGET_MB", "1")  # forces many ACA groups
    g2 = H.HMatrix.batch(batch["bodies"], eta=2.0, leaf=32)
    x = torch.from_numpy(W.random_x(batch["g"].n_dof, 3, seed=5)).cuda()
    assert torch.equal(batch["g"].matvec(x), g2.matvec(x))
    assert g2.info()["rank_mean"] == batch["g"].info()["rank_mean"]
    g2.close()


def test_batch_gmres(batch):
    g = batch["g"]
    bs = [W.smooth_rhs(b["vertices"], b["triangles"], seed=7) for b in batch["bodies"]]
    b = torch.from_numpy(np.concatenate(bs)).cuda()
    x, info = g.solve(b, tol=1e-8, restart=50)
    assert info["status"] == 0
    rel = float(torch.linalg.norm(b - g.matvec(x)) / torch.linalg.norm(b))
    assert rel <= 1e-8
    print("batch gmres:", info, flush=True)
