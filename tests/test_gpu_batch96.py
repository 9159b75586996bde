"""GPU parity at the full batched size (96 ellipsoids and tori, 1.1 M
triangles, eps 1e-5), in the configuration the batched benchmark times:
one handle for all bodies, 8 vectors per body.

Sampled bodies (the smallest, a median one and the largest) are rebuilt by
the oracle; their slices of the batched 8-vector product equal the oracle's
H-matrix products within 1e-10, and their ranks equal the oracle's block by
block. The single-vector product of the whole batch equals the 8-vector
product's first vector.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_batch96_sampled_bodies():
    import gc

    import paper_2205_04752_amd as H
    gc.collect()  # handles of earlier tests release their device memory
    torch.cuda.empty_cache()
    wl = W.workload_c2()
    bodies = wl["bodies"]
    print("case batch96: building 96 bodies", flush=True)
    g = H.HMatrix.batch(bodies, eta=wl["eta"], leaf=wl["leaf"])
    off = g.bodies()
    X = W.random_x(g.n_dof, wl["nrhs"], seed=2)
    Y = g.matvec(torch.from_numpy(X).cuda()).cpu().numpy()
    y1 = g.matvec(torch.from_numpy(X[0]).cuda()).cpu().numpy()
    assert np.linalg.norm(y1 - Y[0]) <= 1e-12 * np.linalg.norm(Y[0])
    nts = np.array([len(b["triangles"]) for b in bodies])
    pick = [int(np.argmin(nts)), int(np.argsort(nts)[len(nts) // 2]), int(np.argmax(nts))]
    st = g.info()
    base = 0
    block_base = []
    for b in bodies:  # block offsets of each body in the batch's canonical order
        block_base.append(base)
        order, blocks = H.plan(b["vertices"], b["triangles"], wl["eta"], wl["leaf"])
        base += len(blocks)
    assert base == st["n_blocks"]
    for i in pick:
        b = bodies[i]
        print(f"case batch96: oracle body {i} ({nts[i]} triangles)", flush=True)
        mesh = O.Mesh(b["vertices"], b["triangles"], b["E"], b["nu"])
        o = O.HMatrix(mesh, wl["eta"], wl["leaf"], eps=b["eps"])
        sl = slice(off[i], off[i + 1])
        yo = o.matvec(np.ascontiguousarray(X[:, sl]))
        rel = np.linalg.norm(Y[:, sl] - yo, axis=1) / np.linalg.norm(yo, axis=1)
        assert rel.max() <= 1e-10, (i, rel)
        ob = o.blocks()
        info = np.zeros(8, dtype=np.int32)
        bad = 0
        for k in np.nonzero(ob[:, 4] == 1)[0]:
            assert H.lib().hmat_block(g._h, int(block_base[i] + k), info.ctypes.data, None, None,
                                      None, None) == 0
            bad += int(info[5] != ob[k, 5])
        assert bad == 0, (i, bad)
    g.close()
