"""PIN-T1: the oracle's cluster tree and block partition (Sec. 2.1).

Checked against the definitions, recomputed here from the raw mesh:
  * tree: sons split their parent; the split is the midpoint of the longest
    axis of the centroid box (ties to the lower axis), son 0 holding
    coordinates <= mid, mesh order kept within each son; leaves hold at most
    `leaf` triangles; `order` is the leaf sequence;
  * partition: exact cover of I x I without overlap; every low-rank block
    satisfies the admissibility condition (eq. adm, eta form, dist > 0) on
    vertex boxes of the supports; every dense block touches a leaf cluster and
    is not admissible; every block's parent pair was neither admissible nor had
    a leaf (leaves of the block-cluster tree); the partition is symmetric.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _vertex_box(V, T, tris):
    P = V[T[tris]].reshape(-1, 3)
    return P.min(axis=0), P.max(axis=0)


def _adm(V, T, order, a, b, eta):
    lo1, hi1 = _vertex_box(V, T, order[a[0]:a[0] + a[1]])
    lo2, hi2 = _vertex_box(V, T, order[b[0]:b[0] + b[1]])
    gap = np.maximum(0.0, np.maximum(lo2 - hi1, lo1 - hi2))
    dist = np.sqrt(np.sum(gap * gap))
    d1 = np.sqrt(np.sum((hi1 - lo1) ** 2))
    d2 = np.sqrt(np.sum((hi2 - lo2) ** 2))
    return dist > 0 and min(d1, d2) <= eta * dist


MESHES = {
    "ico3": lambda: W.icosphere(3),
    "ico4": lambda: W.icosphere(4),
    "torus": lambda: W.torus(1.0, 0.3, 48, 16),
    "box": lambda: W.box_surface(4.0, 1.0, 1.0, 16, 4, 4),
}


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("leaf", [32, 7])
def test_tree_definition(name, leaf):
    V, T = MESHES[name]()
    mesh = O.Mesh(V, T)
    h = O.HMatrix(mesh, 2.0, leaf)
    cl = h.clusters()
    order = h.order
    assert sorted(order.tolist()) == list(range(len(T)))
    cen = ((V[T[:, 0]] + V[T[:, 1]]) + V[T[:, 2]]) / 3.0
    root = cl[0]
    assert root["off"] == 0 and root["len"] == len(T)
    leaves = []
    for c in cl:
        tris = order[c["off"]:c["off"] + c["len"]]
        lo, hi = _vertex_box(V, T, tris)
        assert np.array_equal(lo, c["lo"]) and np.array_equal(hi, c["hi"])
        if c["son0"] < 0:
            assert c["len"] <= leaf or np.ptp(cen[tris], axis=0).max() == 0
            leaves.append(c)
            continue
        s0, s1 = cl[c["son0"]], cl[c["son1"]]
        assert s0["off"] == c["off"] and s0["len"] + s1["len"] == c["len"]
        assert s1["off"] == c["off"] + s0["len"]
        assert s0["len"] > 0 and s1["len"] > 0
        ext = cen[tris].max(axis=0) - cen[tris].min(axis=0)
        ax = int(np.argmax(ext))  # first maximum = lower axis on ties
        mid = 0.5 * (cen[tris, ax].min() + cen[tris, ax].max())
        # sons hold exactly the <= mid / > mid sets, each in the parent's order
        par = tris.tolist()  # parent's own order is its sons' concatenation...
        left = [t for t in par if cen[t, ax] <= mid]
        right = [t for t in par if not cen[t, ax] <= mid]
        assert order[s0["off"]:s0["off"] + s0["len"]].tolist() == left
        assert order[s1["off"]:s1["off"] + s1["len"]].tolist() == right
    # ...and at the root the order before splitting is mesh order: the leaf
    # sequence is then a stable refinement of 0..nt-1 split by split.
    pos = np.concatenate([order[c["off"]:c["off"] + c["len"]] for c in sorted(leaves, key=lambda c: c["off"])])
    assert np.array_equal(pos, order)


def _stable_check(V, T, order, cl):
    """Re-run the splits from mesh order to confirm stability of the whole tree."""
    cen = ((V[T[:, 0]] + V[T[:, 1]]) + V[T[:, 2]]) / 3.0

    def rec(c, tris):
        assert sorted(order[c["off"]:c["off"] + c["len"]].tolist()) == sorted(tris)
        if c["son0"] < 0:
            assert order[c["off"]:c["off"] + c["len"]].tolist() == tris
            return
        t = np.array(tris)
        ext = cen[t].max(axis=0) - cen[t].min(axis=0)
        ax = int(np.argmax(ext))
        mid = 0.5 * (cen[t, ax].min() + cen[t, ax].max())
        rec(cl[c["son0"]], [x for x in tris if cen[x, ax] <= mid])
        rec(cl[c["son1"]], [x for x in tris if not cen[x, ax] <= mid])

    rec(cl[0], list(range(len(T))))


@pytest.mark.parametrize("name", list(MESHES))
def test_tree_stable_from_mesh_order(name):
    V, T = MESHES[name]()
    h = O.HMatrix(O.Mesh(V, T), 2.0, 32)
    _stable_check(V, T, h.order, h.clusters())


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("eta", [2.0, 0.8])
def test_partition_definition(name, eta):
    V, T = MESHES[name]()
    nt = len(T)
    h = O.HMatrix(O.Mesh(V, T), eta, 32)
    B = h.blocks()
    cl = h.clusters()
    order = h.order
    parent = {}
    for i, c in enumerate(cl):
        if c["son0"] >= 0:
            parent[c["son0"]] = i
            parent[c["son1"]] = i
    # canonical order: sorted by (row_off, col_off)
    keys = [(b[0], b[2]) for b in B]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    cover = np.zeros((nt, nt), dtype=np.int8)
    for b in B:
        cover[b[0]:b[0] + b[1], b[2]:b[2] + b[3]] += 1
    assert cover.min() == 1 and cover.max() == 1
    assert int(np.sum(B[:, 1].astype(np.int64) * B[:, 3])) == nt * nt
    index = {(b[0], b[1], b[2], b[3]): b[4] for b in B}
    for b in B:
        r, s = (b[0], b[1]), (b[2], b[3])
        t_id, s_id = b[7], b[8]
        isleaf = cl[t_id]["son0"] < 0 or cl[s_id]["son0"] < 0
        adm = _adm(V, T, order, r, s, eta)
        if b[4] == 1:
            assert adm
        else:
            assert not adm and isleaf
        # symmetric partition, same type
        assert index[(b[2], b[3], b[0], b[1])] == b[4]
        # leaves of the block-cluster tree: the parent pair was refined
        if t_id != 0 or s_id != 0:
            pt, ps = parent[t_id], parent[s_id]
            assert cl[pt]["level"] == cl[t_id]["level"] - 1
            P, S = cl[pt], cl[ps]
            assert not _adm(V, T, order, (P["off"], P["len"]), (S["off"], S["len"]), eta)
            assert P["son0"] >= 0 and S["son0"] >= 0
    # c_sp: blocks per row/column cluster
    csp = max(np.bincount(B[:, 7]).max(), np.bincount(B[:, 8]).max())
    assert h.csp() == csp
