"""Pins of the oracle's adaptive matrix-vector multiplication (Algorithm 2).

Checked against quantities recomputed here from the oracle's ACA crosses as
dense block matrices (no code shared with oracle/amvm.py's row bookkeeping):
  * ACA run for a fixed number of steps resumes exactly (prefixes of a longer
    run), its crosses interpolate their blocks, its rows cycle through the
    three displacement components, and on a matrix whose components decouple
    (coplanar clusters) it reaches every part in its first steps and
    recovers the matrix exactly;
  * gamma_k = ||b_k - b^_k|| with A_k, A^_k assembled densely from the ranks
    recorded at every round;
  * the marked set meets the Doerfler condition gamma_k(P_k) <= (1-theta)
    gamma_k (the Remark after Algorithm 2), every marked block has a row
    entry above the threshold, and only marked blocks grow, by two steps;
  * x = 0 needs no ACA step; blocks whose columns meet no nonzero of x are
    never refined;
  * the result converges to the exact collocation product, and the
    estimator stays within a factor 2 of the true error (the paper's
    efficiency/reliability figure) once the saturation regime is reached.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.amvm import amvm

pytestmark = pytest.mark.filterwarnings("ignore")


def _point_force_x(V, T, p=(5.0, 5.0, 5.0)):
    """Smooth data: x_i = S(c_i - p) e_3 at the centroids (the paper's example)."""
    c = V[T].mean(axis=1)
    return np.concatenate([O.kelvin(ci - np.asarray(p))[:, 2] for ci in c])


@pytest.fixture(scope="module")
def small():
    V, T = W.icosphere(2)
    mesh = O.Mesh(V, T, 1.0, 0.3)
    return V, T, mesh


def _dense_blocks(hm):
    ob = hm.blocks()
    far = {}
    for b in np.nonzero(ob[:, 4] == 1)[0]:
        U, Vv, _, _ = hm.factors(int(b))
        far[int(b)] = (U, Vv)
    return ob, far


def _assemble(hm, ob, far, ranks, extra=0):
    """Dense cluster-order matrix with admissible block b at rank ranks[b] + extra."""
    order = hm.order
    N = 3 * len(order)
    A = np.zeros((N, N))
    for b in range(len(ob)):
        rs = slice(3 * ob[b, 0], 3 * (ob[b, 0] + ob[b, 1]))
        cs = slice(3 * ob[b, 2], 3 * (ob[b, 2] + ob[b, 3]))
        if ob[b, 4]:
            U, Vv = far[b]
            r = min(int(ranks[b]) + extra, U.shape[1])
            A[rs, cs] = U[:, :r] @ Vv[:, :r].T
        else:
            A[rs, cs] = hm.dense_block(b)
    perm = (3 * order[:, None] + np.arange(3)).ravel()
    return A, perm


def test_step_limited_aca_resumes(small):
    """A run paused after r steps continues as the uninterrupted run: the
    crosses of fill_steps(8) are the first 8 of fill_steps(96), bit for bit
    (ACA is sequential; the adaptive multiplication resumes it every round)."""
    V, T, mesh = small
    a = O.HMatrix(mesh, 2.0, 16)
    a.fill_steps(96)
    e = O.HMatrix(mesh, 2.0, 16)
    e.fill_steps(8)
    ob = e.blocks()
    for b in np.nonzero(ob[:, 4] == 1)[0]:
        Ue, Ve, pre, pce = e.factors(int(b))
        Ua, Va, pra, pca = a.factors(int(b))
        k = Ue.shape[1]
        assert k == min(8, Ua.shape[1])
        assert np.array_equal(pre, pra[:k]) and np.array_equal(pce, pca[:k])
        assert np.array_equal(Ue, Ua[:, :k]) and np.array_equal(Ve, Va[:, :k])


def test_step_limited_cross_property(small):
    """Every step-limited cross interpolates its block (Sec. 2.2: the remainder
    vanishes on the pivot rows and columns), with the dense block recomputed
    here entry by entry; on these curved blocks no remainder row vanishes, so
    the pivot rows visit the classes 0, 1, 2, 0, 1, 2, ..."""
    V, T, mesh = small
    a = O.HMatrix(mesh, 2.0, 16)
    a.fill_steps(24)
    ob = a.blocks()
    order = a.order
    A = mesh.dense()
    for b in np.nonzero(ob[:, 4] == 1)[0]:
        U, Vv, pr, pc = a.factors(int(b))
        rt = (3 * order[ob[b, 0]:ob[b, 0] + ob[b, 1], None] + np.arange(3)).ravel()
        cs = (3 * order[ob[b, 2]:ob[b, 2] + ob[b, 3], None] + np.arange(3)).ravel()
        B = A[np.ix_(rt, cs)]
        R = B - U @ Vv.T
        assert np.abs(R[pr, :]).max() <= 1e-13 * np.abs(B).max()
        assert np.abs(R[:, pc]).max() <= 1e-13 * np.abs(B).max()
        assert np.array_equal(pr % 3, np.arange(len(pr)) % 3), (b, pr % 3)


def _decoupled(p, r_in, r_n, seed):
    """3p x 3q matrix whose rows and columns of classes 0, 1 (in-plane) and of
    class 2 (normal) do not couple, with exact ranks r_in and r_n, the way
    the Kelvin tensor decouples on coplanar clusters."""
    rng = np.random.default_rng(seed)
    q = p + 3
    m, n = 3 * p, 3 * q
    rin = np.nonzero(np.arange(m) % 3 != 2)[0]
    cin = np.nonzero(np.arange(n) % 3 != 2)[0]
    rn = np.nonzero(np.arange(m) % 3 == 2)[0]
    cn = np.nonzero(np.arange(n) % 3 == 2)[0]
    B = np.zeros((m, n))
    B[np.ix_(rin, cin)] = rng.standard_normal((len(rin), r_in)) @ rng.standard_normal((r_in, len(cin)))
    if r_n:
        B[np.ix_(rn, cn)] = 10.0 * rng.standard_normal((len(rn), r_n)) @ rng.standard_normal((r_n, len(cn)))
    return B, rn


@pytest.mark.parametrize("r_in,r_n", [(4, 3), (6, 1), (5, 0)])
def test_step_limited_decoupled_classes(r_in, r_n):
    """On a matrix whose in-plane and normal classes decouple, the look-ahead's
    ACA reaches the normal part within its first three steps (the third row is
    the lowest row of class 2, since no cross has entries there yet) and
    recovers the matrix exactly in r_in + r_n crosses. Partial pivoting on
    |u_k| alone would take r_in in-plane steps first: its crosses never have
    entries in class-2 rows."""
    B, rn = _decoupled(20, r_in, r_n, seed=r_in + 7 * r_n)
    out = O.aca_dense_steps(B, kcap=60)
    U, Vv, pr = out["U"], out["V"], out["rows"]
    if r_n:
        assert pr[2] == 2
        assert np.abs(U[:, 2][np.arange(B.shape[0]) % 3 != 2]).max() == 0.0
        assert np.abs(U[rn, 2]).max() > 0.0
    assert U.shape[1] == r_in + r_n, (U.shape[1], pr)
    assert np.linalg.norm(B - U @ Vv.T) <= 1e-12 * np.linalg.norm(B)


def test_rounds_against_dense_recomputation(small):
    V, T, mesh = small
    x = _point_force_x(V, T)
    theta = 0.5
    y, hist, hm = amvm(mesh, x, theta=theta, tol=1e-7, leaf=16, kcap=96)
    ob, far = _dense_blocks(hm)
    assert len(hist) > 3
    for k, rec in enumerate(hist):
        Ak, perm = _assemble(hm, ob, far, rec["ranks"])
        Ah, _ = _assemble(hm, ob, far, rec["ranks"], extra=2)
        xp = x[perm]
        gk = np.linalg.norm((Ak - Ah) @ xp)
        assert abs(gk - rec["gamma"]) <= 1e-12 * max(gk, 1e-300), (k, gk, rec["gamma"])
        if not rec["marked"]:
            continue
        # Doerfler condition, recomputed from the dense difference
        D = Ah - Ak
        keep = np.ones(len(ob), dtype=bool)
        keep[rec["marked"]] = False
        rest = np.zeros(D.shape[0])
        for b in np.nonzero((ob[:, 4] == 1) & keep)[0]:
            rs = slice(3 * ob[b, 0], 3 * (ob[b, 0] + ob[b, 1]))
            cs = slice(3 * ob[b, 2], 3 * (ob[b, 2] + ob[b, 3]))
            rest[rs] += D[rs, cs] @ xp[cs]
        assert np.linalg.norm(rest) <= (1 - theta) * gk * (1 + 1e-10)
        # the threshold of step 3 b (iii), and every marked block reaches it
        N = D.shape[0]
        assert abs(rec["tau"] - (1 - theta) * gk / np.sqrt(hm.csp() * N * N)) <= 1e-12 * rec["tau"]
        for b in rec["marked"]:
            rs = slice(3 * ob[b, 0], 3 * (ob[b, 0] + ob[b, 1]))
            cs = slice(3 * ob[b, 2], 3 * (ob[b, 2] + ob[b, 3]))
            assert np.abs(D[rs, cs] @ xp[cs]).max() >= rec["tau"] * (1 - 1e-12)
        # only marked blocks grow, by two steps (or to their last cross)
        if k + 1 < len(hist):
            nxt = hist[k + 1]["ranks"]
            for b in np.nonzero(ob[:, 4] == 1)[0]:
                if b in rec["marked"]:
                    assert nxt[b] == min(rec["ranks"][b] + 2, far[b][0].shape[1])
                else:
                    assert nxt[b] == rec["ranks"][b]


def test_zero_and_sparse_data(small):
    V, T, mesh = small
    y, hist, hm = amvm(mesh, np.zeros(3 * len(T)), leaf=16)
    assert np.all(y == 0.0) and len(hist) == 1 and hist[0]["gamma"] == 0.0
    # x nonzero on the triangles of one leaf cluster only
    cl = [c for c in hm.clusters() if c["son0"] < 0][3]
    tri = hm.order[cl["off"]:cl["off"] + cl["len"]]
    x = np.zeros(3 * len(T))
    x[(3 * tri[:, None] + np.arange(3)).ravel()] = 1.0
    y, hist, hm = amvm(mesh, x, tol=1e-8, leaf=16, hm=hm)
    ob = hm.blocks()
    final = hist[-1]["ranks"]
    for b in np.nonzero(ob[:, 4] == 1)[0]:
        c0, c1 = ob[b, 2], ob[b, 2] + ob[b, 3]
        if c1 <= cl["off"] or c0 >= cl["off"] + cl["len"]:
            assert final[b] == 0, b


def test_convergence_and_estimator_quality(small):
    V, T, mesh = small
    x = _point_force_x(V, T)
    A = mesh.dense()
    bt = A @ x
    y, hist, hm = amvm(mesh, x, theta=0.5, tol=1e-8, leaf=16, kcap=96)
    assert np.linalg.norm(y - bt) <= 1e-6 * np.linalg.norm(bt)
    ob, far = _dense_blocks(hm)
    ratios = []
    for rec in hist:
        Ak, perm = _assemble(hm, ob, far, rec["ranks"])
        bk = np.zeros_like(x)
        bk[perm] = Ak @ x[perm]
        err = np.linalg.norm(bk - bt)
        if err > 1e-13 * np.linalg.norm(bt):
            ratios.append(rec["gamma"] / err)
    ratios = np.array(ratios[2:])  # after the first rounds (saturation regime)
    assert np.mean((ratios >= 0.5) & (ratios <= 2.0)) >= 0.8, ratios


def test_estimator_within_factor_two_once_accurate(small):
    """The paper's efficiency figure (Sec. 6.1) shows gamma_k / ||b - b_k|| inside
    [1/2, 2] at every point of its range (errors from about 3e-4 down); here every
    round whose error against the exact collocation product is below 1e-3
    relative must lie in that band, and there must be many such rounds."""
    V, T, mesh = small
    x = _point_force_x(V, T)
    bt = mesh.dense() @ x
    y, hist, hm = amvm(mesh, x, theta=0.5, tol=1e-8, leaf=16, kcap=96)
    ob, far = _dense_blocks(hm)
    seen = 0
    for k, rec in enumerate(hist):
        Ak, perm = _assemble(hm, ob, far, rec["ranks"])
        bk = np.zeros_like(x)
        bk[perm] = Ak @ x[perm]
        err = np.linalg.norm(bk - bt)
        if err <= 1e-3 * np.linalg.norm(bt):
            seen += 1
            assert 0.5 <= rec["gamma"] / err <= 2.0, (k, rec["gamma"], err)
    assert seen >= 10, seen


def test_marking_stops_at_first_row(small):
    """Algorithm 2, step 3: rows are taken in decreasing |(b^_k - b_k)_i|; along
    them every block with a row entry at or above the threshold joins P_k, and
    marking ends at the first row after which gamma_k(P_k) <= (1 - theta) gamma_k
    (the minimal-cardinality set of the algorithm). Everything is recomputed here
    from dense block products: the row errors, each block's contribution, the
    Doerfler test after every row group, and completeness above the last row."""
    V, T, mesh = small
    x = _point_force_x(V, T)
    theta = 0.5
    y, hist, hm = amvm(mesh, x, theta=theta, tol=1e-7, leaf=16, kcap=96)
    ob, far = _dense_blocks(hm)
    fars = np.nonzero(ob[:, 4] == 1)[0]
    checked = 0
    for k, rec in enumerate(hist):
        if not rec["marked"]:
            continue
        Ak, perm = _assemble(hm, ob, far, rec["ranks"])
        Ah, _ = _assemble(hm, ob, far, rec["ranks"], extra=2)
        xp = x[perm]
        D = Ah - Ak
        e = D @ xp
        gk = np.linalg.norm(e)
        contrib = {}
        for b in fars:
            rs = slice(3 * ob[b, 0], 3 * (ob[b, 0] + ob[b, 1]))
            cs = slice(3 * ob[b, 2], 3 * (ob[b, 2] + ob[b, 3]))
            contrib[int(b)] = (rs, D[rs, cs] @ xp[cs])
        rows = rec["marked_rows"]
        assert len(rows) == len(rec["marked"])
        groups = []  # (row, [blocks]) in marking order
        for b, i in zip(rec["marked"], rows):
            if groups and groups[-1][0] == i:
                groups[-1][1].append(b)
            else:
                groups.append((i, [b]))
        # rows in decreasing |e_i|, each visited once
        r = [g[0] for g in groups]
        assert len(set(r)) == len(r)
        for a, c in zip(r, r[1:]):
            assert abs(e[c]) <= abs(e[a]) * (1 + 1e-12) + 1e-300, (k, a, c)
        # the Doerfler test fails after every row group but the last
        rest = e.copy()
        for gi, (i, bs) in enumerate(groups):
            for b in bs:
                rs, db = contrib[b]
                assert abs(db[i - rs.start]) >= rec["tau"] * (1 - 1e-12)
                rest[rs] -= db
            nr = np.linalg.norm(rest)
            if gi + 1 < len(groups):
                assert nr > (1 - theta) * gk * (1 + 1e-12), (k, gi, nr, gk)
            else:
                assert nr <= (1 - theta) * gk * (1 + 1e-10), (k, nr, gk)
        # completeness: above the last row, no block over the threshold is left out
        last = abs(e[r[-1]])
        marked = set(rec["marked"])
        for b, (rs, db) in contrib.items():
            if b in marked:
                continue
            big = np.abs(e[rs]) > last * (1 + 1e-9)
            assert not np.any(big & (np.abs(db) >= rec["tau"] * (1 + 1e-9))), (k, b)
        checked += 1
    assert checked >= 3


@pytest.mark.parametrize("name", ["plate20-leaf32", "cube12-leaf16"])
def test_amvm_flat_geometry(name):
    """Coplanar clusters (a flat plate; the faces of the paper's cube): the
    result must still reach the exact collocation product within a few
    tolerances once the estimator reports convergence. With partial pivoting
    on |u_k| alone in the look-ahead, the normal component is never sampled:
    the estimator then converges while the product is off by 0.34 (plate)
    and 2.5e-3 (cube) relative."""
    if name.startswith("plate"):
        V, T = W.plate(20)
        leaf = 32
    else:
        V, T = W.cube_surface(12)
        leaf = 16
    mesh = O.Mesh(V, T, 1.0, 0.3)
    x = _point_force_x(V, T)
    tol = 1e-6
    y, hist, hm = amvm(mesh, x, theta=0.5, tol=tol, leaf=leaf, kcap=96, max_iter=1000)
    bt = mesh.brute_matvec(x[None, :])[0]
    assert hist[-1]["gamma"] <= tol * np.linalg.norm(y) * 1.01
    err = np.linalg.norm(y - bt) / np.linalg.norm(bt)
    assert err <= 20 * tol, err
