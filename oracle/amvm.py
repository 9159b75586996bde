"""Adaptive matrix-vector multiplication (Algorithm 2, Sec. 3) -- test oracle.

Test infrastructure only: plain NumPy over the C oracle's blocks, used by
tests/ and bench.py's CPU baseline, never by the library.

The sequence of H-matrices A_k shares the tree and partition of the
ordinary build; only the ranks of the admissible blocks change.
  * A_0 (the coarse start, a reading of "a coarse H-matrix approximation"):
    dense blocks exact, every admissible block of rank 0.
  * The look-ahead A^_k takes `lookahead` (2) further ACA steps on every
    admissible block; dense blocks are the same in both (Sec. 3).
  * d_b = (A^_k - A_k)_b x_s, the block's rank-2 contribution;
    b^_k - b_k = sum_b d_b and gamma_k = ||b_k - b^_k||_2.
  * Marking (step 3 b): rows in decreasing order of |(b_k - b^_k)_i| (ties:
    lower row first); along them, every admissible block containing row i
    with |(d_b)_i| >= (1 - theta) (c_sp M N)^(-1/2) gamma_k joins P_k
    (blocks of a row in canonical order); stop after the first row at
    which gamma_k(P_k) = ||sum_{b not in P_k} d_b|| <= (1 - theta) gamma_k
    holds, or when the rows run out.
  * A_{k+1} = A^_k on P_k (their rank grows by `lookahead`), A_k elsewhere.
  * Stop when gamma_k <= tol ||b^_k||_2 (reading: the tolerance is relative)
    or after max_iter rounds; the result is b_k.
ACA crosses come from ``HMatrix.fill_steps(kcap)``: ACA without the accuracy
test, so the first r crosses of a block are those of r resumed steps. Its
pivot rows cycle through the three displacement components (the oracle's
cycle_next rule): with no accuracy test, nothing else would send ACA to the
normal component of a coplanar block, whose error the estimator would then
never see. A block
that is exhausted (full rank, every row used, or kcap reached) has no further
crosses and contributes nothing more.
"""
from __future__ import annotations

import numpy as np

from . import HMatrix, Mesh


def amvm(mesh: Mesh, x, theta: float = 0.5, tol: float = 1e-6, max_iter: int = 200,
         eta: float = 2.0, leaf: int = 32, kcap: int = 96, lookahead: int = 2, hm=None):
    """Returns (b in the caller's DOF order, history list of dicts with
    'ranks' (per block at A_k, -1 for dense blocks), 'gamma', 'marked',
    'marked_rows' (the cluster-order row at which each marked block joined
    P_k), 'gamma_rest' (gamma_k(P_k)), 'tau'), and the oracle H-matrix used."""
    if hm is None:
        hm = HMatrix(mesh, eta, leaf)
        hm.fill_steps(kcap)
    ob = hm.blocks()
    order = hm.order
    nt = len(order)
    N = M = 3 * nt
    perm = (3 * order[:, None] + np.arange(3)).ravel()  # cluster DOF -> caller DOF
    xp = np.asarray(x, dtype=np.float64)[perm]
    far = np.nonzero(ob[:, 4] == 1)[0]
    rows = {b: slice(3 * int(ob[b, 0]), 3 * int(ob[b, 0] + ob[b, 1])) for b in range(len(ob))}
    cols = {b: slice(3 * int(ob[b, 2]), 3 * int(ob[b, 2] + ob[b, 3])) for b in range(len(ob))}
    # dense part of every A_k
    bk = np.zeros(M)
    for b in np.nonzero(ob[:, 4] == 0)[0]:
        bk[rows[b]] += hm.dense_block(int(b)) @ xp[cols[b]]
    U, V = {}, {}
    for b in far:
        U[b], V[b], _, _ = hm.factors(int(b))
    # far blocks containing each row, canonical order
    row_blocks = [[] for _ in range(M)]
    for b in far:
        for i in range(rows[b].start, rows[b].stop):
            row_blocks[i].append(int(b))
    csp = hm.csp()
    rank = {int(b): 0 for b in far}
    hist = []
    for _ in range(max_iter):
        d = {}
        e = np.zeros(M)
        for b in far:
            b = int(b)
            r0, r1 = rank[b], min(rank[b] + lookahead, U[b].shape[1])
            if r1 > r0:
                db = U[b][:, r0:r1] @ (V[b][:, r0:r1].T @ xp[cols[b]])
                d[b] = db
                e[rows[b]] += db
        gamma = float(np.linalg.norm(e))
        rk = np.full(len(ob), -1, dtype=np.int64)
        for b in far:
            rk[b] = rank[int(b)]
        rec = dict(ranks=rk, gamma=gamma, marked=[], gamma_rest=gamma, tau=0.0)
        hist.append(rec)
        if gamma <= tol * np.linalg.norm(bk + e) or not d:
            break
        tau = (1.0 - theta) * (csp * M * N) ** -0.5 * gamma
        rec["tau"] = tau
        order_rows = np.argsort(-np.abs(e), kind="stable")
        marked, marked_rows, rest = [], [], e.copy()
        in_p = set()
        for i in order_rows:
            added = False
            for b in row_blocks[i]:
                if b in in_p or b not in d:
                    continue
                if abs(d[b][i - rows[b].start]) >= tau:
                    in_p.add(b)
                    marked.append(b)
                    marked_rows.append(int(i))
                    rest[rows[b]] -= d[b]
                    added = True
            if added and np.linalg.norm(rest) <= (1.0 - theta) * gamma:
                break
        rec["marked"] = marked
        rec["marked_rows"] = marked_rows
        rec["gamma_rest"] = float(np.linalg.norm(rest))
        for b in marked:
            bk[rows[b]] += d[b]
            rank[b] = min(rank[b] + lookahead, U[b].shape[1])
    y = np.zeros(M)
    y[perm] = bk
    return y, hist, hm
