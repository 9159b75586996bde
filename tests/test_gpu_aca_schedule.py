"""ACA launch schedule (hmat_opts aca_small_tri / aca_wide) and its autotuner
(hmat_tune_aca), on the GPU.

The schedule decides which blocks run one wave each and the workgroup size of
the others; it does not change the arithmetic of an entry, a remainder or a
pivot choice, only the order in which ||S_k||^2 is summed. So unless a stop
test lies within rounding of its threshold (not the case here), every
schedule gives the same ranks, pivots and factors: the products are equal
bit for bit, and the default schedule's factors are pinned to the oracle by
the parity tests.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _H():
    import paper_2205_04752_amd as H
    return H


CASES = {
    "ico3-eps1e-6": (lambda: W.icosphere(3), 1e-6),
    "box-eps1e-7": (lambda: W.box_surface(6.0, 1.0, 1.0, 36, 6, 6), 1e-7),
}


@pytest.mark.parametrize("name", list(CASES))
def test_schedules_give_the_same_matrix(name):
    H = _H()
    mk, eps = CASES[name]
    V, T = mk()
    print("case aca schedule:", name, flush=True)
    x = torch.from_numpy(W.random_x(3 * len(T), 2, seed=4)).cuda()
    ref = H.HMatrix(V, T, 1.0, 0.3, 2.0, 32, eps)
    y0 = ref.matvec(x)
    st0 = ref.info()
    ref.close()
    for small in (32, 64, 128, 1024):
        for wide in (0, 1):
            g = H.HMatrix(V, T, 1.0, 0.3, 2.0, 32, eps, aca_schedule=(small, wide))
            st = g.info()
            assert (st["rank_mean"], st["rank_max"], st["n_far"]) == (st0["rank_mean"], st0["rank_max"],
                                                                     st0["n_far"]), (small, wide)
            assert torch.equal(g.matvec(x), y0), (small, wide)
            g.close()


def test_tune_aca_reports_and_picks_the_fastest():
    H = _H()
    V, T = W.icosphere(3)
    r = H.tune_aca(V, T, eps=1e-6, reps=2)
    c = r["candidates"]
    assert len(c) == 6
    assert sorted({(s, w) for s, w, _ in c}) == [(s, w) for s in (32, 64, 128) for w in (0, 1)]
    assert all(ms > 0 for _, _, ms in c)
    assert r["best_ms"] == min(ms for _, _, ms in c)
    assert r["aca_schedule"] == tuple(c[r["best"]][:2])
    # the chosen schedule builds the same matrix as the default
    x = torch.from_numpy(W.random_x(3 * len(T), 1, seed=5)).cuda()
    g0 = H.HMatrix(V, T, 1.0, 0.3, 2.0, 32, 1e-6)
    g1 = H.HMatrix(V, T, 1.0, 0.3, 2.0, 32, 1e-6, aca_schedule=r["aca_schedule"])
    assert torch.equal(g0.matvec(x), g1.matvec(x))
    g0.close()
    g1.close()
    print("tune_aca:", r, flush=True)


def test_fp32_build_schedules():
    """FP32 builds (FP32 ACA at eps >= 1e-5) under another schedule: the same
    matrix as the default schedule's."""
    H = _H()
    V, T = W.icosphere(3)
    x = torch.from_numpy(W.random_x(3 * len(T), 1, seed=6)).cuda()
    g0 = H.HMatrix(V, T, 1.0, 0.3, 2.0, 32, 1e-5, precision=1)
    g1 = H.HMatrix(V, T, 1.0, 0.3, 2.0, 32, 1e-5, precision=1, aca_schedule=(128, 1))
    assert torch.equal(g0.matvec(x, precision=1), g1.matvec(x, precision=1))
    g0.close()
    g1.close()
