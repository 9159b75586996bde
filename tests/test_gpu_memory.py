"""Device-memory reuse across streams and threads.

The library keeps released device buffers and lends them to later
allocations on any stream (ordered by an event recorded at the release), and
keeps a pool of first-pass ACA panel buffers per device that concurrent
builds borrow. Checked here:
  * two threads, each on its own stream, build and multiply a sequence of
    meshes of different sizes and free each handle right away (so buffers
    pass between the threads' streams); every product equals the one from a
    single-threaded run bit for bit, and so do the ranks;
  * products issued right after the build on a side stream, and handles
    freed while the other thread's kernels run, leave the results unchanged
    over three rounds;
  * hmat_release_memory returns the kept memory to the device.
"""
import threading

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _H():
    import paper_2205_04752_amd as H
    return H


def _meshes():
    return [W.icosphere(2), W.torus(1.0, 0.3, 28, 10), W.ellipsoid(4, (1.2, 0.8, 0.5)),
            W.icosphere(3), W.torus(1.0, 0.45, 20, 12), W.icosphere(1)]


def _run(meshes, eps_list, stream, out, key):
    H = _H()
    with torch.cuda.stream(stream):
        res = []
        for (V, T), eps in zip(meshes, eps_list):
            N = 3 * len(T)
            g = H.HMatrix(V, T, 1.0, 0.3, 2.0, 32, eps, stream=stream)
            x = torch.from_numpy(W.random_x(N, 3, seed=N)).cuda()
            y = g.matvec(x, stream=stream)
            stream.synchronize()
            res.append((y.cpu().numpy(), g.info()["rank_mean"]))
            g.close()
        out[key] = res


def test_threads_and_streams_share_buffers():
    meshes = _meshes()
    eps_a = [1e-4, 1e-6, 1e-3, 1e-5, 1e-7, 1e-4]
    eps_b = eps_a[::-1]
    print("case memory: sequential reference", flush=True)
    ref = {}
    s0 = torch.cuda.Stream()
    _run(meshes, eps_a, s0, ref, "a")
    _run(meshes, eps_b, s0, ref, "b")
    for rnd in range(3):
        print(f"case memory: two threads, round {rnd}", flush=True)
        out = {}
        sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
        ta = threading.Thread(target=_run, args=(meshes, eps_a, sa, out, "a"))
        tb = threading.Thread(target=_run, args=(meshes[::-1], eps_b[::-1], sb, out, "b"))
        ta.start()
        tb.start()
        ta.join()
        tb.join()
        assert "a" in out and "b" in out
        for (ya, ra), (yr, rr) in zip(out["a"], ref["a"]):
            assert ra == rr and np.array_equal(ya, yr)
        # thread b ran the meshes in reverse order with reversed eps: compare per mesh
        for (yb, rb), (yr, rr) in zip(out["b"], ref["b"][::-1]):
            assert rb == rr and np.array_equal(yb, yr)


def test_release_memory_returns_cached_memory():
    """hmat_release_memory hands the cached buffers back to the device (free
    device memory rises by at least half of a freed handle's bytes) and later
    builds give the same products bit for bit."""
    H = _H()
    V, T = W.icosphere(4)
    N = 3 * len(T)
    x = torch.from_numpy(W.random_x(N, 2, seed=5)).cuda()
    g = H.HMatrix(V, T, 1.0, 0.3, 2.0, 32, 1e-6)
    held = g.info()["device_bytes"]
    y0 = g.matvec(x).cpu()
    g.close()
    torch.cuda.synchronize()
    free_before, _ = torch.cuda.mem_get_info()
    H.release_memory()
    free_after, _ = torch.cuda.mem_get_info()
    assert free_after - free_before >= held // 2, (free_before, free_after, held)
    g = H.HMatrix(V, T, 1.0, 0.3, 2.0, 32, 1e-6)
    y1 = g.matvec(x).cpu()
    g.close()
    assert torch.equal(y0, y1)
