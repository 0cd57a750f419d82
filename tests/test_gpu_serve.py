"""GPU serving: every request's result is the same alone and in a mix of
concurrent requests (exact, integer pairs), and equals the oracle's join of
the resident build relation with that request."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2411_18183_amd import asjoin as A
    A.lib()
    return A


@pytest.mark.parametrize("sched", ["split", "fused"])
def test_results_identical_alone_and_in_the_mix(A, oracle, wl, sched):
    import torch
    R = wl.served_build_side(scale=0.01)  # 100k resident keys of 256 bytes
    Rk = A.DeviceKeys.from_host(R)
    t = A.asj_build(Rk, flags=A.ASJ_PROBE_SPLIT if sched == "split" else A.ASJ_PROBE_FUSED)
    reqs = [wl.served_request(R, seed=5, request=i, min_size=500, max_size=20000) for i in range(10)]
    want = [oracle.join_hash(R, q) for q in reqs]

    def buffers(q):
        data = torch.from_numpy(q.data).pin_memory()
        off = torch.from_numpy(q.offsets).pin_memory()
        out = torch.empty((q.n, 2), dtype=torch.int32).pin_memory()
        return data, off, out

    # alone: one request in the server at a time
    srv = A.Server(t, slots=3)
    alone = []
    for q in reqs:
        d, o, out = buffers(q)
        info = srv.wait(srv.submit(d, o, out))
        assert info["status"] == 0 and info["batch_requests"] == 1
        alone.append(oracle.sort_pairs(out[:info["count"]].numpy()))
    # mix: all requests (twice over) submitted at once; the server packs and overlaps them
    bufs = [buffers(q) for q in reqs + reqs]
    tickets = [srv.submit(*b) for b in bufs]
    infos = [srv.wait(x) for x in tickets]
    assert max(i["batch_requests"] for i in infos) > 1, "nothing was batched"
    # device time of each request's launch (HIP events): the kernel is part of it
    assert all(0 < i["t_kernel_ms"] <= i["t_device_ms"] for i in infos)
    for k, (info, b) in enumerate(zip(infos, bufs)):
        got = oracle.sort_pairs(b[2][:info["count"]].numpy())
        assert info["status"] == 0
        assert np.array_equal(got, alone[k % len(reqs)]), k
        assert np.array_equal(got, want[k % len(reqs)]), k
    srv.close()
    t.free()


def test_small_budget_serializes_without_losing_requests(A, oracle, wl):
    import torch
    R = wl.served_build_side(scale=0.002)
    t = A.asj_build(A.DeviceKeys.from_host(R))
    reqs = [wl.served_request(R, seed=6, request=i, size=3000) for i in range(6)]
    one = max(q.nbytes for q in reqs) * 2 + 64 * 3000 + (1 << 16)
    srv = A.Server(t, slots=4, hbm_budget=one)
    bufs = []
    for q in reqs:
        out = torch.empty((q.n, 2), dtype=torch.int32).pin_memory()
        bufs.append((torch.from_numpy(q.data), torch.from_numpy(q.offsets), out))
    tickets = [srv.submit(*b) for b in bufs]
    infos = [srv.wait(x) for x in tickets]
    st = srv.stats()
    assert st["peak_budget_used"] <= one
    for q, info, b in zip(reqs, infos, bufs):
        assert info["status"] == 0
        assert np.array_equal(oracle.sort_pairs(b[2][:info["count"]].numpy()), oracle.join_hash(R, q))
    srv.close()
    t.free()
