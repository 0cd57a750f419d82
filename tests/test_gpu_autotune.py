"""The autotuner: it times the whole join over its grid, returns a valid
choice no slower than the defaults it measured, and later calls that leave
the options to the library use that choice -- with output still exactly the
oracle's join."""
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


def capacity(n, lf):
    cap = 64
    while cap * lf < n:
        cap *= 2
    return cap


def phases(A, fn):
    A.timing_enable(True)
    fn()
    names = [n for n, _ in A.timing_read(64)]
    A.timing_enable(False)
    return names


def test_autotune_single_join(A, oracle, wl):
    import torch
    w = wl.large(scale=0.005)
    Rk, Sk = A.DeviceKeys.from_host(w.R), A.DeviceKeys.from_host(w.S)
    out = torch.empty((w.S.n + 1024, 2), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    want = oracle.join_hash(w.R, w.S)
    try:
        res = A.autotune(Rk, Sk, out, cnt)
        assert res["trials"] >= 60 and res["best_ms"] <= res["default_ms"]
        assert res["load_factor"] in (0.25, 0.35, 0.5, 0.7) and res["keys_per_window"] in (4, 8, 16, 32, 64)
        assert res["grid_rounds"] in (1, 2, 4)
        assert int(cnt[0]) == len(want)  # the trial joins were exact too
        t = A.asj_build(Rk)  # options left to the library
        assert t.capacity == capacity(w.R.n, res["load_factor"])
        t.free()
        assert A.asj_build(Rk, load_factor=0.5).capacity == capacity(w.R.n, 0.5)  # explicit options win
        names = phases(A, lambda: A.asj_join(Rk, Sk, out, cnt))
        assert ("probe_verify" in names) == (res["schedule"] == "split")
        assert np.array_equal(oracle.sort_pairs(out[:int(cnt[0])].cpu().numpy()), want)
    finally:
        A.autotune_clear()
    t = A.asj_build(Rk)  # back to the defaults
    assert t.capacity == capacity(w.R.n, 0.5)
    t.free()


def test_autotune_batch(A, oracle, wl):
    import torch
    b = wl.batch(scale=0.002, njoins=12)
    R, S = A.DeviceKeys.from_host(b.R), A.DeviceKeys.from_host(b.S)
    dev = lambda a: torch.from_numpy(np.asarray(a, dtype=np.int64)).cuda()
    caps = np.diff(b.s_seg) + 16
    oseg = np.zeros(b.njoins + 1, dtype=np.int64)
    oseg[1:] = np.cumsum(caps)
    out = torch.empty((int(oseg[-1]), 2), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(b.njoins, dtype=torch.int64, device="cuda")
    try:
        res = A.autotune_batch(R, S, dev(b.r_seg), dev(b.s_seg), out, dev(oseg), cnt)
        assert res["trials"] == 120 and res["best_ms"] <= res["default_ms"]  # 4 x 5 x 2 schedules x 3 grids
        assert res["grid_rounds"] in (1, 2, 4)
        got, gseg, counts, _, _ = A.join_batch(R, S, b.r_seg, b.s_seg)  # options left to the library
        outh = got.cpu().numpy()
        for k in range(b.njoins):
            j = b.join(k)
            want = oracle.join_hash(j.R, j.S)
            assert np.array_equal(oracle.sort_pairs(outh[gseg[k]:gseg[k] + counts[k]]), want), k
    finally:
        A.autotune_clear()
