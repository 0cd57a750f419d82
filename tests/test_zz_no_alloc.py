"""asj_join_noalloc (no device allocation, fixed scratch array) against
asj_join, the entry point it is a variant of, through the C interface.

Two calls in a row share the device's one scratch array, the second with a
smaller input, so what the first call left there must not leak into the
second.  Outputs must be equal as multisets of (r_id, s_id) pairs, with equal
|T| and candidate counts; each is also compared with the oracle.
"""
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


def run_both(A, oracle, R, S, **kw):
    import torch
    Rk, Sk = A.DeviceKeys.from_host(R), A.DeviceKeys.from_host(S)
    # room for every inner pair, paper-literal extra pairs and outer rows
    cap = 2 * len(oracle.join_signature(R, S, verify=False)[0]) + R.n + S.n + 16
    res = []
    for fn in (A.asj_join_noalloc, A.asj_join):
        out = torch.full((cap, 2), -9, dtype=torch.int32, device="cuda")
        cnt = torch.full((2,), -9, dtype=torch.int64, device="cuda")
        fn(Rk, Sk, out, cnt, **kw)
        total, ncand = (int(x) for x in cnt.tolist())
        assert 0 <= total <= cap
        res.append((np.asarray(sorted(map(tuple, out[:total].cpu().numpy().tolist())), dtype=np.int32).reshape(-1, 2),
                    total, ncand))
    return res


def check(A, oracle, R, S, **kw):
    (got, total, ncand), (want, wtotal, wcand) = run_both(A, oracle, R, S, **kw)
    assert total == wtotal and ncand == wcand
    assert np.array_equal(got, want)
    return got


@pytest.mark.parametrize("kind", ["inner", "semi", "anti", "left", "right", "full", "plain", "literal", "f8"])
def test_noalloc_twice_second_smaller(A, oracle, wl, kind):
    kw = {}
    flags = {"inner": 0, "semi": A.ASJ_SEMI, "anti": A.ASJ_ANTI, "left": A.ASJ_LEFT_OUTER,
             "right": A.ASJ_RIGHT_OUTER, "full": A.ASJ_LEFT_OUTER | A.ASJ_RIGHT_OUTER, "plain": A.ASJ_PLAIN,
             "literal": A.ASJ_NO_VERIFY, "f8": 0}[kind]
    if kind == "f8":
        kw.update(f=8, nsym=4)
    # first: at the row limit, with duplicates; second: much smaller
    big = wl.random_small(11, m=A.ASJ_NOALLOC_MAX_BUILD_ROWS, n=14000, max_len=70, alphabet=b"abc\x00")
    small = wl.random_small(12, m=300, n=900, max_len=40, alphabet=b"ab")
    for w in (big, small):
        got = check(A, oracle, w.R, w.S, flags=flags, **kw)
        if kind == "inner":
            assert np.array_equal(got, oracle.join_nested(w.R, w.S))


def test_noalloc_tiny_workload_then_smaller(A, oracle, wl):
    for w in (wl.tiny(), wl.tiny(seed=3, scale=0.3)):
        got = check(A, oracle, w.R, w.S)
        want, _ = oracle.join_signature(w.R, w.S)
        assert np.array_equal(got, want)


def test_noalloc_empty_sides_after_a_join(A, oracle, wl):
    w = wl.tiny(scale=0.2)
    check(A, oracle, w.R, w.S)
    empty = wl.from_keys([])
    for R, S in ((empty, w.S), (w.R, empty), (empty, empty)):
        (got, total, ncand), _ = run_both(A, oracle, R, S)
        assert total == 0 and ncand == 0 and len(got) == 0


def test_noalloc_refuses_what_would_allocate(A, wl):
    import torch
    w = wl.random_small(3, m=A.ASJ_NOALLOC_MAX_BUILD_ROWS + 1, n=10, max_len=8)
    Rk, Sk = A.DeviceKeys.from_host(w.R), A.DeviceKeys.from_host(w.S)
    out = torch.empty((16, 2), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    with pytest.raises(A.AsjError) as e:
        A.asj_join_noalloc(Rk, Sk, out, cnt)
    assert e.value.code == A.ASJ_EINVAL
    small = wl.random_small(4, m=50, n=50, max_len=8)
    Rs, Ss = A.DeviceKeys.from_host(small.R), A.DeviceKeys.from_host(small.S)
    for flags, code in ((A.ASJ_SORTED, A.ASJ_EINVAL), (A.ASJ_GLOBAL_TABLES, A.ASJ_EINVAL),
                        (A.ASJ_PROBE_SPLIT, A.ASJ_EINVAL), (A.ASJ_FINGERPRINT, A.ASJ_EUNSUPPORTED)):
        with pytest.raises(A.AsjError) as e:
            A.asj_join_noalloc(Rs, Ss, out, cnt, flags=flags)
        assert e.value.code == code
    with pytest.raises(A.AsjError) as e:
        A.asj_join_noalloc(Rs, Ss, out, cnt, nsym=4)
    assert e.value.code == A.ASJ_EUNSUPPORTED
