"""GPU parity of the batched path: many joins per launch sequence.

Each join of a batch must produce exactly the oracle's join of its own
relations (as a multiset), the same output as asj_join on that join alone,
and the oracle's candidate count.
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


def flatten(wl, joins):
    """[(R keys, S keys)] -> flattened relations with row-local ids and segment arrays."""
    rk, sk, rid, sid = [], [], [], []
    r_seg, s_seg = [0], [0]
    for R, S in joins:
        rk += R
        sk += S
        rid += list(range(len(R)))
        sid += list(range(len(S)))
        r_seg.append(len(rk))
        s_seg.append(len(sk))
    return wl.from_keys(rk, rid), wl.from_keys(sk, sid), np.array(r_seg), np.array(s_seg)


SCHED = {"split": 0x8, "fused": 0x4}


@pytest.mark.parametrize("sched", sorted(SCHED))
def test_batch_matches_oracle_and_single_joins(A, oracle, wl, sched):
    b = wl.batch(scale=0.003, njoins=20)
    R, S = A.DeviceKeys.from_host(b.R), A.DeviceKeys.from_host(b.S)
    out, oseg, counts, cands, clock = A.join_batch(R, S, b.r_seg, b.s_seg, flags=SCHED[sched])
    outh = out.cpu().numpy()
    for k in range(b.njoins):
        j = b.join(k)
        want, want_cand = oracle.join_signature(j.R, j.S)
        got = outh[oseg[k]:oseg[k] + counts[k]]
        assert counts[k] == len(want), k
        assert np.array_equal(oracle.sort_pairs(got), want), k
        assert cands[k] == want_cand, k
        alone, total, _ = A.join(A.DeviceKeys.from_host(j.R), A.DeviceKeys.from_host(j.S))
        assert np.array_equal(oracle.sort_pairs(alone.cpu().numpy()), oracle.sort_pairs(got)), k
    start = clock[-1]
    assert start > 0 and (clock[:-1] >= start).all()


def test_batch_empty_joins_duplicates_and_caller_workspace(A, oracle, wl):
    import torch
    joins = [
        ([], [b"a", b"b"]),                       # empty build side
        ([b"a", b"b"], []),                       # empty probe side
        ([], []),                                 # both empty
        ([b"k" * 70] * 5 + [b""], [b"k" * 70] * 3 + [b"", b""]),  # duplicates, empty keys
        ([bytes([i % 7]) * (i % 90) for i in range(300)], [bytes([i % 5]) * (i % 130) for i in range(400)]),
        ([b"x" * 5000, b"y" * 4096], [b"x" * 5000, b"y" * 4096, b"y" * 4095]),
    ]
    Rf, Sf, r_seg, s_seg = flatten(wl, joins)
    R, S = A.DeviceKeys.from_host(Rf), A.DeviceKeys.from_host(Sf)
    J = len(joins)
    caps = np.array([max(1, len(a) * len(b)) for a, b in joins])
    out_seg = np.zeros(J + 1, dtype=np.int64)
    out_seg[1:] = np.cumsum(caps)
    ws = torch.empty(A.asj_batch_workspace_bytes(J, Rf.n, Sf.n), dtype=torch.uint8, device="cuda")
    dev = lambda a: torch.from_numpy(np.asarray(a, dtype=np.int64)).cuda()
    out = torch.empty((int(out_seg[-1]), 2), dtype=torch.int32, device="cuda")
    counts = torch.zeros(J, dtype=torch.int64, device="cuda")
    cands = torch.zeros(J, dtype=torch.int64, device="cuda")
    clock = torch.zeros(J + 1, dtype=torch.int64, device="cuda")
    for rep in range(2):  # the second call reuses the workspace and must start clean
        A.asj_join_batch(R, S, dev(r_seg), dev(s_seg), out, dev(out_seg), counts, cands, clock, workspace=ws)
        torch.cuda.synchronize()
        c = counts.cpu().numpy()
        outh = out.cpu().numpy()
        for k, (rk, sk) in enumerate(joins):
            want = oracle.join_nested(wl.from_keys(rk), wl.from_keys(sk))
            assert c[k] == len(want), (rep, k)
            assert np.array_equal(oracle.sort_pairs(outh[out_seg[k]:out_seg[k] + c[k]]), want), (rep, k)


@pytest.mark.parametrize("sched", sorted(SCHED))
@pytest.mark.parametrize("flags_name", ["ASJ_PLAIN", "ASJ_NO_VERIFY"])
def test_batch_plain_and_paper_literal(A, oracle, wl, flags_name, sched):
    joins = [wl.random_small(s, m=60 + 9 * s, n=80 + 5 * s, max_len=[3, 12, 40][s % 3], alphabet=b"ab\x00")
             for s in range(8)]
    Rf, Sf, r_seg, s_seg = flatten(wl, [([w.R.key(i) for i in range(w.R.n)], [w.S.key(i) for i in range(w.S.n)])
                                        for w in joins])
    R, S = A.DeviceKeys.from_host(Rf), A.DeviceKeys.from_host(Sf)
    flags = getattr(A, flags_name) | SCHED[sched]
    out, oseg, counts, cands, _ = A.join_batch(R, S, r_seg, s_seg, flags=flags)
    outh = out.cpu().numpy()
    for k, w in enumerate(joins):
        if flags_name == "ASJ_PLAIN":
            want = oracle.join_nested(w.R, w.S)
        else:
            want, _ = oracle.join_signature(w.R, w.S, verify=False)
        assert counts[k] == len(want)
        assert np.array_equal(oracle.sort_pairs(outh[oseg[k]:oseg[k] + counts[k]]), want)


@pytest.mark.parametrize("case", ["last_bound", "decreasing"])
def test_batch_invalid_segments_report_minus_one(A, wl, case):
    joins = [([b"a", b"b"], [b"a"]), ([b"c"], [b"c", b"d"]), ([b"e"], [b"e"])]
    Rf, Sf, r_seg, s_seg = flatten(wl, joins)
    R, S = A.DeviceKeys.from_host(Rf), A.DeviceKeys.from_host(Sf)
    bad = r_seg.copy()
    if case == "last_bound":
        bad[-1] += 5  # does not end at the last build row
    else:
        bad[1], bad[2] = bad[2], bad[1]  # a segment of negative size
    _, _, counts, _, _ = A.join_batch(R, S, bad, s_seg)
    assert (counts == -1).all()
    _, _, counts, _, _ = A.join_batch(R, S, r_seg, s_seg)  # the same inputs with valid segments
    assert counts.tolist() == [1, 1, 1]
