"""Parity at full workload sizes, in the launch configurations the benchmark
times: asj_join with default options on the large single join (R = 1M,
S = 4M keys, ~4.9 GB) and on the DNA join (R = 200k, S = 1M keys of
1000-10000 bases), asj_join_batch over all 256 joins of the batched
workload (~14 GB) and over 128 independent tiny joins (655 MB), and the
continuous-batching server over the resident 10M-key build side with
requests of up to 1M keys.

Join outputs are compared with the oracle's hash join on the same inputs
(exact multisets of integer pairs): whole joins where the oracle finishes
in about 20 s (large, DNA, every served request), a seeded sample of whole
joins for the batched workload.  Signatures of sampled keys are compared
bit for bit.  On every output, properties that hold at any size are
checked as well: no pair twice, ids inside their join, and the keys of
sampled emitted pairs byte-equal.
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


def note(msg):
    print(f"[fullsize] {msg}", flush=True)


def unique_pairs(p):
    """True when no (r_id, s_id) pair occurs twice."""
    if len(p) == 0:
        return True
    key = (p[:, 0].astype(np.int64) << 32) | p[:, 1].astype(np.int64)
    return len(np.unique(key)) == len(key)


def keys_equal(R, S, pairs, rng, count=20000, r_base=0, s_base=0):
    """Byte-compare the keys of up to `count` sampled emitted pairs."""
    if len(pairs) == 0:
        return True
    pick = rng.choice(len(pairs), size=min(count, len(pairs)), replace=False)
    return all(R.key(r_base + int(pairs[i, 0])) == S.key(s_base + int(pairs[i, 1])) for i in pick)


def gpu_signatures(A, keys):
    return A.asj_signature(keys).cpu().numpy().view(np.uint32).astype(np.uint64)


@pytest.mark.parametrize("name", ["large", "dna"])
def test_full_size_join_equals_oracle(A, oracle, wl, name):
    import torch
    w = getattr(wl, name)()
    note(f"{name}: R={w.R.n} S={w.S.n} bytes={w.R.nbytes + w.S.nbytes}")
    Rk, Sk = A.DeviceKeys.from_host(w.R), A.DeviceKeys.from_host(w.S)
    expected = int(w.meta["expected_matches"])
    out = torch.empty((expected + 1024, 2), dtype=torch.int32, device="cuda")  # the benchmark's capacity
    counts = torch.zeros(2, dtype=torch.int64, device="cuda")
    A.asj_join(Rk, Sk, out, counts)
    total = int(counts[0])
    assert 0 <= total <= expected + 1024
    got = out[:total].cpu().numpy()
    note(f"{name}: GPU |T|={total}; oracle join")
    want = oracle.join_hash(w.R, w.S, cap=expected + 1024)
    assert total == len(want) == expected
    assert np.array_equal(oracle.sort_pairs(got), want)
    assert unique_pairs(got)
    rng = np.random.default_rng([17, len(name)])
    for rel, keys in ((w.R, Rk), (w.S, Sk)):
        sig = gpu_signatures(A, keys)
        idx = np.sort(rng.choice(rel.n, size=min(rel.n, 20000), replace=False))
        assert np.array_equal(sig[idx], oracle.signatures(rel.subset(idx)))


def test_full_size_batch_sampled_joins_equal_oracle(A, oracle, wl):
    b = wl.batch()
    note(f"batch: joins={b.njoins} R={b.R.n} S={b.S.n} bytes={b.R.nbytes + b.S.nbytes}")
    R, S = A.DeviceKeys.from_host(b.R), A.DeviceKeys.from_host(b.S)
    out, oseg, counts, _, _ = A.join_batch(R, S, b.r_seg, b.s_seg)
    outh = out.cpu().numpy()
    rsz, ssz = np.diff(b.r_seg), np.diff(b.s_seg)
    rng = np.random.default_rng(23)
    for k in range(b.njoins):  # properties of every join's output
        p = outh[oseg[k]:oseg[k] + counts[k]]
        assert counts[k] <= oseg[k + 1] - oseg[k], k
        assert ((p[:, 0] >= 0) & (p[:, 0] < rsz[k]) & (p[:, 1] >= 0) & (p[:, 1] < ssz[k])).all(), k
        assert unique_pairs(p), k
        assert keys_equal(b.R, b.S, p, rng, count=200, r_base=int(b.r_seg[k]), s_base=int(b.s_seg[k])), k
    sample = set(rng.choice(b.njoins, size=24, replace=False).tolist())
    sample |= {int(np.argmax(ssz)), int(np.argmin(ssz))}
    for k in sorted(sample):
        j = b.join(k)
        want = oracle.join_hash(j.R, j.S, cap=j.S.n + 1024)
        got = outh[oseg[k]:oseg[k] + counts[k]]
        assert counts[k] == len(want), k
        assert np.array_equal(oracle.sort_pairs(got), want), k
    note(f"batch: {len(sample)} joins equal the oracle; {int(counts.sum())} pairs in all")
    idx = np.sort(rng.choice(b.S.n, size=20000, replace=False))
    assert np.array_equal(gpu_signatures(A, S)[idx], oracle.signatures(b.S.subset(idx)))


def concat(wl, rels):
    """Relations end to end, ids made global so one oracle join covers them all."""
    lens = np.concatenate([r.lengths() for r in rels])
    data = np.concatenate([r.data[:r.offsets[-1]] for r in rels] + [np.zeros(16, np.uint8)])
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    return wl.Relation(data, off, np.arange(len(lens), dtype=np.int32))


def test_full_size_served_requests_equal_oracle(A, oracle, wl):
    import torch
    R = wl.served_build_side()  # 10M resident keys of 256 bytes
    note(f"served: R={R.n} bytes={R.nbytes}")
    t = A.asj_build(A.DeviceKeys.from_host(R))
    reqs = [wl.served_request(R, seed=5, request=i) for i in range(4)]
    reqs.append(wl.served_request(R, seed=5, request=1000, size=1_000_000))
    srv = A.Server(t, slots=4)
    bufs = [(torch.from_numpy(q.data).pin_memory(), torch.from_numpy(q.offsets).pin_memory(),
             torch.empty((q.n, 2), dtype=torch.int32).pin_memory()) for q in reqs]
    tickets = [srv.submit(d, o, out) for d, o, out in bufs]  # all in flight together
    infos = [srv.wait(x) for x in tickets]
    srv.close()
    assert all(x["status"] == 0 for x in infos)
    note(f"served: sizes {[q.n for q in reqs]} batches {[x['batch_requests'] for x in infos]}; oracle join")
    want = oracle.join_hash(R, concat(wl, reqs), cap=sum(q.n for q in reqs) + 1024)
    base = np.concatenate([[0], np.cumsum([q.n for q in reqs])])
    for i, (q, x, (_, _, out)) in enumerate(zip(reqs, infos, bufs)):
        sel = want[(want[:, 1] >= base[i]) & (want[:, 1] < base[i + 1])].copy()
        sel[:, 1] -= base[i]
        got = out[:x["count"]].numpy()
        assert x["count"] == len(sel), i
        assert np.array_equal(oracle.sort_pairs(got), oracle.sort_pairs(sel)), i
        assert unique_pairs(got), i
    t.free()


def test_full_size_host_join_partitioned_equals_oracle(A, oracle, wl):
    """The large join (4.9 GB of keys) from pinned host memory within a 1 GiB
    device budget, the benchmark's partitioned configuration: the build side
    does not fit half the budget, so both relations are partitioned by
    signature bits; the output must be the oracle's whole join."""
    import torch
    w = wl.large()
    expected = int(w.meta["expected_matches"])
    note(f"host join: R={w.R.n} S={w.S.n}, 1 GiB budget")
    Rh, Sh = A.HostKeys.from_host(w.R), A.HostKeys.from_host(w.S)
    out = torch.empty((expected + 1024, 2), dtype=torch.int32)
    total, st = A.asj_join_host(Rh, Sh, out, hbm_budget=1 << 30)
    note(f"host join: |T|={total} stats={st}")
    assert st["partitions"] >= 2 and st["device_peak"] <= 1 << 30
    got = out[:total].numpy()
    want = oracle.join_hash(w.R, w.S, cap=expected + 1024)
    assert total == len(want) == expected
    assert np.array_equal(oracle.sort_pairs(got), want)
    A.asj_join_host_release()


def test_full_size_tiny_instances_batch_equals_oracle(A, oracle, wl):
    """128 independent tiny joins (R = S = 10k keys of 256 B each, 655 MB) in
    one batch, the benchmark's throughput configuration (every join's table
    built in LDS; options left to the library): every join has exactly the
    generator's 2000 matches, every output has the properties above, and a
    seeded sample of whole joins equals the oracle pair for pair."""
    parts = [wl.tiny(seed=1 + i) for i in range(128)]
    def cat(rels):
        lens = np.concatenate([r.lengths() for r in rels])
        data = np.concatenate([r.data[:r.offsets[-1]] for r in rels] + [np.zeros(16, np.uint8)])
        off = np.zeros(len(lens) + 1, dtype=np.int64)
        np.cumsum(lens, out=off[1:])
        return wl.Relation(data, off, np.concatenate([r.ids for r in rels]))
    Rf, Sf = cat([p.R for p in parts]), cat([p.S for p in parts])
    r_seg = np.concatenate([[0], np.cumsum([p.R.n for p in parts])]).astype(np.int64)
    s_seg = np.concatenate([[0], np.cumsum([p.S.n for p in parts])]).astype(np.int64)
    note(f"tiny instances: joins=128 R={Rf.n} S={Sf.n} bytes={Rf.nbytes + Sf.nbytes}")
    R, S = A.DeviceKeys.from_host(Rf), A.DeviceKeys.from_host(Sf)
    out, oseg, counts, cands, _ = A.join_batch(R, S, r_seg, s_seg)
    assert (counts == 2000).all()
    outh = out.cpu().numpy()
    rng = np.random.default_rng(29)
    for k, w in enumerate(parts):
        p = outh[oseg[k]:oseg[k] + counts[k]]
        assert ((p[:, 0] >= 0) & (p[:, 0] < w.R.n) & (p[:, 1] >= 0) & (p[:, 1] < w.S.n)).all(), k
        assert unique_pairs(p), k
        assert keys_equal(w.R, w.S, p, rng, count=100), k
    for k in sorted(rng.choice(128, size=12, replace=False).tolist()):
        want, want_cand = oracle.join_signature(parts[k].R, parts[k].S)
        assert np.array_equal(oracle.sort_pairs(outh[oseg[k]:oseg[k] + counts[k]]), want), k
        assert cands[k] == want_cand, k
    note("tiny instances: 128 joins with 2000 pairs each; 12 sampled joins equal the oracle")
