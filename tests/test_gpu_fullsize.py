"""Parity at full workload sizes, in the launch configurations the benchmark
times.

* The large single join (R = 1M, S = 4M keys, ~4.9 GB) and the DNA join
  (R = 200k, S = 1M keys of 1000-10000 bases) through asj_join: with the
  library defaults, with the autotuner's choice (what the benchmark times:
  options left to the library after asj_autotune on the same inputs), and
  with every probe configuration the autotuner may choose on the
  device-memory table (load factor, keys per window, grid rounds, probe
  schedule).  Every output is compared pair for pair with one oracle
  signature join, candidate count included.
* asj_join_batch over all 256 joins of the batched workload (~14 GB): every
  join compared pair for pair with the oracle's hash join (the oracle calls
  run in a thread pool; they release the GIL).
* 256 independent tiny joins (1.3 GB) in one batch.
* The continuous-batching server over the resident 10M-key build side with
  requests of up to 1M keys, and the partitioned host-memory join.

Join outputs are exact multisets of integer pairs; signatures of sampled
keys are compared bit for bit.  On every output, properties that hold at any
size are checked as well: no pair twice, ids inside their join.
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


def gpu_signatures(A, keys):
    return A.asj_signature(keys).cpu().numpy().view(np.uint32).astype(np.uint64)


# Probe configurations the autotuner may choose for a single join with a
# device-memory table (load factor, keys per window, grid rounds, schedule),
# beside the library defaults and the autotuner's own choice.
BENCH_CONFIGS = ([dict(load_factor=0.25, keys_per_window=k, grid_rounds=g) for k in (4, 8, 16, 32, 64)
                  for g in (1, 2, 4)]
                 + [dict(load_factor=lf, keys_per_window=32, grid_rounds=1) for lf in (0.35, 0.5, 0.7)]
                 + [dict(load_factor=0.25, keys_per_window=32, grid_rounds=1, split=True)])


@pytest.mark.parametrize("name", ["large", "dna"])
def test_full_size_join_equals_oracle(A, oracle, wl, name):
    import torch
    w = getattr(wl, name)()
    note(f"{name}: R={w.R.n} S={w.S.n} bytes={w.R.nbytes + w.S.nbytes}")
    Rk, Sk = A.DeviceKeys.from_host(w.R), A.DeviceKeys.from_host(w.S)
    expected = int(w.meta["expected_matches"])
    cap = expected + 1024  # the benchmark's capacity
    out = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
    counts = torch.zeros(2, dtype=torch.int64, device="cuda")
    note(f"{name}: oracle signature join")
    want, want_cand = oracle.join_signature(w.R, w.S, cap=cap)
    assert len(want) == expected

    def check(label, **kw):
        counts.zero_()
        A.asj_join(Rk, Sk, out, counts, **kw)
        total, ncand = (int(x) for x in counts.tolist())
        assert total == expected, (label, total)
        got = out[:total].cpu().numpy()
        assert np.array_equal(oracle.sort_pairs(got), want), label
        assert ncand == want_cand, (label, ncand, want_cand)
        assert unique_pairs(got), label

    check("defaults")
    tune = A.autotune(Rk, Sk, out, counts)  # the benchmark's setup; later calls leave the options to the library
    note(f"{name}: autotuner chose {tune}")
    check("autotuned")
    A.autotune_clear()
    for cfg in BENCH_CONFIGS:
        cfg = dict(cfg)
        flags = A.ASJ_PROBE_SPLIT if cfg.pop("split", False) else A.ASJ_PROBE_FUSED
        check(str(cfg), flags=flags | A.ASJ_GLOBAL_TABLES, **cfg)
    note(f"{name}: {len(BENCH_CONFIGS) + 2} configurations equal the oracle (|T|={expected}, candidates={want_cand})")
    rng = np.random.default_rng([17, len(name)])
    for rel, keys in ((w.R, Rk), (w.S, Sk)):
        sig = gpu_signatures(A, keys)
        idx = np.sort(rng.choice(rel.n, size=min(rel.n, 20000), replace=False))
        assert np.array_equal(sig[idx], oracle.signatures(rel.subset(idx)))


def oracle_batch(oracle, b, workers=None):
    """The oracle's signature join of every join of a batch workload, as
    (sorted pairs, candidate count) per join.  Join k is passed as views of
    the batch arena (its offsets slice and row-local ids); the C calls
    release the GIL, so the joins run in a thread pool."""
    import os
    from concurrent.futures import ThreadPoolExecutor

    def one(k):
        r0, r1, s0, s1 = (int(x) for x in (b.r_seg[k], b.r_seg[k + 1], b.s_seg[k], b.s_seg[k + 1]))
        R = (b.R.data, b.R.offsets[r0:r1 + 1], b.R.ids[r0:r1])
        S = (b.S.data, b.S.offsets[s0:s1 + 1], b.S.ids[s0:s1])
        return oracle.join_signature(R, S, cap=(s1 - s0) + 1024)

    workers = workers or max(1, min(16, os.cpu_count() or 1))
    # largest joins first, so the pool does not end on one long join
    order = sorted(range(b.njoins), key=lambda k: -(b.s_seg[k + 1] - b.s_seg[k]))
    with ThreadPoolExecutor(workers) as ex:
        res = dict(zip(order, ex.map(one, order)))
    return [res[k] for k in range(b.njoins)]


def check_batch_output(oracle, b, want, outh, oseg, counts, cands, label):
    rsz, ssz = np.diff(b.r_seg), np.diff(b.s_seg)
    for k in range(b.njoins):
        wp, wc = want[k]
        assert counts[k] == len(wp), (label, k, counts[k], len(wp))
        assert counts[k] <= oseg[k + 1] - oseg[k], (label, k)
        p = outh[oseg[k]:oseg[k] + counts[k]]
        assert ((p[:, 0] >= 0) & (p[:, 0] < rsz[k]) & (p[:, 1] >= 0) & (p[:, 1] < ssz[k])).all(), (label, k)
        assert np.array_equal(oracle.sort_pairs(p), wp), (label, k)
        assert cands[k] == wc, (label, k, cands[k], wc)


def test_full_size_batch_all_joins_equal_oracle(A, oracle, wl):
    """All 256 joins of the full-size batched workload, in the library's
    default configuration and in the autotuner's choice (what the benchmark
    times), each compared pair for pair with the oracle, candidate counts
    included."""
    import torch
    b = wl.batch()
    note(f"batch: joins={b.njoins} R={b.R.n} S={b.S.n} bytes={b.R.nbytes + b.S.nbytes}")
    R, S = A.DeviceKeys.from_host(b.R), A.DeviceKeys.from_host(b.S)
    out, oseg, counts, cands, _ = A.join_batch(R, S, b.r_seg, b.s_seg)
    outh = out.cpu().numpy()
    note("batch: oracle joins")
    want = oracle_batch(oracle, b)
    check_batch_output(oracle, b, want, outh, oseg, counts, cands, "defaults")
    note(f"batch: all {b.njoins} joins equal the oracle; {int(counts.sum())} pairs")
    dev = lambda a: torch.from_numpy(np.asarray(a, dtype=np.int64)).cuda()
    r_seg, s_seg, out_seg = dev(b.r_seg), dev(b.s_seg), dev(oseg)
    J = b.njoins
    tune = A.autotune_batch(R, S, r_seg, s_seg, out, out_seg, torch.zeros(J, dtype=torch.int64, device="cuda"))
    note(f"batch: autotuner chose {tune}")
    cnt = torch.zeros(J, dtype=torch.int64, device="cuda")
    cnd = torch.zeros(J, dtype=torch.int64, device="cuda")
    ws = torch.empty(A.asj_batch_workspace_bytes(J, b.R.n, b.S.n), dtype=torch.uint8, device="cuda")
    out.fill_(-7)
    A.asj_join_batch(R, S, r_seg, s_seg, out, out_seg, cnt, cnd, None, workspace=ws)
    check_batch_output(oracle, b, want, out.cpu().numpy(), oseg, cnt.cpu().numpy(), cnd.cpu().numpy(), "autotuned")
    A.autotune_clear()
    rng = np.random.default_rng(23)
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
    """256 independent tiny joins (R = S = 10k keys of 256 B each, 1.3 GB) in
    one batch, the benchmark's throughput configuration (every join's table
    built in LDS, stated with ASJ_LOCAL_ONLY; options left to the library):
    every join has exactly the
    generator's 2000 matches and equals the oracle pair for pair, candidate
    counts included."""
    J = 256
    parts = [wl.tiny(seed=1 + i) for i in range(J)]
    def cat(rels):
        lens = np.concatenate([r.lengths() for r in rels])
        data = np.concatenate([r.data[:r.offsets[-1]] for r in rels] + [np.zeros(16, np.uint8)])
        off = np.zeros(len(lens) + 1, dtype=np.int64)
        np.cumsum(lens, out=off[1:])
        return wl.Relation(data, off, np.concatenate([r.ids for r in rels]))
    Rf, Sf = cat([p.R for p in parts]), cat([p.S for p in parts])
    r_seg = np.concatenate([[0], np.cumsum([p.R.n for p in parts])]).astype(np.int64)
    s_seg = np.concatenate([[0], np.cumsum([p.S.n for p in parts])]).astype(np.int64)
    b = wl.BatchWorkload(f"tiny x{J}", Rf, Sf, r_seg, s_seg)
    note(f"tiny instances: joins={J} R={Rf.n} S={Sf.n} bytes={Rf.nbytes + Sf.nbytes}")
    R, S = A.DeviceKeys.from_host(Rf), A.DeviceKeys.from_host(Sf)
    want = oracle_batch(oracle, b)
    # as timed: the batch states that every join has an LDS table; and without the statement
    for flags in (A.ASJ_LOCAL_ONLY, 0):
        out, oseg, counts, cands, _ = A.join_batch(R, S, r_seg, s_seg, flags=flags)
        assert (counts == 2000).all()
        check_batch_output(oracle, b, want, out.cpu().numpy(), oseg, counts, cands, f"{b.name} flags={flags:#x}")
    note(f"tiny instances: all {J} joins (2000 pairs each) equal the oracle, with and without ASJ_LOCAL_ONLY")
