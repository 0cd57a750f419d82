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


# fused: joins with at most 10240 build rows get LDS tables (every join in
# these small batches); fused_global: device-memory tables for all
SCHED = {"split": 0x8, "fused": 0x4, "fused_global": 0x4 | 0x400}


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


def region_batch_joins(seed):
    """Build sides whose segments have runs that leave their 4096-slot
    regions: a key repeated 6000 times, a segment about 95% full, an empty
    build side and a small join; every probe side holds each distinct build
    key once (so that a row missing from its table loses its pair) plus
    random keys."""
    rng = np.random.default_rng(seed)

    def rand(k):
        lens = rng.integers(1, 24, size=k)
        off = np.zeros(k + 1, dtype=np.int64)
        np.cumsum(lens, out=off[1:])
        data = rng.integers(0, 256, size=int(off[-1]), dtype=np.uint8).tobytes()
        return [data[off[i]:off[i + 1]] for i in range(k)]

    builds = [[b"same key"] * 6000 + rand(14000), [], rand(5000), rand(31000)]
    joins = []
    for rk in builds:
        uniq = list(dict.fromkeys(rk))
        joins.append((rk, [uniq[i] for i in rng.permutation(len(uniq))] + rand(500)))
    return joins


def test_batch_segment_with_more_regions_than_a_block_counts(A, oracle, wl):
    """A segment of 2^27 slots (700k build rows at load factor 0.01) has
    32768 regions: a partition block counts the first 8192 regions from its
    first row's in LDS and takes one device atomic per row for the others.
    Beside it, a small join; both equal the oracle, every build key probed."""
    rng = np.random.default_rng(77)

    def keys(k):
        lens = rng.integers(1, 24, size=k)
        off = np.zeros(k + 1, dtype=np.int64)
        np.cumsum(lens, out=off[1:])
        data = rng.integers(0, 256, size=int(off[-1]), dtype=np.uint8).tobytes()
        return [data[off[i]:off[i + 1]] for i in range(k)]

    joins = []
    for nr in (700_000, 20_000):
        rk = keys(nr) + [b"hot key"] * 50
        uniq = list(dict.fromkeys(rk))
        joins.append((rk, [uniq[i] for i in rng.permutation(len(uniq))] + keys(1000)))
    R, S, r_seg, s_seg = flatten(wl, joins)
    out, oseg, counts, cands, _ = A.join_batch(A.DeviceKeys.from_host(R), A.DeviceKeys.from_host(S), r_seg, s_seg,
                                               flags=SCHED["fused_global"], load_factor=0.01)
    outh = out.cpu().numpy()
    for k, (rk, sk) in enumerate(joins):
        want, want_cand = oracle.join_signature(wl.from_keys(rk), wl.from_keys(sk))
        got = outh[oseg[k]:oseg[k] + counts[k]]
        assert counts[k] == len(want) and np.array_equal(oracle.sort_pairs(got), want), k
        assert cands[k] == want_cand, k


@pytest.mark.parametrize("plain", [False, True])
@pytest.mark.parametrize("sched", sorted(SCHED))
def test_batch_segments_built_by_regions(A, oracle, wl, sched, plain):
    """Batch segments are built region by region (rows scattered into the
    4096-slot regions of their home slots, each region placed in LDS and
    written whole, the rows that leave their region or find its slots all
    taken placed afterwards from their home slot, wrapping at the segment's
    end).  At load factor 0.95 one segment is about 95% full and another
    holds a key repeated beyond a region's slots; every join must equal the
    oracle's, with every build key probed."""
    joins = region_batch_joins(11)
    R, S, r_seg, s_seg = flatten(wl, joins)
    flags = SCHED[sched] | (A.ASJ_PLAIN if plain else 0)
    out, oseg, counts, cands, _ = A.join_batch(A.DeviceKeys.from_host(R), A.DeviceKeys.from_host(S), r_seg, s_seg,
                                               flags=flags, load_factor=0.95)
    outh = out.cpu().numpy()
    for k, (rk, sk) in enumerate(joins):
        want, want_cand = oracle.join_signature(wl.from_keys(rk), wl.from_keys(sk))
        got = outh[oseg[k]:oseg[k] + counts[k]]
        assert counts[k] == len(want) and np.array_equal(oracle.sort_pairs(got), want), k
        if not plain:
            assert cands[k] == want_cand, k


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_batch_random_shapes_built_by_regions(A, oracle, wl, seed):
    """Seeded batches of 2-40 joins whose build sides are empty, a few rows,
    around the LDS-table limit or up to 60k rows (some with a fifth of their
    rows on three repeated keys), at load factors from 0.25 to 0.97, under
    every schedule: each join equals the oracle's, with its candidate count;
    every distinct build key is probed."""
    rng = np.random.default_rng([seed, 41])

    def keys(k, hot=None, dup=0.0):
        lens = rng.integers(1, 21, size=k)
        off = np.zeros(k + 1, dtype=np.int64)
        np.cumsum(lens, out=off[1:])
        data = rng.integers(0, 256, size=int(off[-1]), dtype=np.uint8).tobytes()
        out = [data[off[i]:off[i + 1]] for i in range(k)]
        for i in np.flatnonzero(rng.uniform(size=k) < dup):
            out[i] = hot[int(rng.integers(0, len(hot)))]
        return out

    joins = []
    for _ in range(int(rng.integers(2, 41))):
        nr = int(rng.choice([0, int(rng.integers(1, 200)), int(rng.integers(5000, 15000)),
                             int(rng.integers(20000, 60000))]))
        rk = keys(nr, keys(3), float(rng.choice([0.0, 0.2])))
        uniq = list(dict.fromkeys(rk))
        joins.append((rk, [uniq[i] for i in rng.permutation(len(uniq))] + keys(int(rng.integers(0, 300)))))
    R, S, r_seg, s_seg = flatten(wl, joins)
    lf = float(rng.choice([0.25, 0.5, 0.9, 0.97]))
    wants = [oracle.join_signature(wl.from_keys(rk), wl.from_keys(sk)) for rk, sk in joins]
    for sched in sorted(SCHED):
        out, oseg, counts, cands, _ = A.join_batch(A.DeviceKeys.from_host(R), A.DeviceKeys.from_host(S), r_seg, s_seg,
                                                   flags=SCHED[sched], load_factor=lf)
        outh = out.cpu().numpy()
        for k, (want, want_cand) in enumerate(wants):
            got = outh[oseg[k]:oseg[k] + counts[k]]
            assert counts[k] == len(want) and np.array_equal(oracle.sort_pairs(got), want), (sched, k)
            assert cands[k] == want_cand, (sched, k)


def concat(wl, parts):
    """Workloads -> one batch: flattened relations (row-local ids) and segments."""
    def cat(rels):
        lens = np.concatenate([r.lengths() for r in rels])
        data = np.concatenate([r.data[:r.offsets[-1]] for r in rels] + [np.zeros(16, np.uint8)])
        off = np.zeros(len(lens) + 1, dtype=np.int64)
        np.cumsum(lens, out=off[1:])
        return wl.Relation(data, off, np.concatenate([r.ids for r in rels]))
    seg = lambda rels: np.concatenate([[0], np.cumsum([r.n for r in rels])]).astype(np.int64)
    return cat([p.R for p in parts]), cat([p.S for p in parts]), seg([p.R for p in parts]), seg([p.S for p in parts])


KINDS = {"inner": 0, "semi": 0x40, "anti": 0x80, "left": 0x100, "right": 0x800, "full": 0x900}


@pytest.mark.parametrize("plain", [False, True])
@pytest.mark.parametrize("kind", sorted(KINDS))
def test_batch_lds_tables_beside_device_tables(A, oracle, wl, kind, plain):
    """Joins on both sides of the LDS-table limit (10240 build rows) in one
    batch, one of them with every key repeated about 20 times on both sides
    (long runs of equal signatures in one bucket), probe sides long enough
    that a join's windows are shared by several blocks: every join equals
    the oracle's, and the run with device-memory tables for all joins."""
    sizes = [(1, 300, 24), (700, 5000, 70), (10239, 12000, 130), (10240, 12000, 9), (10241, 9000, 64),
             (25000, 30000, 33), (64, 64, 200)]
    parts = []
    for i, (m, n, L) in enumerate(sizes):
        alphabet = np.frombuffer(b"ab", dtype=np.uint8) if L == 9 else None  # 512 distinct keys
        parts.append(wl.fixed_length(seed=40 + i, m=m, n=n, key_len=L, copy_frac=0.3, alphabet=alphabet))
    Rf, Sf, r_seg, s_seg = concat(wl, parts)
    R, S = A.DeviceKeys.from_host(Rf), A.DeviceKeys.from_host(Sf)
    flags = KINDS[kind] | (A.ASJ_PLAIN if plain else 0)
    caps = None
    if kind != "inner":
        caps = np.diff(s_seg) + np.diff(r_seg) + 16
    else:
        caps = np.array([21 * n + 64 for _, n, _ in sizes])
    got, oseg, counts, _, _ = A.join_batch(R, S, r_seg, s_seg, caps=caps, flags=flags)
    ref, rseg, rcounts, _, _ = A.join_batch(R, S, r_seg, s_seg, caps=caps, flags=flags | A.ASJ_GLOBAL_TABLES)
    goth, refh = got.cpu().numpy(), ref.cpu().numpy()
    for k, w in enumerate(parts):
        want = oracle.join_nested(w.R, w.S) if kind == "inner" and w.R.n * w.S.n < 4_000_000 else None
        if kind == "inner" and want is None:
            want, _ = oracle.join_signature(w.R, w.S)
        elif kind != "inner":
            want = oracle.join_variant(w.R, w.S, kind)
        mine = oracle.sort_pairs(goth[oseg[k]:oseg[k] + counts[k]])
        assert counts[k] == len(want) and np.array_equal(mine, want), (kind, plain, k)
        assert rcounts[k] == counts[k], (kind, plain, k)
        assert np.array_equal(oracle.sort_pairs(refh[rseg[k]:rseg[k] + rcounts[k]]), mine), (kind, plain, k)


@pytest.mark.parametrize("extra", [0, 0x400])
@pytest.mark.parametrize("kind", [k for k in sorted(KINDS) if k != "inner"])
def test_batch_kinds_with_empty_sides(A, oracle, wl, kind, extra):
    """Semi, anti and outer joins in a batch that opens and ends with empty
    joins and mixes empty build sides, empty probe sides, both empty and a
    join above the LDS-table limit: the rows without a partner (build rows
    found through the segment bounds) go to their own join's output."""
    big_r = [b"%07d" % i for i in range(10300)]
    big_s = [b"%07d" % (3 * i) for i in range(5000)] + [b"q%d" % i for i in range(700)]
    joins = [
        ([], []),
        ([], [b"a", b"b", b"a"]),
        ([b"a", b"b", b"b"], []),
        ([], []),
        ([b"k" * 40] * 3 + [b"", b"z"], [b"k" * 40, b"", b"", b"y"]),
        (big_r, big_s),
        ([b"a"], []),
        ([], [b"a"]),
        ([], []),
    ]
    Rf, Sf, r_seg, s_seg = flatten(wl, joins)
    R, S = A.DeviceKeys.from_host(Rf), A.DeviceKeys.from_host(Sf)
    caps = np.array([len(a) + len(b) + 16 for a, b in joins])
    got, oseg, counts, _, _ = A.join_batch(R, S, r_seg, s_seg, caps=caps, flags=KINDS[kind] | extra)
    goth = got.cpu().numpy()
    for k, (rk, sk) in enumerate(joins):
        want = oracle.join_variant(wl.from_keys(rk), wl.from_keys(sk), kind)
        mine = oracle.sort_pairs(goth[oseg[k]:oseg[k] + counts[k]])
        assert counts[k] == len(want) and np.array_equal(mine, want), (kind, extra, k)


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


@pytest.mark.parametrize("kind", ["inner", "left", "full"])
def test_batch_local_only_flag(A, oracle, wl, kind):
    """ASJ_LOCAL_ONLY skips the device-memory table build: a batch whose
    joins all have at most 10240 build rows gives the oracle's output with
    it; one join above the limit fails the whole call on the device (every
    count -1), and the flag is refused beside the split schedule or
    device-memory tables."""
    sizes = [(1, 300, 24), (700, 5000, 70), (10240, 12000, 130), (0, 50, 8), (64, 0, 200), (5000, 5000, 9)]
    parts = [wl.fixed_length(seed=70 + i, m=m, n=n, key_len=L, copy_frac=0.3 if m else 0.0)
             for i, (m, n, L) in enumerate(sizes)]
    Rf, Sf, r_seg, s_seg = concat(wl, parts)
    R, S = A.DeviceKeys.from_host(Rf), A.DeviceKeys.from_host(Sf)
    flags = KINDS[kind] | A.ASJ_LOCAL_ONLY
    caps = np.diff(s_seg) + np.diff(r_seg) + 16
    got, oseg, counts, cands, _ = A.join_batch(R, S, r_seg, s_seg, caps=caps, flags=flags)
    goth = got.cpu().numpy()
    for k, w in enumerate(parts):
        want = oracle.join_variant(w.R, w.S, kind) if kind != "inner" else oracle.join_signature(w.R, w.S)[0]
        assert counts[k] == len(want), (kind, k)
        assert np.array_equal(oracle.sort_pairs(goth[oseg[k]:oseg[k] + counts[k]]), want), (kind, k)
    if kind == "inner":
        assert all(cands[k] == oracle.join_signature(w.R, w.S)[1] for k, w in enumerate(parts))
    big = parts + [wl.fixed_length(seed=90, m=10241, n=2000, key_len=40, copy_frac=0.3)]
    Rb, Sb, rb_seg, sb_seg = concat(wl, big)
    _, _, bcounts, _, _ = A.join_batch(A.DeviceKeys.from_host(Rb), A.DeviceKeys.from_host(Sb), rb_seg, sb_seg,
                                        flags=flags)
    assert (bcounts == -1).all()
    for extra in (A.ASJ_GLOBAL_TABLES, A.ASJ_PROBE_SPLIT):
        with pytest.raises(A.AsjError):
            A.join_batch(R, S, r_seg, s_seg, caps=caps, flags=flags | extra)


def test_batch_local_only_workspace(A, oracle, wl):
    """A batch that states ASJ_LOCAL_ONLY builds no device table, so its
    workspace needs no table-build scratch: asj_batch_workspace_bytes gives
    less with the flag, a caller workspace of exactly that size serves the
    flagged batch (equal to the oracle), and the same batch without the flag
    refuses it as too small."""
    import torch
    parts = [wl.fixed_length(seed=110 + i, m=m, n=n, key_len=L, copy_frac=0.3)
             for i, (m, n, L) in enumerate([(3000, 4000, 20), (10240, 9000, 64), (500, 800, 9)])]
    Rf, Sf, r_seg, s_seg = concat(wl, parts)
    R, S = A.DeviceKeys.from_host(Rf), A.DeviceKeys.from_host(Sf)
    J, opts = len(parts), dict(load_factor=0.5, keys_per_window=32)
    small = A.asj_batch_workspace_bytes(J, R.n, S.n, flags=A.ASJ_LOCAL_ONLY, **opts)
    assert small < A.asj_batch_workspace_bytes(J, R.n, S.n, **opts)
    dev = lambda a: torch.from_numpy(np.asarray(a, dtype=np.int64)).cuda()
    caps = np.diff(s_seg) + 16
    oseg = np.concatenate([[0], np.cumsum(caps)])
    out = torch.empty((int(oseg[-1]), 2), dtype=torch.int32, device="cuda")
    counts = torch.zeros(J, dtype=torch.int64, device="cuda")
    ws = torch.empty(small, dtype=torch.uint8, device="cuda")
    A.asj_join_batch(R, S, dev(r_seg), dev(s_seg), out, dev(oseg), counts, workspace=ws, flags=A.ASJ_LOCAL_ONLY,
                     **opts)
    c, outh = counts.cpu().numpy(), out.cpu().numpy()
    for k, w in enumerate(parts):
        want = oracle.join_signature(w.R, w.S)[0]
        assert c[k] == len(want) and np.array_equal(oracle.sort_pairs(outh[oseg[k]:oseg[k] + c[k]]), want), k
    with pytest.raises(A.AsjError):
        A.asj_join_batch(R, S, dev(r_seg), dev(s_seg), out, dev(oseg), counts, workspace=ws, **opts)


@pytest.mark.parametrize("sig", [(16, 1), (8, 2), (8, 4)])
@pytest.mark.parametrize("verify", [True, False])
def test_batch_lds_tables_other_signatures(A, oracle, wl, sig, verify):
    """Every signature width the batches offer, on LDS tables and on
    device-memory tables, at several window sizes and grids: pairs and
    candidate counts equal the oracle's signature join with the same
    parameters (with verify=False, the paper-literal signature-equal pairs)."""
    f, nsym = sig
    parts = [wl.random_small(60 + s, m=200 + 150 * s, n=900 + 100 * s, max_len=[3, 12, 70, 200][s % 4],
                             alphabet=b"abc\x00") for s in range(5)]
    Rf, Sf, r_seg, s_seg = concat(wl, parts)
    R, S = A.DeviceKeys.from_host(Rf), A.DeviceKeys.from_host(Sf)
    flags = 0 if verify else A.ASJ_NO_VERIFY
    wants = [oracle.join_signature(w.R, w.S, f=f, nsym=nsym, verify=verify) for w in parts]
    for extra, kpw, rounds in ((0, 64, 1), (0, 16, 2), (A.ASJ_GLOBAL_TABLES, 32, 4)):
        out, oseg, counts, cands, _ = A.join_batch(R, S, r_seg, s_seg, f=f, nsym=nsym, flags=flags | extra,
                                                   keys_per_window=kpw, grid_rounds=rounds,
                                                   caps=np.array([len(w[0]) + 16 for w in wants]))
        outh = out.cpu().numpy()
        for k, (want, want_cand) in enumerate(wants):
            assert counts[k] == len(want), (extra, kpw, k)
            assert np.array_equal(oracle.sort_pairs(outh[oseg[k]:oseg[k] + counts[k]]), want), (extra, kpw, k)
            assert cands[k] == want_cand, (extra, kpw, k)


@pytest.mark.parametrize("njoins", [12, 40])
@pytest.mark.parametrize("extra", [0, 0x400, 0x800])
def test_batch_graph_replays_equal_eager(A, oracle, wl, extra, njoins):
    """A batch call with a caller workspace, captured into a HIP graph and
    replayed three times with eager work (another batch on other inputs, a
    torch op) and synchronizations between the replays: every replay leaves
    the eager call's counts and pairs (LDS tables, device-memory tables, and
    the right outer join's unmatched-build kernel)."""
    import torch
    b = wl.batch(scale=0.003, njoins=njoins)
    other = wl.batch(seed=9, scale=0.002, njoins=5)
    R, S = A.DeviceKeys.from_host(b.R), A.DeviceKeys.from_host(b.S)
    R2, S2 = A.DeviceKeys.from_host(other.R), A.DeviceKeys.from_host(other.S)
    _, oseg, counts, _, _ = A.join_batch(R, S, b.r_seg, b.s_seg, flags=extra,
                                         caps=np.diff(b.s_seg) + np.diff(b.r_seg) + 16)
    J = b.njoins
    dev = lambda a: torch.from_numpy(np.asarray(a, dtype=np.int64)).cuda()
    r_seg, s_seg, out_seg = dev(b.r_seg), dev(b.s_seg), dev(oseg)
    ws = torch.empty(A.asj_batch_workspace_bytes(J, b.R.n, b.S.n, flags=extra), dtype=torch.uint8, device="cuda")
    out = torch.full((int(oseg[-1]), 2), -7, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(J, dtype=torch.int64, device="cuda")
    call = lambda: A.asj_join_batch(R, S, r_seg, s_seg, out, out_seg, cnt, None, None, workspace=ws, flags=extra)
    call()
    torch.cuda.synchronize()
    eager_cnt = cnt.cpu().numpy().copy()
    eager = [oracle.sort_pairs(out[oseg[k]:oseg[k] + eager_cnt[k]].cpu().numpy()) for k in range(J)]
    assert (eager_cnt == counts).all()
    st = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=st):
        call()
    for rep in range(3):
        out.fill_(-7)
        cnt.zero_()
        A.join_batch(R2, S2, other.r_seg, other.s_seg)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        c = cnt.cpu().numpy()
        assert (c == eager_cnt).all(), rep
        for k in range(J):
            assert np.array_equal(oracle.sort_pairs(out[oseg[k]:oseg[k] + c[k]].cpu().numpy()), eager[k]), (rep, k)


def test_batch_thousands_of_tiny_joins(A, oracle, wl):
    """3000 joins of 0-6 rows each (more joins than one plan-kernel pass of
    1024, many joins per block share, empty build and probe sides): every
    join equals the oracle's, with LDS tables and with device-memory tables."""
    rng = np.random.default_rng(77)
    alphabet = [b"", b"a", b"b", b"ab", b"ba", b"abc"]
    joins = []
    for _ in range(3000):
        m, n = int(rng.integers(0, 7)), int(rng.integers(0, 7))
        joins.append(([alphabet[i] for i in rng.integers(0, len(alphabet), m)],
                      [alphabet[i] for i in rng.integers(0, len(alphabet), n)]))
    Rf, Sf, r_seg, s_seg = flatten(wl, joins)
    R, S = A.DeviceKeys.from_host(Rf), A.DeviceKeys.from_host(Sf)
    caps = np.array([max(1, len(a) * len(b)) for a, b in joins])
    for extra in (0, A.ASJ_GLOBAL_TABLES):
        out, oseg, counts, _, _ = A.join_batch(R, S, r_seg, s_seg, caps=caps, flags=extra)
        outh = out.cpu().numpy()
        for k, (rk, sk) in enumerate(joins):
            want = sorted((i, j) for j, s in enumerate(sk) for i, r in enumerate(rk) if r == s)
            got = sorted(map(tuple, outh[oseg[k]:oseg[k] + counts[k]].tolist()))
            assert counts[k] == len(want) and got == want, (extra, k)
