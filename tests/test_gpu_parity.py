"""GPU parity: the HIP path against the oracle, through the C interface.

Signatures must be bit-exact (integer work); join outputs must be equal as
multisets of (r_id, s_id) pairs (compared sorted; several orders are
correct); candidate counts must equal the oracle's signature-equal pair
count exactly.
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


def gpu_sigs(A, rel, f=16, nsym=2):
    keys = A.DeviceKeys.from_host(rel)
    out = A.asj_signature(keys, f, nsym).cpu().numpy()
    if f * nsym == 64:  # two words per key, the low word first
        return out.view(np.uint64)
    return out.view(np.uint32).astype(np.uint64)


# fused: asj_join with at most 10240 build rows builds its table in LDS;
# fused_global: the device-memory table for every size
SCHEDULES = ["split", "fused", "fused_global"]


def sched_flag(A, sched):
    return {"split": A.ASJ_PROBE_SPLIT, "fused": A.ASJ_PROBE_FUSED,
            "fused_global": A.ASJ_PROBE_FUSED | A.ASJ_GLOBAL_TABLES}[sched]


def gpu_join(A, R, S, sched=None, **kw):
    if sched is not None:
        kw["flags"] = kw.get("flags", 0) | sched_flag(A, sched)
    Rk, Sk = A.DeviceKeys.from_host(R), A.DeviceKeys.from_host(S)
    pairs, total, ncand = A.join(Rk, Sk, **kw)
    return pairs.cpu().numpy(), total, ncand


def adversarial_keys(rng):
    lens = (list(range(0, 140)) + [255, 256, 257, 511, 512, 513, 1023, 1024, 1025, 2047, 2049, 4095, 4096, 4097,
                                   4159, 4160, 4161, 8191, 8192, 8193, 10000, 12345, 65536, 131067, 131068, 131072])
    keys = []
    for i, L in enumerate(lens):
        kind = i % 4
        if kind == 0:
            keys.append(rng.integers(0, 256, size=L, dtype=np.uint8).tobytes())
        elif kind == 1:
            keys.append(b"\xff" * L)
        elif kind == 2:
            keys.append(bytes(L))
        else:
            keys.append(rng.integers(0x20, 0x7F, size=L, dtype=np.uint8).tobytes())
    return keys


@pytest.mark.parametrize("shift", [0, 1, 2, 3, 5, 15, 16])
@pytest.mark.parametrize("params", [(16, 2), (16, 1), (8, 4), (8, 2), (16, 4)])
def test_signature_bitexact_adversarial(A, oracle, wl, shift, params):
    rng = np.random.default_rng(100 + shift)
    rel = wl.unaligned_copy(wl.from_keys(adversarial_keys(rng)), shift)
    f, nsym = params
    assert np.array_equal(gpu_sigs(A, rel, f, nsym), oracle.signatures(rel, f, nsym))


@pytest.mark.parametrize("name,scale", [("tiny", 1.0), ("large", 0.01), ("dna", 0.004)])
def test_signature_bitexact_workloads(A, oracle, wl, name, scale):
    w = getattr(wl, name)(scale=scale)
    for rel in (w.R, w.S):
        assert np.array_equal(gpu_sigs(A, rel), oracle.signatures(rel))
    assert np.array_equal(gpu_sigs(A, w.S, 16, 4), oracle.signatures(w.S, 16, 4))


def test_signature_bitexact_batch_keys(A, oracle, wl):
    b = wl.batch(scale=0.002, njoins=16)
    assert np.array_equal(gpu_sigs(A, b.S), oracle.signatures(b.S))


def test_signature_many_windows_and_ragged_tail(A, oracle, wl):
    # 64-key windows with every chunk count from 0 to ~70 and a ragged last window
    rng = np.random.default_rng(7)
    lens = rng.integers(0, 4500, size=64 * 37 + 13)
    lens[::5] = rng.integers(0, 65, size=len(lens[::5]))
    keys = [rng.integers(0, 256, size=int(L), dtype=np.uint8).tobytes() for L in lens]
    rel = wl.from_keys(keys)
    assert np.array_equal(gpu_sigs(A, rel), oracle.signatures(rel))


# Keys long enough that a chunk's 64-chunk block index has several octal
# digits (position factors from the device-memory pairs): 12 KB (blocks up
# to 2, the LDS pair alone), 12.3 KB, 1 MB, 3 MB and 20 MB (block index up to
# 5120 = 0o12000), beside short keys, in an unaligned arena.
@pytest.mark.parametrize("params", [(16, 2), (16, 4), (16, 1), (8, 2)])
def test_signature_very_long_keys(A, oracle, wl, params):
    rng = np.random.default_rng(sum(params))
    lens = [12288, 12288 + 5, 3 * 4096 + 64, (1 << 20) + 3, 3 * (1 << 20) + 17, 7, 0, 20 * (1 << 20) + 1, 130]
    keys = [rng.integers(0, 256, size=L, dtype=np.uint8).tobytes() for L in lens]
    rel = wl.unaligned_copy(wl.from_keys(keys), 3)
    f, nsym = params
    assert np.array_equal(gpu_sigs(A, rel, f, nsym), oracle.signatures(rel, f, nsym))


# Above 10240 keys the signature kernel sizes its windows from the keys'
# mean length (4 .. 64 keys, about eight passes of 64 chunks each): mean
# lengths chosen so that each window size is taken, with short keys and
# empty keys mixed in, a ragged last window and an unaligned arena.
@pytest.mark.parametrize("mean,params", [(400, (16, 2)), (1000, (16, 2)), (2000, (16, 4)), (4000, (16, 2)),
                                         (8000, (16, 2)), (2000, (8, 4)), (700, (16, 1))])
def test_signature_every_window_size(A, oracle, wl, mean, params):
    rng = np.random.default_rng(mean + params[1])
    n = 10240 + 1 + int(rng.integers(0, 300))
    lens = rng.integers(mean // 2, mean + mean // 2 + 1, size=n)
    short = rng.uniform(size=n) < 0.05
    lens[short] = rng.integers(0, 70, size=int(short.sum()))
    data = rng.integers(0, 256, size=int(lens.sum()) + 16, dtype=np.uint8)
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    rel = wl.unaligned_copy(wl.Relation(data, off, np.arange(n, dtype=np.int32)), int(mean) % 7)
    f, nsym = params
    assert np.array_equal(gpu_sigs(A, rel, f, nsym), oracle.signatures(rel, f, nsym))


@pytest.mark.parametrize("sched", SCHEDULES)
@pytest.mark.parametrize("seed", range(10))
def test_join_small_random(A, oracle, wl, seed, sched):
    alphabets = [b"ab\x00", b"a", b"\x00", bytes(range(256)), b"xy"]
    w = wl.random_small(seed, m=int(50 + 37 * seed), n=int(70 + 53 * seed), max_len=[1, 3, 9, 40, 300][seed % 5],
                        alphabet=alphabets[seed % 5])
    if seed % 2:
        w.R.ids = (np.random.default_rng(seed).permutation(w.R.n) + 1000).astype(np.int32)
        w.S.ids = (np.random.default_rng(seed + 1).permutation(w.S.n) + 7000).astype(np.int32)
    want = oracle.join_nested(w.R, w.S)
    _, want_cand = oracle.join_signature(w.R, w.S)
    got, total, ncand = gpu_join(A, w.R, w.S, sched=sched)
    assert total == len(want)
    assert np.array_equal(oracle.sort_pairs(got), want)
    assert ncand == want_cand


@pytest.mark.parametrize("sched", SCHEDULES)
@pytest.mark.parametrize("name,scale", [("tiny", 1.0), ("large", 0.02), ("dna", 0.01)])
def test_join_workloads(A, oracle, wl, name, scale, sched):
    w = getattr(wl, name)(scale=scale)
    want, want_cand = oracle.join_signature(w.R, w.S)
    got, total, ncand = gpu_join(A, w.R, w.S, sched=sched)
    assert total == len(want) == w.meta["expected_matches"]
    assert np.array_equal(oracle.sort_pairs(got), want)
    assert ncand == want_cand


def test_join_batch_members(A, oracle, wl):
    b = wl.batch(scale=0.003, njoins=10)
    for k in range(b.njoins):
        j = b.join(k)
        want, want_cand = oracle.join_signature(j.R, j.S)
        got, total, ncand = gpu_join(A, j.R, j.S)
        assert total == len(want)
        assert np.array_equal(oracle.sort_pairs(got), want)
        assert ncand == want_cand


@pytest.mark.parametrize("sched", SCHEDULES)
@pytest.mark.parametrize("seed", range(4))
def test_plain_baseline_join(A, oracle, wl, seed, sched):
    w = wl.random_small(seed, m=300, n=500, max_len=[2, 9, 80, 700][seed], alphabet=b"ab\x00")
    got, total, _ = gpu_join(A, w.R, w.S, sched=sched, flags=A.ASJ_PLAIN)
    want = oracle.join_nested(w.R, w.S)
    assert total == len(want) and np.array_equal(oracle.sort_pairs(got), want)
    t = wl.tiny(scale=0.5)
    got, total, _ = gpu_join(A, t.R, t.S, sched=sched, flags=A.ASJ_PLAIN)
    assert np.array_equal(oracle.sort_pairs(got), oracle.join_hash(t.R, t.S))


@pytest.mark.parametrize("sched", SCHEDULES)
@pytest.mark.parametrize("seed", range(4))
def test_paper_literal_no_verify(A, oracle, wl, seed, sched):
    w = wl.random_small(seed, m=200, n=300, max_len=[2, 6, 30, 3][seed], alphabet=b"a\x00")
    want, want_cand = oracle.join_signature(w.R, w.S, verify=False)
    got, total, ncand = gpu_join(A, w.R, w.S, sched=sched, flags=A.ASJ_NO_VERIFY)
    assert total == len(want) == ncand == want_cand
    assert np.array_equal(oracle.sort_pairs(got), want)


@pytest.mark.parametrize("sched", SCHEDULES)
def test_variant_signature_joins(A, oracle, wl, sched):
    w = wl.random_small(3, m=400, n=600, max_len=50, alphabet=b"ab\x00")
    for f, nsym in ((16, 1), (8, 4), (8, 2)):
        want, want_cand = oracle.join_signature(w.R, w.S, f=f, nsym=nsym)
        got, total, ncand = gpu_join(A, w.R, w.S, sched=sched, f=f, nsym=nsym)
        assert np.array_equal(oracle.sort_pairs(got), want)
        assert ncand == want_cand


@pytest.mark.parametrize("sched", SCHEDULES)
def test_fingerprint_control_equals_oracle(A, oracle, wl, sched):
    """The baseline's key hash stored as a fingerprint: the same exact join;
    its candidates (fingerprint-equal pairs) include every output pair."""
    cases = [wl.random_small(seed, m=300, n=500, max_len=[2, 9, 80, 700][seed], alphabet=b"ab\x00")
             for seed in range(4)]
    cases.append(wl.tiny(scale=0.5))
    cases.append(wl.large(scale=0.002))
    for i, w in enumerate(cases):
        want = oracle.join_hash(w.R, w.S)
        got, total, ncand = gpu_join(A, w.R, w.S, sched=sched, flags=A.ASJ_FINGERPRINT)
        assert total == len(want) and np.array_equal(oracle.sort_pairs(got), want), i
        assert ncand >= total, i
    for bad in (A.ASJ_FINGERPRINT | A.ASJ_PLAIN, A.ASJ_FINGERPRINT | A.ASJ_NO_VERIFY):
        with pytest.raises(A.AsjError) as ei:
            gpu_join(A, cases[0].R, cases[0].S, flags=bad)
        assert ei.value.code == A.ASJ_EINVAL
    b = wl.batch(scale=0.001, njoins=2)
    with pytest.raises(A.AsjError) as ei:
        A.join_batch(A.DeviceKeys.from_host(b.R), A.DeviceKeys.from_host(b.S), b.r_seg, b.s_seg,
                     flags=A.ASJ_FINGERPRINT)
    assert ei.value.code == A.ASJ_EUNSUPPORTED


def test_sig64_joins_equal_oracle(A, oracle, wl):
    """64-bit signatures (f = 16, n = 4; fused schedule): exact pairs, exact
    candidate counts (pairs of equal 64-bit signature), and the paper-literal
    output on signature equality."""
    for seed in range(4):
        w = wl.random_small(seed, m=300 + 50 * seed, n=700, max_len=[2, 9, 70, 300][seed], alphabet=b"ab\x00")
        want, want_cand = oracle.join_signature(w.R, w.S, f=16, nsym=4)
        got, total, ncand = gpu_join(A, w.R, w.S, f=16, nsym=4)
        assert total == len(want) and np.array_equal(oracle.sort_pairs(got), want), seed
        assert ncand == want_cand, seed
        lit, lit_cand = oracle.join_signature(w.R, w.S, f=16, nsym=4, verify=False)
        got, total, ncand = gpu_join(A, w.R, w.S, f=16, nsym=4, flags=A.ASJ_NO_VERIFY)
        assert np.array_equal(oracle.sort_pairs(got), lit) and ncand == lit_cand, seed
        for kind, flag in (("semi", A.ASJ_SEMI), ("anti", A.ASJ_ANTI)):
            got, _, _ = gpu_join(A, w.R, w.S, f=16, nsym=4, flags=flag)
            assert np.array_equal(oracle.sort_pairs(got), oracle.join_variant(w.R, w.S, kind)), (seed, kind)
    t = wl.tiny(scale=0.5)
    got, total, ncand = gpu_join(A, t.R, t.S, f=16, nsym=4)
    assert np.array_equal(oracle.sort_pairs(got), oracle.join_hash(t.R, t.S)) and ncand == total


def test_sig64_separates_two_component_collisions(A, oracle, wl):
    """Keys that differ by a three-symbol Reed-Solomon codeword of the
    two-component code (its generator vanishes at alpha and alpha^2) share
    the {16, 2} signature but not the {16, 4} one: the paper-literal join
    matches them with two components and not with four."""
    import random
    rng = random.Random(5)
    g0, g1 = oracle.gf_exp(16, 3), oracle.gf_exp(16, 1) ^ oracle.gf_exp(16, 2)  # (y + a)(y + a^2), g2 = 1
    base = [rng.randrange(1, 65536) for _ in range(200)]
    key = lambda sy: b"".join(int(v).to_bytes(2, "little") for v in sy)
    variants = []
    for i in (0, 31, 32, 77, 150, 197):  # inside a chunk, across chunk boundaries, at the end
        t = rng.randrange(1, 65536)
        k = list(base)
        k[i] ^= oracle.mul_table(16, g0, t)
        k[i + 1] ^= oracle.mul_table(16, g1, t)
        k[i + 2] ^= t
        variants.append(key(k))
    R, S = wl.from_keys([key(base)]), wl.from_keys([key(base)] + variants)
    s2 = oracle.signatures(S, 16, 2)
    assert (s2 == s2[0]).all() and len(set(oracle.signatures(S, 16, 4).tolist())) == len(variants) + 1
    got, total, ncand = gpu_join(A, R, S, flags=A.ASJ_NO_VERIFY)
    assert total == ncand == len(variants) + 1
    got, total, ncand = gpu_join(A, R, S, flags=A.ASJ_NO_VERIFY, f=16, nsym=4)
    assert total == ncand == 1 and got.tolist() == [[0, 0]]
    assert np.array_equal(gpu_sigs(A, S, 16, 4), oracle.signatures(S, 16, 4))


def test_sig64_unsupported_forms(A, wl):
    import torch
    w = wl.random_small(1, m=20, n=20)
    with pytest.raises(A.AsjError) as ei:
        gpu_join(A, w.R, w.S, sched="split", f=16, nsym=4)
    assert ei.value.code == A.ASJ_EUNSUPPORTED
    b = wl.batch(scale=0.001, njoins=2)
    R, S = A.DeviceKeys.from_host(b.R), A.DeviceKeys.from_host(b.S)
    with pytest.raises(A.AsjError) as ei:
        A.join_batch(R, S, b.r_seg, b.s_seg, f=16, nsym=4)
    assert ei.value.code == A.ASJ_EUNSUPPORTED
    out = torch.empty((64, 2), dtype=torch.int32)
    with pytest.raises(A.AsjError) as ei:
        A.asj_join_host(A.HostKeys.from_host(w.R, pin=False), A.HostKeys.from_host(w.S, pin=False), out,
                        f=16, nsym=4)
    assert ei.value.code == A.ASJ_EUNSUPPORTED


@pytest.mark.parametrize("sched", SCHEDULES)
def test_duplicate_keys_multimap(A, oracle, wl, sched):
    keys_r = [b"k" * 100] * 150 + [b"x" * 7] * 3 + [b""] * 4 + [bytes([i % 7]) * (i % 300) for i in range(500)]
    keys_s = [b"k" * 100] * 40 + [b""] * 5 + [b"x" * 7] + [bytes([i % 5]) * (i % 200) for i in range(700)]
    R, S = wl.from_keys(keys_r), wl.from_keys(keys_s)
    want = oracle.join_hash(R, S)
    got, total, _ = gpu_join(A, R, S, sched=sched, cap=10)  # forces the second call
    assert total == len(want) >= 150 * 40
    assert np.array_equal(oracle.sort_pairs(got), want)


def test_overflow_reports_full_count(A, oracle, wl):
    import torch
    w = wl.tiny(scale=0.3)
    Rk, Sk = A.DeviceKeys.from_host(w.R), A.DeviceKeys.from_host(w.S)
    want = oracle.join_hash(w.R, w.S)
    cap = len(want) // 3
    out = torch.full((cap, 2), -1, dtype=torch.int32, device="cuda")
    counts = torch.zeros(2, dtype=torch.int64, device="cuda")
    A.asj_join(Rk, Sk, out, counts)
    assert int(counts[0]) == len(want)
    part = {tuple(p) for p in out.cpu().numpy().tolist()}
    assert len(part) == cap and part <= {tuple(p) for p in want.tolist()}


def test_empty_relations(A, oracle, wl):
    empty = wl.from_keys([])
    some = wl.from_keys([b"a", b"", b"bb"])
    for R, S in ((empty, some), (some, empty), (empty, empty)):
        got, total, ncand = gpu_join(A, R, S)
        assert total == 0 and len(got) == 0 and ncand == 0
    allempty = wl.from_keys([b""] * 5)
    got, total, _ = gpu_join(A, allempty, wl.from_keys([b""] * 3))
    assert total == 15


def test_build_once_probe_twice_on_two_streams(A, oracle, wl):
    import torch
    w = wl.large(scale=0.005)
    Rk, Sk = A.DeviceKeys.from_host(w.R), A.DeviceKeys.from_host(w.S)
    t = A.asj_build(Rk)
    assert t.status() == A.ASJ_OK
    cap = t.capacity
    assert cap & (cap - 1) == 0 and cap >= 2 * w.R.n
    want = oracle.join_hash(w.R, w.S)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for st in (s1, s2):
        out = torch.empty((len(want) + 10, 2), dtype=torch.int32, device="cuda")
        cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
        A.asj_probe(t, Sk, out, cnt, stream=st)
        outs.append((out, cnt))
    torch.cuda.synchronize()
    for out, cnt in outs:
        n = int(cnt[0])
        assert n == len(want)
        assert np.array_equal(oracle.sort_pairs(out[:n].cpu().numpy()), want)
    t.free()


def test_rejects_bad_parameters(A, wl):
    rel = A.DeviceKeys.from_host(wl.from_keys([b"abc"]))
    with pytest.raises(A.AsjError) as e:
        A.asj_signature(rel, 8, 3)  # valid width, no kernel for it
    assert e.value.code == A.ASJ_EUNSUPPORTED
    with pytest.raises(A.AsjError) as e:
        A.asj_signature(rel, 16, 3)  # 48 bits: valid, no kernel for it
    assert e.value.code == A.ASJ_EUNSUPPORTED
    with pytest.raises(A.AsjError) as e:
        A.asj_signature(rel, 16, 5)  # 80 bits do not fit the 64-bit signature word
    assert e.value.code == A.ASJ_EINVAL
    with pytest.raises(A.AsjError) as e:
        A.asj_signature(rel, 12, 2)
    assert e.value.code == A.ASJ_EINVAL
    with pytest.raises(A.AsjError):
        A.asj_build(rel, load_factor=1.5)
    with pytest.raises(A.AsjError):
        A.asj_build(rel, flags=A.ASJ_PLAIN | A.ASJ_NO_VERIFY)


@pytest.mark.parametrize("sched", SCHEDULES)
def test_grid_rounds_do_not_change_the_output(A, oracle, wl, sched):
    """The probe grid (1 .. 8 rounds of resident blocks) only changes which
    wave takes which window."""
    w = wl.large(scale=0.004)
    want = oracle.join_hash(w.R, w.S)
    for rounds in (1, 2, 3, 8):
        got, total, _ = gpu_join(A, w.R, w.S, sched=sched, grid_rounds=rounds)
        assert total == len(want) and np.array_equal(oracle.sort_pairs(got), want), rounds
    with pytest.raises(A.AsjError) as ei:
        gpu_join(A, w.R, w.S, grid_rounds=9)
    assert ei.value.code == A.ASJ_EINVAL


def test_contradictory_schedule_flags_rejected(A, wl):
    w = wl.random_small(1, m=10, n=10)
    with pytest.raises(A.AsjError):
        gpu_join(A, w.R, w.S, flags=A.ASJ_PROBE_FUSED | A.ASJ_PROBE_SPLIT)


@pytest.mark.parametrize("sched", SCHEDULES)
def test_plain_baseline_long_shared_prefixes(A, oracle, wl, sched):
    """Keys that agree on their first 64 bytes (or more) and differ later, at
    lengths around the chunk boundaries: the plain join's first-chunk compare
    passes them on and the remaining chunks must decide."""
    rng = np.random.default_rng(31)
    prefix = bytes(rng.integers(0, 256, size=300, dtype=np.uint8))
    keys_r, keys_s = [], []
    for i, L in enumerate([1, 63, 64, 65, 100, 127, 128, 129, 191, 192, 193, 300] * 6):
        base = bytearray(prefix[:L])
        base[-1] = i % 256
        keys_r.append(bytes(base))
        near = bytearray(base)
        near[-1] ^= 0x5A  # differs only in its last byte
        keys_s += [bytes(base), bytes(near)]
    R, S = wl.from_keys(keys_r), wl.from_keys(keys_s)
    want = oracle.join_nested(R, S)
    for flags in (A.ASJ_PLAIN, 0):
        got, total, _ = gpu_join(A, R, S, sched=sched, flags=flags)
        assert total == len(want) and np.array_equal(oracle.sort_pairs(got), want)


def is_sorted_pairs(p):
    if len(p) < 2:
        return True
    a = p[:, 0].astype(np.int64) * (1 << 33) + p[:, 1].astype(np.int64)
    return bool((np.diff(a) >= 0).all())


@pytest.mark.parametrize("sched", SCHEDULES)
@pytest.mark.parametrize("seed", range(4))
def test_sorted_output_equals_sorted_oracle(A, oracle, wl, sched, seed):
    """ASJ_SORTED: the pairs come back in (r_id, s_id) order -- compared as
    arrays, with no sorting on the host -- including negative ids, heavy
    duplicates and the two-call pattern."""
    w = wl.random_small(seed, m=300 + 50 * seed, n=900, max_len=[3, 9, 70, 200][seed], alphabet=b"ab\x00")
    rng = np.random.default_rng(seed)
    w.R.ids = (rng.permutation(w.R.n) - w.R.n // 2).astype(np.int32)  # negative and positive ids
    w.S.ids = (rng.permutation(w.S.n) * 7 - 3000).astype(np.int32)
    want = oracle.join_nested(w.R, w.S)
    got, total, _ = gpu_join(A, w.R, w.S, sched=sched, flags=A.ASJ_SORTED, cap=16)
    assert total == len(want)
    assert np.array_equal(got, want)


def test_sorted_output_larger_and_truncated(A, oracle, wl):
    import torch
    w = wl.large(scale=0.02)
    Rk, Sk = A.DeviceKeys.from_host(w.R), A.DeviceKeys.from_host(w.S)
    want = oracle.join_hash(w.R, w.S)
    got, total, _ = A.join(Rk, Sk, flags=A.ASJ_SORTED)
    assert total == len(want) and np.array_equal(got.cpu().numpy(), want)
    # out_cap below |T|: the stored pairs are sorted and belong to T
    cap = len(want) // 3
    out = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    A.asj_join(Rk, Sk, out, cnt, flags=A.ASJ_SORTED)
    assert int(cnt[0]) == len(want)
    part = out.cpu().numpy()
    assert is_sorted_pairs(part)
    key = lambda p: set(map(tuple, p.tolist()))
    assert key(part) <= key(want) and len(key(part)) == cap
    # no result at all
    empty_s = wl.from_keys([b"\x01nothing"] * 10)
    got, total, _ = A.join(Rk, A.DeviceKeys.from_host(empty_s), flags=A.ASJ_SORTED)
    assert total == 0


def test_sorted_not_supported_for_batches(A, wl):
    w = wl.random_small(1, m=10, n=10)
    R, S = A.DeviceKeys.from_host(w.R), A.DeviceKeys.from_host(w.S)
    with pytest.raises(A.AsjError):
        A.join_batch(R, S, [0, w.R.n], [0, w.S.n], flags=A.ASJ_SORTED)


def swapped(wl, rel, at):
    """The relation with offsets[at] and offsets[at + 1] swapped (decreasing,
    every offset still inside the arena)."""
    off = rel.offsets.copy()
    off[at], off[at + 1] = off[at + 1], off[at]
    return wl.Relation(rel.data, off, rel.ids)


@pytest.mark.parametrize("sched", SCHEDULES)
def test_validate_flag(A, oracle, wl, sched):
    import torch
    w = wl.tiny(scale=0.3)
    flags = A.ASJ_VALIDATE | sched_flag(A, sched)
    # valid inputs: the output is unchanged
    got, total, _ = gpu_join(A, w.R, w.S, flags=flags)
    assert np.array_equal(oracle.sort_pairs(got), oracle.join_hash(w.R, w.S))
    # a decreasing probe offset: nothing is joined, |T| = -1
    bad_s = swapped(wl, w.S, 5)
    Rk, Sk = A.DeviceKeys.from_host(w.R), A.DeviceKeys.from_host(bad_s)
    out = torch.empty((w.S.n, 2), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    A.asj_join(Rk, Sk, out, cnt, flags=flags)
    assert int(cnt[0]) == -1
    # a decreasing build offset: the table reports ASJ_EINVAL and probes yield -1
    t = A.asj_build(A.DeviceKeys.from_host(swapped(wl, w.R, 7)), flags=flags)
    assert t.status() == A.ASJ_EINVAL
    A.asj_probe(t, A.DeviceKeys.from_host(w.S), out, cnt)
    assert int(cnt[0]) == -1
    t.free()


def test_validate_flag_batch(A, oracle, wl):
    b = wl.batch(scale=0.002, njoins=6)
    R = A.DeviceKeys.from_host(b.R)
    S_ok = A.DeviceKeys.from_host(b.S)
    out, oseg, counts, _, _ = A.join_batch(R, S_ok, b.r_seg, b.s_seg, flags=A.ASJ_VALIDATE)
    outh = out.cpu().numpy()
    for k in range(b.njoins):
        j = b.join(k)
        assert np.array_equal(oracle.sort_pairs(outh[oseg[k]:oseg[k] + counts[k]]), oracle.join_hash(j.R, j.S))
    S_bad = A.DeviceKeys.from_host(swapped(wl, b.S, 3))
    _, _, counts, _, _ = A.join_batch(R, S_bad, b.r_seg, b.s_seg, flags=A.ASJ_VALIDATE)
    assert (counts == -1).all()


KINDS = {"semi": 0x40, "anti": 0x80, "left": 0x100, "right": 0x800, "full": 0x900}


@pytest.mark.parametrize("sched", SCHEDULES)
@pytest.mark.parametrize("kind", sorted(KINDS))
def test_join_variants_equal_oracle(A, oracle, wl, kind, sched):
    """Semi, anti and left outer joins of the probe relation: exact pair
    multisets against the oracle's definitions, with the signature join, the
    plain join and the paper-literal (unverified) match."""
    for seed in range(3):
        w = wl.random_small(seed, m=150 + 40 * seed, n=300, max_len=[2, 9, 70][seed], alphabet=b"ab\x00")
        got, total, _ = gpu_join(A, w.R, w.S, sched=sched, flags=KINDS[kind])
        want = oracle.join_variant(w.R, w.S, kind)
        assert total == len(want) and np.array_equal(oracle.sort_pairs(got), want), seed
        got, total, _ = gpu_join(A, w.R, w.S, sched=sched, flags=KINDS[kind] | A.ASJ_PLAIN)
        assert np.array_equal(oracle.sort_pairs(got), want), seed
        got, total, _ = gpu_join(A, w.R, w.S, sched=sched, flags=KINDS[kind] | A.ASJ_NO_VERIFY)
        assert np.array_equal(oracle.sort_pairs(got), oracle.join_variant(w.R, w.S, kind, verify=False)), seed
    t = wl.tiny(scale=0.5)
    got, total, _ = gpu_join(A, t.R, t.S, sched=sched, flags=KINDS[kind] | A.ASJ_SORTED)
    assert np.array_equal(got, oracle.join_variant(t.R, t.S, kind))  # sorted on the device


def test_join_variants_batch_and_served(A, oracle, wl):
    import torch
    b = wl.batch(scale=0.002, njoins=8)
    R, S = A.DeviceKeys.from_host(b.R), A.DeviceKeys.from_host(b.S)
    for kind in ("anti", "left", "right", "full"):
        caps = 2 * np.diff(b.s_seg) + np.diff(b.r_seg) + 16
        out, oseg, counts, _, _ = A.join_batch(R, S, b.r_seg, b.s_seg, caps=caps, flags=KINDS[kind])
        outh = out.cpu().numpy()
        for k in range(b.njoins):
            j = b.join(k)
            assert np.array_equal(oracle.sort_pairs(outh[oseg[k]:oseg[k] + counts[k]]),
                                  oracle.join_variant(j.R, j.S, kind)), (kind, k)
    Rs = wl.served_build_side(scale=0.002)
    t = A.asj_build(A.DeviceKeys.from_host(Rs), flags=A.ASJ_SEMI)
    srv = A.Server(t, slots=2)
    reqs = [wl.served_request(Rs, seed=5, request=i, min_size=300, max_size=3000) for i in range(4)]
    bufs = [(torch.from_numpy(q.data).pin_memory(), torch.from_numpy(q.offsets).pin_memory(),
             torch.empty((q.n, 2), dtype=torch.int32).pin_memory()) for q in reqs]
    infos = [srv.wait(srv.submit(d, o, out)) for d, o, out in bufs]
    srv.close()
    for q, x, (_, _, out) in zip(reqs, infos, bufs):
        assert x["status"] == 0
        assert np.array_equal(oracle.sort_pairs(out[:x["count"]].numpy()), oracle.join_variant(Rs, q, "semi"))
    t.free()


def test_two_join_kinds_rejected(A, wl):
    w = wl.random_small(1, m=10, n=10)
    with pytest.raises(A.AsjError):
        gpu_join(A, w.R, w.S, flags=KINDS["semi"] | KINDS["anti"])


@pytest.mark.parametrize("kind", ["right", "full"])
def test_outer_build_side_kinds_rejected_by_server_and_host_join(A, wl, kind):
    """The right and full outer joins list build rows that a call's probe rows
    left unmatched; the server (many overlapping requests on one table) and
    the host-memory join (S in pieces) do not offer them."""
    w = wl.random_small(2, m=50, n=50)
    t = A.asj_build(A.DeviceKeys.from_host(w.R), flags=KINDS[kind])
    with pytest.raises(A.AsjError) as ei:
        A.Server(t, slots=1)
    assert ei.value.code == A.ASJ_EUNSUPPORTED
    t.free()
    import torch
    out = torch.empty((16, 2), dtype=torch.int32).pin_memory()
    with pytest.raises(A.AsjError) as ei:
        A.asj_join_host(A.HostKeys.from_host(w.R), A.HostKeys.from_host(w.S), out, flags=KINDS[kind])
    assert ei.value.code == A.ASJ_EUNSUPPORTED


def test_right_outer_probe_calls_report_their_own_unmatched_rows(A, oracle, wl):
    """One table, two probe relations: each asj_probe call lists the build rows
    that its own probe rows did not match."""
    import torch
    w = wl.random_small(4, m=300, n=200, max_len=6, alphabet=b"ab")
    w2 = wl.random_small(5, m=10, n=150, max_len=6, alphabet=b"ab")
    t = A.asj_build(A.DeviceKeys.from_host(w.R), flags=KINDS["right"])
    for S in (w.S, w2.S, w.S):
        want = oracle.join_variant(w.R, S, "right")
        out = torch.empty((len(want) + 8, 2), dtype=torch.int32, device="cuda")
        cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
        A.asj_probe(t, A.DeviceKeys.from_host(S), out, cnt)
        n = int(cnt[0])
        assert n == len(want)
        assert np.array_equal(oracle.sort_pairs(out[:n].cpu().numpy()), want)
    t.free()


def region_case(wl, case):
    """A build side, its load factor, and a probe side holding every distinct
    build key once (so that a build row missing from the table loses its
    pair) plus 2000 random keys."""
    rng = np.random.default_rng(sum(map(ord, case)))

    def rand(k):
        lens = rng.integers(1, 24, size=k)
        off = np.zeros(k + 1, dtype=np.int64)
        np.cumsum(lens, out=off[1:])
        data = rng.integers(0, 256, size=int(off[-1]), dtype=np.uint8).tobytes()
        return [data[off[i]:off[i + 1]] for i in range(k)]

    rk, lf = {
        # region builds (327680 rows or more)
        "nearly_full": lambda: (rand(524000), 0.9999),                       # 2^19 slots, 512-slot regions
        "one_key": lambda: ([b"same key"] * 6000 + rand(334000), 0.3),       # 2048-slot regions
        "one_key_sparse": lambda: ([b"same key"] * 6000 + rand(334000), 0.08),  # 2^23 slots, 4096-slot regions
        # two-pass builds
        "small_nearly_full": lambda: (rand(16383), 0.9999),
        "small_one_key": lambda: ([b"same key"] * 6000 + rand(3000), 0.5),
        "empty": lambda: ([], 0.5),
    }[case]()
    uniq = list(dict.fromkeys(rk))
    sk = [uniq[i] for i in rng.permutation(len(uniq))] + rand(2000)
    return wl.from_keys(rk), wl.from_keys(sk), lf


_REGION_CASES = {}  # case -> relations, load factor and the oracle's join


@pytest.mark.parametrize("plain", [False, True])
@pytest.mark.parametrize("sched", ["split", "fused_global"])
@pytest.mark.parametrize("case", ["nearly_full", "one_key", "one_key_sparse", "small_nearly_full", "small_one_key",
                                  "empty"])
def test_device_table_every_row_found(A, oracle, wl, case, sched, plain):
    """Device-memory tables of 327680 build rows or more are built region by
    region (rows grouped by the region of their home slot, each region placed
    in LDS); rows whose run leaves their region, or that find its slots all
    taken by others homed there, are placed from their home slot in device
    memory, past the table's end at slot 0.  Smaller tables take the
    two-pass insert.  Nearly full tables, a key repeated beyond a region's
    slots and an empty build side must give the oracle's join and, with
    signatures, its candidate count, with every build key probed."""
    if case not in _REGION_CASES:
        R, S, lf = region_case(wl, case)
        _REGION_CASES[case] = (R, S, lf, oracle.join_signature(R, S))
    R, S, lf, (want, want_cand) = _REGION_CASES[case]
    flags = A.ASJ_PLAIN if plain else 0
    got, total, ncand = gpu_join(A, R, S, sched=sched, flags=flags, load_factor=lf)
    assert total == len(want) and np.array_equal(oracle.sort_pairs(got), want)
    if not plain:
        assert ncand == want_cand
    if case == "one_key" and sched == "split":
        # a build side that fails validation: the region build places no row
        # (but still writes every region), the table reports ASJ_EINVAL and
        # a probe of it yields -1
        t = A.asj_build(A.DeviceKeys.from_host(swapped(wl, R, 1000)), flags=flags | A.ASJ_VALIDATE,
                        load_factor=lf)
        assert t.status() == A.ASJ_EINVAL
        import torch
        out = torch.empty((S.n, 2), dtype=torch.int32, device="cuda")
        cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
        A.asj_probe(t, A.DeviceKeys.from_host(S), out, cnt)
        assert int(cnt[0]) == -1
        t.free()


@pytest.mark.parametrize("m", [10239, 10240, 10241])
def test_single_join_at_the_lds_table_limit(A, oracle, wl, m):
    """asj_join with one build row below, at and above the LDS-table limit
    (10240 rows: a table built in LDS by every probing block; 10241: the
    device-memory table): inner join with candidate counts, and the outer
    kinds whose unmatched build rows come from the per-row match marks,
    with caller ids on both sides."""
    w = wl.random_small(m, m=m, n=12000, alphabet=bytes(range(256)), lengths=[3, 8, 16, 33, 64, 130])
    w.R.ids = (np.random.default_rng(m).permutation(w.R.n) + 500).astype(np.int32)
    w.S.ids = (np.random.default_rng(m + 1).permutation(w.S.n) + 90000).astype(np.int32)
    want, want_cand = oracle.join_signature(w.R, w.S)
    got, total, ncand = gpu_join(A, w.R, w.S)
    assert total == len(want) and ncand == want_cand
    assert np.array_equal(oracle.sort_pairs(got), want)
    for kind in ("left", "right", "full"):
        got, total, _ = gpu_join(A, w.R, w.S, flags=KINDS[kind])
        want = oracle.join_variant(w.R, w.S, kind)
        assert total == len(want) and np.array_equal(oracle.sort_pairs(got), want), kind


# ---------------------------------------------------------------------------
# Arenas without padding: the header promises that `data` needs none (only
# 4-byte words holding key bytes are read), and a key's bytes must be masked
# against whatever follows it.  The keys go into device buffers whose bytes
# before the first key and after offsets[n] are non-zero junk, or into a
# buffer of exactly offsets[n] bytes.
# ---------------------------------------------------------------------------

def junk_keys(A, rel, shift, junk, exact=False):
    import torch
    off = rel.offsets - rel.offsets[0]
    nbytes = int(off[-1])
    body = torch.from_numpy(np.ascontiguousarray(rel.data[rel.offsets[0]:rel.offsets[0] + nbytes]))
    if exact:
        buf = torch.empty(shift + nbytes, dtype=torch.uint8, device="cuda")
    else:
        buf = torch.empty(shift + nbytes + 67, dtype=torch.uint8, device="cuda")
    g = torch.Generator().manual_seed(int(junk))
    buf.copy_(torch.randint(1, 256, (buf.numel(),), dtype=torch.uint8, generator=g))  # never zero
    if nbytes:
        buf[shift:shift + nbytes].copy_(body)
    offs = torch.from_numpy(off + shift).cuda()
    ids = torch.from_numpy(rel.ids).cuda() if rel.ids is not None else None
    return A.DeviceKeys(buf, offs, ids)


@pytest.mark.parametrize("exact", [False, True])
@pytest.mark.parametrize("shift", [0, 1, 3, 6])
@pytest.mark.parametrize("params", [(16, 2), (16, 1), (8, 4), (8, 2), (16, 4)])
def test_signature_no_padding_junk_around_keys(A, oracle, wl, shift, params, exact):
    rng = np.random.default_rng(300 + shift)
    keys = adversarial_keys(rng)[:150] + [b"x" * L for L in (1, 2, 3, 5, 63, 65, 127)]
    rel = wl.from_keys(keys)
    f, nsym = params
    out = A.asj_signature(junk_keys(A, rel, shift, 1000 + shift, exact), f, nsym).cpu().numpy()
    got = out.view(np.uint64) if f * nsym == 64 else out.view(np.uint32).astype(np.uint64)
    assert np.array_equal(got, oracle.signatures(rel, f, nsym))


def junk_join_relations(wl, seed):
    rng = np.random.default_rng([seed, 42])
    def mk(count, max_len):
        lens = rng.integers(0, max_len + 1, size=count)
        short = rng.uniform(size=count) < 0.4
        lens[short] = rng.integers(0, 70, size=int(short.sum()))
        return [rng.integers(0, 3, size=int(L), dtype=np.uint8).tobytes() for L in lens]
    rk = mk(700 + 13 * seed, 300)
    sk = mk(1500 + 29 * seed, 300)
    for i in range(len(sk)):
        if rng.uniform() < 0.35:
            sk[i] = rk[int(rng.integers(0, len(rk)))]
    # the last key of each relation is short, so its tail is read at the arena's end
    rk[-1] = rk[-1][:1 + seed % 60]
    sk[-1] = sk[-1][:2 + seed % 50]
    return wl.from_keys(rk), wl.from_keys(sk)


@pytest.mark.parametrize("exact", [False, True])
@pytest.mark.parametrize("mode", ["split", "fused", "fused_global", "plain", "sig64"])
@pytest.mark.parametrize("seed", range(3))
def test_join_no_padding_junk_around_keys(A, oracle, wl, seed, mode, exact):
    import torch
    R, S = junk_join_relations(wl, seed)
    kw = {}
    if mode == "plain":
        kw["flags"] = A.ASJ_PLAIN
    elif mode == "sig64":
        kw.update(nsym=4, flags=A.ASJ_PROBE_FUSED | A.ASJ_GLOBAL_TABLES)
    else:
        kw["flags"] = sched_flag(A, mode)
    Rk = junk_keys(A, R, 1 + seed, 2000 + seed, exact)
    Sk = junk_keys(A, S, 3 + seed, 3000 + seed, exact)
    pairs, total, ncand = A.join(Rk, Sk, **kw)
    want = oracle.join_nested(R, S)
    assert total == len(want)
    assert np.array_equal(oracle.sort_pairs(pairs.cpu().numpy()), want)
    if mode != "plain":
        _, want_cand = oracle.join_signature(R, S, 16, 4 if mode == "sig64" else 2)
        assert ncand == want_cand


@pytest.mark.parametrize("exact", [False, True])
@pytest.mark.parametrize("flags", ["default", "global", "plain"])
def test_batch_no_padding_junk_around_keys(A, oracle, wl, flags, exact):
    parts = [junk_join_relations(wl, s) for s in range(5)]
    def cat(rels):
        keys = [r.key(k) for r in rels for k in range(r.n)]
        return wl.from_keys(keys, np.concatenate([r.ids for r in rels]))
    Rf, Sf = cat([p[0] for p in parts]), cat([p[1] for p in parts])
    r_seg = np.concatenate([[0], np.cumsum([p[0].n for p in parts])]).astype(np.int64)
    s_seg = np.concatenate([[0], np.cumsum([p[1].n for p in parts])]).astype(np.int64)
    fl = {"default": 0, "global": A.ASJ_GLOBAL_TABLES, "plain": A.ASJ_PLAIN}[flags]
    out, oseg, counts, cands, _ = A.join_batch(junk_keys(A, Rf, 2, 51, exact), junk_keys(A, Sf, 5, 52, exact),
                                               r_seg, s_seg, flags=fl)
    outh = out.cpu().numpy()
    for k, (R, S) in enumerate(parts):
        want, want_cand = oracle.join_signature(R, S)
        assert counts[k] == len(want), k
        assert np.array_equal(oracle.sort_pairs(outh[oseg[k]:oseg[k] + counts[k]]), want), k
        if flags != "plain":
            assert cands[k] == want_cand, k
