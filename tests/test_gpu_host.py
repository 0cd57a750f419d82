"""asj_join_host: relations in host memory, joined within a device-memory
budget -- the build side resident and the probe side streamed (one
partition), or the Grace-style partitioned join (several partitions).

Every output is compared with the oracle's join (exact multisets of
(r_id, s_id) pairs, the join kinds by their definitions); the partitioning
must not change what the join computes.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

KINDS = {"inner": 0, "semi": 0x40, "anti": 0x80, "left": 0x100}


@pytest.fixture(scope="module")
def A():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2411_18183_amd import asjoin as A
    A.lib()
    return A


def host_join(A, R, S, cap=None, pin=True, **kw):
    """One call with the given capacity, else the two-call pattern (the first
    call reports |T|, the second stores every pair)."""
    import torch
    Rh, Sh = A.HostKeys.from_host(R, pin=pin), A.HostKeys.from_host(S, pin=pin)
    fixed = cap is not None
    if cap is None:
        cap = 1024
    out = torch.empty((cap, 2), dtype=torch.int32)
    total, stats = A.asj_join_host(Rh, Sh, out, **kw)
    if total > cap and not fixed:
        cap = total
        out = torch.empty((cap, 2), dtype=torch.int32)
        total2, stats = A.asj_join_host(Rh, Sh, out, **kw)
        assert total2 == total
    return out[:min(total, cap)].numpy(), total, stats


def want_for(oracle, R, S, kind, verify=True):
    if kind == "inner":
        return oracle.join_hash(R, S) if verify else oracle.join_signature(R, S, verify=False)[0]
    return oracle.join_variant(R, S, kind, verify=verify)


@pytest.mark.parametrize("parts", [1, 2, 8, 64])
@pytest.mark.parametrize("kind", sorted(KINDS))
def test_host_join_small_relations(A, oracle, wl, kind, parts):
    """Duplicates, empty keys and NUL bytes; signature, plain and paper-literal matches."""
    for seed in range(3):
        w = wl.random_small(seed, m=150 + 40 * seed, n=300, max_len=[2, 9, 70][seed], alphabet=b"ab\x00")
        print(f"[host] kind={kind} parts={parts} seed={seed}", flush=True)
        got, total, st = host_join(A, w.R, w.S, flags=KINDS[kind], partitions=parts)
        want = want_for(oracle, w.R, w.S, kind)
        assert total == len(want) and np.array_equal(oracle.sort_pairs(got), want), seed
        assert st["partitions"] == parts
        got, total, _ = host_join(A, w.R, w.S, flags=KINDS[kind] | A.ASJ_PLAIN, partitions=parts)
        assert np.array_equal(oracle.sort_pairs(got), want), seed
        got, total, _ = host_join(A, w.R, w.S, flags=KINDS[kind] | A.ASJ_NO_VERIFY, partitions=parts)
        assert np.array_equal(oracle.sort_pairs(got), want_for(oracle, w.R, w.S, kind, verify=False)), seed


@pytest.mark.parametrize("parts", [1, 4])
@pytest.mark.parametrize("sched", ["fused", "split"])
def test_host_join_streams_pieces_within_a_small_budget(A, oracle, wl, parts, sched):
    """R = S = 10k keys of 256 B in arenas that start off the 4-byte grid,
    4 MB of device memory: the probe side goes through in several pieces."""
    w = wl.tiny(scale=1.0)
    R, S = wl.unaligned_copy(w.R, 3), wl.unaligned_copy(w.S, 1)
    flag = {"fused": A.ASJ_PROBE_FUSED, "split": A.ASJ_PROBE_SPLIT}[sched]
    budget = 4 << 20 if parts == 4 else 8 << 20
    print(f"[host] tiny parts={parts} sched={sched} budget={budget}", flush=True)
    got, total, st = host_join(A, R, S, flags=flag, partitions=parts, hbm_budget=budget)
    want = oracle.join_hash(R, S)
    assert total == len(want) == 2000 and np.array_equal(oracle.sort_pairs(got), want)
    assert st["partitions"] == parts and st["pieces"] >= 2 and st["device_peak"] <= budget
    if parts > 1:
        assert st["chunks"] >= 4  # both relations, more than one chunk each
        keys = R.nbytes + S.nbytes
        assert 2 * keys <= st["bytes_h2d"] <= 3 * keys  # partitioning pass + join pass
    got, total, st = host_join(A, R, S, flags=flag | KINDS["anti"], partitions=parts, hbm_budget=budget)
    assert np.array_equal(oracle.sort_pairs(got), oracle.join_variant(R, S, "anti"))


def test_host_join_budget_chooses_partitions(A, oracle, wl):
    """Left to the library, the partition count grows until the largest
    build partition fits half the budget; a roomy budget keeps R resident."""
    w = wl.tiny(scale=1.0)
    want = oracle.join_hash(w.R, w.S)
    got, total, st = host_join(A, w.R, w.S, hbm_budget=3 << 20)
    assert st["partitions"] >= 2 and st["device_peak"] <= 3 << 20
    assert np.array_equal(oracle.sort_pairs(got), want)
    got, total, st = host_join(A, w.R, w.S, hbm_budget=1 << 30)
    assert st["partitions"] == 1 and st["chunks"] == 0 and st["pieces"] == 1
    assert np.array_equal(oracle.sort_pairs(got), want)
    got, total, st = host_join(A, w.R, w.S, pin=False, hbm_budget=3 << 20)  # pageable host memory
    assert np.array_equal(oracle.sort_pairs(got), want)


def test_host_join_edge_cases(A, oracle, wl):
    import torch
    e = wl.from_keys([])
    w = wl.random_small(4, m=60, n=90, max_len=5, alphabet=b"a\x00")
    for parts in (1, 4):
        # empty build side: the inner join is empty, the anti join is every probe row
        got, total, _ = host_join(A, e, w.S, partitions=parts)
        assert total == 0
        got, total, _ = host_join(A, e, w.S, flags=KINDS["anti"], partitions=parts)
        assert np.array_equal(oracle.sort_pairs(got), oracle.join_variant(e, w.S, "anti"))
        # empty probe side, both empty
        assert host_join(A, w.R, e, partitions=parts)[1] == 0
        assert host_join(A, e, e, flags=KINDS["left"], partitions=parts)[1] == 0
        # every key empty: all pairs match
        z = wl.from_keys([b""] * 7)
        got, total, _ = host_join(A, z, z, partitions=parts)
        assert total == 49 and np.array_equal(oracle.sort_pairs(got), oracle.join_hash(z, z))
        # output capacity below |T|: the count is whole, the stored pairs are a subset
        want = oracle.join_hash(w.R, w.S)
        got, total, _ = host_join(A, w.R, w.S, cap=5, partitions=parts)
        assert total == len(want) and len(got) == 5
        wantset = {tuple(p) for p in want.tolist()}
        assert all(tuple(p) in wantset for p in got.tolist())
        got, total, _ = host_join(A, w.R, w.S, cap=0, partitions=parts)
        assert total == len(want)
    # a build side of one repeated key cannot be split by partitioning
    d = wl.from_keys([b"k" * 200] * 3000)
    with pytest.raises(A.AsjError) as ei:
        host_join(A, d, d, cap=16, hbm_budget=1 << 20)
    assert ei.value.code == A.ASJ_ENOMEM
    # sorted output is not offered here
    with pytest.raises(A.AsjError) as ei:
        host_join(A, w.R, w.S, flags=A.ASJ_SORTED)
    assert ei.value.code == A.ASJ_EUNSUPPORTED
    torch.cuda.synchronize()
