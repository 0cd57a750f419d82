"""Pins for the oracle: checks against what the paper and the mathematics fix.

The paper prints no worked signature value, so the oracle is pinned by
hand-derived closed forms (tests/golden/closed_forms.txt), by the field
axioms and the primitivity of alpha (Section 3.1), by the change-detection
guarantee the paper states for n-symbol signatures (Section 3.1), by
Reed-Solomon codewords (the signature is P(alpha^j), so multiples of
prod_j (y + alpha^j) sign to zero), and by brute-force joins on tiny inputs
(Section 2 and Section 3.2).
"""
import os
import random

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "closed_forms.txt")
METHODS = (0, 1, 2)


def load_golden():
    exps, sigs = [], []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if not line:
                continue
            p = line.split()
            if p[0] == "exp":
                exps.append((int(p[1]), int(p[2]), int(p[3], 16)))
            elif p[0] == "sig":
                key = b"" if p[3] == "-" else bytes.fromhex(p[3])
                sigs.append((int(p[1]), int(p[2]), key, int(p[4], 16)))
    return exps, sigs


# --- a third GF multiply, written here only to build test inputs (codewords)
def py_gf_mul(a, b, f=16):
    poly = 0x1100B if f == 16 else 0x11D
    r = 0
    while b:
        if b & 1:
            r ^= a
        b >>= 1
        a <<= 1
        if a >> f:
            a ^= poly
    return r


def py_poly_mul(p, q, f=16):
    out = [0] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            out[i + j] ^= py_gf_mul(a, b, f)
    return out


def py_alpha_pow(e, f=16):
    v = 1
    for _ in range(e):
        v = py_gf_mul(v, 2, f)
    return v


def symbols_to_key(sym, f=16):
    if f == 8:
        return bytes(sym)
    return b"".join(int(s).to_bytes(2, "little") for s in sym)


def key_to_symbols(key):
    if len(key) % 2:
        key = key + b"\x00"
    return [key[2 * i] | (key[2 * i + 1] << 8) for i in range(len(key) // 2)]


# ---------------------------------------------------------------------------
# field (Section 3.1)
# ---------------------------------------------------------------------------

def test_golden_field_powers(oracle):
    exps, _ = load_golden()
    assert exps
    for f, e, want in exps:
        assert oracle.gf_exp(f, e) == want, (f, e)


def test_alpha_is_primitive(oracle):
    # every non-zero element is a power of alpha (Section 3.1)
    assert oracle.alpha_order(16) == 65535
    assert oracle.alpha_order(8) == 255


def test_log_antilog_inverse_gf16(oracle):
    L = oracle.lib()
    seen = set()
    for v in range(1, 65536):
        e = L.or_gf_log(16, v)
        assert L.or_gf_exp(16, e) == v
        seen.add(e)
    assert len(seen) == 65535


def test_table_multiply_equals_clmul_gf8_exhaustive(oracle):
    L = oracle.lib()
    for a in range(256):
        for b in range(256):
            assert L.or_mul_table(8, a, b) == L.or_mul_clmul(8, a, b)


def test_table_multiply_equals_clmul_gf16(oracle):
    L = oracle.lib()
    rng = random.Random(11)
    edges = [0, 1, 2, 0x8805, 0x8000, 0xFFFF, 0x100B]
    pairs = [(a, b) for a in edges for b in edges] + [(rng.randrange(65536), rng.randrange(65536)) for _ in range(100000)]
    for a, b in pairs:
        assert L.or_mul_table(16, a, b) == L.or_mul_clmul(16, a, b), (a, b)


def test_clmul_matches_independent_python_multiply(oracle):
    rng = random.Random(12)
    for _ in range(3000):
        a, b = rng.randrange(65536), rng.randrange(65536)
        assert oracle.mul_clmul(16, a, b) == py_gf_mul(a, b, 16)
        a8, b8 = a & 0xFF, b & 0xFF
        assert oracle.mul_clmul(8, a8, b8) == py_gf_mul(a8, b8, 8)


def test_field_axioms(oracle):
    mul = lambda a, b: oracle.mul_table(16, a, b)
    rng = random.Random(13)
    for _ in range(5000):
        a, b, c = (rng.randrange(65536) for _ in range(3))
        assert mul(a, b) == mul(b, a)
        assert mul(mul(a, b), c) == mul(a, mul(b, c))
        assert mul(a, b ^ c) == mul(a, b) ^ mul(a, c)
        assert mul(a, 1) == a and mul(a, 0) == 0
        if a:
            inv = oracle.gf_exp(16, (65535 - oracle.gf_log(16, a)) % 65535)
            assert mul(a, inv) == 1


# ---------------------------------------------------------------------------
# signature (Section 3.1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("method", METHODS)
def test_golden_signatures(oracle, method):
    _, sigs = load_golden()
    assert sigs
    for f, nsym, key, want in sigs:
        assert oracle.signature(key, f, nsym, method) == want, (f, nsym, key.hex(), method)


@pytest.mark.parametrize("f,nsym", [(16, 2), (16, 4), (8, 4), (8, 2), (16, 1)])
def test_three_formulations_agree(oracle, f, nsym):
    rng = np.random.default_rng(14)
    keys = [rng.integers(0, 256, size=int(L), dtype=np.uint8).tobytes()
            for L in list(range(0, 40)) + list(rng.integers(40, 3000, size=60))]
    a = oracle.signatures(keys, f, nsym, 0)
    b = oracle.signatures(keys, f, nsym, 1)
    c = oracle.signatures(keys, f, nsym, 2)
    assert (a == b).all() and (a == c).all()


def test_zero_symbols_do_not_change_the_signature(oracle):
    rng = np.random.default_rng(15)
    for L in range(0, 64):
        k = rng.integers(0, 256, size=L, dtype=np.uint8).tobytes()
        pad = b"\x00" * (2 if L % 2 == 0 else 1)
        assert oracle.signature(k) == oracle.signature(k + pad)
        assert oracle.signature(k) == oracle.signature(k + pad + b"\x00\x00" * 7)


def test_linearity_under_xor(oracle):
    rng = np.random.default_rng(16)
    for L in list(range(0, 50)) + [255, 256, 1000, 4097]:
        p = rng.integers(0, 256, size=L, dtype=np.uint8)
        q = rng.integers(0, 256, size=L, dtype=np.uint8)
        for f, nsym in ((16, 2), (8, 4), (16, 4)):
            sp = oracle.signature(p.tobytes(), f, nsym)
            sq = oracle.signature(q.tobytes(), f, nsym)
            assert oracle.signature((p ^ q).tobytes(), f, nsym) == sp ^ sq


def test_concatenation_identity(oracle):
    # sig_j(P || Q) = sig_j(P) + alpha^(j |P|) sig_j(Q), |P| in symbols (P of even byte length)
    rng = np.random.default_rng(17)
    for _ in range(200):
        lp = 2 * int(rng.integers(0, 300))
        lq = int(rng.integers(0, 300))
        P = rng.integers(0, 256, size=lp, dtype=np.uint8).tobytes()
        Q = rng.integers(0, 256, size=lq, dtype=np.uint8).tobytes()
        s = oracle.signature(P + Q)
        sp, sq = oracle.signature(P), oracle.signature(Q)
        for j in (1, 2):
            comp = lambda v: (v >> (16 * (j - 1))) & 0xFFFF
            shift = oracle.gf_exp(16, j * (lp // 2))
            assert comp(s) == comp(sp) ^ py_gf_mul(comp(sq), shift)


def test_single_symbol_closed_form(oracle):
    rng = random.Random(18)
    for _ in range(300):
        i = rng.randrange(0, 200)
        p = rng.randrange(1, 65536)
        key = symbols_to_key([0] * i + [p])
        want = py_gf_mul(p, py_alpha_pow(i)) | (py_gf_mul(p, py_alpha_pow(2 * i)) << 16)
        assert oracle.signature(key) == want


def test_detects_every_one_symbol_change(oracle):
    # Section 3.1: any change of up to n symbols is detected with certainty
    rng = random.Random(19)
    base = [rng.randrange(65536) for _ in range(64)]
    s0 = oracle.signature(symbols_to_key(base))
    keys = []
    for i in range(64):
        for _ in range(4):
            k = list(base)
            k[i] ^= rng.randrange(1, 65536)
            keys.append(symbols_to_key(k))
    sigs = oracle.signatures(keys)
    assert (sigs != s0).all()


def test_detects_every_two_symbol_change(oracle):
    rng = random.Random(20)
    base = [rng.randrange(65536) for _ in range(40)]
    s0 = oracle.signature(symbols_to_key(base))
    keys = []
    for i in range(40):
        for i2 in range(i + 1, 40):
            k = list(base)
            k[i] ^= rng.randrange(1, 65536)
            k[i2] ^= rng.randrange(1, 65536)
            keys.append(symbols_to_key(k))
    assert (oracle.signatures(keys) != s0).all()


def test_four_symbol_signature_detects_four_changes(oracle):
    rng = random.Random(21)
    base = [rng.randrange(65536) for _ in range(12)]
    s0 = oracle.signature(symbols_to_key(base), 16, 4)
    import itertools
    keys = []
    for pos in itertools.combinations(range(12), 4):
        k = list(base)
        for i in pos:
            k[i] ^= rng.randrange(1, 65536)
        keys.append(symbols_to_key(k))
    assert (oracle.signatures(keys, 16, 4) != s0).all()


@pytest.mark.parametrize("nsym", [1, 2, 3, 4])
def test_reed_solomon_codewords_sign_to_zero(oracle, nsym):
    # component j is P(alpha^j); a multiple of prod_j (y + alpha^j) vanishes at every alpha^j
    rng = random.Random(22 + nsym)
    gen = [1]
    for j in range(1, nsym + 1):
        gen = py_poly_mul(gen, [py_alpha_pow(j), 1])
    for _ in range(20):
        q = [rng.randrange(65536) for _ in range(rng.randrange(1, 60))]
        cw = py_poly_mul(q, gen)
        key = symbols_to_key(cw)
        assert oracle.signature(key, 16, nsym) == 0
        p = [rng.randrange(65536) for _ in range(len(cw))]
        pk = symbols_to_key(p)
        mixed = symbols_to_key([a ^ b for a, b in zip(p, cw)])
        assert oracle.signature(mixed, 16, nsym) == oracle.signature(pk, 16, nsym)


def test_bound_is_tight_three_symbol_change_can_collide(oracle):
    # (y + alpha)(y + alpha^2) has three non-zero coefficients: adding it to
    # a key changes 3 symbols and keeps the 2-symbol signature.
    gen = py_poly_mul([py_alpha_pow(1), 1], [py_alpha_pow(2), 1])
    assert all(g != 0 for g in gen) and len(gen) == 3
    base = list(range(1, 21))
    for off in (0, 5, 17):
        changed = list(base)
        for i, g in enumerate(gen):
            changed[off + i] ^= g
        assert oracle.signature(symbols_to_key(changed)) == oracle.signature(symbols_to_key(base))


def test_byte_order_reading(oracle):
    # a symbol is the little-endian pair (byte 2i, byte 2i+1)
    for v in (0x0102, 0xABCD, 0x00FF, 0xFF00):
        k = v.to_bytes(2, "little")
        assert oracle.signature(k) == v | (v << 16)


# ---------------------------------------------------------------------------
# joins (Section 2, Section 3.2)
# ---------------------------------------------------------------------------

def brute_sig_pairs(oracle, R, S, f=16, nsym=2):
    sr = oracle.signatures(R, f, nsym)
    ss = oracle.signatures(S, f, nsym)
    a, b = np.nonzero(sr[:, None] == ss[None, :])
    rid, sid = R.ids[a], S.ids[b]
    return oracle.sort_pairs(np.stack([rid, sid], axis=1) if len(a) else np.zeros((0, 2), np.int32))


@pytest.mark.parametrize("seed", range(12))
def test_joins_agree_on_small_random_inputs(oracle, wl, seed):
    alphabets = [b"ab\x00", b"a", b"\x00", bytes(range(256))]
    w = wl.random_small(seed, m=int(20 + 7 * seed), n=int(30 + 11 * seed), max_len=[0, 3, 9, 40][seed % 4] or 1,
                        alphabet=alphabets[seed % 4])
    R, S = w.R, w.S
    if seed % 3 == 1:  # permuted ids
        R.ids = np.random.default_rng(seed).permutation(R.n).astype(np.int32) + 1000
        S.ids = np.random.default_rng(seed + 1).permutation(S.n).astype(np.int32) + 5000
    nested = oracle.join_nested(R, S)
    hashed = oracle.join_hash(R, S)
    sig, ncand = oracle.join_signature(R, S)
    assert np.array_equal(nested, hashed)
    assert np.array_equal(nested, sig)
    literal, ncand2 = oracle.join_signature(R, S, verify=False)
    brute = brute_sig_pairs(oracle, R, S)
    assert np.array_equal(literal, brute)
    assert ncand == ncand2 == len(brute)
    # the exact join is a sub-multiset of the paper-literal output
    lit = {tuple(p) for p in literal.tolist()}
    assert all(tuple(p) in lit for p in nested.tolist())


def test_literal_join_differs_on_trailing_nul(oracle, wl):
    # reading: zero symbols contribute nothing, so "ab" and "ab\0\0" share a
    # signature; only byte verification separates them
    R = wl.from_keys([b"ab", b"", b"\x00\x00"])
    S = wl.from_keys([b"ab\x00\x00", b"", b"ab"])
    exact, ncand = oracle.join_signature(R, S)
    literal, _ = oracle.join_signature(R, S, verify=False)
    assert exact.tolist() == [[0, 2], [1, 1]]
    assert len(literal) > len(exact)
    assert ncand == len(literal)


def test_tiny_workload_ground_truth(oracle, wl):
    w = wl.tiny()
    pairs, ncand = oracle.join_signature(w.R, w.S)
    assert len(pairs) == 2000 == w.meta["expected_matches"]
    assert np.array_equal(pairs, oracle.join_hash(w.R, w.S))
    assert ncand >= 2000
    # every matched S row is one of the copied rows and holds its source bytes
    for r, s in pairs[:50].tolist():
        assert w.R.key(r) == w.S.key(s)


def test_large_workload_ground_truth_scaled(oracle, wl):
    w = wl.large(scale=0.005)
    pairs, _ = oracle.join_signature(w.R, w.S)
    assert len(pairs) == w.meta["expected_matches"]
    assert np.array_equal(pairs, oracle.join_hash(w.R, w.S))
    lens = w.R.lengths()
    assert lens.min() >= 64 and lens.max() <= 4096
    assert all(w.R.key(k)[:48] == w.R.key(0)[:48] for k in range(0, w.R.n, 97))


def test_dna_workload_ground_truth_scaled(oracle, wl):
    w = wl.dna(scale=0.004)
    pairs, ncand = oracle.join_signature(w.R, w.S)
    assert len(pairs) == w.meta["expected_matches"]
    assert np.array_equal(pairs, oracle.join_hash(w.R, w.S))
    # a near-duplicate differs from its source in exactly one byte, hence in
    # one symbol, so it can never share the source's signature (Section 3.1)
    kind, src = w.meta["kind"], w.meta["src"]
    near = np.flatnonzero(kind == 2)
    ss = oracle.signatures(w.S.subset(near))
    sr = oracle.signatures(w.R.subset(src[near]))
    assert (ss != sr).all()
    for t in near[:200]:
        a, b = np.frombuffer(w.S.key(t), np.uint8), np.frombuffer(w.R.key(src[t]), np.uint8)
        assert len(a) == len(b) and int((a != b).sum()) == 1


def test_batch_workload_joins_scaled(oracle, wl):
    b = wl.batch(scale=0.002, njoins=12)
    for k in range(b.njoins):
        j = b.join(k)
        pairs, _ = oracle.join_signature(j.R, j.S)
        assert np.array_equal(pairs, oracle.join_hash(j.R, j.S))
        assert len(pairs) >= int(0.1 * j.S.n) or j.S.n < 40


def test_fixed_length_workload_structure(oracle, wl):
    w = wl.fixed_length(seed=3, m=500, n=2000, key_len=9)
    assert (w.R.lengths() == 9).all() and (w.S.lengths() == 9).all()
    assert w.meta["copies"] == 400
    pairs = oracle.join_hash(w.R, w.S)
    assert len(pairs) >= 400  # every copy matches its source row (more only through equal random keys)


def _brute_variant(R_keys, S_keys, S_ids, kind):
    """Semi / anti / left, right and full outer join by explicit Python loops
    over the keys (build ids = build row indexes)."""
    out = []
    for s, sid in zip(S_keys, S_ids):
        hits = [r for r, rk in enumerate(R_keys) if rk == s]
        if kind == "semi" and hits:
            out.append((-1, sid))
        elif kind in ("anti", "left", "full") and not hits:
            out.append((-1, sid))
        if kind in ("left", "right", "full"):
            out += [(r, sid) for r in hits]
    if kind in ("right", "full"):
        out += [(r, -1) for r, rk in enumerate(R_keys) if rk not in S_keys]
    return sorted(out)


@pytest.mark.parametrize("seed", range(5))
def test_join_variants_equal_brute_force(oracle, wl, seed):
    w = wl.random_small(seed, m=40 + 7 * seed, n=60 + 5 * seed, max_len=[2, 5, 9, 30, 3][seed], alphabet=b"ab\x00")
    R_keys = [w.R.key(i) for i in range(w.R.n)]
    S_keys = [w.S.key(i) for i in range(w.S.n)]
    S_ids = [int(x) for x in w.S.ids]
    assert [int(x) for x in w.R.ids] == list(range(w.R.n))  # build ids are row indexes here
    for kind in ("semi", "anti", "left", "right", "full"):
        got = [tuple(map(int, p)) for p in oracle.join_variant(w.R, w.S, kind)]
        assert got == _brute_variant(R_keys, S_keys, S_ids, kind), kind


def test_join_variant_invariants(oracle, wl):
    w = wl.tiny(scale=0.2)
    inner = oracle.join_hash(w.R, w.S)
    semi, anti, left = (oracle.join_variant(w.R, w.S, k) for k in ("semi", "anti", "left"))
    assert len(semi) + len(anti) == w.S.n                      # every probe row is in exactly one of them
    assert not set(semi[:, 1]) & set(anti[:, 1])
    assert set(semi[:, 1]) == set(inner[:, 1])
    assert np.array_equal(left, oracle.sort_pairs(np.concatenate([inner, anti])))
    assert len(semi) == 400 and (semi[:, 0] == -1).all()      # the recipe's copies are the matches
    right, full = (oracle.join_variant(w.R, w.S, k) for k in ("right", "full"))
    lonely_r = right[right[:, 1] == -1]
    assert len(lonely_r) + len(set(inner[:, 0])) == w.R.n   # every build row is matched or listed once
    assert not set(lonely_r[:, 0]) & set(inner[:, 0])
    assert np.array_equal(right, oracle.sort_pairs(np.concatenate([inner, lonely_r])))
    assert np.array_equal(full, oracle.sort_pairs(np.concatenate([inner, anti, lonely_r])))
