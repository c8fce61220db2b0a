"""Pins for the serial oracle: hand-worked streams, published hash vectors, library
routines, invariants, brute force on tiny inputs and planted mistakes."""
import json
import os
import random

import numpy as np
import pytest

import oracle
from oracle import tiny
import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
MASK32 = 0xFFFFFFFF
FIELDS = ("count", "sum", "min", "max")


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def golden_inputs(g):
    kind = g["kind"]
    if kind == oracle.TEXT_WORDS:
        elems = np.frombuffer(g["text"].encode(), np.uint8)
        return dict(offsets=g["starts"], lengths=g["lengths"], elements=elems)
    d = dict(offsets=g["offsets"], elements=np.array(g["elements"], np.uint32))
    if "thresholds" in g:
        d["parent_param"] = np.array(g["thresholds"], np.uint32)
    return d


def c_run(kind, **kw):
    return oracle.run(kind, emit_outputs=True, **kw)


def tiny_run(kind, offsets, elements, lengths=None, parent_param=None, param=(0, 0, 0, 0)):
    return tiny.run(kind, offsets, elements, lengths, parent_param, param)


def as_records(r):
    return [(int(r.count[p]), int(r.sum[p]), int(r.min[p]), int(r.max[p])) for p in range(len(r.count))]


GOLDEN_FILES = ["e1_modfilter.json", "e2_hash_expand.json", "e3_text_words.json", "e4_graph_thresh.json"]


@pytest.mark.parametrize("name", GOLDEN_FILES)
def test_golden_c_oracle(name):
    g = load(name)
    kw = golden_inputs(g)
    r = c_run(g["kind"], param=tuple(g.get("param", (0, 0, 0, 0))), **kw)
    for f in FIELDS:
        assert [int(v) for v in getattr(r, f)] == g["expected"][f], f
    assert r.out.tolist() == g["outputs"]


@pytest.mark.parametrize("name", GOLDEN_FILES)
def test_golden_tiny_oracle(name):
    g = load(name)
    kw = golden_inputs(g)
    recs, outs = tiny_run(g["kind"], param=tuple(g.get("param", (0, 0, 0, 0))), **kw)
    exp = list(zip(*(g["expected"][f] for f in FIELDS)))
    assert recs == [tuple(e) for e in exp]
    assert outs == g["outputs"]


# ---- the hash is MurmurHash3's finalizer: pin it with the published MurmurHash3_x86_32 vectors ----

def _rotl(x, r):
    return ((x << r) | (x >> (32 - r))) & MASK32


def murmur3_x86_32(data, seed):
    """MurmurHash3_x86_32 body and tail; the final avalanche is the oracle's fmix32."""
    c1, c2 = 0xCC9E2D51, 0x1B873593
    h = seed & MASK32
    nb = len(data) // 4
    for i in range(nb):
        k = int.from_bytes(data[4 * i:4 * i + 4], "little")
        k = _rotl((k * c1) & MASK32, 15)
        k = (k * c2) & MASK32
        h ^= k
        h = _rotl(h, 13)
        h = (h * 5 + 0xE6546B64) & MASK32
    tail = data[4 * nb:]
    k = 0
    if len(tail) >= 3:
        k ^= tail[2] << 16
    if len(tail) >= 2:
        k ^= tail[1] << 8
    if len(tail) >= 1:
        k ^= tail[0]
        k = _rotl((k * c1) & MASK32, 15)
        h ^= (k * c2) & MASK32
    h ^= len(data)
    return oracle.fmix32(h)


MURMUR_VECTORS = [
    (b"", 0, 0x00000000),
    (b"", 1, 0x514E28B7),
    (b"", 0xFFFFFFFF, 0x81F16F39),
    (b"\0\0\0\0", 0, 0x2362F9DE),
    (b"aaaa", 0x9747B28C, 0x5A97808A),
    (b"aaa", 0x9747B28C, 0x283E0130),
    (b"aa", 0x9747B28C, 0x5D211726),
    (b"a", 0x9747B28C, 0x7FA09EA6),
    (b"abcd", 0x9747B28C, 0xF0478627),
    (b"abc", 0x9747B28C, 0xC84A62DD),
    (b"ab", 0x9747B28C, 0x74875592),
    (b"Hello, world!", 0x9747B28C, 0x24884CBA),
    (b"The quick brown fox jumps over the lazy dog", 0x9747B28C, 0x2FA826CD),
]


@pytest.mark.parametrize("data,seed,expected", MURMUR_VECTORS)
def test_fmix32_against_published_murmur3_vectors(data, seed, expected):
    assert murmur3_x86_32(data, seed) == expected


def test_hash_salts_and_tiny_agree():
    rng = random.Random(5)
    for _ in range(2000):
        x = rng.getrandbits(32)
        s = rng.randrange(4)
        assert oracle.hash32(x, s) == tiny.salted_hash(x, s)
        assert oracle.hash32(x, s) == oracle.fmix32(x ^ ((0x9E3779B9 * (s + 1)) & MASK32))


def test_fmix32_is_a_bijection_on_a_window():
    # every step of the finalizer is invertible, so distinct inputs give distinct outputs
    xs = range(0, 1 << 16)
    assert len({oracle.fmix32(x) for x in xs}) == 1 << 16


# ---- library cross-checks ----

def segment_sums(vals, offsets):
    cs = np.zeros(len(vals) + 1, np.uint64)
    np.cumsum(vals.astype(np.uint64), out=cs[1:])
    off = np.asarray(offsets, np.int64)
    return cs[off[1:]] - cs[off[:-1]]


def segment_minmax(vals, mask, offsets):
    P = len(offsets) - 1
    mn = np.full(P, MASK32, np.uint32)
    mx = np.zeros(P, np.uint32)
    parent = np.repeat(np.arange(P), np.diff(np.asarray(offsets, np.int64)))
    np.minimum.at(mn, parent[mask], vals[mask])
    np.maximum.at(mx, parent[mask], vals[mask])
    return mn, mx


@pytest.mark.parametrize("modulus,residue", [(1, 0), (4, 0), (4, 3), (7, 5)])
def test_modfilter_matches_numpy_reductions(modulus, residue):
    offsets, vals = workloads.modfilter_workload(seed=11, n_parents=700, max_size=64)
    r = oracle.run(oracle.MODFILTER, offsets, vals, param=(modulus, residue, 0, 0), emit_outputs=True)
    mask = vals % modulus == residue
    parent = np.repeat(np.arange(len(offsets) - 1), np.diff(offsets.astype(np.int64)))
    assert np.array_equal(r.count, np.bincount(parent[mask], minlength=len(offsets) - 1))
    assert np.array_equal(r.sum, segment_sums(np.where(mask, vals, 0), offsets))
    mn, mx = segment_minmax(vals, mask, offsets)
    assert np.array_equal(r.min, mn) and np.array_equal(r.max, mx)
    assert np.array_equal(r.out, vals[mask])
    if modulus == 1:
        assert np.array_equal(r.count, np.diff(offsets))


def test_graph_threshold_matches_numpy_reductions():
    offsets, w, thr, _ = workloads.graph_workload(seed=9, n_vertices=3000, n_edges=50000, cap=2000)
    r = oracle.run(oracle.GRAPH_THRESH, offsets, w, parent_param=thr, emit_outputs=True)
    parent = np.repeat(np.arange(3000), np.diff(offsets.astype(np.int64)))
    mask = w < thr[parent]
    assert np.array_equal(r.count, np.bincount(parent[mask], minlength=3000))
    assert np.array_equal(r.sum, segment_sums(np.where(mask, w, 0), offsets))
    assert np.array_equal(r.out, w[mask])


def test_text_words_matches_str_split():
    text, starts, lengths = workloads.text_workload(seed=13, total_bytes=200000, mean_len=40.0,
                                                    max_len=600)
    r = oracle.run(oracle.TEXT_WORDS, starts, text, lengths=lengths, emit_outputs=True)
    raw = text.tobytes()
    all_lens = []
    for p in range(len(starts)):
        line = raw[starts[p]:starts[p] + lengths[p]].decode()
        words = [w for w in line.split(" ") if w]
        assert r.count[p] == len(words)
        assert r.max[p] == (max(len(w) for w in words) if words else 0)
        assert r.sum[p] == sum(len(w) for w in words)
        all_lens.extend(len(w) for w in words)
    assert r.out.tolist() == all_lens


def numpy_hash(x, salt):
    x = x.astype(np.uint64) ^ np.uint64((0x9E3779B9 * (salt + 1)) & MASK32)
    m = np.uint64(MASK32)
    x ^= x >> np.uint64(16)
    x = (x * np.uint64(0x85EBCA6B)) & m
    x ^= x >> np.uint64(13)
    x = (x * np.uint64(0xC2B2AE35)) & m
    x ^= x >> np.uint64(16)
    return x


def test_hash_expand_matches_vectorized_numpy():
    offsets = workloads.uniform_offsets(21, 900, 40)
    vals = workloads.hash_values(21, int(offsets[-1]))
    r = oracle.run(oracle.HASH_EXPAND, offsets, vals, emit_outputs=True)
    h0 = numpy_hash(vals, 0)
    c = np.where(h0 & np.uint64(1), (h0 >> np.uint64(1)) & np.uint64(3), 0).astype(np.int64)
    kids = np.stack([numpy_hash(vals, j + 1) for j in range(3)], axis=1)
    take = np.arange(3)[None, :] < c[:, None]
    out = kids[take]                       # row-major: element order, then child order
    assert np.array_equal(r.out.astype(np.uint64), out)
    parent = np.repeat(np.arange(900), np.diff(offsets.astype(np.int64)))
    kid_parent = np.repeat(parent, c)
    assert np.array_equal(r.count, np.bincount(kid_parent, minlength=900))
    cs = np.zeros(len(out) + 1, np.uint64)
    np.cumsum(out, out=cs[1:])
    ko = np.concatenate([[0], np.cumsum(np.bincount(kid_parent, minlength=900))])
    assert np.array_equal(r.sum, cs[ko[1:]] - cs[ko[:-1]])


# ---- invariants and brute force ----

def random_case(kind, rng, P=None):
    P = P if P is not None else rng.randrange(0, 25)
    sizes = [rng.choice([0, 0, 1, 2, 3, 5, 8, 13, 40]) for _ in range(P)]
    offsets = workloads.sizes_to_offsets(np.array(sizes, np.uint64)) if P else np.zeros(1, np.uint32)
    n = int(offsets[-1])
    if kind == oracle.TEXT_WORDS:
        # lines separated by newlines: starts/lengths with a one-byte gap
        starts, pos, buf = [], 0, []
        for s in sizes:
            starts.append(pos)
            buf.extend(rng.choice(b"  ab") for _ in range(s))
            buf.append(10)
            pos += s + 1
        return dict(offsets=np.array(starts, np.uint32), lengths=np.array(sizes, np.uint32),
                    elements=np.array(buf, np.uint8))
    vals = np.array([rng.choice([0, 1, 4, 8, MASK32, MASK32 - 1, rng.getrandbits(32)]) for _ in range(n)],
                    np.uint32)
    d = dict(offsets=offsets, elements=vals)
    if kind == oracle.GRAPH_THRESH:
        d["parent_param"] = np.array([rng.choice([0, 1, 5, MASK32, rng.getrandbits(32)]) for _ in range(P)],
                                     np.uint32)
    return d


KINDS = [oracle.MODFILTER, oracle.HASH_EXPAND, oracle.TEXT_WORDS, oracle.GRAPH_THRESH]


def spans(kw):
    return list(tiny.regions(kw["offsets"], kw.get("lengths")))


@pytest.mark.parametrize("kind", KINDS)
def test_c_and_tiny_oracles_agree_and_invariants_hold(kind):
    rng = random.Random(100 + kind)
    for _ in range(150):
        kw = random_case(kind, rng)
        r = c_run(kind, **kw)
        recs, outs = tiny_run(kind, **kw)
        assert as_records(r) == recs
        assert r.out.tolist() == outs
        counts = r.count.astype(np.int64)
        assert counts.sum() == len(outs)                      # sum of counts = surviving total
        base = np.concatenate([[0], np.cumsum(counts)])
        for p, (s, e) in enumerate(spans(kw)):
            sl = outs[base[p]:base[p + 1]]                     # region p's slice of the stream
            if sl:
                assert (len(sl), sum(sl), min(sl), max(sl)) == recs[p]
            else:
                assert recs[p] == (0, 0, MASK32, 0)
            n = e - s
            kmax = {oracle.MODFILTER: 1, oracle.HASH_EXPAND: 3, oracle.TEXT_WORDS: 1,
                    oracle.GRAPH_THRESH: 1}[kind]
            assert len(sl) <= kmax * n
            if kind == oracle.TEXT_WORDS:
                assert len(sl) <= (n + 1) // 2 and (max(sl) if sl else 0) <= n


def test_every_output_derives_from_its_own_region():
    rng = random.Random(7)
    for _ in range(100):
        kw = random_case(oracle.HASH_EXPAND, rng)
        r = c_run(oracle.HASH_EXPAND, **kw)
        base = np.concatenate([[0], np.cumsum(r.count.astype(np.int64))])
        vals = kw["elements"]
        for p, (s, e) in enumerate(spans(kw)):
            allowed = {tiny.salted_hash(int(x), j + 1) for x in vals[s:e] for j in range(3)}
            assert set(r.out[base[p]:base[p + 1]].tolist()) <= allowed


def test_edge_cases():
    # no parents
    r = c_run(oracle.MODFILTER, offsets=np.zeros(1, np.uint32), elements=np.zeros(0, np.uint32))
    assert len(r.count) == 0 and len(r.out) == 0
    # all parents empty
    r = c_run(oracle.HASH_EXPAND, offsets=np.zeros(6, np.uint32), elements=np.zeros(0, np.uint32))
    assert r.count.tolist() == [0] * 5 and r.min.tolist() == [MASK32] * 5 and r.max.tolist() == [0] * 5
    # one parent holds the whole stream
    vals = workloads.hash_values(3, 5000)
    whole = c_run(oracle.HASH_EXPAND, offsets=np.array([0, 5000], np.uint32), elements=vals)
    split = c_run(oracle.HASH_EXPAND, offsets=workloads.fixed_offsets(5000, 1), elements=vals)
    assert whole.count[0] == split.count.sum() and whole.sum[0] == split.sum.sum()
    assert whole.min[0] == split.min.min() and whole.max[0] == split.max.max()
    assert np.array_equal(whole.out, split.out)
    # L = 1 everywhere: every record is that element's own result
    for p in range(0, 5000, 499):
        recs, _ = tiny_run(oracle.HASH_EXPAND, [0, 1], [int(vals[p])])
        assert recs[0] == (int(split.count[p]), int(split.sum[p]), int(split.min[p]), int(split.max[p]))
    # a single element 0 under the mod filter survives with sum 0
    r = c_run(oracle.MODFILTER, offsets=np.array([0, 1], np.uint32), elements=np.array([0], np.uint32))
    assert (int(r.count[0]), int(r.sum[0])) == (1, 0)


def test_bad_regions_are_rejected():
    with pytest.raises(ValueError):
        oracle.run(oracle.MODFILTER, [0, 5], np.zeros(3, np.uint32))


# ---- planted mistakes: each must be caught by the pins above ----

def _golden_agrees(stage_patch, agg_identity=(0, 0, MASK32, 0)):
    """Re-run the golden cases through a mutated copy of the tiny oracle."""
    orig = tiny.stages_for
    try:
        tiny.stages_for = stage_patch(orig)
        ok = True
        for name in GOLDEN_FILES:
            g = load(name)
            kw = golden_inputs(g)
            recs, outs = tiny_run(g["kind"], param=tuple(g.get("param", (0, 0, 0, 0))), **kw)
            recs = [r if r[0] else agg_identity for r in recs]
            exp = [tuple(e) for e in zip(*(g["expected"][f] for f in FIELDS))]
            ok &= recs == exp and outs == g["outputs"]
        return ok
    finally:
        tiny.stages_for = orig


def test_planted_mistakes_are_caught():
    assert _golden_agrees(lambda orig: orig)

    def flip_mod(orig):
        def f(kind, param=(0, 0, 0, 0)):
            if kind == tiny.MODFILTER:
                return [lambda x, reg: [x] if x % 4 != 0 else []]
            return orig(kind, param)
        return f

    def child_salt_off_by_one(orig):
        def f(kind, param=(0, 0, 0, 0)):
            if kind == tiny.HASH_EXPAND:
                return [lambda x, reg: [x] if tiny.salted_hash(x, 0) & 1 else [],
                        lambda x, reg: [tiny.salted_hash(x, j) for j in range((tiny.salted_hash(x, 0) >> 1) & 3)]]
            return orig(kind, param)
        return f

    def word_start_ignores_line_start(orig):
        def f(kind, param=(0, 0, 0, 0)):
            if kind == tiny.TEXT_WORDS:
                st = orig(kind, param)
                return [lambda i, reg: [i] if i > 0 and reg["line"][i] != 32 and reg["line"][i - 1] == 32 else [],
                        st[1]]
            return orig(kind, param)
        return f

    def non_strict_threshold(orig):
        def f(kind, param=(0, 0, 0, 0)):
            if kind == tiny.GRAPH_THRESH:
                return [lambda w, reg: [w] if w <= reg["threshold"] else []]
            return orig(kind, param)
        return f

    for mutant in (flip_mod, child_salt_off_by_one, word_start_ignores_line_start, non_strict_threshold):
        assert not _golden_agrees(mutant), mutant.__name__
    # a wrong identity for empty regions is caught too
    assert not _golden_agrees(lambda orig: orig, agg_identity=(0, 0, 0, 0))


# ---- tree topology (§2.1): the filter feeds the expansion and a second sink ----

def test_tree_first_sink_is_the_linear_pipeline():
    """The tree's first sink sees exactly the linear pipeline's items: its records and output
    stream equal the hash/expand oracle's (the pinned linear case)."""
    offsets = workloads.uniform_offsets(41, 700, 60)
    vals = workloads.hash_values(41, int(offsets[-1]))
    t = oracle.run(oracle.HASH_TREE, offsets, vals, emit_outputs=True)
    h = oracle.run(oracle.HASH_EXPAND, offsets, vals, emit_outputs=True)
    for f in ("count", "sum", "min", "max", "out"):
        assert np.array_equal(getattr(t, f), getattr(h, f)), f


def test_tree_second_sink_matches_vectorized_numpy():
    """The second sink holds, per region, the count and the sum of the elements whose H(x,0) has
    bit 0 set: a numpy replay of the hash (written here) and bincount with int64 sums."""
    offsets = workloads.uniform_offsets(42, 900, 40)
    vals = workloads.hash_values(42, int(offsets[-1]))
    t = oracle.run(oracle.HASH_TREE, offsets, vals)
    keep = (numpy_hash(vals, 0) & np.uint64(1)).astype(bool)
    parent = np.repeat(np.arange(900), np.diff(offsets.astype(np.int64)))
    assert np.array_equal(t.kept_count, np.bincount(parent[keep], minlength=900))
    sums = np.bincount(parent[keep], weights=None, minlength=900) * 0
    np.add.at(sums, parent[keep], vals[keep].astype(np.int64))
    assert np.array_equal(t.kept_sum.astype(np.int64), sums)
    # invariants: survivors never exceed the region, children never exceed three per survivor
    sizes = np.diff(offsets.astype(np.int64))
    assert (t.kept_count <= sizes).all() and (t.count <= 3 * t.kept_count.astype(np.int64)).all()


def test_tree_c_and_tiny_oracles_agree():
    rng = random.Random(7)
    for _ in range(30):
        P = rng.randrange(0, 20)
        sizes = [rng.choice([0, 1, 2, 5, 17, 40]) for _ in range(P)]
        offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)
        vals = np.array([rng.getrandbits(32) for _ in range(int(offsets[-1]))], np.uint32)
        t = oracle.run(oracle.HASH_TREE, offsets, vals, emit_outputs=True)
        recs, second, outs = tiny.run_tree(offsets, vals)
        assert [tuple(int(v) for v in r) for r in zip(t.count, t.sum, t.min, t.max)] == recs
        assert [(int(c), int(s)) for c, s in zip(t.kept_count, t.kept_sum)] == second
        assert t.out.tolist() == outs


def test_tree_planted_mistake_is_caught():
    """A second sink that takes every element instead of the filter's survivors differs from the
    oracle on a seeded stream."""
    offsets = workloads.uniform_offsets(43, 200, 30)
    vals = workloads.hash_values(43, int(offsets[-1]))
    t = oracle.run(oracle.HASH_TREE, offsets, vals)
    wrong = [(e - s) for s, e in tiny.regions(offsets)]
    assert [int(c) for c in t.kept_count] != wrong
