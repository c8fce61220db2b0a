"""GPU parity: the HIP path through the C ABI against the serial oracle, element by
element, on seeded inputs (integer results: bit-exact)."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import workloads
import paper_2006_07478_amd as rs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
STRATS = [rs.RS_TAG, rs.RS_SIGNAL]
# with lane-resolved signals, offered for u32 kinds at widths up to 256
ALL3 = STRATS + [rs.RS_SIGNAL_LANES]
SNAME = {rs.RS_TAG: "tag", rs.RS_SIGNAL: "signal", rs.RS_SIGNAL_LANES: "lanes", rs.RS_ENUM_TAG: "enum+tag"}


def strats(kind, width):
    """The strategies offered for a kind and an ensemble width."""
    out = ALL3 if kind != rs.RS_TEXT_WORDS and width <= 256 else STRATS
    if kind in (rs.RS_HASH_EXPAND, rs.RS_TEXT_WORDS):   # enumeration, then tags: kinds with a second stage
        out = out + [rs.RS_ENUM_TAG]
    return out


def skip_unoffered(kind, strategy, width):
    if strategy not in strats(kind, width):
        pytest.skip("lane-resolved signals are offered for u32 kinds at widths up to 256, enumeration "
                    "with tags downstream for kinds with a second stage")
ALL = rs.RS_COUNT | rs.RS_SUM | rs.RS_MIN | rs.RS_MAX
WIDTHS = [64, 128, 256, 512, 1024]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check(got, ref, fields=("count", "sum", "min", "max"), where=""):
    for f in fields:
        g, r = got[f], getattr(ref, f)
        if not np.array_equal(g, r):
            bad = np.nonzero(g != r)[0]
            raise AssertionError(f"{where}: field {f} differs at {len(bad)} parents, first {bad[:5].tolist()}: "
                                 f"gpu {g[bad[:5]].tolist()} oracle {r[bad[:5]].tolist()}")


def run_one(kind, strategy, width, offsets, elements, lengths=None, parent_param=None, param=(0, 0, 0, 0),
            fields=ALL, device=False, flags=0, queue_depth=0):
    import torch
    with rs.Pipeline(kind, strategy=strategy, ensemble_width=width, agg_fields=fields, param=param,
                     flags=flags, queue_depth=queue_depth) as p:
        if device:
            to = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a).view(
                np.int32 if a.dtype == np.uint32 else np.uint8)).cuda()
            sid = p.push(to(offsets), to(elements), lengths=to(lengths), parent_param=to(parent_param),
                         n_elements=len(elements))
        else:
            sid = p.push(offsets, elements, lengths=lengths, parent_param=parent_param)
        p.run()
        out = p.read(sid)
        st = p.stats(sid) if flags & rs.RS_COLLECT_STATS else None
    return out, st


# ---- hand-worked streams ----

@pytest.mark.parametrize("name", ["e1_modfilter.json", "e2_hash_expand.json", "e3_text_words.json",
                                  "e4_graph_thresh.json"])
@pytest.mark.parametrize("strategy", ALL3)
@pytest.mark.parametrize("width", [64, 256])
def test_golden_streams(name, strategy, width):
    g = json.load(open(os.path.join(GOLDEN, name)))
    say("golden", name, SNAME[strategy], width)
    kind = g["kind"]
    skip_unoffered(kind, strategy, width)
    if kind == rs.RS_TEXT_WORDS:
        elems = np.frombuffer(g["text"].encode(), np.uint8)
        got, _ = run_one(kind, strategy, width, np.array(g["starts"], np.uint32), elems,
                         lengths=np.array(g["lengths"], np.uint32))
    else:
        got, _ = run_one(kind, strategy, width, np.array(g["offsets"], np.uint32), np.array(g["elements"], np.uint32),
                         parent_param=np.array(g["thresholds"], np.uint32) if "thresholds" in g else None,
                         param=tuple(g.get("param", (0, 0, 0, 0))))
    for f in ("count", "sum", "min", "max"):
        assert [int(v) for v in got[f]] == g["expected"][f], f


# ---- sum app, 4096 parents with sizes in [0, 64] ----

@pytest.mark.parametrize("strategy", ALL3)
@pytest.mark.parametrize("width", [64, 128, 256, 512])
@pytest.mark.parametrize("device", [False, True])
def test_sum_app_4096_parents(strategy, width, device):
    skip_unoffered(rs.RS_MODFILTER, strategy, width)
    say("sum app", SNAME[strategy], width, "device" if device else "host")
    offsets, vals = workloads.modfilter_workload(seed=1, n_parents=4096, max_size=64)
    ref = oracle.run(oracle.MODFILTER, offsets, vals, param=(4, 0, 0, 0))
    got, _ = run_one(rs.RS_MODFILTER, strategy, width, offsets, vals, param=(4, 0, 0, 0),
                     fields=rs.RS_COUNT | rs.RS_SUM, device=device)
    check(got, ref, ("count", "sum"), "sum app")


@pytest.mark.parametrize("modulus,residue", [(1, 0), (7, 3), (4, 2)])
def test_modfilter_parameters(modulus, residue):
    offsets, vals = workloads.modfilter_workload(seed=17, n_parents=3000, max_size=90)
    ref = oracle.run(oracle.MODFILTER, offsets, vals, param=(modulus, residue, 0, 0))
    for strategy in ALL3:
        got, _ = run_one(rs.RS_MODFILTER, strategy, 256, offsets, vals, param=(modulus, residue, 0, 0))
        check(got, ref, where=f"mod {modulus} {residue}")


# ---- boundary-frequency sweep, reduced size: several tiles and a ragged tail ----

@pytest.mark.parametrize("L", [1, 4, 16, 64, 256, 1024, 4096])
@pytest.mark.parametrize("strategy", ALL3)
def test_hash_expand_fixed_L(L, strategy):
    n = (1 << 18) + 13                     # not a multiple of the region length or of 4
    say("hash/expand L", L, SNAME[strategy])
    offsets = workloads.fixed_offsets(n, L)
    vals = workloads.hash_values(2, n)
    ref = oracle.run(oracle.HASH_EXPAND, offsets, vals)
    got, _ = run_one(rs.RS_HASH_EXPAND, strategy, 256, offsets, vals)
    check(got, ref, where=f"L={L}")


@pytest.mark.parametrize("width", [64, 128, 512])
@pytest.mark.parametrize("strategy", ALL3)
def test_hash_expand_widths_variable_regions(width, strategy):
    skip_unoffered(rs.RS_HASH_EXPAND, strategy, width)
    say("hash/expand width", width, SNAME[strategy])
    offsets = workloads.uniform_offsets(5, 3000, 300)
    vals = workloads.hash_values(5, int(offsets[-1]))
    ref = oracle.run(oracle.HASH_EXPAND, offsets, vals)
    got, _ = run_one(rs.RS_HASH_EXPAND, strategy, width, offsets, vals)
    check(got, ref, where=f"width {width}")


# ---- edge cases ----

@pytest.mark.parametrize("strategy", ALL3)
def test_edge_cases(strategy):
    say("edge cases", SNAME[strategy])
    # all parents empty
    offs = np.zeros(1001, np.uint32)
    got, _ = run_one(rs.RS_HASH_EXPAND, strategy, 256, offs, np.zeros(4, np.uint32))
    assert (got["count"] == 0).all() and (got["min"] == 0xFFFFFFFF).all() and (got["max"] == 0).all()
    # one parent holds the whole stream
    vals = workloads.hash_values(3, 200003)
    offs = np.array([0, 200003], np.uint32)
    ref = oracle.run(oracle.HASH_EXPAND, offs, vals)
    got, _ = run_one(rs.RS_HASH_EXPAND, strategy, 256, offs, vals)
    check(got, ref, where="one parent")
    # a single element 0 under the mod filter
    got, _ = run_one(rs.RS_MODFILTER, strategy, 64, np.array([0, 1], np.uint32), np.array([0], np.uint32),
                     fields=rs.RS_COUNT | rs.RS_SUM)
    assert int(got["count"][0]) == 1 and int(got["sum"][0]) == 0
    # regions that do not start at element 0 and skip elements at the end
    vals = workloads.hash_values(4, 5000)
    offs = np.array([7, 7, 100, 2500, 4990], np.uint32)
    ref = oracle.run(oracle.HASH_EXPAND, offs, vals)
    got, _ = run_one(rs.RS_HASH_EXPAND, strategy, 128, offs, vals)
    check(got, ref, where="offset start")


def test_zero_parents():
    with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=rs.RS_TAG, ensemble_width=256) as p:
        sid = p.push(np.zeros(1, np.uint32), np.zeros(4, np.uint32))
        p.run()
        got = p.read(sid)
        assert all(len(v) == 0 for v in got.values())


# ---- text and graph kinds ----

@pytest.mark.parametrize("strategy", STRATS)
@pytest.mark.parametrize("width", [64, 256])
def test_text_words(strategy, width):
    say("text", SNAME[strategy], width)
    text, starts, lengths = workloads.text_workload(seed=3, total_bytes=1 << 20)
    ref = oracle.run(oracle.TEXT_WORDS, starts, text, lengths=lengths)
    got, _ = run_one(rs.RS_TEXT_WORDS, strategy, width, starts, text, lengths=lengths)
    check(got, ref, where="text")


@pytest.mark.parametrize("strategy", STRATS)
def test_text_long_lines_and_long_words(strategy):
    say("text long", SNAME[strategy])
    text, starts, lengths = workloads.text_workload(seed=8, total_bytes=1 << 20, mean_len=3000.0, max_len=65536,
                                                    space_per_65536=300)
    ref = oracle.run(oracle.TEXT_WORDS, starts, text, lengths=lengths)
    got, _ = run_one(rs.RS_TEXT_WORDS, strategy, 256, starts, text, lengths=lengths)
    check(got, ref, where="text long")


@pytest.mark.parametrize("strategy", ALL3)
@pytest.mark.parametrize("width", [64, 256])
def test_graph_threshold(strategy, width):
    say("graph", SNAME[strategy], width)
    offsets, w, thr, _ = workloads.graph_workload(seed=4, n_vertices=1 << 14, n_edges=1 << 18, cap=20000)
    ref = oracle.run(oracle.GRAPH_THRESH, offsets, w, parent_param=thr)
    got, _ = run_one(rs.RS_GRAPH_THRESH, strategy, width, offsets, w, parent_param=thr)
    check(got, ref, where="graph")


# ---- batching, replay, statistics ----

def test_batched_streams_equal_alone():
    say("batched")
    shapes = [(5000, 1.0), (20000, 37.5), (100000, 700.0), (3000, 4096.0), (1, 1.0), (77777, 3.0)]
    streams = [workloads.serving_stream(5, s, n, m) for s, (n, m) in enumerate(shapes)]
    for strategy in ALL3:
        with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=strategy, ensemble_width=256) as p:
            ids = [p.push(o, v) for o, v in streams]
            p.run()
            for sid, (o, v) in zip(ids, streams):
                check(p.read(sid), oracle.run(oracle.HASH_EXPAND, o, v), where="batched")


def test_run_again_replays_bit_exact():
    """Replays equal the oracle, and every replay processes every element: a replay that skipped
    claims would leave the earlier launch's (equal) aggregates in place, so the statistics, which
    accumulate over launches, count the first node's items per launch as well."""
    n = 1 << 20
    offsets = workloads.fixed_offsets(n, 64)
    vals = workloads.hash_values(2, n)
    ref = oracle.run(oracle.HASH_EXPAND, offsets, vals)
    for strategy in ALL3:
        with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=strategy, ensemble_width=256) as p:   # graph replays
            sid = p.push(offsets, vals)
            p.run()
            for _ in range(4):
                p.run_again()
                check(p.read(sid), ref, where="replay")
        with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=strategy, ensemble_width=256, flags=rs.RS_COLLECT_STATS) as p:
            sid = p.push(offsets, vals)
            p.run()
            assert p.stats(sid).items[0] == n
            for i in range(4):
                p.run_again()
                check(p.read(sid), ref, where="replay")
                assert p.stats(sid).items[0] == (i + 2) * n, f"replay {i}: claims skipped"


def test_signal_occupancy_matches_closed_form():
    """Enumerating-node firings at fixed L: ceil(L/w) per region, L/(w ceil(L/w)) occupancy."""
    w = 256
    for L in (1, 100, 256, 300, 4096):
        n = L * 512
        offsets = workloads.fixed_offsets(n, L)
        vals = workloads.hash_values(2, n)
        _, st = run_one(rs.RS_HASH_EXPAND, rs.RS_SIGNAL, w, offsets, vals, flags=rs.RS_COLLECT_STATS)
        fires = 512 * -(-L // w)
        assert st.firings[0] == fires and st.items[0] == n
        assert st.signals[0] == 512 and st.signals[2] == 512
        assert st.full[0] == 512 * (L // w)
        _, st_t = run_one(rs.RS_HASH_EXPAND, rs.RS_TAG, w, offsets, vals, flags=rs.RS_COLLECT_STATS)
        assert st_t.items[0] == n and st_t.signals[0] == 0


@pytest.mark.parametrize("strategy", ALL3)
@pytest.mark.parametrize("mx", [1, 7, 64, 300, 5000])
def test_variable_size_regions(strategy, mx):
    """Region sizes uniform in [0, max] (the variable-size sweep): records equal the oracle's,
    and for signals the enumerating node fires ceil(n_p/w) times per region, full floor(n_p/w)."""
    say("variable sizes", SNAME[strategy], mx)
    n = 300007
    offsets = workloads.variable_offsets(11, n, mx)
    vals = workloads.hash_values(12, n)
    ref = oracle.run(oracle.HASH_EXPAND, offsets, vals)
    sizes = np.diff(offsets.astype(np.int64))
    for w in (64, 256):
        got, st = run_one(rs.RS_HASH_EXPAND, strategy, w, offsets, vals, flags=rs.RS_COLLECT_STATS)
        check(got, ref, where=f"variable max={mx} {SNAME[strategy]} w={w}")
        assert st.items[0] == n
        if strategy == rs.RS_SIGNAL:
            assert st.firings[0] == int(np.sum(-(-sizes // w)))
            assert st.full[0] == int(np.sum(sizes // w))
            assert st.signals[0] == len(sizes)


@pytest.mark.parametrize("width", [64, 128, 256, 512, 1024])
def test_tags_many_mid_size_regions(width):
    """Tags, ensembles that span many regions of several items each (the lanes of one region fold
    within each 8-lane block before one of them adds to the region's slot), at every width.  Hash
    values use all 32 bits, so the folded sums carry past 32 bits; all-ones values, which a mod-4
    filter with residue 3 keeps, fill both 16-bit halves of every folded sum."""
    say("tags, mid-size regions, width", width)
    n = 200003
    offsets = workloads.variable_offsets(21, n, 48)   # sizes U[0, 48]: about 18 items a region
    vals = workloads.hash_values(22, n)
    ref = oracle.run(oracle.HASH_EXPAND, offsets, vals)
    got, _ = run_one(rs.RS_HASH_EXPAND, rs.RS_TAG, width, offsets, vals)
    check(got, ref, where=f"hash/expand, sizes U[0,48], w={width}")
    m = (1 << 17) + 5
    offsets = workloads.fixed_offsets(m, 17)
    ones = np.full(m, 0xFFFFFFFF, np.uint32)
    ref = oracle.run(oracle.MODFILTER, offsets, ones, param=(4, 3, 0, 0))
    assert int(ref.count[0]) == 17 and int(ref.sum[0]) == 17 * 0xFFFFFFFF
    got, _ = run_one(rs.RS_MODFILTER, rs.RS_TAG, width, offsets, ones, param=(4, 3, 0, 0))
    check(got, ref, where=f"all-ones, L=17, w={width}")


def test_lane_signals_flow_and_occupancy():
    """Lane-resolved signals: every region's end is signalled once on each edge (empty regions
    included), and ensembles span boundaries, so the enumerating node stays near full where the
    plain signal strategy fills L/(w ceil(L/w)) of its lanes."""
    w = 256
    for L in (1, 5, 100, 300):
        n = 200003
        offsets = workloads.fixed_offsets(n, L)
        vals = workloads.hash_values(2, n)
        P = len(offsets) - 1
        got, st = run_one(rs.RS_HASH_EXPAND, rs.RS_SIGNAL_LANES, w, offsets, vals, flags=rs.RS_COLLECT_STATS)
        check(got, oracle.run(oracle.HASH_EXPAND, offsets, vals), where=f"lanes L={L}")
        assert st.items[0] == n
        assert st.signals[0] == P and st.signals[1] == P and st.signals[2] == P
        occ = st.items[0] / (st.firings[0] * w)
        if L >= 64:
            # a firing is cut short only at the end of a claim
            assert occ > 0.9, (L, occ)
        else:
            # the 64-entry signal queue bounds an ensemble to the regions whose ends fit in it,
            # still far above the plain signal strategy's L / (w ceil(L/w))
            assert occ > 2 * L / (w * -(-L // w)), (L, occ)
    # empty regions everywhere between single elements
    offsets = np.repeat(np.arange(0, 1001, dtype=np.uint32), 3)
    vals = workloads.hash_values(3, 1000)
    got, st = run_one(rs.RS_HASH_EXPAND, rs.RS_SIGNAL_LANES, 64, offsets, vals, flags=rs.RS_COLLECT_STATS)
    check(got, oracle.run(oracle.HASH_EXPAND, offsets, vals), where="lanes empty regions")
    assert st.signals[0] == len(offsets) - 1


def test_lane_signals_not_offered_for_text_or_wide_ensembles():
    with pytest.raises(rs.RsError) as ei:
        rs.Pipeline(rs.RS_TEXT_WORDS, strategy=rs.RS_SIGNAL_LANES, ensemble_width=64)
    assert ei.value.code == rs.RS_EINVAL
    with pytest.raises(rs.RsError) as ei:
        rs.Pipeline(rs.RS_HASH_EXPAND, strategy=rs.RS_SIGNAL_LANES, ensemble_width=512)
    assert ei.value.code == rs.RS_EINVAL


# ---- ordered output stream ----

def run_outputs(kind, strategy, width, offsets, elements, lengths=None, parent_param=None):
    with rs.Pipeline(kind, strategy=strategy, ensemble_width=width, agg_fields=ALL, emit_outputs=True) as p:
        sid = p.push(offsets, elements, lengths=lengths, parent_param=parent_param)
        p.run()
        return p.read(sid), p.outputs(sid)


@pytest.mark.parametrize("strategy", ALL3)
@pytest.mark.parametrize("L", [1, 7, 300, 5000])
def test_output_stream_hash_expand(strategy, L):
    say("outputs hash/expand", SNAME[strategy], L)
    n = 150001
    offsets = workloads.fixed_offsets(n, L)
    vals = workloads.hash_values(9, n)
    ref = oracle.run(oracle.HASH_EXPAND, offsets, vals, emit_outputs=True)
    got, out = run_outputs(rs.RS_HASH_EXPAND, strategy, 256, offsets, vals)
    check(got, ref, where="outputs agg")
    assert len(out) == len(ref.out) and np.array_equal(out, ref.out)


@pytest.mark.parametrize("strategy", ALL3)
@pytest.mark.parametrize("L", [3, 37, 4096])
def test_output_stream_large_claims(strategy, L):
    """An ordered output stream of at least 2048 claims of 32 ensembles (w = 64: 2^22 elements and
    up), where claims hold twice the parents (at L = 4096 a claim is one parent either way):
    outputs and records equal the oracle's."""
    say("outputs, large claims", SNAME[strategy], L)
    n = (1 << 22) + 19
    offsets = workloads.fixed_offsets(n, L)
    vals = workloads.hash_values(23, n)
    ref = oracle.run(oracle.HASH_EXPAND, offsets, vals, emit_outputs=True)
    got, out = run_outputs(rs.RS_HASH_EXPAND, strategy, 64, offsets, vals)
    check(got, ref, where=f"outputs agg, L={L}")
    assert len(out) == len(ref.out) and np.array_equal(out, ref.out)


@pytest.mark.parametrize("strategy", ALL3)
def test_output_stream_other_kinds(strategy):
    say("outputs other kinds", SNAME[strategy])
    offsets, vals = workloads.modfilter_workload(seed=1, n_parents=4096, max_size=64)
    ref = oracle.run(oracle.MODFILTER, offsets, vals, emit_outputs=True)
    _, out = run_outputs(rs.RS_MODFILTER, strategy, 128, offsets, vals)
    assert np.array_equal(out, ref.out)
    offsets, w, thr, _ = workloads.graph_workload(seed=4, n_vertices=1 << 13, n_edges=1 << 17, cap=20000)
    ref = oracle.run(oracle.GRAPH_THRESH, offsets, w, parent_param=thr, emit_outputs=True)
    _, out = run_outputs(rs.RS_GRAPH_THRESH, strategy, 64, offsets, w, parent_param=thr)
    assert np.array_equal(out, ref.out)
    if strategy not in strats(rs.RS_TEXT_WORDS, 256):
        return
    text, starts, lengths = workloads.text_workload(seed=3, total_bytes=1 << 19)
    ref = oracle.run(oracle.TEXT_WORDS, starts, text, lengths=lengths, emit_outputs=True)
    _, out = run_outputs(rs.RS_TEXT_WORDS, strategy, 256, starts, text, lengths=lengths)
    assert np.array_equal(out, ref.out)


def test_output_stream_batched_and_replayed():
    say("outputs batched/replayed")
    shapes = [(5000, 1.0), (60000, 37.5), (100000, 700.0), (1, 1.0)]
    streams = [workloads.serving_stream(5, s, n, m) for s, (n, m) in enumerate(shapes)]
    for strategy in ALL3:
        with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=strategy, ensemble_width=256, emit_outputs=True) as p:
            ids = [p.push(o, v) for o, v in streams]
            p.run()
            for rep in range(3):
                if rep:
                    p.run_again()
                for sid, (o, v) in zip(ids, streams):
                    ref = oracle.run(oracle.HASH_EXPAND, o, v, emit_outputs=True)
                    assert np.array_equal(p.outputs(sid), ref.out)
                    check(p.read(sid), ref, where="outputs batched")


# ---- borrowed device streams with malformed regions are reported, never read out of bounds ----

def test_malformed_device_regions_are_rejected():
    import torch
    say("malformed device regions")
    vals = torch.from_numpy(workloads.hash_values(1, 4096).view(np.int32)).cuda()
    bad_offsets = [np.array([0, 100, 50, 4096], np.uint32),          # decreasing
                   np.array([0, 100, 5000], np.uint32)]               # past n_elements
    for offs in bad_offsets:
        for strategy in ALL3:
            with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=strategy, ensemble_width=256) as p:
                sid = p.push(torch.from_numpy(offs.view(np.int32)).cuda(), vals, n_elements=4096)
                p.run()
                with pytest.raises(rs.RsError) as ei:
                    p.read(sid)
                assert ei.value.code == rs.RS_EINVAL
    # one malformed stream among good ones in a batch: only it is refused
    good = workloads.fixed_offsets(4096, 16)
    ref = oracle.run(oracle.HASH_EXPAND, good, workloads.hash_values(1, 4096))
    with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=rs.RS_TAG, ensemble_width=256) as p:
        g = torch.from_numpy(good.view(np.int32)).cuda()
        ids = [p.push(g, vals, n_elements=4096),
               p.push(torch.from_numpy(bad_offsets[0].view(np.int32)).cuda(), vals, n_elements=4096),
               p.push(g, vals, n_elements=4096)]
        p.run()
        check(p.read(ids[0]), ref, where="good stream before the malformed one")
        with pytest.raises(rs.RsError) as ei:
            p.read(ids[1])
        assert ei.value.code == rs.RS_EINVAL
        check(p.read(ids[2]), ref, where="good stream after the malformed one")
    # text lines that overlap
    text = torch.from_numpy(np.frombuffer(b"ab cd\nef gh\n" + b" " * 4, np.uint8).copy()).cuda()
    with rs.Pipeline(rs.RS_TEXT_WORDS, strategy=rs.RS_TAG, ensemble_width=64) as p:
        sid = p.push(torch.tensor([0, 3], dtype=torch.int32).cuda(), text,
                     lengths=torch.tensor([5, 5], dtype=torch.int32).cuda(), n_elements=12)
        p.run()
        with pytest.raises(rs.RsError):
            p.read(sid)


def test_host_validation_messages():
    with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=rs.RS_TAG, ensemble_width=64) as p:
        with pytest.raises(rs.RsError) as ei:
            p.push(np.array([0, 5, 3], np.uint32), np.zeros(8, np.uint32))
        assert ei.value.code == rs.RS_EINVAL and "decrease" in str(ei.value)
        with pytest.raises(rs.RsError):
            p.push(np.array([0, 9], np.uint32), np.zeros(8, np.uint32))
    with rs.Pipeline(rs.RS_GRAPH_THRESH, strategy=rs.RS_TAG, ensemble_width=64) as p:
        with pytest.raises(rs.RsError):
            p.push(np.array([0, 2], np.uint32), np.zeros(2, np.uint32))   # thresholds missing


# ---- autotuner ----

def test_autotuned_pipeline_matches_oracle(tmp_path, monkeypatch):
    monkeypatch.setenv("RS_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    say("autotune")
    for L in (2, 3000):
        offsets = workloads.fixed_offsets(1 << 19, L)
        vals = workloads.hash_values(2, 1 << 19)
        ref = oracle.run(oracle.HASH_EXPAND, offsets, vals)
        for _ in range(2):   # second pipeline hits the cache
            with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=rs.RS_AUTO, ensemble_width=0,
                             flags=rs.RS_COLLECT_STATS) as p:
                sid = p.push(offsets, vals)
                p.run()
                check(p.read(sid), ref, where=f"autotune L={L}")
                st = p.stats(sid)
                assert st.ensemble_width in WIDTHS
                assert st.strategy in strats(rs.RS_HASH_EXPAND, st.ensemble_width)
                assert st.queue_depth in (2 * st.ensemble_width, 4 * st.ensemble_width)
    n_lines = lambda: len([l for l in (tmp_path / "tune.txt").read_text().split("\n") if l.strip()])
    assert n_lines() == 2
    # pipelines that fix different strategies keep their own cached choices side by side: the
    # second round tunes nothing
    counts = []
    for _ in range(2):
        for s in (rs.RS_SIGNAL, rs.RS_TAG):
            with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=s, ensemble_width=0, flags=rs.RS_COLLECT_STATS) as p:
                sid = p.push(offsets, vals)
                p.run()
                check(p.read(sid), ref, where=f"fixed strategy {s}, tuned width")
                assert p.stats(sid).strategy == s
        counts.append(n_lines())
    assert counts[0] <= 4 and counts[1] == counts[0]


# ---- every configuration the autotuner can pick ----

# Claims hold at most 255 parents, and a launch has at most 20 one-wave workgroups per compute
# unit (5120 on 256 CUs), each taking two or more claims by index before any from a counter: with
# regions of about 4 items, 2^22 parents make over 16000 claims, so every candidate's launch takes
# claims both by index and from the counters.
CAND_PARENTS = 1 << 22


def candidate_inputs(kind):
    if kind == rs.RS_TEXT_WORDS:
        text, starts, lengths = workloads.text_workload(seed=31, total_bytes=40 << 20, mean_len=8.0, max_len=300)
        return dict(offsets=starts, elements=text, lengths=lengths), oracle.run(
            oracle.TEXT_WORDS, starts, text, lengths=lengths)
    if kind == rs.RS_GRAPH_THRESH:
        offsets, w, thr, _ = workloads.graph_workload(seed=32, n_vertices=CAND_PARENTS, n_edges=CAND_PARENTS * 4)
        return dict(offsets=offsets, elements=w, parent_param=thr), oracle.run(
            oracle.GRAPH_THRESH, offsets, w, parent_param=thr)
    offsets = workloads.uniform_offsets(33, CAND_PARENTS, 8)
    vals = workloads.hash_values(34, int(offsets[-1]))
    ok = oracle.MODFILTER if kind == rs.RS_MODFILTER else oracle.HASH_EXPAND
    param = (4, 0, 0, 0) if kind == rs.RS_MODFILTER else (0, 0, 0, 0)
    return dict(offsets=offsets, elements=vals, param=param), oracle.run(ok, offsets, vals, param=param)


_CAND = {}


@pytest.mark.parametrize("width", WIDTHS)
@pytest.mark.parametrize("strategy", ALL3 + [rs.RS_ENUM_TAG])
@pytest.mark.parametrize("kind", [rs.RS_MODFILTER, rs.RS_HASH_EXPAND, rs.RS_TEXT_WORDS, rs.RS_GRAPH_THRESH])
def test_every_autotune_candidate(kind, strategy, width):
    """Each (kind, strategy, width) that RS_AUTO may select, against the oracle (§3.3: the SIMD rule
    holds at any ensemble width)."""
    skip_unoffered(kind, strategy, width)
    if kind not in _CAND:
        _CAND.clear()
        _CAND[kind] = candidate_inputs(kind)
    inp, ref = _CAND[kind]
    say("candidate", kind, SNAME[strategy], width)
    fields = rs.DEFAULT_FIELDS[kind]
    got, _ = run_one(kind, strategy, width, inp["offsets"], inp["elements"], lengths=inp.get("lengths"),
                     parent_param=inp.get("parent_param"), param=inp.get("param", (0, 0, 0, 0)), fields=fields,
                     device=True)
    check(got, ref, [n for n, bit, _ in rs.FIELDS if fields & bit], f"candidate {kind} {SNAME[strategy]} w={width}")


@pytest.mark.parametrize("factor", [4, 8])
@pytest.mark.parametrize("width", [64, 256])
@pytest.mark.parametrize("strategy", ALL3 + [rs.RS_ENUM_TAG])
@pytest.mark.parametrize("kind", [rs.RS_MODFILTER, rs.RS_HASH_EXPAND, rs.RS_TEXT_WORDS, rs.RS_GRAPH_THRESH])
def test_queue_depths(kind, strategy, width, factor):
    """Queue depths 4w and 8w (every other test runs the default 2w; the autotuner picks 2w or 4w)
    against the oracle: a node fires against the space left in its downstream queue (§3.2), so the
    depth changes when nodes fire, never what they compute."""
    skip_unoffered(kind, strategy, width)
    if kind not in _CAND:
        _CAND.clear()
        _CAND[kind] = candidate_inputs(kind)
    inp, ref = _CAND[kind]
    say("queue depth", kind, SNAME[strategy], width, factor * width)
    fields = rs.DEFAULT_FIELDS[kind]
    got, st = run_one(kind, strategy, width, inp["offsets"], inp["elements"], lengths=inp.get("lengths"),
                      parent_param=inp.get("parent_param"), param=inp.get("param", (0, 0, 0, 0)), fields=fields,
                      device=True, queue_depth=factor * width, flags=rs.RS_COLLECT_STATS)
    assert st.queue_depth == factor * width
    check(got, ref, [n for n, bit, _ in rs.FIELDS if fields & bit],
          f"queue depth {factor}w {kind} {SNAME[strategy]} w={width}")


def test_lookback_give_up_reports_a_device_error(monkeypatch):
    """A look-back wait bounded at zero: a claim that finds a predecessor's count unpublished gives
    up at once, writes no outputs and raises the launch's error flag.  Every wave still finishes:
    the run either reports RS_EDEVICE or, when no claim had to wait, returns the exact stream.  A
    pipeline with the normal bound then runs exactly."""
    n = 1 << 22
    offsets = workloads.fixed_offsets(n, 16)
    vals = workloads.hash_values(2, n)
    ref = oracle.run(oracle.HASH_EXPAND, offsets, vals, emit_outputs=True)
    say("look-back give-up")
    monkeypatch.setenv("RS_LOOKBACK_WAIT_US", "0")
    with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=rs.RS_TAG, ensemble_width=256, emit_outputs=True) as p:
        sid = p.push(offsets, vals)
        try:
            p.run()
            check(p.read(sid), ref, where="zero bound")
            assert np.array_equal(p.outputs(sid), ref.out)
        except rs.RsError as e:
            assert e.code == rs.RS_EDEVICE and "watchdog" in str(e)
    monkeypatch.delenv("RS_LOOKBACK_WAIT_US")
    with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=rs.RS_TAG, ensemble_width=256, emit_outputs=True) as p:
        sid = p.push(offsets, vals)
        p.run()
        check(p.read(sid), ref, where="normal bound")
        assert np.array_equal(p.outputs(sid), ref.out)


# ---- serving: continuous batching under an HBM budget ----

def test_serving_results_equal_alone_and_in_the_mix():
    say("serving")
    n_req = 48
    shapes_n, shapes_m = workloads.stream_shapes(seed=5, n_streams=n_req, lo_n=1e3, hi_n=2e5)
    reqs = [workloads.serving_stream(5, s, int(shapes_n[s]), float(shapes_m[s])) for s in range(n_req)]
    arrivals = np.sort(workloads.arrivals(6, n_req, 2000.0))
    refs = [oracle.run(oracle.HASH_EXPAND, o, v) for o, v in reqs]
    budget = 3 * 1024 * 1024   # total footprint is about 10 MB: admission must gate
    for per_stream in (False, True):
        with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=rs.RS_TAG, ensemble_width=256, hbm_budget_bytes=budget) as p:
            results, timings = p.serve(reqs, arrivals, per_stream=per_stream)
        for i in range(n_req):
            assert timings[i]["status"] == 0
            assert timings[i]["completed"] >= timings[i]["arrival"]
            check(results[i], refs[i], where=f"serve request {i}")
        if not per_stream:
            assert len({t["batch"] for t in timings}) < n_req     # requests shared launches
    # each request alone gives the same result
    for i in (0, 7, 31):
        got, _ = run_one(rs.RS_HASH_EXPAND, rs.RS_SIGNAL, 128, *reqs[i])
        check(got, refs[i], where=f"alone {i}")


def test_serving_device_requests_into_device_outputs():
    """RS_SERVE_DEVICE_OUT: device-resident requests whose aggregates the kernel writes straight
    into the caller's device arrays equal the oracle, batched and one launch per request."""
    import torch
    say("serving device outputs")
    n_req = 40
    shapes_n, shapes_m = workloads.stream_shapes(seed=5, n_streams=n_req, lo_n=1e3, hi_n=2e5)
    reqs = [workloads.serving_stream(5, s, int(shapes_n[s]), float(shapes_m[s])) for s in range(n_req)]
    arrivals = np.sort(workloads.arrivals(6, n_req, 4000.0))
    refs = [oracle.run(oracle.HASH_EXPAND, o, v) for o, v in reqs]
    dev = [(torch.from_numpy(o.view(np.int32)).cuda(), torch.from_numpy(v.view(np.int32)).cuda()) for o, v in reqs]
    tdt = {np.uint32: torch.int32, np.uint64: torch.int64}
    for per_stream in (False, True):
        outs = []
        for o, v in reqs:
            P = len(o) - 1
            outs.append({name: torch.full((max(P, 1),), -1, dtype=tdt[dt], device="cuda")
                         for name, bit, dt in rs.FIELDS if rs.DEFAULT_FIELDS[rs.RS_HASH_EXPAND] & bit})
        with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=rs.RS_TAG, ensemble_width=256) as p:
            results, timings = p.serve(dev, arrivals, per_stream=per_stream, device_out=outs)
        torch.cuda.synchronize()
        for i in range(n_req):
            assert timings[i]["status"] == 0
            got = {k: t.cpu().numpy().view(dict(count=np.uint32, sum=np.uint64, min=np.uint32,
                                                   max=np.uint32)[k]) for k, t in results[i].items()}
            check(got, refs[i], where=f"device-out request {i} per_stream={per_stream}")
    with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=rs.RS_TAG, ensemble_width=256) as p:
        missing = [dict(outs[0])]
        missing[0].pop("min")
        with pytest.raises(rs.RsError) as ei:
            p.serve(dev[:1], [0.0], device_out=missing)
        assert ei.value.code == rs.RS_EINVAL


def test_serving_rejects_a_request_larger_than_the_budget():
    o, v = workloads.serving_stream(5, 0, 100000, 10.0)
    with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=rs.RS_TAG, ensemble_width=256, hbm_budget_bytes=1000) as p:
        with pytest.raises(rs.RsError) as ei:
            p.serve([(o, v)], [0.0])
        assert ei.value.code == rs.RS_EBUDGET


def test_kernel_times_cover_every_timed_launch():
    """RS_TIME_KERNEL: one device time per run/run_again, in launch order, inside the host-side
    span of the launches, and the timed launches still compute the oracle's results."""
    import time
    import torch
    say("kernel times")
    n, L = 1 << 20, 256
    offsets = workloads.fixed_offsets(n, L)
    vals = workloads.hash_values(7, n)
    ref = oracle.run(oracle.HASH_EXPAND, offsets, vals)
    with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=rs.RS_SIGNAL, ensemble_width=128, flags=rs.RS_TIME_KERNEL) as p:
        sid = p.push(offsets, vals)
        p.run()
        first = p.kernel_times()
        assert len(first) == 1 and first[0] > 0.0
        assert p.kernel_times() == []   # consumed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            p.run_again(rs.RS_RUN_ASYNC)
        got_t = p.kernel_times()
        span_ms = (time.perf_counter() - t0) * 1e3
        assert len(got_t) == 5 and all(t > 0.0 for t in got_t)
        assert sum(got_t) <= span_ms
        check(p.read(sid), ref, where="timed launches")
    with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=rs.RS_TAG, ensemble_width=128) as p:
        with pytest.raises(rs.RsError) as ei:
            p.kernel_times()
        assert ei.value.code == rs.RS_EINVAL


# ---- per-stage choice: enumeration in the first stage, tags after it (the second taxi version) ----

@pytest.mark.parametrize("L", [1, 4, 16, 64, 256, 1024, 4096])
def test_enum_tag_hash_fixed_L(L):
    n = (1 << 18) + 13
    say("enum+tag hash/expand L", L)
    offsets = workloads.fixed_offsets(n, L)
    vals = workloads.hash_values(2, n)
    ref = oracle.run(oracle.HASH_EXPAND, offsets, vals)
    got, st = run_one(rs.RS_HASH_EXPAND, rs.RS_ENUM_TAG, 256, offsets, vals, flags=rs.RS_COLLECT_STATS)
    check(got, ref, where=f"enum+tag L={L}")
    # the enumerating node's ensembles stop at region ends, as under signals; no signal travels
    assert st.items[0] == n and st.firings[0] >= len(offsets) - 1
    assert sum(st.signals) == 0


@pytest.mark.parametrize("width", WIDTHS)
def test_enum_tag_widths(width):
    say("enum+tag widths", width)
    offsets = workloads.uniform_offsets(5, 3000, 300)
    vals = workloads.hash_values(5, int(offsets[-1]))
    ref = oracle.run(oracle.HASH_EXPAND, offsets, vals)
    got, _ = run_one(rs.RS_HASH_EXPAND, rs.RS_ENUM_TAG, width, offsets, vals)
    check(got, ref, where=f"enum+tag hash width {width}")
    text, starts, lengths = workloads.text_workload(seed=3, total_bytes=1 << 20)
    ref = oracle.run(oracle.TEXT_WORDS, starts, text, lengths=lengths)
    got, _ = run_one(rs.RS_TEXT_WORDS, rs.RS_ENUM_TAG, width, starts, text, lengths=lengths)
    check(got, ref, ("count", "max"), where=f"enum+tag text width {width}")


@pytest.mark.parametrize("name", ["e2_hash_expand.json", "e3_text_words.json"])
@pytest.mark.parametrize("width", [64, 256])
def test_enum_tag_golden_streams(name, width):
    test_golden_streams(name, rs.RS_ENUM_TAG, width)


def test_enum_tag_edge_cases():
    say("enum+tag edge cases")
    offs = np.zeros(1001, np.uint32)
    got, _ = run_one(rs.RS_HASH_EXPAND, rs.RS_ENUM_TAG, 256, offs, np.zeros(4, np.uint32))
    assert (got["count"] == 0).all() and (got["min"] == 0xFFFFFFFF).all() and (got["max"] == 0).all()
    vals = workloads.hash_values(3, 200003)
    offs = np.array([0, 200003], np.uint32)
    check(run_one(rs.RS_HASH_EXPAND, rs.RS_ENUM_TAG, 256, offs, vals)[0], oracle.run(oracle.HASH_EXPAND, offs, vals),
          where="enum+tag one parent")
    vals = workloads.hash_values(4, 5000)
    offs = np.array([7, 7, 100, 2500, 4990], np.uint32)
    check(run_one(rs.RS_HASH_EXPAND, rs.RS_ENUM_TAG, 128, offs, vals)[0], oracle.run(oracle.HASH_EXPAND, offs, vals),
          where="enum+tag offset start")


@pytest.mark.parametrize("L", [1, 7, 300, 5000])
def test_enum_tag_output_stream(L):
    say("enum+tag outputs", L)
    n = 150001
    offsets = workloads.fixed_offsets(n, L)
    vals = workloads.hash_values(9, n)
    ref = oracle.run(oracle.HASH_EXPAND, offsets, vals, emit_outputs=True)
    got, out = run_outputs(rs.RS_HASH_EXPAND, rs.RS_ENUM_TAG, 256, offsets, vals)
    check(got, ref, where="enum+tag outputs agg")
    assert len(out) == len(ref.out) and np.array_equal(out, ref.out)
    text, starts, lengths = workloads.text_workload(seed=3, total_bytes=1 << 19)
    ref = oracle.run(oracle.TEXT_WORDS, starts, text, lengths=lengths, emit_outputs=True)
    _, out = run_outputs(rs.RS_TEXT_WORDS, rs.RS_ENUM_TAG, 256, starts, text, lengths=lengths)
    assert np.array_equal(out, ref.out)


@pytest.mark.parametrize("width", [64, 128, 256])
def test_taxi_shape_three_versions(width):
    """The paper's three taxi versions on taxi-shaped text (lines of 1397 characters on average,
    about 45 markers each): both stages enumerated (signals), the first enumerated and tags
    after it, neither enumerated (tags).  Each equals the oracle; the first stage's full-ensemble
    share is high under enumeration and the second's is low under signals only."""
    text, starts, lengths = workloads.taxi_workload(seed=9, total_bytes=1 << 23)
    ref = oracle.run(oracle.TEXT_WORDS, starts, text, lengths=lengths)
    full = {}
    for s in (rs.RS_SIGNAL, rs.RS_ENUM_TAG, rs.RS_TAG):
        say("taxi", SNAME[s], width)
        got, st = run_one(rs.RS_TEXT_WORDS, s, width, starts, text, lengths=lengths, fields=rs.RS_COUNT | rs.RS_MAX,
                          flags=rs.RS_COLLECT_STATS)
        check(got, ref, ("count", "max"), where=f"taxi {SNAME[s]} w={width}")
        full[s] = [st.full[k] / max(1, st.firings[k]) for k in range(3)]
    assert full[rs.RS_SIGNAL][0] > 0.5 and full[rs.RS_ENUM_TAG][0] > 0.5     # stage 1: long regions
    assert full[rs.RS_ENUM_TAG][1] > full[rs.RS_SIGNAL][1]                  # stage 2: tags fill ensembles


# ---- tree topology: the filter feeds the expansion and a second sink (RS_HASH_TREE) ----

TREE_FIELDS = ("count", "sum", "min", "max", "kept_count", "kept_sum")
TREE_STRATS = ALL3 + [rs.RS_ENUM_TAG]


@pytest.mark.parametrize("L", [1, 5, 16, 64, 256, 1000, 4096])
@pytest.mark.parametrize("strategy", TREE_STRATS)
def test_tree_fixed_L(L, strategy):
    n = (1 << 18) + 13
    say("tree L", L, SNAME[strategy])
    offsets = workloads.fixed_offsets(n, L)
    vals = workloads.hash_values(2, n)
    ref = oracle.run(oracle.HASH_TREE, offsets, vals)
    got, _ = run_one(rs.RS_HASH_TREE, strategy, 256, offsets, vals, fields=rs.DEFAULT_FIELDS[rs.RS_HASH_TREE])
    check(got, ref, TREE_FIELDS, f"tree L={L} {SNAME[strategy]}")


@pytest.mark.parametrize("width", WIDTHS)
@pytest.mark.parametrize("strategy", TREE_STRATS)
def test_tree_widths_variable_regions(width, strategy):
    skip_unoffered(rs.RS_HASH_TREE, strategy, width)
    say("tree width", width, SNAME[strategy])
    offsets = workloads.uniform_offsets(5, 3000, 300)
    vals = workloads.hash_values(5, int(offsets[-1]))
    ref = oracle.run(oracle.HASH_TREE, offsets, vals)
    got, _ = run_one(rs.RS_HASH_TREE, strategy, width, offsets, vals, fields=rs.DEFAULT_FIELDS[rs.RS_HASH_TREE],
                     device=True)
    check(got, ref, TREE_FIELDS, f"tree width {width} {SNAME[strategy]}")


@pytest.mark.parametrize("strategy", TREE_STRATS)
def test_tree_edge_cases_and_second_sink_alone(strategy):
    say("tree edge cases", SNAME[strategy])
    offs = np.zeros(1001, np.uint32)
    got, _ = run_one(rs.RS_HASH_TREE, strategy, 256, offs, np.zeros(4, np.uint32),
                     fields=rs.DEFAULT_FIELDS[rs.RS_HASH_TREE])
    assert (got["kept_count"] == 0).all() and (got["kept_sum"] == 0).all() and (got["count"] == 0).all()
    vals = workloads.hash_values(4, 5000)
    offs = np.array([7, 7, 100, 2500, 4990], np.uint32)
    ref = oracle.run(oracle.HASH_TREE, offs, vals)
    got, _ = run_one(rs.RS_HASH_TREE, strategy, 128, offs, vals, fields=rs.DEFAULT_FIELDS[rs.RS_HASH_TREE])
    check(got, ref, TREE_FIELDS, "tree offset start")
    # the second sink alone
    got, _ = run_one(rs.RS_HASH_TREE, strategy, 64, offs, vals, fields=rs.RS_KEPT_COUNT | rs.RS_KEPT_SUM)
    check(got, ref, ("kept_count", "kept_sum"), "tree second sink alone")


@pytest.mark.parametrize("strategy", TREE_STRATS)
def test_tree_output_stream_and_batch(strategy):
    """The first sink's ordered output stream equals the linear pipeline's; a batch of streams of
    very different region lengths gives each stream's own records."""
    say("tree outputs and batch", SNAME[strategy])
    n = 150001
    offsets = workloads.fixed_offsets(n, 37)
    vals = workloads.hash_values(9, n)
    ref = oracle.run(oracle.HASH_TREE, offsets, vals, emit_outputs=True)
    with rs.Pipeline(rs.RS_HASH_TREE, strategy=strategy, ensemble_width=256, emit_outputs=True) as p:
        sid = p.push(offsets, vals)
        p.run()
        got, out = p.read(sid), p.outputs(sid)
    check(got, ref, TREE_FIELDS, "tree outputs agg")
    assert np.array_equal(out, ref.out)
    shapes = [(5000, 1.0), (60000, 37.5), (100000, 700.0), (7, 3.0)]
    ins = [workloads.serving_stream(51, i, nn, m) for i, (nn, m) in enumerate(shapes)]
    with rs.Pipeline(rs.RS_HASH_TREE, strategy=strategy, ensemble_width=128) as p:
        ids = [p.push(o, v) for o, v in ins]
        p.run()
        for i, (o, v) in zip(ids, ins):
            check(p.read(i), oracle.run(oracle.HASH_TREE, o, v), TREE_FIELDS, "tree batch")


# ---- fused runs across region boundaries near multiples of w ----

@pytest.mark.parametrize("strategy", [rs.RS_TAG, rs.RS_SIGNAL, rs.RS_SIGNAL_LANES, rs.RS_ENUM_TAG])
@pytest.mark.parametrize("kind", [rs.RS_HASH_EXPAND, rs.RS_HASH_TREE])
def test_fused_runs_around_region_boundaries(kind, strategy):
    """Region lengths just below, at and above multiples of w = 256 (and empty, single-element and
    long regions) in a seeded order: fused runs start, cross region ends and stop at every kind of
    boundary, including the cached next-region bound that lets a run under tags skip the region
    table."""
    say("fused boundaries", kind, SNAME[strategy])
    rng = np.random.default_rng(11)
    menu = np.array([0, 1, 3, 255, 256, 257, 511, 512, 513, 768, 1024, 1280, 4096, 5000], np.int64)
    sizes = rng.choice(menu, size=1500)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)
    vals = workloads.hash_values(5, int(offsets[-1]))
    oc = oracle.HASH_TREE if kind == rs.RS_HASH_TREE else oracle.HASH_EXPAND
    ref = oracle.run(oc, offsets, vals)
    fields = rs.DEFAULT_FIELDS[kind]
    got, _ = run_one(kind, strategy, 256, offsets, vals, fields=fields)
    check(got, ref, TREE_FIELDS if kind == rs.RS_HASH_TREE else ("count", "sum", "min", "max"),
          f"fused boundaries {kind} {SNAME[strategy]}")
