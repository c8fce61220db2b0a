"""GPU parity at the full workload sizes, in the launch configuration the benchmark
times (strategy fixed, ensemble width from the autotuner), against the serial oracle
on every parent (integer results: bit-exact)."""
import os
import sys

import numpy as np
import pytest

import oracle
import workloads
import paper_2006_07478_amd as rs

pytestmark = pytest.mark.gpu

STRATS = [rs.RS_TAG, rs.RS_SIGNAL]
ALL3 = STRATS + [rs.RS_SIGNAL_LANES]   # lane-resolved signals: u32 kinds
SNAME = {rs.RS_TAG: "tag", rs.RS_SIGNAL: "signal", rs.RS_SIGNAL_LANES: "lanes"}


@pytest.fixture(scope="module", autouse=True)
def gpu(tmp_path_factory):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    os.environ.setdefault("RS_AUTOTUNE_CACHE", str(tmp_path_factory.mktemp("tune") / "cache.txt"))
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32 if a.dtype == np.uint32 else np.uint8)).cuda()


def check(got, ref, fields, where):
    for f in fields:
        g, r = got[f], getattr(ref, f)
        if not np.array_equal(g, r):
            bad = np.nonzero(g != r)[0]
            raise AssertionError(f"{where}: {f} differs at {len(bad)} parents, first {bad[:5].tolist()}")


def run_dev(kind, strategy, offsets, elements, lengths=None, parent_param=None, fields=None):
    with rs.Pipeline(kind, strategy=strategy, ensemble_width=0, agg_fields=fields) as p:
        sid = p.push(dev(offsets), dev(elements), lengths=None if lengths is None else dev(lengths),
                     parent_param=None if parent_param is None else dev(parent_param), n_elements=len(elements))
        p.run()
        return p.read(sid), p.stats(sid)


@pytest.mark.parametrize("L", [1, 4, 16, 64, 256, 1024, 4096])
def test_hash_expand_2p26(L):
    n = 1 << 26
    offsets = workloads.fixed_offsets(n, L)
    vals = workloads.hash_values(2, n)
    ref = oracle.run(oracle.HASH_EXPAND, offsets, vals)
    for s in ALL3:
        say("2^26 hash/expand L", L, SNAME[s])
        got, st = run_dev(rs.RS_HASH_EXPAND, s, offsets, vals)
        say("   ensemble width", st.ensemble_width)
        check(got, ref, ("count", "sum", "min", "max"), f"2^26 L={L} {SNAME[s]}")


def test_output_stream_2p26():
    """The ordered output stream at the headline size, as the benchmark times it (widths from the
    autotuner): every output item in order, and the records."""
    n = 1 << 26
    offsets = workloads.fixed_offsets(n, 4096)
    vals = workloads.hash_values(2, n)
    ref = oracle.run(oracle.HASH_EXPAND, offsets, vals, emit_outputs=True)
    for s in ALL3:
        say("2^26 output stream L 4096", SNAME[s])
        with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=s, ensemble_width=0, emit_outputs=True) as p:
            sid = p.push(dev(offsets), dev(vals), n_elements=n)
            p.run()
            got, out = p.read(sid), p.outputs(sid)
        check(got, ref, ("count", "sum", "min", "max"), f"2^26 outputs {SNAME[s]}")
        assert len(out) == len(ref.out) and np.array_equal(out, ref.out), f"2^26 output items {SNAME[s]}"


def test_output_stream_2p26_L16():
    """The ordered output stream at 2^26 elements in regions of 16, with the widths the autotuner
    picks: claims of 255 parents, over 16000 of them, whose look-backs once waited on claims
    owned by waves that had not started.  Claims now come from one ascending counter."""
    n = 1 << 26
    offsets = workloads.fixed_offsets(n, 16)
    vals = workloads.hash_values(2, n)
    ref = oracle.run(oracle.HASH_EXPAND, offsets, vals, emit_outputs=True)
    for s in ALL3:
        say("2^26 output stream L 16", SNAME[s])
        with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=s, ensemble_width=0, emit_outputs=True) as p:
            sid = p.push(dev(offsets), dev(vals), n_elements=n)
            p.run()
            say("   ensemble width", p.stats(sid).ensemble_width)
            got, out = p.read(sid), p.outputs(sid)
        check(got, ref, ("count", "sum", "min", "max"), f"2^26 L=16 outputs {SNAME[s]}")
        assert len(out) == len(ref.out) and np.array_equal(out, ref.out), f"2^26 L=16 output items {SNAME[s]}"


@pytest.mark.parametrize("mx", [16, 32, 2048])
def test_variable_sizes_2p26(mx):
    """The variable-size sweep at its full size: region sizes uniform in [0, max] (max = 32: tags
    fold many mid-size regions per 8-lane block)."""
    n = 1 << 26
    offsets = workloads.variable_offsets(13, n, mx)
    vals = workloads.hash_values(2, n)
    ref = oracle.run(oracle.HASH_EXPAND, offsets, vals)
    for s in ALL3:
        say("2^26 variable sizes max", mx, SNAME[s])
        got, st = run_dev(rs.RS_HASH_EXPAND, s, offsets, vals)
        check(got, ref, ("count", "sum", "min", "max"), f"2^26 variable max={mx} {SNAME[s]}")


def test_taxi_shape_1gib():
    """The taxi-shaped text at 1 GiB under the three versions of §5 (signals; enumeration then
    tags; tags)."""
    text, starts, lengths = workloads.taxi_workload(seed=9, total_bytes=1 << 30)
    say("taxi 1 GiB:", len(starts), "lines")
    ref = oracle.run(oracle.TEXT_WORDS, starts, text, lengths=lengths)
    for s in (rs.RS_SIGNAL, rs.RS_ENUM_TAG, rs.RS_TAG):
        say("taxi 1 GiB", s)
        got, st = run_dev(rs.RS_TEXT_WORDS, s, starts, text, lengths=lengths, fields=rs.RS_COUNT | rs.RS_MAX)
        check(got, ref, ("count", "max"), f"taxi {s}")


def test_enum_tag_2p26():
    """Enumeration then tags at the headline size, short and long regions."""
    n = 1 << 26
    vals = workloads.hash_values(2, n)
    for L in (16, 4096):
        offsets = workloads.fixed_offsets(n, L)
        ref = oracle.run(oracle.HASH_EXPAND, offsets, vals)
        say("2^26 enum+tag L", L)
        got, _ = run_dev(rs.RS_HASH_EXPAND, rs.RS_ENUM_TAG, offsets, vals)
        check(got, ref, ("count", "sum", "min", "max"), f"2^26 enum+tag L={L}")


def test_text_1gib():
    text, starts, lengths = workloads.text_workload(seed=3, total_bytes=1 << 30)
    say("text 1 GiB:", len(starts), "lines")
    ref = oracle.run(oracle.TEXT_WORDS, starts, text, lengths=lengths)
    for s in STRATS:
        say("text 1 GiB", SNAME[s])
        got, st = run_dev(rs.RS_TEXT_WORDS, s, starts, text, lengths=lengths,
                          fields=rs.RS_COUNT | rs.RS_MAX)
        check(got, ref, ("count", "max"), f"text {SNAME[s]}")


def test_graph_2p24_vertices_2p28_edges():
    offsets, w, thr, beta = workloads.graph_workload(seed=4)
    say("graph: beta", beta, "max degree", int(np.diff(offsets.astype(np.int64)).max()))
    ref = oracle.run(oracle.GRAPH_THRESH, offsets, w, parent_param=thr)
    for s in ALL3:
        say("graph", SNAME[s])
        got, st = run_dev(rs.RS_GRAPH_THRESH, s, offsets, w, parent_param=thr, fields=rs.RS_COUNT | rs.RS_SUM)
        check(got, ref, ("count", "sum"), f"graph {SNAME[s]}")


def test_serving_512_streams_one_batch():
    n, m = workloads.stream_shapes(seed=5, n_streams=512)
    say("512 streams,", int(n.sum()), "elements")
    with rs.Pipeline(rs.RS_HASH_EXPAND, strategy=rs.RS_AUTO, ensemble_width=0) as p:
        ids, streams = [], []
        for s in range(512):
            o, v = workloads.serving_stream(5, s, int(n[s]), float(m[s]))
            ids.append(p.push(o, v))
            streams.append((o, v))
        p.run()
        for s in range(512):
            o, v = streams[s]
            ref = oracle.run(oracle.HASH_EXPAND, o, v)
            check(p.read(ids[s]), ref, ("count", "sum", "min", "max"), f"stream {s}")


@pytest.mark.parametrize("L", [16, 4096])
def test_tree_2p26(L):
    """The tree topology at the headline size, widths from the autotuner."""
    n = 1 << 26
    offsets = workloads.fixed_offsets(n, L)
    vals = workloads.hash_values(2, n)
    ref = oracle.run(oracle.HASH_TREE, offsets, vals)
    for s in ALL3 + [rs.RS_ENUM_TAG]:
        say("2^26 tree L", L, s)
        got, _ = run_dev(rs.RS_HASH_TREE, s, offsets, vals, fields=rs.DEFAULT_FIELDS[rs.RS_HASH_TREE])
        check(got, ref, ("count", "sum", "min", "max", "kept_count", "kept_sum"), f"2^26 tree L={L} {s}")
