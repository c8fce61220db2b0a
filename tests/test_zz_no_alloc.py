"""The entry point that allocates nothing (run_noalloc) against the pipeline entry points
(pipeline_create / stream_push / run / read_aggregates) on the same device-resident inputs:
bit-identical aggregates on two calls in a row, the second with a smaller input, so that the
device state the calls share is shown to be cleared between them.  Both are also checked against
the serial oracle."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2006_07478_amd as rs
import workloads

pytestmark = pytest.mark.gpu


def _torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _dev(torch, a):
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a.view(np.int32)).cuda()


FIELDS = (("count", rs.RS_COUNT, np.uint32), ("sum", rs.RS_SUM, np.uint64), ("min", rs.RS_MIN, np.uint32),
          ("max", rs.RS_MAX, np.uint32))


def _reference(torch, kind, strategy, width, streams, fields):
    out = []
    with rs.Pipeline(kind, strategy=strategy, ensemble_width=width, agg_fields=fields) as p:
        ids = []
        for offs, vals, pp in streams:
            ids.append(p.push(_dev(torch, offs), _dev(torch, vals), parent_param=None if pp is None else _dev(torch, pp),
                              n_elements=len(vals)))
        p.run()
        out = [p.read(i) for i in ids]
    return out


def _noalloc(torch, kind, strategy, width, streams, fields):
    n = len(streams)
    d = rs.rs_pipeline_desc()
    d.abi_version = rs.ABI_VERSION
    d.kind = kind
    d.strategy = strategy
    d.agg_fields = fields
    d.ensemble_width = width
    sd = (rs.rs_stream_desc * n)()
    ov = (rs.rs_agg_view * n)()
    keep, res = [], []
    for i, (offs, vals, pp) in enumerate(streams):
        P = len(offs) - 1
        o, v = _dev(torch, offs), _dev(torch, vals)
        keep += [o, v]
        sd[i].mem = rs.RS_MEM_DEVICE
        sd[i].elem_bytes = 4
        sd[i].n_parents = P
        sd[i].n_elements = len(vals)
        sd[i].offsets = o.data_ptr()
        sd[i].lengths = None
        sd[i].elements = v.data_ptr()
        if pp is not None:
            t = _dev(torch, pp)
            keep.append(t)
            sd[i].parent_param = t.data_ptr()
        dst = {}
        for name, bit, dt in FIELDS:
            if fields & bit:
                a = torch.full((max(P, 1),), 7, dtype=torch.int64 if dt == np.uint64 else torch.int32, device="cuda")
                dst[name] = a
                setattr(ov[i], name, a.data_ptr())
        res.append((dst, P))
    torch.cuda.synchronize()
    rs.run_noalloc(d, sd, n, ov, None, rs.RS_RUN_SYNC)
    return [{k: a.cpu().numpy().view(np.uint64 if k == "sum" else np.uint32)[:P] for k, a in dst.items()}
            for dst, P in res]


def _check(got, ref, want, fields, what):
    for name, bit, _ in FIELDS:
        if fields & bit:
            assert np.array_equal(got[name], ref[name]), f"{what}: {name} differs from the pipeline entry points"
            assert np.array_equal(got[name], getattr(want, name)), f"{what}: {name} differs from the oracle"


def _hash_streams(scale):
    n1, n2, n3 = 300_000 // scale, 200_000 // scale, 65_536 // scale
    return [(workloads.fixed_offsets(n1, 37), workloads.hash_values(11, n1), None),
            (workloads.variable_offsets(12, n2, 40), workloads.hash_values(12, n2), None),
            (workloads.fixed_offsets(n3, 4096), workloads.hash_values(13, n3), None)]


@pytest.mark.parametrize("strategy", [rs.RS_TAG, rs.RS_SIGNAL, rs.RS_SIGNAL_LANES])
def test_noalloc_equals_the_pipeline_entry_points_twice(strategy):
    torch = _torch()
    fields = rs.RS_COUNT | rs.RS_SUM | rs.RS_MIN | rs.RS_MAX
    for call, streams in enumerate((_hash_streams(1), _hash_streams(8)[:1])):   # the second call is smaller
        ref = _reference(torch, rs.RS_HASH_EXPAND, strategy, 256, streams, fields)
        got = _noalloc(torch, rs.RS_HASH_EXPAND, strategy, 256, streams, fields)
        for i, (offs, vals, _) in enumerate(streams):
            want = oracle.run(oracle.HASH_EXPAND, offs, vals)
            _check(got[i], ref[i], want, fields, f"call {call} stream {i} strategy {strategy}")


def test_noalloc_graph_kind_with_context_twice():
    torch = _torch()
    fields = rs.RS_COUNT | rs.RS_SUM
    for call, (nv, ne) in enumerate(((20_000, 320_000), (3_000, 40_000))):
        offs, w, thr, _ = workloads.graph_workload(4 + call, nv, ne)
        streams = [(offs, w, thr)]
        ref = _reference(torch, rs.RS_GRAPH_THRESH, rs.RS_TAG, 128, streams, fields)
        got = _noalloc(torch, rs.RS_GRAPH_THRESH, rs.RS_TAG, 128, streams, fields)
        want = oracle.run(oracle.GRAPH_THRESH, offs, w, parent_param=thr)
        _check(got[0], ref[0], want, fields, f"graph call {call}")
