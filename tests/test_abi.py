"""The C-ABI library loads on a machine without a GPU, exports every entry point that
include/regionstream.h declares, and rejects malformed pipeline descriptions before
touching the device."""
import ctypes
import os
import re

import pytest

import paper_2006_07478_amd as rs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "regionstream.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_abi():
    names = declared_functions()
    for required in ("pipeline_create", "stream_push", "run", "read_aggregates"):
        assert required in names
    assert set(names) == set(rs.ABI_FUNCTIONS)


def test_library_exports_every_declared_symbol():
    L = rs.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_no_extra_exports():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", rs.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.split() and l.split()[1] == "T"}
    exported = {n for n in exported if not n.startswith("_")}
    assert exported == set(declared_functions())


def _desc(**kw):
    d = rs.rs_pipeline_desc()
    d.abi_version = rs.ABI_VERSION
    d.kind = rs.RS_HASH_EXPAND
    d.strategy = rs.RS_TAG
    d.agg_fields = rs.RS_COUNT | rs.RS_SUM
    d.ensemble_width = 256
    for k, v in kw.items():
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("bad", [
    dict(abi_version=99), dict(kind=0), dict(kind=9), dict(strategy=7), dict(agg_fields=0),
    dict(agg_fields=16), dict(ensemble_width=100), dict(ensemble_width=2048), dict(queue_depth=300),
    dict(queue_depth=256), dict(queue_depth=4096), dict(emit_outputs=2), dict(agg_fields=16),
    dict(kind=6), dict(kind=5, agg_fields=64),
])
def test_bad_descriptions_are_rejected_on_the_host(bad):
    h = ctypes.c_void_p()
    rc = rs.lib().pipeline_create(ctypes.byref(_desc(**bad)), ctypes.byref(h))
    assert rc == rs.RS_EINVAL
    assert h.value is None
    assert rs.rs_last_error()


def test_null_arguments():
    assert rs.lib().pipeline_create(None, None) == rs.RS_EINVAL
    assert rs.lib().run(None, 0) == rs.RS_EINVAL
    assert rs.lib().read_aggregates(None, 1, None, 0) == rs.RS_EINVAL
    assert rs.lib().pipeline_destroy(None) == rs.RS_OK


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    monkeypatch.setattr(rs, "_lib", None)
    monkeypatch.setattr(rs, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        rs.lib()


def test_noalloc_rejects_more_streams_than_its_scratch_holds():
    """The no-allocation entry point refuses a call beyond its fixed table (16 streams) before
    touching any device."""
    d = _desc()
    n = rs.NOALLOC_MAX_STREAMS + 1
    sd = (rs.rs_stream_desc * n)()
    ov = (rs.rs_agg_view * n)()
    with pytest.raises(rs.RsError) as e:
        rs.run_noalloc(d, sd, n, ov)
    assert e.value.code == rs.RS_EINVAL and "16 streams" in str(e.value)


def test_noalloc_needs_an_explicit_configuration():
    """Autotuning allocates, so the no-allocation entry point takes an explicit strategy and width."""
    for kw in ({"strategy": rs.RS_AUTO}, {"ensemble_width": 0}, {"emit_outputs": 1}):
        d = _desc(**kw)
        sd = (rs.rs_stream_desc * 1)()
        ov = (rs.rs_agg_view * 1)()
        with pytest.raises(rs.RsError) as e:
            rs.run_noalloc(d, sd, 1, ov)
        assert e.value.code == rs.RS_EINVAL
