"""ctypes binding of libregionstream.so (include/regionstream.h).

Argument marshalling only: every step of the computation runs in the library's
HIP kernels.  Functions keep the C names; ``Pipeline`` is a small convenience
wrapper that accepts numpy arrays (copied by the library) or torch device
tensors (borrowed by pointer).  If the library has not been built this module
raises on first use rather than falling back to anything else.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libregionstream.so")

ABI_VERSION = 1
RS_OK, RS_EINVAL, RS_ENOMEM, RS_EDEVICE, RS_EBUDGET, RS_ENOTREADY, RS_ESTATE, RS_ENOTFOUND = 0, -1, -2, -3, -4, -5, -6, -7
RS_TAG, RS_SIGNAL, RS_AUTO, RS_SIGNAL_LANES, RS_ENUM_TAG = 0, 1, 2, 3, 4
RS_MODFILTER, RS_HASH_EXPAND, RS_TEXT_WORDS, RS_GRAPH_THRESH, RS_HASH_TREE = 1, 2, 3, 4, 5
RS_COUNT, RS_SUM, RS_MIN, RS_MAX, RS_KEPT_COUNT, RS_KEPT_SUM = 1, 2, 4, 8, 16, 32
RS_MEM_HOST, RS_MEM_DEVICE = 0, 1
RS_RUN_SYNC, RS_RUN_ASYNC, RS_RUN_PER_STREAM = 0, 1, 2
RS_SERVE_DEVICE_OUT = 8
RS_READ_BLOCK, RS_NONBLOCK, RS_READ_DEVICE, RS_READ_RELEASE = 0, 1, 2, 4
RS_COLLECT_STATS, RS_NO_GRAPH, RS_TIME_KERNEL = 1, 2, 4

STATUS_NAMES = {0: "RS_OK", -1: "RS_EINVAL", -2: "RS_ENOMEM", -3: "RS_EDEVICE", -4: "RS_EBUDGET",
                -5: "RS_ENOTREADY", -6: "RS_ESTATE", -7: "RS_ENOTFOUND"}

ABI_FUNCTIONS = ["pipeline_create", "pipeline_set_stream", "stream_push", "run", "run_again",
                 "read_aggregates", "read_outputs", "rs_stats", "kernel_times", "stream_release", "serve", "hbm_probe",
                 "run_noalloc", "pipeline_destroy", "rs_last_error"]
NOALLOC_MAX_STREAMS = 16


class RsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class rs_pipeline_desc(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("kind", ctypes.c_uint32), ("strategy", ctypes.c_uint32),
                ("agg_fields", ctypes.c_uint32), ("ensemble_width", ctypes.c_uint32),
                ("queue_depth", ctypes.c_uint32), ("emit_outputs", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("hbm_budget_bytes", ctypes.c_uint64), ("param", ctypes.c_uint32 * 4)]


class rs_stream_desc(ctypes.Structure):
    _fields_ = [("mem", ctypes.c_uint32), ("elem_bytes", ctypes.c_uint32), ("n_parents", ctypes.c_uint64),
                ("n_elements", ctypes.c_uint64), ("offsets", ctypes.c_void_p), ("lengths", ctypes.c_void_p),
                ("elements", ctypes.c_void_p), ("parent_param", ctypes.c_void_p)]


class rs_agg_view(ctypes.Structure):
    _fields_ = [("count", ctypes.c_void_p), ("sum", ctypes.c_void_p), ("min", ctypes.c_void_p),
                ("max", ctypes.c_void_p), ("kept_count", ctypes.c_void_p), ("kept_sum", ctypes.c_void_p)]


class rs_stats_t(ctypes.Structure):
    _fields_ = [("firings", ctypes.c_uint64 * 3), ("items", ctypes.c_uint64 * 3), ("full", ctypes.c_uint64 * 3),
                ("signals", ctypes.c_uint64 * 3), ("ensemble_width", ctypes.c_uint32),
                ("queue_depth", ctypes.c_uint32), ("strategy", ctypes.c_uint32), ("n_workgroups", ctypes.c_uint32),
                ("n_outputs", ctypes.c_uint64)]


class rs_request(ctypes.Structure):
    _fields_ = [("arrival_s", ctypes.c_double), ("stream", rs_stream_desc)]


class rs_request_timing(ctypes.Structure):
    _fields_ = [("arrival_s", ctypes.c_double), ("pushed_s", ctypes.c_double), ("launched_s", ctypes.c_double),
                ("completed_s", ctypes.c_double), ("batch", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("pad", ctypes.c_uint32)]


_lib = None


def lib():
    """Load the in-tree HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, u32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
        L.pipeline_create.argtypes = [ctypes.POINTER(rs_pipeline_desc), ctypes.POINTER(vp)]
        L.pipeline_set_stream.argtypes = [vp, vp]
        L.stream_push.argtypes = [vp, ctypes.POINTER(rs_stream_desc), ctypes.POINTER(u64)]
        L.run.argtypes = [vp, u32]
        L.run_again.argtypes = [vp, u32]
        L.read_aggregates.argtypes = [vp, u64, ctypes.POINTER(rs_agg_view), u32]
        L.read_outputs.argtypes = [vp, u64, vp, u64, ctypes.POINTER(u64), u32]
        L.rs_stats.argtypes = [vp, u64, ctypes.POINTER(rs_stats_t)]
        L.kernel_times.argtypes = [vp, vp, u32, ctypes.POINTER(u32)]
        L.stream_release.argtypes = [vp, u64]
        L.serve.argtypes = [vp, ctypes.POINTER(rs_request), u64, ctypes.POINTER(rs_agg_view),
                            ctypes.POINTER(rs_request_timing), u32]
        L.pipeline_destroy.argtypes = [vp]
        L.hbm_probe.argtypes = [vp, vp, u64, vp]
        L.run_noalloc.argtypes = [ctypes.POINTER(rs_pipeline_desc), ctypes.POINTER(rs_stream_desc), u32,
                                  ctypes.POINTER(rs_agg_view), vp, u32]
        L.rs_last_error.restype = ctypes.c_char_p
        L.rs_last_error.argtypes = []
        for name in ABI_FUNCTIONS[:-1]:
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def rs_last_error():
    return lib().rs_last_error().decode()


def _check(rc):
    if rc != RS_OK:
        raise RsError(rc, rs_last_error())
    return rc


# ---- the C entry points, same names ----

def pipeline_create(desc):
    h = ctypes.c_void_p()
    _check(lib().pipeline_create(ctypes.byref(desc), ctypes.byref(h)))
    return h


def pipeline_set_stream(p, hip_stream):
    return _check(lib().pipeline_set_stream(p, hip_stream))


def stream_push(p, sdesc):
    sid = ctypes.c_uint64()
    _check(lib().stream_push(p, ctypes.byref(sdesc), ctypes.byref(sid)))
    return sid.value


def run(p, flags=RS_RUN_SYNC):
    return _check(lib().run(p, flags))


def run_again(p, flags=RS_RUN_SYNC):
    return _check(lib().run_again(p, flags))


def read_aggregates(p, stream_id, view, flags=RS_READ_BLOCK):
    return _check(lib().read_aggregates(p, stream_id, ctypes.byref(view), flags))


def read_outputs(p, stream_id, out_ptr, cap, flags=RS_READ_BLOCK):
    n = ctypes.c_uint64()
    _check(lib().read_outputs(p, stream_id, out_ptr, cap, ctypes.byref(n), flags))
    return n.value


def rs_stats(p, stream_id):
    st = rs_stats_t()
    _check(lib().rs_stats(p, stream_id, ctypes.byref(st)))
    return st


def kernel_times(p, cap=4096):
    ms = np.zeros(max(cap, 1), np.float32)
    n = ctypes.c_uint32(0)
    _check(lib().kernel_times(p, ms.ctypes.data, cap, ctypes.byref(n)))
    return ms[:min(n.value, cap)].tolist()


def stream_release(p, stream_id):
    return _check(lib().stream_release(p, stream_id))


def serve(p, reqs, n, out, timing, flags=0):
    return _check(lib().serve(p, reqs, n, out, timing, flags))


def hbm_probe(src_ptr, dst_ptr, nbytes, hip_stream=None):
    return _check(lib().hbm_probe(src_ptr, dst_ptr, nbytes, hip_stream))


def run_noalloc(desc, streams, n_streams, out, hip_stream=None, flags=RS_RUN_SYNC):
    """streams: ctypes array of rs_stream_desc (device memory); out: ctypes array of rs_agg_view
    (device pointers)."""
    return _check(lib().run_noalloc(ctypes.byref(desc), streams, n_streams, out, hip_stream, flags))


def pipeline_destroy(p):
    return _check(lib().pipeline_destroy(p))


# ---- convenience wrapper ----

def _ptr(x):
    """Host numpy array -> (pointer, keepalive); torch tensor -> its device pointer."""
    if x is None:
        return None, None
    if isinstance(x, np.ndarray):
        x = np.ascontiguousarray(x)
        return x.ctypes.data, x
    return x.data_ptr(), x


FIELDS = (("count", RS_COUNT, np.uint32), ("sum", RS_SUM, np.uint64), ("min", RS_MIN, np.uint32),
          ("max", RS_MAX, np.uint32), ("kept_count", RS_KEPT_COUNT, np.uint32), ("kept_sum", RS_KEPT_SUM, np.uint64))

DEFAULT_FIELDS = {RS_MODFILTER: RS_COUNT | RS_SUM, RS_HASH_EXPAND: RS_COUNT | RS_SUM | RS_MIN | RS_MAX,
                  RS_TEXT_WORDS: RS_COUNT | RS_MAX, RS_GRAPH_THRESH: RS_COUNT | RS_SUM,
                  RS_HASH_TREE: RS_COUNT | RS_SUM | RS_MIN | RS_MAX | RS_KEPT_COUNT | RS_KEPT_SUM}


class Pipeline:
    def __init__(self, kind, strategy=RS_AUTO, agg_fields=None, ensemble_width=0, queue_depth=0,
                 emit_outputs=False, flags=0, hbm_budget_bytes=0, param=(0, 0, 0, 0)):
        d = rs_pipeline_desc()
        d.abi_version = ABI_VERSION
        d.kind = kind
        d.strategy = strategy
        d.agg_fields = DEFAULT_FIELDS[kind] if agg_fields is None else agg_fields
        d.ensemble_width = ensemble_width
        d.queue_depth = queue_depth
        d.emit_outputs = int(bool(emit_outputs))
        d.flags = flags
        d.hbm_budget_bytes = hbm_budget_bytes
        for i, v in enumerate(param):
            d.param[i] = v
        self.desc = d
        self.kind = kind
        self.h = pipeline_create(d)
        self._keep = {}
        self._np = {}

    def close(self):
        if self.h is not None:
            pipeline_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, hip_stream_ptr):
        pipeline_set_stream(self.h, hip_stream_ptr)

    def _desc(self, offsets, elements, lengths=None, parent_param=None, n_elements=None):
        dev = not isinstance(elements, np.ndarray)
        s = rs_stream_desc()
        s.mem = RS_MEM_DEVICE if dev else RS_MEM_HOST
        s.elem_bytes = 1 if self.kind == RS_TEXT_WORDS else 4
        if lengths is not None:
            s.n_parents = len(lengths)
        else:
            s.n_parents = max(len(offsets) - 1, 0)
        s.n_elements = len(elements) if n_elements is None else n_elements
        keep = []
        for name, arr, dtype in (("offsets", offsets, np.uint32), ("lengths", lengths, np.uint32),
                                 ("elements", elements, None), ("parent_param", parent_param, np.uint32)):
            if arr is None:
                setattr(s, name, None)
                continue
            if not dev:
                arr = np.ascontiguousarray(arr, dtype=dtype if dtype is not None else arr.dtype)
            ptr, k = _ptr(arr)
            keep.append(k)
            setattr(s, name, ptr)
        return s, keep, dev

    def push(self, offsets, elements, lengths=None, parent_param=None, n_elements=None):
        """Push one stream.  numpy inputs are copied (RS_MEM_HOST); torch tensors are borrowed."""
        s, keep, dev = self._desc(offsets, elements, lengths, parent_param, n_elements)
        sid = stream_push(self.h, s)
        if dev:
            self._keep[sid] = keep          # borrowed device memory must outlive the stream
        self._np[sid] = int(s.n_parents)
        return sid

    def run(self, flags=RS_RUN_SYNC):
        run(self.h, flags)

    def run_again(self, flags=RS_RUN_SYNC):
        run_again(self.h, flags)

    def read(self, sid, flags=RS_READ_BLOCK):
        """Return a dict of the stored aggregate fields as numpy arrays."""
        P = self._np[sid]
        v = rs_agg_view()
        out = {}
        for name, bit, dt in FIELDS:
            if self.desc.agg_fields & bit:
                a = np.zeros(max(P, 1), dt)
                out[name] = a
                setattr(v, name, a.ctypes.data)
        read_aggregates(self.h, sid, v, flags)
        return {k: a[:P] for k, a in out.items()}

    def outputs(self, sid, flags=RS_READ_BLOCK):
        """The ordered surviving-item stream of a stream (pipelines with emit_outputs)."""
        n = read_outputs(self.h, sid, None, 0, flags)
        out = np.zeros(max(n, 1), np.uint32)
        read_outputs(self.h, sid, out.ctypes.data, n, flags)
        return out[:n]

    def stats(self, sid):
        return rs_stats(self.h, sid)

    def kernel_times(self, cap=4096):
        """Pipeline-kernel device times (ms) of the launches since the last call (RS_TIME_KERNEL)."""
        return kernel_times(self.h, cap)

    def serve(self, requests, arrivals, per_stream=False, read=True, device_out=None):
        """Run the native serving loop over requests = [(offsets, elements[, lengths, parent_param])]
        arriving at the given times (seconds, sorted).  Returns (results, timings): results[i] is a
        dict of aggregate arrays (or None when read is False) and timings a list of dicts.
        device_out: a list of dicts of device tensors (one per stored field, n_parents entries
        each, per request) that the kernel writes directly (RS_SERVE_DEVICE_OUT); results[i] is
        then that dict."""
        n = len(requests)
        reqs = (rs_request * max(n, 1))()
        outs = (rs_agg_view * max(n, 1))()
        tim = (rs_request_timing * max(n, 1))()
        keep, results = [], []
        for i, r in enumerate(requests):
            r = tuple(r) + (None,) * (4 - len(r))
            s, k, _ = self._desc(r[0], r[1], r[2], r[3])
            keep.append(k)
            reqs[i].arrival_s = float(arrivals[i])
            reqs[i].stream = s
            P = int(s.n_parents)
            res = None
            if device_out is not None:
                res = device_out[i]
                for name, bit, dt in FIELDS:
                    if self.desc.agg_fields & bit and res.get(name) is not None:
                        setattr(outs[i], name, res[name].data_ptr())
            elif read:
                res = {}
                for name, bit, dt in FIELDS:
                    if self.desc.agg_fields & bit:
                        a = np.zeros(max(P, 1), dt)
                        res[name] = a
                        setattr(outs[i], name, a.ctypes.data)
            results.append((res, P))
        flags = (RS_RUN_PER_STREAM if per_stream else 0) | (RS_SERVE_DEVICE_OUT if device_out is not None else 0)
        serve(self.h, reqs, n, outs if (read or device_out is not None) else None, tim, flags)
        out = [None if res is None else {k: a[:P] for k, a in res.items()} for res, P in results]
        timings = [dict(arrival=t.arrival_s, pushed=t.pushed_s, launched=t.launched_s, completed=t.completed_s,
                        batch=t.batch, status=t.status) for t in tim[:n]]
        return out, timings

    def release(self, sid):
        stream_release(self.h, sid)
        self._keep.pop(sid, None)
        self._np.pop(sid, None)
