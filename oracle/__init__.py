"""Serial CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never does; it shares
no code with it.

* ``oracle.c`` -- the plain serial definition of enumeration and aggregation
  (§4, §4.1 of Timcheck & Buhler), compiled with gcc into ``liboracle.so`` and
  called here through ctypes.
* ``tiny.py`` -- an independent pure-Python rendering of the same definition
  for small inputs.
* ``credit_sim.py`` -- a step-by-step model of the credit protocol (§3.1-§3.3)
  used to check Lemma 1, Lemma 2 and the SIMD rule on small streams.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.c")

MODFILTER, HASH_EXPAND, TEXT_WORDS, GRAPH_THRESH, HASH_TREE = 1, 2, 3, 4, 5

_lib = None


def build(force=True):
    """Compile oracle.c into liboracle.so with the host C compiler."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                           SRC_PATH, "-o", tmp])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.oracle_run.restype = ctypes.c_int
        L.oracle_run.argtypes = [ctypes.c_int, u32p, ctypes.c_uint64, u32p, u32p, ctypes.c_void_p,
                                 ctypes.c_uint64, u32p, u32p, u64p, u32p, u32p, u32p,
                                 ctypes.c_uint64, u64p]
        L.oracle_run_tree.restype = ctypes.c_int
        L.oracle_run_tree.argtypes = [ctypes.c_int, u32p, ctypes.c_uint64, u32p, u32p, ctypes.c_void_p,
                                      ctypes.c_uint64, u32p, u32p, u64p, u32p, u32p, u32p, u64p, u32p,
                                      ctypes.c_uint64, u64p]
        L.oracle_fmix32.restype = ctypes.c_uint32
        L.oracle_fmix32.argtypes = [ctypes.c_uint32]
        L.oracle_hash.restype = ctypes.c_uint32
        L.oracle_hash.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        _lib = L
    return _lib


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class Result:
    """Per-parent aggregates (structure of arrays) plus the optional surviving-item stream; for
    the tree kind also the second sink's kept_count and kept_sum."""

    def __init__(self, count, sum_, min_, max_, out, kept_count=None, kept_sum=None):
        self.count, self.sum, self.min, self.max, self.out = count, sum_, min_, max_, out
        self.kept_count, self.kept_sum = kept_count, kept_sum

    def __repr__(self):
        return f"Result(count={self.count}, sum={self.sum}, min={self.min}, max={self.max}, out={self.out})"


def run(kind, offsets, elements, lengths=None, parent_param=None, param=(0, 0, 0, 0),
        emit_outputs=False):
    """Run the serial oracle.

    offsets: CSR offsets [P+1] (lengths None) or region starts [P] (lengths given).
    elements: uint32 array (kinds 1, 2, 4, 5) or uint8 array (kind 3).
    Returns a Result with count/sum/min/max arrays and, if asked, the output stream.
    """
    offsets = np.ascontiguousarray(offsets, dtype=np.uint32)
    if lengths is not None:
        lengths = np.ascontiguousarray(lengths, dtype=np.uint32)
        n_par = len(lengths)
    else:
        n_par = max(len(offsets) - 1, 0)
        if len(offsets) == 0:
            offsets = np.zeros(1, np.uint32)
    edt = np.uint8 if kind == TEXT_WORDS else np.uint32
    elements = np.ascontiguousarray(elements, dtype=edt)
    if parent_param is not None:
        parent_param = np.ascontiguousarray(parent_param, dtype=np.uint32)
    prm = np.ascontiguousarray(np.array(param, dtype=np.uint32).reshape(4))
    count = np.zeros(n_par, np.uint32)
    sum_ = np.zeros(n_par, np.uint64)
    mn = np.zeros(n_par, np.uint32)
    mx = np.zeros(n_par, np.uint32)
    n_out = ctypes.c_uint64(0)
    L = lib()
    out = None
    cap = 0
    if emit_outputs:
        # first pass sizes the stream, second pass fills it
        rc = L.oracle_run(kind, _ptr(prm, ctypes.c_uint32), n_par, _ptr(offsets, ctypes.c_uint32),
                          _ptr(lengths, ctypes.c_uint32), elements.ctypes.data, len(elements),
                          _ptr(parent_param, ctypes.c_uint32), None, None, None, None,
                          None, 0, ctypes.byref(n_out))
        if rc != 0:
            raise ValueError(f"oracle_run failed: {rc}")
        cap = n_out.value
        out = np.zeros(max(cap, 1), np.uint32)
    kc = ks = None
    if kind == HASH_TREE:
        kc = np.zeros(n_par, np.uint32)
        ks = np.zeros(n_par, np.uint64)
    rc = L.oracle_run_tree(kind, _ptr(prm, ctypes.c_uint32), n_par, _ptr(offsets, ctypes.c_uint32),
                           _ptr(lengths, ctypes.c_uint32), elements.ctypes.data, len(elements),
                           _ptr(parent_param, ctypes.c_uint32), _ptr(count, ctypes.c_uint32),
                           _ptr(sum_, ctypes.c_uint64), _ptr(mn, ctypes.c_uint32), _ptr(mx, ctypes.c_uint32),
                           _ptr(kc, ctypes.c_uint32), _ptr(ks, ctypes.c_uint64),
                           _ptr(out, ctypes.c_uint32), cap, ctypes.byref(n_out))
    if rc != 0:
        raise ValueError(f"oracle_run failed: {rc}")
    if out is not None:
        out = out[:n_out.value].copy()
    return Result(count, sum_, mn, mx, out, kc, ks)


def fmix32(x):
    return int(lib().oracle_fmix32(int(x) & 0xFFFFFFFF))


def hash32(x, salt):
    return int(lib().oracle_hash(int(x) & 0xFFFFFFFF, int(salt) & 0xFFFFFFFF))
