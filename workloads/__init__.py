"""Seeded synthetic inputs, shared by the oracle side and the GPU side.

Holds none of the method's arithmetic: only counter-based draws of region
sizes, element values, text bytes, out-degrees, weights and arrival times
(``gen.c``, built with gcc into ``libworkloads.so``).  Inputs stand in for the
paper's workloads: the sum app over regions of a large integer array (§5), a
line-structured text stream shaped like the taxi app's input (§5) and edges
grouped by source vertex (§1).
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libworkloads.so")
SRC_PATH = os.path.join(HERE, "gen.c")

_lib = None

MASK64 = 0xFFFFFFFFFFFFFFFF
GOLDEN64 = 0x9E3779B97F4A7C15


def build(force=True):
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", SRC_PATH,
                           "-o", tmp, "-lm"])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        u64, u32, dbl, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double, ctypes.c_void_p
        L.gen_mix64.restype = u64
        L.gen_mix64.argtypes = [u64]
        L.gen_uniform_sizes.argtypes = [u64, u32, u64, vp]
        L.gen_parent_values.argtypes = [u64, u64, vp, vp]
        L.gen_hash_values.argtypes = [u64, u64, u64, vp]
        L.gen_text.restype = u64
        L.gen_text.argtypes = [u64, u64, dbl, u32, u32, vp, vp, vp, u64]
        L.gen_graph_offsets.restype = dbl
        L.gen_graph_offsets.argtypes = [u64, u64, u64, dbl, u32, vp, vp]
        L.gen_u32_stream.argtypes = [u64, u64, u64, vp]
        L.gen_stream_shapes.argtypes = [u64, u64, dbl, dbl, dbl, vp, vp]
        L.gen_geometric_offsets.restype = u64
        L.gen_geometric_offsets.argtypes = [u64, u64, dbl, vp, u64]
        L.gen_arrivals.argtypes = [u64, u64, dbl, vp]
        _lib = L
    return _lib


def mix64_py(z):
    """SplitMix64 output function in Python (for checking the C generator)."""
    z = (z + GOLDEN64) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def mix64(z):
    return int(lib().gen_mix64(int(z) & MASK64))


def sizes_to_offsets(sizes):
    off = np.zeros(len(sizes) + 1, np.uint64)
    np.cumsum(np.asarray(sizes, np.uint64), out=off[1:])
    if off[-1] >= 2 ** 32:
        raise ValueError("stream too large for u32 offsets")
    return off.astype(np.uint32)


# ---- sum app over regions of an integer array ----

def modfilter_workload(seed=1, n_parents=4096, max_size=64):
    """Parents with sizes uniform in [0, max_size] and values mix64-derived per (parent, index)."""
    sizes = np.zeros(n_parents, np.uint32)
    lib().gen_uniform_sizes(seed, max_size, n_parents, sizes.ctypes.data)
    offsets = sizes_to_offsets(sizes)
    values = np.zeros(max(int(offsets[-1]), 1), np.uint32)
    lib().gen_parent_values(seed, n_parents, offsets.ctypes.data, values.ctypes.data)
    return offsets, values[:int(offsets[-1])]


def hash_values(seed, n, first=0):
    out = np.zeros(max(n, 1), np.uint32)
    lib().gen_hash_values(seed, first, n, out.ctypes.data)
    return out[:n]


def fixed_offsets(n, L):
    """CSR offsets for regions of fixed length L (the last region is shorter if L does not divide n)."""
    r = (n + L - 1) // L
    off = np.minimum(np.arange(r + 1, dtype=np.uint64) * L, n)
    return off.astype(np.uint32)


def hash_fixed_workload(seed=2, n=1 << 26, L=4096):
    return fixed_offsets(n, L), hash_values(seed, n)


def uniform_offsets(seed, n_parents, max_size):
    sizes = np.zeros(n_parents, np.uint32)
    lib().gen_uniform_sizes(seed, max_size, n_parents, sizes.ctypes.data)
    return sizes_to_offsets(sizes)


def variable_offsets(seed, n, max_size):
    """Regions with sizes uniform in [0, max_size] that cover exactly n elements: sizes are
    drawn until their sum reaches n, and the last region is cut to fit (the variable-size
    sweep)."""
    if max_size == 0:
        return np.zeros(4097, np.uint32)   # 4096 empty regions: nothing can cover n
    mean = max_size / 2.0
    P = int(np.ceil(n / mean * 1.1)) + 64
    while True:
        sizes = np.zeros(P, np.uint32)
        lib().gen_uniform_sizes(seed, max_size, P, sizes.ctypes.data)
        ends = np.cumsum(sizes, dtype=np.int64)
        if ends[-1] >= n:
            break
        P *= 2
    last = int(np.searchsorted(ends, n))     # first region whose end reaches n
    offsets = np.zeros(last + 2, np.uint32)
    offsets[1:] = np.minimum(ends[:last + 1], n)
    return offsets


# ---- line-structured text ----

def text_workload(seed=3, total_bytes=1 << 30, mean_len=80.0, max_len=65536, space_per_65536=11796):
    """Returns (text uint8[total_bytes], line starts uint32[R], line lengths uint32[R])."""
    L = lib()
    n_lines = L.gen_text(seed, total_bytes, mean_len, max_len, space_per_65536, None, None, None, 0)
    starts = np.zeros(max(n_lines, 1), np.uint32)
    lengths = np.zeros(max(n_lines, 1), np.uint32)
    text = np.zeros(max(total_bytes, 1), np.uint8)
    k = L.gen_text(seed, total_bytes, mean_len, max_len, space_per_65536, text.ctypes.data,
                   starts.ctypes.data, lengths.ctypes.data, n_lines)
    assert k == n_lines
    return text[:total_bytes], starts[:n_lines], lengths[:n_lines]


# The shape of the paper's second application (§5): long lines (1397 characters on average)
# holding about 45 markers each, a marker being where a word starts.  A line is geometric in
# length with that mean; a byte is a space with probability 2195/65536, so a line of L bytes
# holds about L p (1 - p) = 45 words.  Synthetic bytes only: no record of the application's
# input is used.
TAXI_MEAN_LINE = 1397.0
TAXI_SPACE_PER_65536 = 2195


def taxi_workload(seed=9, total_bytes=1 << 30):
    """Returns (text, line starts, line lengths) shaped like the paper's taxi input."""
    return text_workload(seed=seed, total_bytes=total_bytes, mean_len=TAXI_MEAN_LINE, max_len=65536,
                         space_per_65536=TAXI_SPACE_PER_65536)


# ---- edges grouped by source vertex ----

def graph_offsets(seed=4, n_vertices=1 << 24, n_edges=1 << 28, alpha=1.1, cap=100000):
    scratch = np.zeros(max(n_vertices, 1), np.float64)
    offsets = np.zeros(n_vertices + 1, np.uint32)
    beta = lib().gen_graph_offsets(seed, n_vertices, n_edges, alpha, cap, scratch.ctypes.data,
                                   offsets.ctypes.data)
    return offsets, beta


def u32_stream(seed, stream, n):
    out = np.zeros(max(n, 1), np.uint32)
    lib().gen_u32_stream(seed, stream, n, out.ctypes.data)
    return out[:n]


WEIGHT_STREAM = 0x3E16
THRESHOLD_STREAM = 0x7412


def graph_workload(seed=4, n_vertices=1 << 24, n_edges=1 << 28, alpha=1.1, cap=100000):
    """Returns (CSR offsets, edge weights, per-vertex thresholds, beta)."""
    offsets, beta = graph_offsets(seed, n_vertices, n_edges, alpha, cap)
    weights = u32_stream(seed, WEIGHT_STREAM, n_edges)
    thresholds = u32_stream(seed, THRESHOLD_STREAM, n_vertices)
    return offsets, weights, thresholds, beta


# ---- batched serving ----

def stream_shapes(seed=5, n_streams=512, lo_n=1e3, hi_n=1e7, max_mean=4096.0):
    n = np.zeros(n_streams, np.uint64)
    m = np.zeros(n_streams, np.float64)
    lib().gen_stream_shapes(seed, n_streams, lo_n, hi_n, max_mean, n.ctypes.data, m.ctypes.data)
    return n, m


def geometric_offsets(seed, n_elems, mean_len):
    L = lib()
    r = L.gen_geometric_offsets(seed, n_elems, mean_len, None, 0)
    off = np.zeros(r + 1, np.uint32)
    r2 = L.gen_geometric_offsets(seed, n_elems, mean_len, off.ctypes.data, r)
    assert r2 == r
    return off


def serving_stream(seed, s, n_elems, mean_len):
    """Stream s of a serving batch: geometric regions of the given mean and hash-generated values."""
    seed_s = mix64((seed + s) & MASK64)
    return geometric_offsets(seed_s, int(n_elems), float(mean_len)), hash_values(seed_s, int(n_elems))


def arrivals(seed, n, rate):
    t = np.zeros(max(n, 1), np.float64)
    lib().gen_arrivals(seed, n, rate, t.ctypes.data)
    return t[:n]
