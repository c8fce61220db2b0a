"""Seeded input generators: published SplitMix64 outputs, the C generator against a
Python mirror, and the size/shape invariants of every synthetic workload."""
import numpy as np

import workloads as W


def test_splitmix64_published_sequence():
    # SplitMix64 seeded with 1234567: published first outputs of the reference generator
    seq = [W.mix64((1234567 + k * W.GOLDEN64) & W.MASK64) for k in range(5)]
    assert seq == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                   4593380528125082431, 16408922859458223821]
    assert all(W.mix64(z) == W.mix64_py(z) for z in (0, 1, 2 ** 63, W.MASK64, 0xDEADBEEF))


def test_modfilter_workload_matches_python_mirror():
    off, vals = W.modfilter_workload(seed=1, n_parents=64, max_size=64)
    b = W.mix64_py(1 ^ 0x5EED)
    sizes = [W.mix64_py((b + p) & W.MASK64) % 65 for p in range(64)]
    assert np.diff(off).tolist() == sizes
    assert sizes[:8] == [22, 16, 13, 59, 64, 26, 36, 43]
    base = W.mix64_py(1)
    for p in (0, 5, 63):
        exp = [W.mix64_py(base ^ ((p << 32) | i)) & 0xFFFFFFFF for i in range(sizes[p])]
        assert vals[off[p]:off[p + 1]].tolist() == exp
    full_off, _ = W.modfilter_workload()
    assert len(full_off) == 4097 and np.diff(full_off).max() <= 64 and (np.diff(full_off) == 0).any()


def test_hash_values_and_fixed_offsets():
    v = W.hash_values(2, 8)
    base = W.mix64_py(2)
    assert v.tolist() == [W.mix64_py(base + i) & 0xFFFFFFFF for i in range(8)]
    assert W.hash_values(2, 5, first=3).tolist() == v[3:8].tolist()
    off = W.fixed_offsets(1 << 12, 64)
    assert len(off) == 65 and off[-1] == 4096 and set(np.diff(off).tolist()) == {64}
    off = W.fixed_offsets(10, 4)
    assert off.tolist() == [0, 4, 8, 10]


def test_text_workload_shape():
    total = 1 << 20
    text, starts, lengths = W.text_workload(seed=3, total_bytes=total)
    assert len(text) == total and text[-1] == 10
    ends = starts.astype(np.int64) + lengths
    assert (text[ends] == 10).all()                          # every line ends with a newline
    assert starts[0] == 0 and (starts[1:] == ends[:-1] + 1).all()
    assert ends[-1] == total - 1
    nl = np.zeros(total, bool)
    nl[ends] = True
    body = text[~nl]
    assert ((body == 32) | ((body >= 97) & (body <= 122))).all()
    assert abs((body == 32).mean() - 0.18) < 0.005
    assert abs(lengths[:-1].mean() - 80) < 4 and lengths.max() <= 65536
    assert (lengths == 0).any()


def test_graph_workload_shape():
    off, beta = W.graph_offsets(seed=4, n_vertices=1 << 16, n_edges=1 << 20, cap=100000)
    deg = np.diff(off.astype(np.int64))
    assert off[0] == 0 and off[-1] == 1 << 20 and (deg >= 0).all() and deg.max() <= 100000
    assert (deg == 0).mean() > 0.2                          # many degree-0 vertices
    assert deg.max() > 50 * deg.mean()                      # heavy tail
    assert beta > 0


def test_serving_shapes_and_streams():
    n, m = W.stream_shapes(seed=5, n_streams=512)
    assert ((n >= 1000) & (n <= 10 ** 7)).all() and ((m >= 1) & (m <= 4096)).all()
    off, vals = W.serving_stream(5, 3, 5000, 7.5)
    assert off[0] == 0 and off[-1] == 5000 and (np.diff(off.astype(np.int64)) >= 0).all()
    assert len(vals) == 5000
    t = W.arrivals(6, 100, 50.0)
    assert (np.diff(t) > 0).all() and abs(t[-1] / 100 - 1 / 50.0) < 0.01


def test_variable_offsets_cover_exactly_n():
    """Variable-size sweep regions: sizes in [0, max], the whole stream covered exactly once,
    only the last region cut short, and the same draw for the same seed."""
    for mx, n in ((1, 5000), (7, 100003), (64, 100003), (4096, 1 << 20)):
        o = W.variable_offsets(3, n, mx).astype(np.int64)
        d = np.diff(o)
        assert o[0] == 0 and o[-1] == n
        assert d.min() >= 0 and d.max() <= mx
        assert np.array_equal(o, W.variable_offsets(3, n, mx).astype(np.int64))
        # the uncut sizes come from the same generator as uniform_offsets
        full = np.diff(W.uniform_offsets(3, len(d), mx).astype(np.int64))
        assert np.array_equal(d[:-1], full[:-1]) and d[-1] <= full[-1]
        # sizes look uniform on [0, mx]: the mean of many draws is near mx / 2
        if len(d) > 1000:
            assert abs(d[:-1].mean() - mx / 2) < 0.05 * mx + 0.05
    e = W.variable_offsets(3, 1000, 0)
    assert len(e) == 4097 and not e.any()


def test_taxi_shape():
    """The taxi-shaped text: mean line length near 1397 characters and about 45 markers (word
    starts) per line, the two figures the paper gives for its second application (§5)."""
    import oracle
    text, starts, lengths = W.taxi_workload(seed=9, total_bytes=1 << 24)
    assert abs(float(lengths.mean()) / W.TAXI_MEAN_LINE - 1.0) < 0.06
    assert text[-1] == ord("\n") and len(text) == 1 << 24
    words = oracle.run(oracle.TEXT_WORDS, starts, text, lengths=lengths).count
    assert abs(float(words.mean()) / 45.0 - 1.0) < 0.08
