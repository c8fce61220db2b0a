"""Pure-Python oracle for small inputs (test infrastructure only).

An independent rendering of the serial definition that ``oracle.c`` implements,
written separately (own hash code, list-valued stages) so that the two can be
checked against each other.  It follows §4.1 of Timcheck & Buhler: each parent
is enumerated into element indices, each element is fetched under its parent's
context and sent through the stages, which map one item to an ordered list of
zero or more items (§2.1), and the aggregating node's begin/run/end bracket
every region, so every parent gets one record.
"""

MASK32 = 0xFFFFFFFF
MASK64 = 0xFFFFFFFFFFFFFFFF

MODFILTER, HASH_EXPAND, TEXT_WORDS, GRAPH_THRESH, HASH_TREE = 1, 2, 3, 4, 5


def murmur_fmix32(h):
    """MurmurHash3's 32-bit finalizer."""
    h &= MASK32
    h ^= h >> 16
    h = (h * 0x85EBCA6B) & MASK32
    h ^= h >> 13
    h = (h * 0xC2B2AE35) & MASK32
    h ^= h >> 16
    return h


def salted_hash(x, salt):
    """H(x, s) = fmix32(x xor (0x9E3779B9 * (s + 1) mod 2^32))."""
    return murmur_fmix32((x ^ ((0x9E3779B9 * (salt + 1)) & MASK32)) & MASK32)


def stages_for(kind, param=(0, 0, 0, 0)):
    """Return the list of stage functions g(item, region) -> list of items."""
    if kind == MODFILTER:
        m = param[0] or 4
        r = param[1]
        return [lambda x, reg: [x] if x % m == r else []]
    if kind == HASH_EXPAND:
        def keep(x, reg):
            return [x] if salted_hash(x, 0) & 1 else []

        def expand(x, reg):
            c = (salted_hash(x, 0) >> 1) & 3
            return [salted_hash(x, j + 1) for j in range(c)]
        return [keep, expand]
    if kind == TEXT_WORDS:
        def word_start(i, reg):
            line = reg["line"]
            return [i] if line[i] != 0x20 and (i == 0 or line[i - 1] == 0x20) else []

        def word_length(i, reg):
            line = reg["line"]
            j = i
            while j < len(line) and line[j] != 0x20:
                j += 1
            return [j - i]
        return [word_start, word_length]
    if kind == GRAPH_THRESH:
        return [lambda w, reg: [w] if w < reg["threshold"] else []]
    raise ValueError(kind)


def regions(offsets, lengths=None):
    """Yield (start, end) of every parent's region."""
    if lengths is None:
        for p in range(len(offsets) - 1):
            yield int(offsets[p]), int(offsets[p + 1])
    else:
        for p in range(len(lengths)):
            yield int(offsets[p]), int(offsets[p]) + int(lengths[p])


def run(kind, offsets, elements, lengths=None, parent_param=None, param=(0, 0, 0, 0)):
    """Return (records, outputs): records[p] = (count, sum, min, max); outputs in serial order."""
    stages = stages_for(kind, param)
    records = []
    outputs = []
    for p, (s, e) in enumerate(regions(offsets, lengths)):
        region = {"line": [int(b) for b in elements[s:e]] if kind == TEXT_WORDS else None,
                  "threshold": int(parent_param[p]) if parent_param is not None else None}
        survivors = []
        for i in range(e - s):
            # enumeration yields the index; the element is fetched under the parent
            items = [i] if kind == TEXT_WORDS else [int(elements[s + i])]
            for g in stages:
                items = [y for it in items for y in g(it, region)]
            survivors.extend(items)
        outputs.extend(survivors)
        if survivors:
            records.append((len(survivors) & MASK32, sum(survivors) & MASK64,
                            min(survivors), max(survivors)))
        else:
            records.append((0, 0, MASK32, 0))
    return records, outputs


def run_tree(offsets, elements):
    """The tree topology of §2.1 on the hash stages: the filter's survivors go both to the
    expansion, whose children reach the first sink, and to a second sink of their own.  Returns
    (records, second, outputs): records[p] = (count, sum, min, max) of the children,
    second[p] = (count, sum) of the survivors, outputs the children in serial order."""
    keep, expand = stages_for(HASH_EXPAND)
    records, second, outputs = [], [], []
    for s, e in regions(offsets):
        kids, kept = [], []
        for i in range(e - s):
            survivors = keep(int(elements[s + i]), None)
            kept.extend(survivors)
            for x in survivors:
                kids.extend(expand(x, None))
        outputs.extend(kids)
        records.append((len(kids) & MASK32, sum(kids) & MASK64, min(kids), max(kids)) if kids
                       else (0, 0, MASK32, 0))
        second.append((len(kept) & MASK32, sum(kept) & MASK64))
    return records, second, outputs
