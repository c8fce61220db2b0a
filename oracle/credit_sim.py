"""Step-by-step model of the credit protocol for precise signals (test infrastructure only).

This follows §3 of Timcheck & Buhler in the paper's own terms:

* Between successive nodes n1 -> n2 there is a finite data queue Q and a finite
  signal queue S (§3.1).  Each signal carries a credit: if S is empty when n1
  emits the signal, the credit is the number of items queued on Q (rule 1);
  otherwise it is the number of items n1 emitted since the signal at the tail of
  S (rule 2).  n1 keeps a counter of emitted items that resets at every signal.
* n2 keeps a current credit counter, initially 0.  With no signal queued it
  consumes data freely (rule 1); with a signal queued and counter > 0 it may
  consume at most counter items, decrementing it (rule 2a); with counter 0 it
  either moves the head signal's credit into the counter or, if that credit is
  0, consumes the signal (rule 2b).
* A firing has a data phase (consume min(queued, downstream space, counter if
  a signal is pending) items) and then, if the counter is 0, a signal phase
  that consumes signals until none are left or the counter becomes > 0 (§3.2).
  A node is fireable when it has pending input and room downstream for the
  outputs of at least one input.
* On a SIMD processor the ensemble is additionally capped at the SIMD width and,
  when a signal is queued, at the counter, so that no ensemble holds items from
  both sides of a signal (§3.3).
* Enumeration (§4.2) emits element indices bracketed by a start and an end
  signal per parent; downstream nodes switch their current parent on these
  signals and run begin()/end(); the aggregating node emits one record per
  parent at end().

Every item also carries a hidden copy of the region it came from.  The model
never computes with it; the checks use it to assert the SIMD rule and that
every node's current parent matches the items it processes.  The scheduler
picks a random fireable node with a random ensemble cap, which exercises
Lemma 1 (precise delivery) and Lemma 2 (termination without deadlock) on
arbitrary schedules.
"""
import random
from collections import deque

from . import tiny

MASK32 = 0xFFFFFFFF
MASK64 = 0xFFFFFFFFFFFFFFFF


class ProtocolViolation(AssertionError):
    pass


class Edge:
    """Data queue Q and signal queue S from one node to the next (§3.1)."""

    def __init__(self, cap, sig_cap):
        self.Q = deque()
        self.S = deque()          # entries: [credit, payload, items emitted before it]
        self.cap = cap
        self.sig_cap = sig_cap
        self.since_signal = 0     # sender's emitted-items counter (rule 2)
        self.emitted = 0          # total data items emitted so far

    def space(self):
        return self.cap - len(self.Q)

    def sig_space(self):
        return self.sig_cap - len(self.S)

    def push_data(self, item):
        if len(self.Q) >= self.cap:
            raise ProtocolViolation("data queue overflow")
        self.Q.append(item)
        self.since_signal += 1
        self.emitted += 1

    def push_signal(self, payload):
        if len(self.S) >= self.sig_cap:
            raise ProtocolViolation("signal queue overflow")
        credit = len(self.Q) if not self.S else self.since_signal   # rules 1 and 2
        self.since_signal = 0
        self.S.append([credit, payload, self.emitted])
        return credit


class Item:
    __slots__ = ("value", "region")

    def __init__(self, value, region):
        self.value = value
        self.region = region      # hidden; only the checks read it


class Node:
    """A pipeline node with a current credit counter and a current parent."""

    def __init__(self, name, kmax, stage=None, aggregate=False):
        self.name = name
        self.kmax = kmax          # a-priori maximum outputs per input (§3.2 fireability)
        self.stage = stage        # g(value, region_context) -> list of values
        self.aggregate = aggregate
        self.inp = None
        self.out = None
        self.counter = 0          # current credit counter, initially 0
        self.consumed = 0         # data items consumed from inp
        self.parent = None        # current parent, set by start signals
        self.acc = None
        self.records = {}
        self.ensembles = []       # (node, size) of every data firing

    def pending(self):
        return bool(self.inp.Q) or bool(self.inp.S)

    def fireable(self):
        if not self.pending():
            return False
        if self.aggregate:
            return True           # the sink side is unbounded
        data_ok = bool(self.inp.Q) and self.out.space() >= self.kmax
        sig_ok = bool(self.inp.S) and self.counter == 0 and self.out.sig_space() >= 1
        return data_ok or sig_ok

    def fire(self, cap, contexts, log):
        q, s = self.inp.Q, self.inp.S
        # data phase
        n = len(q)
        if not self.aggregate:
            n = min(n, self.out.space() // self.kmax)
        if s:
            n = min(n, self.counter)   # rule 2a; also the SIMD rule of §3.3
        n = min(n, cap)
        if n > 0:
            ens = [q.popleft() for _ in range(n)]
            if s:
                self.counter -= n
            self.consumed += n
            regions = {it.region for it in ens}
            if len(regions) != 1:
                raise ProtocolViolation(f"{self.name}: ensemble mixes regions {sorted(regions)}")
            if self.parent is None or regions != {self.parent}:
                raise ProtocolViolation(f"{self.name}: items of region {regions} seen under parent {self.parent}")
            self.ensembles.append(n)
            log.append((self.name, "data", [it.value for it in ens]))
            for it in ens:
                if self.aggregate:
                    self._accumulate(it.value)
                else:
                    for y in self.stage(it.value, contexts[self.parent]):
                        self.out.push_data(Item(y, it.region))
        # signal phase
        if self.counter == 0:
            while s and (self.aggregate or self.out.sig_space() >= 1):
                head = s[0]
                if head[0] > 0:                 # rule 2b: move credit into the counter
                    self.counter += head[0]
                    head[0] = 0
                    break
                s.popleft()                     # rule 2b: consume the signal
                if self.consumed != head[2]:    # Lemma 1
                    raise ProtocolViolation(
                        f"{self.name}: signal {head[1]} received after {self.consumed} items, "
                        f"emitted after {head[2]}")
                log.append((self.name, "signal", head[1]))
                self._signal(head[1])

    def _signal(self, payload):
        kind, p = payload
        if kind == "start":
            self.parent = p
            if self.aggregate:
                self.acc = [0, 0, MASK32, 0]    # begin()
        else:
            if self.parent != p:
                raise ProtocolViolation(f"{self.name}: end of {p} while in {self.parent}")
            if self.aggregate:
                self.records[p] = tuple(self.acc)   # end(): one record per parent
            self.parent = None
        if not self.aggregate:
            self.out.push_signal(payload)

    def _accumulate(self, y):
        a = self.acc
        a[0] = (a[0] + 1) & MASK32
        a[1] = (a[1] + y) & MASK64
        a[2] = min(a[2], y)
        a[3] = max(a[3], y)


class Enumerator:
    """Source: opens each parent into its element stream between start and end signals (§4.2)."""

    def __init__(self, sizes, fetch, out):
        self.sizes = list(sizes)
        self.fetch = fetch            # fetch(p, i) -> first-stage item for element i of parent p
        self.out = out
        self.p = 0
        self.i = 0
        self.started = False
        self.ensembles = []

    def pending(self):
        return self.p < len(self.sizes)

    def fireable(self):
        if not self.pending():
            return False
        if not self.started or self.i == self.sizes[self.p]:
            return self.out.sig_space() >= 1
        return self.out.space() >= 1

    def fire(self, cap, log):
        if not self.started:
            self.out.push_signal(("start", self.p))
            self.started = True
            log.append(("enum", "signal", ("start", self.p)))
            return
        left = self.sizes[self.p] - self.i
        if left == 0:
            self.out.push_signal(("end", self.p))
            log.append(("enum", "signal", ("end", self.p)))
            self.p += 1
            self.i = 0
            self.started = False
            return
        n = min(left, cap, self.out.space())
        for _ in range(n):
            self.out.push_data(Item(self.fetch(self.p, self.i), self.p))
            self.i += 1
        self.ensembles.append(n)
        log.append(("enum", "data", n))


def simulate(kind, offsets, elements, lengths=None, parent_param=None, param=(0, 0, 0, 0),
             width=8, rng=None, cap_range=(1, 3), sig_cap_range=(1, 4), max_steps=None,
             policy="random"):
    """Run the pipeline enumerate -> stages -> aggregate under a random schedule.

    policy "random" fires a random fireable node with a random ensemble cap in [1, width];
    "downstream" fires the most downstream fireable node with the full width.

    Returns (records list in parent order, event log, per-node ensemble sizes).
    Raises ProtocolViolation if Lemma 1, the SIMD rule or the parent bookkeeping fails,
    and AssertionError if the run does not terminate within the step bound (Lemma 2).
    """
    rng = rng or random.Random(0)
    stages = tiny.stages_for(kind, param)
    spans = list(tiny.regions(offsets, lengths))
    sizes = [e - s for s, e in spans]
    contexts = []
    for p, (s, e) in enumerate(spans):
        contexts.append({"line": [int(b) for b in elements[s:e]] if kind == tiny.TEXT_WORDS else None,
                         "threshold": int(parent_param[p]) if parent_param is not None else None})

    def fetch(p, i):
        return i if kind == tiny.TEXT_WORDS else int(elements[spans[p][0] + i])

    kmax = {tiny.MODFILTER: [1], tiny.HASH_EXPAND: [1, 3], tiny.TEXT_WORDS: [1, 1],
            tiny.GRAPH_THRESH: [1]}[kind]
    nodes = []
    edges = []
    # queue capacity of an edge is at least the a-priori maximum of the node feeding it
    first = Edge(rng.randint(*cap_range), rng.randint(*sig_cap_range))
    edges.append(first)
    src = Enumerator(sizes, fetch, first)
    prev = first
    for si, g in enumerate(stages):
        nxt = Edge(kmax[si] * rng.randint(*cap_range), rng.randint(*sig_cap_range))
        edges.append(nxt)
        n = Node(f"stage{si + 1}", kmax[si], stage=g)
        n.inp, n.out = prev, nxt
        nodes.append(n)
        prev = nxt
    agg = Node("aggregate", 0, aggregate=True)
    agg.inp = prev
    nodes.append(agg)

    total_items = sum(sizes)
    bound = max_steps or (50 + 20 * (total_items * 4 + 2 * len(sizes)) * (len(nodes) + 1))
    log = []
    steps = 0
    while True:
        cands = [n for n in nodes if n.fireable()]
        if src.fireable():
            cands.append(src)
        if not cands:
            if src.pending() or any(n.pending() for n in nodes):
                raise AssertionError("deadlock: pending input but no fireable node")   # Lemma 2
            break
        if policy == "downstream":
            ready = [n for n in nodes if n.fireable()]
            pick = ready[-1] if ready else src
            cap = width
        else:
            pick = rng.choice(cands)
            cap = rng.randint(1, width)
        if pick is src:
            src.fire(cap, log)
        else:
            pick.fire(cap, contexts, log)
        steps += 1
        if steps > bound:
            raise AssertionError("no termination within the step bound")            # Lemma 2
    records = [agg.records[p] for p in range(len(sizes))]
    ens = {"enum": src.ensembles}
    for n in nodes:
        ens[n.name] = n.ensembles
    return records, log, ens


def tag_replay(kind, offsets, elements, lengths=None, parent_param=None, param=(0, 0, 0, 0),
               width=8, rng=None):
    """The tagging alternative: every item carries its region id, so ensembles may mix regions.

    Elements are enumerated in chunks of random size up to `width` that ignore region
    boundaries; each chunk runs the stages per item under its tag's context, and the
    aggregating node reduces each chunk by tag and merges the partials per region.
    """
    rng = rng or random.Random(0)
    stages = tiny.stages_for(kind, param)
    spans = list(tiny.regions(offsets, lengths))
    stream = []
    for p, (s, e) in enumerate(spans):
        for i in range(e - s):
            stream.append((p, i if kind == tiny.TEXT_WORDS else int(elements[s + i])))
    ctx = [{"line": [int(b) for b in elements[s:e]] if kind == tiny.TEXT_WORDS else None,
            "threshold": int(parent_param[p]) if parent_param is not None else None}
           for p, (s, e) in enumerate(spans)]
    acc = [[0, 0, MASK32, 0] for _ in spans]
    pos = 0
    while pos < len(stream):
        n = rng.randint(1, width)
        chunk = stream[pos:pos + n]
        pos += n
        items = chunk
        for g in stages:
            items = [(t, y) for (t, v) in items for y in g(v, ctx[t])]
        part = {}
        for t, y in items:                       # segmented reduction keyed by tag
            a = part.setdefault(t, [0, 0, MASK32, 0])
            a[0] += 1
            a[1] += y
            a[2] = min(a[2], y)
            a[3] = max(a[3], y)
        for t, a in part.items():                # merge partials into the region's aggregate
            r = acc[t]
            r[0] = (r[0] + a[0]) & MASK32
            r[1] = (r[1] + a[1]) & MASK64
            r[2] = min(r[2], a[2])
            r[3] = max(r[3], a[3])
    return [tuple(a) for a in acc]


def two_node_trace(events):
    """Replay the credit protocol on one edge n1 -> n2 (the situation of Fig. 2(b)).

    events: sequence of ("d", name) data emissions and ("s", name) signal emissions by n1,
            interleaved with ("fire", cap) firings of n2.
    Returns (credits given to each signal, list of n2 firing outcomes) where an outcome is
    ("data", [names]) or ("signal", name) or ("credit", amount).
    """
    e = Edge(10 ** 9, 10 ** 9)
    counter = 0
    credits = {}
    outcomes = []
    for ev in events:
        if ev[0] == "d":
            e.push_data(ev[1])
        elif ev[0] == "s":
            credits[ev[1]] = e.push_signal(ev[1])
        else:
            cap = ev[1]
            n = len(e.Q)
            if e.S:
                n = min(n, counter)
            n = min(n, cap)
            if n:
                outcomes.append(("data", [e.Q.popleft() for _ in range(n)]))
                if e.S:
                    counter -= n
            if counter == 0:
                while e.S:
                    head = e.S[0]
                    if head[0] > 0:
                        counter += head[0]
                        outcomes.append(("credit", head[0]))
                        head[0] = 0
                        break
                    e.S.popleft()
                    outcomes.append(("signal", head[1]))
    return credits, outcomes
