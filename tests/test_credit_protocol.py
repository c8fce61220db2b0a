"""The credit protocol of §3 replayed step by step: the worked example of Fig. 2(b),
Lemma 1 (precise delivery), Lemma 2 (termination), the SIMD rule of §3.3, and
equality of the signal and tag strategies with the serial oracle."""
import json
import os
import random

import numpy as np
import pytest

from oracle import credit_sim, tiny
import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_worked_example_fig2b():
    with open(os.path.join(GOLDEN, "e5_credit_protocol.json")) as f:
        g = json.load(f)
    for case in g["cases"]:
        events = [tuple(e) for e in case["events"]]
        credits, outcomes = credit_sim.two_node_trace(events)
        assert credits == case["credits"]
        assert [list(o) for o in outcomes] == [list(o) for o in case["outcomes"]]


def small_case(kind, rng):
    P = rng.randrange(0, 9)
    sizes = [rng.choice([0, 1, 2, 3, 7, 12]) for _ in range(P)]
    if kind == tiny.TEXT_WORDS:
        starts, buf, pos = [], [], 0
        for s in sizes:
            starts.append(pos)
            buf.extend(rng.choice(b" ab") for _ in range(s))
            buf.append(10)
            pos += s + 1
        return dict(offsets=starts, lengths=sizes, elements=np.array(buf, np.uint8))
    off = [0]
    for s in sizes:
        off.append(off[-1] + s)
    vals = np.array([rng.getrandbits(32) if rng.random() < 0.7 else rng.choice([0, 4, 8]) for _ in range(off[-1])],
                    np.uint32)
    d = dict(offsets=off, elements=vals)
    if kind == tiny.GRAPH_THRESH:
        d["parent_param"] = np.array([rng.getrandbits(32) for _ in range(P)], np.uint32)
    return d


@pytest.mark.parametrize("kind", [1, 2, 3, 4])
def test_random_schedules_deliver_precisely_and_match_oracle(kind):
    """Random fireable node, random ensemble cap, minimal queues: Lemma 1, the SIMD
    rule and the parent bookkeeping are asserted inside the model; the records must
    equal the serial oracle's and the run must terminate (Lemma 2)."""
    rng = random.Random(kind)
    for trial in range(120):
        kw = small_case(kind, rng)
        recs, log, ens = credit_sim.simulate(kind, width=rng.choice([1, 2, 4, 8]), rng=rng, **kw)
        expect, _ = tiny.run(kind, kw["offsets"], kw["elements"], kw.get("lengths"), kw.get("parent_param"))
        assert recs == expect


def test_minimal_queues_still_terminate():
    rng = random.Random(3)
    kw = small_case(2, rng)
    for _ in range(30):
        recs, _, _ = credit_sim.simulate(2, width=16, rng=rng, cap_range=(1, 1), sig_cap_range=(1, 1), **kw)
        assert recs == tiny.run(2, kw["offsets"], kw["elements"])[0]


def test_violation_is_detected_when_credit_is_ignored(monkeypatch):
    """Planted mistake: a receiver that ignores the counter mixes regions in one ensemble."""
    orig = credit_sim.Node.fire

    def greedy_fire(self, cap, contexts, log):
        saved = self.counter
        self.counter = 10 ** 9 if self.inp.S else self.counter
        try:
            orig(self, cap, contexts, log)
        finally:
            if self.counter >= 10 ** 8:
                self.counter = saved
    monkeypatch.setattr(credit_sim.Node, "fire", greedy_fire)
    caught = 0
    rng = random.Random(1)
    for _ in range(40):
        kw = dict(offsets=[0, 3, 6, 9], elements=np.arange(9, dtype=np.uint32) * 4)
        try:
            credit_sim.simulate(1, width=8, rng=rng, cap_range=(8, 8), sig_cap_range=(4, 4), **kw)
        except AssertionError:
            caught += 1
    assert caught > 0


@pytest.mark.parametrize("kind", [1, 2, 3, 4])
def test_tag_strategy_matches_oracle(kind):
    rng = random.Random(50 + kind)
    for _ in range(150):
        kw = small_case(kind, rng)
        got = credit_sim.tag_replay(kind, width=rng.choice([1, 3, 8, 64]), rng=rng, **kw)
        assert got == tiny.run(kind, kw["offsets"], kw["elements"], kw.get("lengths"), kw.get("parent_param"))[0]


def test_enumeration_occupancy_closed_form():
    """With full-width firings the enumerator fires ceil(n_p / w) times per parent, so its
    occupancy is sum n_p / (w * sum ceil(n_p / w)); at fixed L that is L / (w ceil(L / w))."""
    w = 8
    for L in (1, 3, 8, 9, 16, 17):
        offsets = workloads.fixed_offsets(L * 6, L)
        vals = workloads.hash_values(1, L * 6)
        recs, log, ens = credit_sim.simulate(1, offsets=offsets, elements=vals, width=w,
                                             rng=random.Random(1), cap_range=(64, 64),
                                             sig_cap_range=(8, 8), policy="downstream")
        assert recs == tiny.run(1, offsets, vals)[0]
        sizes = ens["enum"]
        assert len(sizes) == 6 * -(-L // w)
        occ = sum(sizes) / (w * len(sizes))
        assert abs(occ - L / (w * -(-L // w))) < 1e-12
