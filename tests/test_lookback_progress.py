"""CPU model of the ordered output stream's look-back (§4's context-free output stream, kept
in serial order): whether the claims' waits can deadlock, under the claim ownership of the
persistent kernel, when not every wave of a launch is resident.

The old ownership (claims by wave index, held two ahead) deadlocks once the grid exceeds the
resident slots, or when two launches share them; claims from one ascending counter, taken only
by running waves (still held two ahead), always finish with the exact prefixes; and a bounded
wait ends every wave even under the old ownership."""
import random

import pytest

from lookback_model import Launch, in_order, interleaved, simulate


def counts(rng, n):
    return [rng.randrange(0, 50) for _ in range(n)]


def prefixes_ok(L):
    run = 0
    for c in range(L.C):
        run += L.counts[c]
        if L.flag[c] != 2 or L.value[c] != run:
            return False
    return True


def test_by_index_ownership_deadlocks_below_full_residency():
    # 4 waves, 8 claims, 2 slots: waves 0 and 1 finish claims 0 and 1, then wait in the
    # look-back of claims 4 and 5 on claims 2 and 3, which belong to waves never dispatched
    L = Launch(8, 4, by_index=True, counts=[1] * 8)
    assert simulate([L], slots=2, dispatch_order=in_order(1, 4)) == "deadlock"
    assert L.flag[4] == 1 and L.flag[2] == 0


def test_by_index_ownership_progresses_when_every_wave_is_resident():
    rng = random.Random(1)
    for trial in range(40):
        W = rng.randrange(1, 12)
        C = rng.randrange(1, 60)
        L = Launch(C, W, by_index=True, counts=counts(rng, C))
        assert simulate([L], slots=W, dispatch_order=in_order(1, W), seed=trial) == "done"
        assert prefixes_ok(L)


def test_by_index_ownership_two_launches_sharing_slots_can_deadlock():
    # each launch alone fits the slots; two of them on different queues interleave
    outcomes = set()
    for seed in range(60):
        rng = random.Random(seed)
        W, C = 6, 30
        Ls = [Launch(C, W, by_index=True, counts=counts(rng, C)) for _ in range(2)]
        outcomes.add(simulate(Ls, slots=W, dispatch_order=interleaved(2, W, seed), seed=seed))
    assert "deadlock" in outcomes


@pytest.mark.parametrize("prefetch_heavy", [False, True])
def test_ascending_counter_always_finishes_with_exact_prefixes(prefetch_heavy):
    rng = random.Random(7 + prefetch_heavy)
    for trial in range(150):
        W = rng.randrange(1, 14)
        C = rng.randrange(1, 80) if not prefetch_heavy else rng.randrange(1, 2 * W + 3)
        slots = rng.randrange(1, W + 1)           # any residency, down to one wave at a time
        n_launches = rng.choice([1, 2])
        Ls = [Launch(C, W, by_index=False, counts=counts(rng, C)) for _ in range(n_launches)]
        order = in_order(n_launches, W) if rng.random() < 0.5 else interleaved(n_launches, W, trial)
        assert simulate(Ls, slots=slots, dispatch_order=order, seed=trial) == "done", (W, C, slots)
        for L in Ls:
            assert prefixes_ok(L)


def test_bounded_wait_ends_every_wave_and_poisons_successors():
    L = Launch(8, 4, by_index=True, counts=[1] * 8)
    assert simulate([L], slots=2, dispatch_order=in_order(1, 4), wait_bound=20) == "gave_up"
    assert all(L.finished)
    # a claim that gave up publishes flag 3, and no claim after it holds a prefix built on it
    first_bad = min(c for c in range(8) if L.flag[c] == 3)
    run = 0
    for c in range(first_bad):
        run += L.counts[c]
        assert L.flag[c] == 2 and L.value[c] == run
    for c in range(first_bad + 1, 8):
        if L.flag[c] == 2:
            # only claims whose walk met an intact prefix before the bad claim
            assert L.value[c] == sum(L.counts[:c + 1])


def test_bounded_wait_leaves_healthy_runs_exact():
    rng = random.Random(3)
    for trial in range(40):
        W = rng.randrange(1, 10)
        C = rng.randrange(1, 50)
        L = Launch(C, W, by_index=False, counts=counts(rng, C))
        slots = rng.randrange(1, W + 1)
        assert simulate([L], slots=slots, dispatch_order=in_order(1, W), seed=trial, wait_bound=10_000) == "done"
        assert prefixes_ok(L)
