"""Step-by-step CPU model of how the persistent pipeline kernel's waves own claims and how an
ordered output stream's decoupled look-back waits on them.

It models scheduling only (no stage arithmetic): which wave owns which claim and when, which
waves are resident on the GPU, and the look-back words each claim publishes.  It follows the
kernel's rules:

- claim ownership, as in ``take_claim``: with ``by_index`` a wave first takes
  max(2, 7/8 of the claims / waves) claims by its index (b, b + W, b + 2W, ...), then claims from
  the launch's counter; without it every claim comes from the counter, in increasing order;
- claims are held two ahead: a wave takes two claims before it starts, and the claim after next
  whenever it starts one;
- a claim first counts its outputs and publishes its count (flag 1), then walks back over its
  predecessors, adding counts until it meets an inclusive prefix (flag 2); a predecessor with
  nothing published blocks the walk; then it publishes its own inclusive prefix (flag 2) and does
  its work;
- with a wait bound, a walk that has been blocked on one predecessor for that many steps gives
  up: the claim publishes flag 3 (no valid prefix), and a walk that meets flag 3 gives up too;
- residency: at most ``slots`` waves are resident at once (shared by every launch in the model);
  waves are dispatched in the given order as slots free up, and a wave leaves its slot when it
  has no claim left.

``simulate`` returns the outcome: "done" (every claim finished, with its inclusive prefix),
"deadlock" (no resident wave can move and no wave can be dispatched), or "gave_up" (every claim
finished, some with flag 3).
"""
import random


class Launch:
    def __init__(self, n_claims, n_waves, by_index, counts, work_steps=2):
        self.C = n_claims
        self.W = n_waves
        self.by_index = by_index
        self.counts = counts                  # output count of each claim
        self.work = work_steps
        self.counter = 0                      # the claim counter
        self.flag = [0] * n_claims            # look-back flag of each claim
        self.value = [0] * n_claims           # published count or inclusive prefix
        self.finished = [False] * n_claims
        n_static = max(2, (n_claims // 8 * 7) // n_waves) if by_index else 0
        self.n_static = n_static

    def take(self, wave):
        """take_claim: the next claim of this wave, or None."""
        while wave.n_static < self.n_static:
            c = wave.index + wave.n_static * self.W
            wave.n_static += 1
            if c < self.C:
                return c
            wave.n_static = self.n_static
        first = self.n_static * self.W if self.by_index else 0
        first = min(first, self.C)
        k = self.counter
        self.counter += 1
        return first + k if first + k < self.C else None


class Wave:
    def __init__(self, launch, index):
        self.launch = launch
        self.index = index
        self.n_static = 0
        self.held = []            # claims owned, in the order they will be worked
        self.phase = None         # None (between claims), "count", "walk", "work"
        self.cur = None
        self.walk_i = None
        self.prefix = 0
        self.blocked_for = 0
        self.work_left = 0
        self.started = False

    def start(self):
        self.started = True
        for _ in range(2):
            c = self.launch.take(self)
            if c is not None:
                self.held.append(c)

    def exhausted(self):
        return self.phase is None and not self.held

    def step(self, wait_bound):
        """Advance one step; returns True when the wave moved."""
        L = self.launch
        if self.phase is None:
            if not self.held:
                return False
            self.cur = self.held.pop(0)
            c = L.take(self)                  # the claim after next is taken as this one starts
            if c is not None:
                self.held.append(c)
            self.phase = "count"
            return True
        if self.phase == "count":
            L.flag[self.cur] = 1
            L.value[self.cur] = L.counts[self.cur]
            self.phase = "walk"
            self.walk_i = self.cur - 1
            self.prefix = 0
            self.blocked_for = 0
            return True
        if self.phase == "walk":
            if self.walk_i < 0:
                return self._publish(ok=True)
            f = L.flag[self.walk_i]
            if f == 0:
                if wait_bound is None:
                    return False
                # a bounded wait: its clock advances, and past the bound the walk gives up
                self.blocked_for += 1
                if self.blocked_for > wait_bound:
                    return self._publish(ok=False)
                return True
            self.blocked_for = 0
            if f == 3:
                return self._publish(ok=False)
            self.prefix += L.value[self.walk_i]
            if f == 2:
                return self._publish(ok=True)
            self.walk_i -= 1
            return True
        if self.phase == "work":
            self.work_left -= 1
            if self.work_left <= 0:
                L.finished[self.cur] = True
                self.phase = None
            return True
        raise AssertionError(self.phase)

    def _publish(self, ok):
        L = self.launch
        if ok:
            L.flag[self.cur] = 2
            L.value[self.cur] = self.prefix + L.counts[self.cur]
        else:
            L.flag[self.cur] = 3
            L.value[self.cur] = 0
        self.phase = "work"
        self.work_left = L.work
        return True


def simulate(launches, slots, dispatch_order, seed=0, wait_bound=None, max_steps=1_000_000):
    """Run the launches' waves on `slots` resident slots.  dispatch_order lists (launch index,
    wave index) pairs in the order the hardware dispatches them.  Each round, resident waves
    move in a random order (seeded)."""
    rng = random.Random(seed)
    waves = {(li, b): Wave(L, b) for li, L in enumerate(launches) for b in range(L.W)}
    pending = list(dispatch_order)
    resident = []
    for _ in range(max_steps):
        # dispatch into free slots
        while pending and len(resident) < slots:
            w = waves[pending.pop(0)]
            w.start()
            resident.append(w)
        moved = False
        order = resident[:]
        rng.shuffle(order)
        for w in order:
            if rng.random() < 0.8:            # not every wave moves every round
                moved |= w.step(wait_bound)
        before = len(resident)
        resident = [w for w in resident if not w.exhausted()]
        freed = len(resident) < before
        if all(all(L.finished) for L in launches) and not pending:
            gave_up = any(f == 3 for L in launches for f in L.flag)
            return "gave_up" if gave_up else "done"
        if not moved and not freed and not (pending and len(resident) < slots):
            # every wave gets a chance to move before the state counts as stuck
            if not any(w.step(wait_bound) for w in resident):
                return "deadlock"
    raise AssertionError("simulation did not settle")


def in_order(n_launches, n_waves):
    """Dispatch order of launches run back to back: launch 0's waves in index order, then the next."""
    return [(li, b) for li in range(n_launches) for b in range(n_waves)]


def interleaved(n_launches, n_waves, seed):
    """Two launches on different queues: their waves reach free slots in an arbitrary interleaving,
    each launch's waves in index order."""
    rng = random.Random(seed)
    queues = [[(li, b) for b in range(n_waves)] for li in range(n_launches)]
    out = []
    while any(queues):
        q = rng.choice([q for q in queues if q])
        out.append(q.pop(0))
    return out
