"""CPU model of the device barrier's protocol (the counter barrier of the
device header): an arrival word holding the phase number (high 32 bits) and
the arrivals of the phase (low 32 bits), and a generation word holding the
completed phases.  Random interleavings of the arrivals' steps, reads of
the generation word that may return any older value still allowed by
per-location coherence, and a different number of arrivals in every phase
(slots are shared by calls with different work-group counts, which run as
separate launches in stream order) must never let an arrival leave a phase
before every arrival of that phase has arrived, and must never deadlock.  A model of the steps, not of the
kernel: it pins the protocol the kernel implements."""
import random

import pytest


class Memory:
    """Two words; the generation keeps its history so a read may return any
    value at or after the last one this reader saw (coherence)."""

    def __init__(self):
        self.cnt = 0
        self.gen_hist = [0]

    def fetch_add_cnt(self):
        old = self.cnt
        self.cnt += 1
        return old

    def read_gen(self, seen_idx, rng):
        idx = rng.randint(seen_idx, len(self.gen_hist) - 1)
        return idx, self.gen_hist[idx]


def run_model(units_per_phase, seed, mem=None):
    """Consecutive phases with the same member count are barriers inside one
    launch: members run ahead into the next phase freely.  A phase with a
    different member count is a later launch in stream order: it starts
    only after every member of the previous phase has left it."""
    rng = random.Random(seed)
    mem = Memory() if mem is None else mem
    arrived, left = {}, {}
    nagents = max(units_per_phase)
    nph = len(units_per_phase)
    state = {a: {"phase": 0, "step": "arrive", "next": None, "seen": 0} for a in range(nagents)}

    def may_start(p):
        return p == 0 or units_per_phase[p] == units_per_phase[p - 1] or \
            left.get(p - 1, 0) == units_per_phase[p - 1]

    def leave(a, p):
        left[p] = left.get(p, 0) + 1
        state[a]["phase"] = p + 1
        state[a]["step"] = "arrive"

    done = set()
    steps = 0
    while len(done) < nagents:
        steps += 1
        assert steps < 200_000, "no progress: deadlock"
        a = rng.choice([x for x in range(nagents) if x not in done])
        s = state[a]
        p = s["phase"]
        if p == nph:
            done.add(a)
            continue
        units = units_per_phase[p]
        if s["step"] == "arrive":
            if not may_start(p):
                continue
            if a >= units:                          # not a member of this launch
                if left.get(p, 0) == units:         # it has ended
                    s["phase"] += 1
                    s["seen"] = len(mem.gen_hist) - 1
                continue
            old = mem.fetch_add_cnt()
            assert (old >> 32) == p, "arrival in the wrong phase"
            arrived[p] = arrived.get(p, 0) + 1
            nxt = (old >> 32) + 1
            if (old & 0xFFFFFFFF) == units - 1:
                mem.cnt = nxt << 32                 # reset with the next phase number
                mem.gen_hist.append(nxt)            # then release the generation
                s["seen"] = len(mem.gen_hist) - 1
                leave(a, p)
            else:
                s["step"], s["next"] = "wait", nxt
        else:
            s["seen"], g = mem.read_gen(s["seen"], rng)
            if g == s["next"]:
                assert arrived[p] == units, "left the phase before every arrival"
                leave(a, p)
    return mem


@pytest.mark.parametrize("seed", range(40))
def test_barrier_phases_hold_under_any_interleaving(seed):
    rng = random.Random(1000 + seed)
    units = [rng.choice([1, 2, 3, 5, 8]) for _ in range(12)]
    mem = run_model(units, seed)
    assert mem.gen_hist[-1] == len(units) and mem.cnt == len(units) << 32


def timed_out_phase(units):
    """Memory after a barrier phase in which one of `units` members never
    arrived: the others added themselves, waited out the spin limit and left
    (the kernel latches a timeout and ends), so the count still holds
    units - 1 arrivals of phase 0 and the generation never moved."""
    mem = Memory()
    for _ in range(units - 1):
        mem.fetch_add_cnt()
    return mem


@pytest.mark.parametrize("units", [2, 3, 8])
def test_stale_words_after_a_timeout_release_the_next_barrier_early(units):
    """Left as they are, the words of a timed-out phase make the next
    barrier's first arrival the "last" one: it leaves before the others
    arrive.  Clearing them (what the host does once it reads a latched
    timeout with the device idle) gives a barrier that holds again."""
    early = 0
    for seed in range(30):
        try:
            run_model([units] * 4, seed, mem=timed_out_phase(units))
        except AssertionError as e:
            assert "before every arrival" in str(e) or "wrong phase" in str(e)
            early += 1
    assert early == 30
    for seed in range(30):
        mem = run_model([units] * 4, seed, mem=Memory())   # the cleared words
        assert mem.gen_hist[-1] == 4 and mem.cnt == 4 << 32


def run_old_model(units, nphases, seed, limit=20_000):
    """The earlier protocol: read the generation, arrive on a count that the
    last arrival resets, wait until the generation changes.  The read and
    the arrival are unordered (relaxed, different lines), so either may be
    performed first.  Returns False when the schedule deadlocks."""
    rng = random.Random(seed)
    cnt, gen = 0, 0
    st = {a: {"phase": 0, "todo": None, "g": None} for a in range(units)}
    steps = 0
    while any(x["phase"] < nphases for x in st.values()):
        steps += 1
        if steps > limit:
            return False
        a = rng.choice([x for x in st if st[x]["phase"] < nphases])
        x = st[a]
        if x["todo"] is None:
            x["todo"] = ["read", "add"] if rng.random() < 0.5 else ["add", "read"]
        if x["todo"]:
            op = x["todo"].pop(0)
            if op == "read":
                x["g"] = gen
            else:
                cnt += 1
                if cnt == units:          # last arrival
                    cnt, gen = 0, gen + 1
                    x["last"] = True
            continue
        if x.pop("last", False) or gen != x["g"]:
            x["phase"] += 1
            x["todo"], x["g"] = None, None
    return True


def test_reading_the_generation_apart_from_the_arrival_can_deadlock():
    """The model finds the earlier protocol's failure: a read of the
    generation performed after the arrival can see the phase's own
    completion and wait for a change that needs its own next arrival."""
    assert not all(run_old_model(4, 6, seed) for seed in range(200))
