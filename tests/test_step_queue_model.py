"""A host model of the one-launch step's tile queue (sweep_step_persistent),
run on the CPU with the launch tables the library builds for the batch its
GPU tests use.

Each workgroup repeatedly takes the next queue index (head), finds its phase
(x, y or z tiles), its volume (slot) and the tile within the volume, waits
until every tile of that volume's previous phase is done (the done counter
of (phase - 1, slot) reaches the previous phase's tile count), works, and
counts its tile done.  Past the end of the queue it leaves; the last
workgroup to leave resets head, the done counters and the exit count for the
next launch.  The device runs this with atomics on a coarse-grained
workspace; here every counter operation is atomic and sequentially
consistent, and a seeded scheduler interleaves the workgroups one action at a
time, with only `resident` workgroups on the device at once (the others start,
in index order, as residents leave), as the hardware dispatcher does.

What the model shows: for every grid size and residency tried, every launch
ends, each tile runs exactly once, no tile starts before its volume's
previous phase is complete, and the counters are zero again after each
launch.  So with counters that behave as atomics, the queue cannot stall;
the stall seen on the GPU (the path is switched off) therefore lies in how
the counters behave on the device, which this model cannot reproduce."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2110_13368_amd import workloads as W

TILE = 64


def queue_tables(shapes):
    """The host's tables for the one-launch step: per axis, the exclusive tile
    prefix over the volumes (count + 1 entries), and the first queue index of
    each phase."""
    prefix, phase_start = [], [0]
    for axis in range(3):
        acc, row = 0, []
        for shp in shapes:
            row.append(acc)
            vol = shp[0] * shp[1] * shp[2]
            acc += (vol // shp[axis] + TILE - 1) // TILE
        row.append(acc)
        prefix.append(row)
        phase_start.append(phase_start[-1] + acc)
    return prefix, phase_start


def find_slot(prefix, count, tile):
    """Largest k in [0, count) with prefix[k] <= tile (the device's search)."""
    lo, hi = 0, count - 1
    while lo < hi:
        mid = (lo + hi + 1) >> 1
        if prefix[mid] <= tile:
            lo = mid
        else:
            hi = mid - 1
    return lo


class Launch:
    def __init__(self, shapes, grid, resident, rng, counters=None):
        self.prefix, self.ps = queue_tables(shapes)
        self.count = len(shapes)
        self.grid, self.resident, self.rng = grid, resident, rng
        # counters: head, exited, done[3][count]
        self.c = counters if counters is not None else {"head": 0, "exited": 0,
                                                        "done": np.zeros((3, self.count), np.int64)}
        self.runs = np.zeros(self.ps[3], np.int64)  # times each queue index was worked on
        self.started = {}  # queue index -> action number its work started
        self.finished = {}

    def run(self, max_actions=10_000_000):
        c, ps = self.c, self.ps
        waiting = list(range(self.grid))  # not yet dispatched, in index order
        state = {}  # workgroup -> (state, data)
        actions = 0
        while waiting or state:
            while waiting and len(state) < self.resident:
                state[waiting.pop(0)] = ("take", None)
            wg = list(state)[self.rng.integers(len(state))]
            st, d = state[wg]
            actions += 1
            assert actions < max_actions, "launch does not end"
            if st == "take":
                t = c["head"]
                c["head"] += 1
                if t >= ps[3]:
                    prev = c["exited"]
                    c["exited"] += 1
                    if prev == self.grid - 1:  # the last to leave resets the counters
                        c["head"] = 0
                        c["done"][:] = 0
                        c["exited"] = 0
                    del state[wg]
                    continue
                phase = 0 if t < ps[1] else (1 if t < ps[2] else 2)
                tp = t - ps[phase]
                slot = find_slot(self.prefix[phase], self.count, tp)
                assert self.prefix[phase][slot] <= tp < self.prefix[phase][slot + 1]
                state[wg] = ("wait" if phase > 0 else "work", (t, phase, slot, int(self.rng.integers(1, 6))))
            elif st == "wait":
                t, phase, slot, work = d
                pp = self.prefix[phase - 1]
                need = pp[slot + 1] - pp[slot]
                if c["done"][phase - 1, slot] >= need:
                    state[wg] = ("work", d)
            elif st == "work":
                t, phase, slot, work = d
                if t not in self.started:
                    self.started[t] = actions
                    self.runs[t] += 1
                if work > 1:
                    state[wg] = ("work", (t, phase, slot, work - 1))
                else:
                    self.finished[t] = actions
                    c["done"][phase, slot] += 1
                    state[wg] = ("take", None)
        return actions

    def check(self):
        ps = self.ps
        assert np.all(self.runs == 1), "a tile ran more or less than once"
        # every tile of a volume's previous phase finished before any of its tiles started
        for phase in (1, 2):
            for slot in range(self.count):
                lo, hi = self.prefix[phase][slot], self.prefix[phase][slot + 1]
                plo, phi = self.prefix[phase - 1][slot], self.prefix[phase - 1][slot + 1]
                if hi == lo or phi == plo:
                    continue
                first_start = min(self.started[ps[phase] + t] for t in range(lo, hi))
                last_prev = max(self.finished[ps[phase - 1] + t] for t in range(plo, phi))
                assert last_prev < first_start, (phase, slot)
        assert self.c["head"] == 0 and self.c["exited"] == 0 and not self.c["done"].any()


def test_queue_tables_match_the_split_sweep_tiling():
    prefix, ps = queue_tables([(9, 10, 11), (64, 1, 1), (65, 3, 2)])
    assert prefix[0] == [0, 2, 3, 4]  # x-lines 110, 1, 6: 2, 1, 1 tiles of 64 lines
    assert prefix[1] == [0, 2, 3, 6]  # y-lines 99, 64, 130
    assert prefix[2] == [0, 2, 3, 7]  # z-lines 90, 64, 195
    assert ps == [0, 4, 10, 17]


@pytest.mark.parametrize("grid,resident", [(1, 1), (7, 3), (300, 300), (300, 40), (10_000, 512)])
def test_queue_ends_runs_every_tile_once_in_order(grid, resident):
    wl = W.batched(n_sims=5, edge_range=(9, 75), cells_range=(100, 2000))
    shapes = [s.shape for s in wl.sims for _ in range(s.n_sub)]
    _, ps = queue_tables(shapes)
    grid = min(grid, ps[3])  # the runtime never launches more workgroups than tiles
    rng = np.random.default_rng(2110 + grid + resident)
    first = Launch(shapes, grid, min(resident, grid), rng)
    first.run()
    first.check()
    # a second launch (the next step's graph replay) starts from the reset counters
    second = Launch(shapes, grid, min(resident, grid), rng, counters=first.c)
    second.run()
    second.check()
