"""Pins of the oracle's cache side of a run-time channel exchange (Sec. 5.2:
what the cache holds for a replaced channel is no longer valid) against the
LRU rules it must keep (Sec. 5.3): the channel's bricks leave, nothing else
moves, and the freed slots are the first taken, in ascending index."""
from __future__ import annotations

import numpy as np

import oracle


def _sim():
    V = oracle.make_volume((64, 64, 16), (1, 1, 1), 3, 16, 8, 3, (4, 4, 4), 4)
    sim = oracle.CacheSim(V, 60)
    rng = np.random.default_rng(4)
    up = rng.permutation(sim.total)[:80]  # more than the slots: evictions happen too
    for f, part in enumerate(np.array_split(up, 4)):
        sim.stream(f + 1, part)
    return V, sim


def test_only_the_channels_bricks_leave():
    V, sim = _sim()
    before = sim.page_table()
    per = sim.total // V.n_channels
    sim.evict_channel(1)
    after = sim.page_table()
    chan = lambda i: sim.id_to_dense[i] // per
    assert {i: s for i, s in before.items() if chan(i) != 1} == after
    assert any(chan(i) == 1 for i in before)
    assert not any(chan(i) == 1 for i in after)
    freed = sorted(s for i, s in before.items() if chan(i) == 1)
    assert sorted(np.nonzero(sim.slot_brick < 0)[0].tolist()) == freed


def test_freed_slots_are_taken_first_in_ascending_order():
    V, sim = _sim()
    per = sim.total // V.n_channels
    sim.evict_channel(0)
    freed = np.nonzero(sim.slot_brick < 0)[0]
    assert len(freed) > 2
    new = [b for b in range(per, sim.total) if sim.res_slot[b] < 0][:len(freed) - 1]
    flags, ev, slots = sim.stream(9, new)
    assert (flags == 1).all() and (ev < 0).all()
    assert np.array_equal(slots, freed[:len(new)])
