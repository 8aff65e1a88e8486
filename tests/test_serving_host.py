"""Host logic of the serving loop on the CPU: the first-fit output arena
against a brute-force model of the address space, and the latency summary's
treatment of unfinished and shed requests."""
from __future__ import annotations

import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

pytest.importorskip("torch")
from paper_2309_04393_amd import serving  # noqa: E402


def _arena(size):
    a = serving.Arena.__new__(serving.Arena)  # bookkeeping only, no device buffer
    a.size, a.free_off, a.free_len, a.used, a.peak = size, [0], [size], 0, 0
    return a


@given(st.lists(st.tuples(st.booleans(), st.integers(1, 3000)), min_size=1, max_size=60))
@settings(max_examples=200, deadline=None)
def test_arena_matches_first_fit_model(ops):
    """Allocations are 256-byte aligned, never overlap, take the lowest free
    offset that fits (first fit), and frees coalesce back to one range."""
    size = 16384
    a = _arena(size)
    used = np.zeros(size // 256, bool)  # the model: one flag per 256-byte unit
    live = []
    for is_alloc, n in ops:
        if is_alloc or not live:
            units = (n + 255) // 256
            # first fit in the model
            expect = None
            for u in range(len(used) - units + 1):
                if not used[u:u + units].any():
                    expect = u
                    break
            got = a.alloc(n)
            if expect is None:
                assert got is None
                continue
            assert got == (expect * 256, units * 256)
            used[expect:expect + units] = True
            live.append(got)
        else:
            o, ln = live.pop(n % len(live))
            a.free(o, ln)
            used[o // 256:(o + ln) // 256] = False
        assert a.used == int(used.sum()) * 256
        # free list = the model's free runs, sorted and coalesced
        runs, u = [], 0
        while u < len(used):
            if not used[u]:
                v = u
                while v < len(used) and not used[v]:
                    v += 1
                runs.append((u * 256, (v - u) * 256))
                u = v
            else:
                u += 1
        assert list(zip(a.free_off, a.free_len)) == runs
    for o, ln in live:
        a.free(o, ln)
    assert a.free_off == [0] and a.free_len == [size] and a.used == 0


def test_latency_summary_unfinished_and_shed():
    R = serving.Request
    mk = lambda rid, arr, done, shed=False: R(rid, 0, arr, 8, 8, {}, [], None, done=done, shed=shed)
    trace = [mk(0, 0.0, 0.010), mk(1, 0.0, 0.020), mk(2, 0.0, 0.030), mk(3, 0.0, math.nan, shed=True)]
    s = serving.latency_summary(trace)
    assert s["n"] == 3 and s["completed"] == 3  # the shed request is not counted
    assert abs(s["p50_ms"] - 20.0) < 1e-9 and abs(s["max_ms"] - 30.0) < 1e-9
    trace.append(mk(4, 0.0, math.nan))  # unfinished, not shed: infinitely late
    s = serving.latency_summary(trace)
    assert s["n"] == 4 and s["completed"] == 3
    assert s["p99_ms"] is None  # the 99th percentile is unbounded
    assert abs(s["p50_completed_ms"] - 20.0) < 1e-9
