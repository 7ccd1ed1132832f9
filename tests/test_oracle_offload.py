"""Pins of the oracle's ADMM-Offload planner (Section 5.1) on hand-worked timelines,
and parity of the library's planner (lam_offload_plan / lam_offload_evaluate, host
code) with it on those and on random timelines.

Hand-worked cases (phases of 1 s each, sizes 10 bytes):
* A used in phase 0 over [0, 0.5], B in phase 1 over [0.2, 0.6], link 100 B/s (transfers
  of 0.1 s): A offloaded over [0.5, 0.6] and prefetched over [2.9, 3.0], B offloaded over
  [1.6, 1.7] and prefetched over [3.9, 4.0]; they are never present together, so the
  peak is 10 and M = 10, T = 0.
* the same with a 20 B/s link (transfers of 0.5 s): A's offload ends at 1.0 while B's
  prefetch for phase 1 starts at 0.5, so both are present over [0.5, 1.0]: M = 0 and the
  planner keeps everything resident.
* A and C both used in phase 0 over [0, 0.5], 20 B/s: offloads [0.5, 1.0] and [1.0, 1.5];
  both prefetches are planned for [2.5, 3.0], the second waits for the first and ends at
  3.5, half a second after phase 0 starts: T = 0.5.
* a transfer longer than the gap is dropped (constraint 3); dead gaps (the next phase
  writes first) cost no transfer: two variables each written and used in its own phase
  are never present together.
"""
import random

import pytest

from oracle import lam_oracle as O

AB = {"A": {0: (0.0, 0.5, False)}, "B": {1: (0.2, 0.6, False)}}


def test_disjoint_uses_fast_link():
    best = O.offload_plan([1.0, 1.0, 1.0], {"A": 10.0, "B": 10.0}, AB, 0.0, 100.0)
    assert best[0] == {"A", "B"} and best[1] == 10.0 and best[2] == 0.0
    ab = {v: (round(a, 12), round(z, 12)) for v, a, z in best[4]}
    assert ab == {"A": (0.6, 2.9), "B": (1.7, 3.9)}


def test_disjoint_uses_slow_link_saves_nothing():
    best = O.offload_plan([1.0, 1.0, 1.0], {"A": 10.0, "B": 10.0}, AB, 0.0, 20.0)
    assert best[0] == frozenset() and best[3] == 0.0
    M, T, _ = O.offload_evaluate(["A", "B"], [1.0, 1.0, 1.0], {"A": 10.0, "B": 10.0}, AB, 20.0)
    assert M == 0.0 and T == 0.0


def test_prefetch_contention_delays():
    acc = {"A": {0: (0.0, 0.5, False)}, "C": {0: (0.0, 0.5, False)}}
    M, T, absent = O.offload_evaluate(["A", "C"], [1.0, 1.0, 1.0], {"A": 10.0, "C": 10.0}, acc, 20.0)
    assert M == 0.0 and T == pytest.approx(0.5)
    assert sorted((v, a, z) for v, a, z in absent) == [("A", 1.0, 2.5), ("C", 1.5, 3.0)]


def test_gap_too_short_is_dropped_and_dead_gaps_are_free():
    # A: gap of 2.5 s, transfers of 3 s: dropped (constraint 3), nothing absent
    M, T, absent = O.offload_evaluate(["A"], [1.0, 1.0, 1.0], {"A": 10.0}, {"A": {0: (0.0, 0.5, False)}}, 10.0 / 3.0)
    assert absent == [] and M == 0.0 and T == 0.0
    # G written first in phase 0 and K in phase 1, each used over [0, 0.5] of its phase: both dead outside,
    # absent from their last use to their next phase's start with no transfer even on a 1 mB/s link;
    # they are never present together (peak 10, M = 10)
    acc = {"G": {0: (0.0, 0.5, True)}, "K": {1: (0.0, 0.5, True)}}
    best = O.offload_plan([1.0, 1.0, 1.0], {"G": 10.0, "K": 10.0}, acc, 0.0, 1e-3)
    assert best[0] == {"G", "K"} and best[1] == 10.0 and best[2] == 0.0
    assert sorted(best[4]) == [("G", 0.5, 3.0), ("K", 1.5, 4.0)]


def test_budget():
    sizes = {"A": 10.0, "B": 10.0}
    assert O.offload_plan([1.0, 1.0, 1.0], sizes, AB, 5.0, 100.0, budget=15.0)[0] == {"A", "B"}
    assert O.offload_plan([1.0, 1.0, 1.0], sizes, AB, 5.0, 20.0, budget=15.0)[3] == -1.0


def _random_case(rng):
    P = rng.randint(2, 4)
    phase = [rng.uniform(0.2, 2.0) for _ in range(P)]
    nv = rng.randint(1, 5)
    sizes, acc = {}, {}
    for i in range(nv):
        name = f"v{i}"
        sizes[name] = float(rng.choice([1, 2, 3, 6])) * 1e9
        ks = sorted(rng.sample(range(P), rng.randint(1, P)))
        a = {}
        for k in ks:
            f = rng.uniform(0.0, phase[k])
            l = rng.uniform(f, phase[k])
            a[k] = (f, l, rng.random() < 0.3)
        acc[name] = a
    return phase, sizes, acc, rng.uniform(0.0, 2e9), rng.choice([5e9, 25e9, 50e9, 200e9])


def _lib_vars(sizes, acc, cands=None):
    return {n: {"bytes": sizes[n], "access": acc[n], "candidate": cands is None or n in cands} for n in sizes}


def test_library_planner_matches_oracle():
    from paper_2511_01893_amd import lam as L
    rng = random.Random(11)
    cases = [([1.0, 1.0, 1.0], {"A": 10.0, "B": 10.0}, AB, 0.0, link) for link in (100.0, 20.0)]
    cases += [_random_case(rng) for _ in range(150)]
    chosen = 0
    for phase, sizes, acc, resident, link in cases:
        budget = None if rng.random() < 0.5 else resident + sum(sizes.values()) * rng.uniform(0.5, 1.0)
        o = O.offload_plan(phase, sizes, acc, resident, link, budget=budget)
        g = L.offload_plan(phase, _lib_vars(sizes, acc), resident, link, budget)
        assert set(g["offload"]) == set(o[0]), (phase, sizes, acc, link)
        assert g["M"] == o[1] and g["T"] == o[2] and g["MT"] == o[3]
        chosen += bool(o[0])
        for plan in (list(sizes), list(sizes)[:1]):
            om, ot, _ = O.offload_evaluate(plan, phase, sizes, acc, link)
            ge = L.offload_evaluate(phase, _lib_vars(sizes, acc), resident, link, plan)
            assert ge["M"] == om and ge["T"] == ot
    assert chosen > 10


def test_library_planner_argument_errors():
    from paper_2511_01893_amd import lam as L
    v = _lib_vars({"A": 1.0}, {"A": {0: (0.0, 0.5, False)}})
    with pytest.raises(L.LamError):
        L.offload_plan([1.0, -1.0], v, 0.0, 1e9)
    with pytest.raises(L.LamError):
        L.offload_plan([1.0], _lib_vars({"A": 1.0}, {"A": {0: (0.6, 0.5, False)}}), 0.0, 1e9)
    with pytest.raises(L.LamError):
        L.offload_plan([1.0], v, 0.0, 0.0)


def test_dead_gaps_abutting_at_a_phase_boundary():
    """G written and used in phase 0 only, D written in phase 1 and read in phase 2: both gaps are
    dead, G is absent through phases 1-2 and D through phase 0, so they are never present together
    and M is one size with no transfer, whatever the phase durations.  D's absence ends where phase
    1 starts, the instant G's begins: a folded end computed as (start + period) mod period can land
    an ulp early and count both as present (it did for phases of 75.77, 3.59 and 0.67 ms)."""
    rng = random.Random(5)
    cases = [[0.07577, 0.00359, 0.00067], [0.07637, 0.00352, 0.00066]]
    cases += [[rng.uniform(1e-4, 0.2) for _ in range(3)] for _ in range(300)]
    for ph in cases:
        a = {"G": {0: (0.0, ph[0], True)}, "D": {1: (0.0, ph[1], True), 2: (0.0, ph[2], False)}}
        M, T, _ = O.offload_evaluate(["G", "D"], ph, {"G": 5.0, "D": 5.0}, a, 1e9)
        assert M == 5.0 and T == 0.0, ph


def test_library_dead_gaps_abutting_at_a_phase_boundary():
    from paper_2511_01893_amd import lam as L
    for ph in ([0.07577, 0.00359, 0.00067], [0.07637, 0.00352, 0.00066]):
        a = {"G": {0: (0.0, ph[0], True)}, "D": {1: (0.0, ph[1], True), 2: (0.0, ph[2], False)}}
        r = L.offload_evaluate(ph, _lib_vars({"G": 5.0, "D": 5.0}, a), 0.0, 1e9, ["G", "D"])
        assert r["M"] == 5.0 and r["T"] == 0.0, ph
