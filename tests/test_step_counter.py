"""The clause phase's step protocol, modelled on the host.

The sweep kernels cut a clause phase into T steps of 64 records; W waves take
them from a workgroup counter that hands out pairs of consecutive steps
(2j, 2j + 1), and the counter runs on across the sweeps of an item, each
sweep owning P = ceil(T/2) + W - (T mod 2) pair numbers.  This checks, for
random interleavings of the waves, that every step of every sweep is taken
exactly once and that a sweep consumes exactly P pair numbers, so the next
sweep's numbering starts where the kernel expects it.
"""
import random

import pytest


def pairs_per_sweep(T, W):
    return (T + 1) // 2 + W - (T & 1)


def run_sweep(T, W, counter, base, rng):
    taken = []

    def take(prev):
        if prev >= 0 and prev % 2 == 0:
            return prev + 1
        p = counter[0]
        counter[0] += 1
        return 2 * (p - base)

    state = [take(-1) for _ in range(W)]     # every wave takes a first pair
    live = [w for w in range(W) if state[w] < T]
    while live:
        w = rng.choice(live)                 # any wave may be the next to finish a step
        taken.append(state[w])
        state[w] = take(state[w])
        if state[w] >= T:
            live.remove(w)
    return taken


@pytest.mark.parametrize("T", [0, 1, 2, 3, 7, 8, 64, 95, 96, 1537])
@pytest.mark.parametrize("W", [1, 2, 4, 16])
def test_every_step_once_and_P_numbers_per_sweep(T, W):
    rng = random.Random(T * 131 + W)
    counter = [0]
    P = pairs_per_sweep(T, W)
    for s in range(5):
        base = s * P
        assert counter[0] == base
        taken = run_sweep(T, W, counter, base, rng)
        assert sorted(taken) == list(range(T))
    assert counter[0] == 5 * P


def test_a_counter_off_by_one_pair_is_caught():
    # the step-count formula without the odd-T correction leaves the next
    # sweep's numbering one pair short, so it would skip a pair of steps
    T, W = 7, 4
    rng = random.Random(1)
    counter = [0]
    wrong_P = (T + 1) // 2 + W
    run_sweep(T, W, counter, 0, rng)
    assert counter[0] != wrong_P
