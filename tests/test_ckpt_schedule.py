"""The checkpointed sweep's lane schedule, checked on the CPU (no GPU).

A wavefront's lanes each replay every segment of their tape forward and
then reverse it, one step a trip; each lane waits first_gap trips before
replaying its first segment and again after reversing it (the rule in the
sweep's source: L = r_max when that adds no trips, else L = K when the
2 K (F_max + 1) trips are at most a quarter more than 2 S_max, else no
wait).  Restated here, the schedule must give every lane exactly S replay
steps and S reverse steps in the sweep's order, end, keep every trip of an
aligned wavefront all-replay or all-reverse, and take no more trips than
the rule allows.
"""
import numpy as np
import pytest


def first_gaps(steps, k):
    r = [(s - 1) % k + 1 if s > 0 else 0 for s in steps]
    f = [(s - q) // k if s > 0 else 0 for s, q in zip(steps, r)]
    r_max, f_max, s_max = max(r), max(f), max(steps)
    if r_max + k * f_max <= s_max:
        return [r_max - q for q in r], "r_max"
    if 4 * k * (f_max + 1) <= 5 * s_max:
        return [k - q for q in r], "k"
    return [0] * len(steps), None


def run(steps, k):
    """Trips of one wavefront: (number, mixed trips, per-lane step order)."""
    gaps, mode = first_gaps(steps, k)
    lanes = []
    for s, g in zip(steps, gaps):
        lanes.append(dict(i=s, slot=(s - 1) % k if s > 0 else 0, rebuild=s > 0, j=0,
                          seg=(s - 1) % k + 1 if s > 0 else 0, wait=g, gap=g, live=True,
                          order=[]))
    trips = mixed = 0
    while any(l["live"] for l in lanes):
        trips += 1
        assert trips < 10 * (2 * max(steps) + 2 * k + 1)
        kinds = set()
        for l in lanes:
            if not l["live"]:
                continue
            if l["wait"] > 0:
                l["wait"] -= 1
                continue
            if not l["rebuild"] and l["i"] == 0:
                l["live"] = False
                continue
            if l["rebuild"]:
                # replay step j of the segment that ends at mesh point i
                l["order"].append(("replay", l["i"] - l["seg"] + l["j"] + 1))
                kinds.add("replay")
                l["j"] += 1
                if l["j"] == l["seg"]:
                    l["rebuild"] = False
                continue
            kinds.add("reverse")
            l["order"].append(("reverse", l["i"]))
            l["i"] -= 1
            l["slot"] -= 1
            if l["slot"] < 0 and l["i"] > 0:
                l["slot"], l["rebuild"], l["j"], l["seg"] = k - 1, True, 0, k
                l["wait"], l["gap"] = l["gap"], 0
        mixed += kinds == {"replay", "reverse"}
    return trips, mixed, mode, [l["order"] for l in lanes]


def expected_order(s, k):
    """Segments from the last: replay its steps forward, then reverse them."""
    out = []
    end = s
    while end > 0:
        start = ((end - 1) // k) * k
        out += [("replay", m) for m in range(start + 1, end + 1)]
        out += [("reverse", m) for m in range(end, start, -1)]
        end = start
    return out


@pytest.mark.parametrize("k", [16, 32, 64, 128, 256])   # the segment lengths the library takes
def test_schedule_order_alignment_and_trips(k):
    rng = np.random.default_rng(k)
    for trial in range(60):
        spread = [0, 3, 25, 200][trial % 4]
        steps = sorted(int(x) for x in rng.normal(300, spread, 64).clip(0, None))
        if trial % 7 == 0:
            steps[int(rng.integers(0, 64))] = 0     # a failed or empty lane
        trips, mixed, mode, orders = run(steps, k)
        for s, o in zip(steps, orders):
            assert o == expected_order(s, k)
        s_max = max(steps)
        if mode is not None:
            assert mixed == 0
        if mode == "r_max" or mode is None:
            assert trips == 2 * s_max + 1 if s_max > 0 else trips <= 1
        else:
            assert trips - 1 <= (5 * 2 * s_max) // 4 + 2 * k


def test_straddling_wavefront_is_padded_or_left():
    # step counts on both sides of a multiple of K: r wraps from K to 1
    steps = [255, 256, 257, 258] * 16
    gaps, mode = first_gaps(steps, 64)
    assert mode == "k" and min(gaps) == 0 and max(gaps) == 63
    gaps, mode = first_gaps(steps, 256)        # padding to 256 would double the trips
    assert mode is None and gaps == [0] * 64
