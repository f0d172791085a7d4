"""Pins of the overlap histogram and the annealing schedule (oracle.overlap)
to closed forms and brute force."""
import math

import numpy as np

from oracle import overlap, physics


def test_all_configurations_closed_form():
    """Over all 2^n configurations, a configuration has C(n, k) partners with k
    agreeing sites (k < n), so the unordered pairs number 2^(n-1) C(n, k)."""
    n = 10
    c = overlap.overlap_counts(physics.all_configs(n))
    want = [2 ** (n - 1) * math.comb(n, k) for k in range(n)] + [0]
    assert c.tolist() == want


def test_brute_force_pair_loop_and_flip_relation():
    rng = np.random.default_rng(3)
    s = np.where(rng.random((23, 17)) < 0.3, -1, 1).astype(np.int8)
    c = overlap.overlap_counts(s)
    ref = np.zeros(18, dtype=np.int64)
    for a in range(23):
        for b in range(a + 1, 23):
            ref[int((s[a] == s[b]).sum())] += 1
    assert np.array_equal(c, ref) and c.sum() == 23 * 22 // 2
    # S and its global flip -S: pairs inside S or inside -S keep k, the cross
    # pairs (a, -b), a != b, have n - k, and the 23 pairs (a, -a) have k = 0
    cb = overlap.overlap_counts(np.concatenate([s, -s]))
    want = 2 * ref + 2 * ref[::-1]
    want[0] += 23
    assert np.array_equal(cb, want)


def test_annealing_schedule_endpoints():
    T0, nw, neq, na = 2.0, 1200, 5, 500
    T = [overlap.anneal_temperature(i, T0, nw, neq, na) for i in range(0, nw + neq * na + 20)]
    assert T[nw] == T0 and T[nw + neq - 1] == T0 and T[nw + neq] == T0 - T0 / na
    assert T[nw + neq * na] == 0.0 and T[-1] == 0.0
    assert all(a >= b for a, b in zip(T, T[1:]))
    assert len(set(T)) == na + 1
