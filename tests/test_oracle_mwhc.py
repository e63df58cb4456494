"""Pins of the oracle's MWHC variant (section 4.1): 3-partite edges, the
peelability threshold of random 3-hypergraphs, the peel-only failure rule,
exact values and the filter's false-positive rate."""
import math

import numpy as np

import oracle as O
import synthetic as S


def test_geometry_is_three_parts_of_c_m_over_3():
    for m in (0, 1, 1000, 65536, 10 ** 6):
        g = O.geometry(m, 3, mwhc=True)
        assert (g["c_num"], g["c_den"], g["mwhc"]) == (123, 100, 1)
        assert g["part"] == max(1, math.ceil(1.23 * m / 3)) and g["V"] == 3 * g["part"]


def test_edges_are_three_partite_and_uniform_in_each_part():
    part = 1000
    offs = [[], [], []]
    rng = np.random.default_rng(1)
    for lo in rng.integers(0, 2 ** 63, 20000, dtype=np.int64).tolist():
        v = O.edge_mwhc(lo, part, 0)
        for i in range(3):
            assert i * part <= v[i] < (i + 1) * part
            offs[i].append(v[i] - i * part)
    for o in offs:  # mean and spread of a uniform variable on [0, part)
        o = np.asarray(o, dtype=np.float64)
        assert abs(o.mean() - (part - 1) / 2) < 5 * part / math.sqrt(12 * o.size)
        assert abs(o.std() - part / math.sqrt(12)) < 0.02 * part
    # a different local seed gives a different edge from the same signature
    assert O.edge_mwhc(12345, part, 0) != O.edge_mwhc(12345, part, 1)


def _first_attempt_failures(c, sizes, trials):
    fails = tot = 0
    for m in sizes:
        for t in range(trials):
            keys = S.member_keys(m, 5000 + 13 * m + t).numpy().view(np.uint64)
            B = O.build(keys, b=8, is_filter=True, h=0, seed=t, tmax=1, c=c, mwhc=True)
            fails += B.status
            tot += 1
    return fails / tot


def test_peelability_threshold_of_random_3_hypergraphs():
    """Random 3-hypergraphs peel w.h.p. above c = 1.2217 (section 3.1) and
    almost never below it; 1.23 is above."""
    sizes = (20000, 50000)
    assert _first_attempt_failures((123, 100), sizes, 4) <= 0.25
    assert _first_attempt_failures((130, 100), sizes, 4) <= 0.25
    assert _first_attempt_failures((115, 100), sizes, 4) >= 0.75


def test_peel_only_rule_and_values():
    keys = S.member_keys(30000, 61).numpy().view(np.uint64)
    vals = S.values(30000, 16, 61).numpy().view(np.uint64)
    B = O.build(keys, vals, b=16, is_filter=False, h=2, seed=3, mwhc=True)
    assert B.status == 0
    assert all(f[2] == 2 and f[3] > 0 for f in B.failures)
    assert np.array_equal(O.query(B, keys), vals)
    # a key listed twice with two values never peels: every attempt fails
    k2 = keys.copy()
    v2 = vals.copy()
    k2[10] = k2[20]
    v2[10] = v2[20] ^ 1
    B2 = O.build(k2, v2, b=16, is_filter=False, h=0, seed=3, tmax=4, mwhc=True)
    assert B2.status == 1 and [f[1] for f in B2.failures] == [0, 1, 2, 3]
    assert all(f[2] == 2 for f in B2.failures)


def test_filter_false_positive_rate():
    n, b = 40000, 8
    keys = S.member_keys(n, 62).numpy().view(np.uint64)
    B = O.build(keys, b=b, is_filter=True, h=1, seed=0, mwhc=True)
    assert O.query(B, keys).min() == 1
    neg = S.negative_keys(n, 200000, 62).numpy().view(np.uint64)
    fp = int(O.query(B, neg).sum())
    p = 2.0 ** -b
    assert abs(fp - 200000 * p) <= 5 * math.sqrt(200000 * p * (1 - p))
