"""Algorithm 1 (Sec. 3.5) in the oracle: the paper's worked example, the
bounds of Sec. 3.7, the clamped last round, and parallel == sequential on a
real glass (CPU only)."""
import math
import os

import numpy as np
import pytest

import aqs_synth as S
import oracle as O
from oracle.alg1 import adaptive_k, aqs_parallel, aqs_sequential, chain_plan

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load_example():
    kv, cases = {}, []
    for line in open(os.path.join(GOLD, "alg1_worked_example.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, *v = line.split()
        if k == "case":
            cases.append(v)
        else:
            kv[k] = v
    return kv, cases


class Mock:
    """Configurations are (strain index, basin label) pairs.  The true path
    stays in basin 0; an anchor at strain index m lands in basin
    wrong[m] if given (a misprediction), else 0; fine steps keep the basin."""

    def __init__(self, wrong=None):
        self.wrong = wrong or {}
        self.calls = []

    def level1(self, r_star, m):
        k, b = r_star
        if m == 0:               # r^c_0 = r_star, already an inherent structure
            return (k, b)
        return (k + m, ("anchor", k + m))

    def level2(self, anchors, lengths):
        out = []
        for (k, tag), ln in zip(anchors, lengths):
            basin = self.wrong.get(k, 0) if isinstance(tag, tuple) else tag
            outgoing = (k, basin)
            out.append((outgoing, (k + ln, basin)))
        self.calls.append(list(lengths))
        return out

    @staticmethod
    def equal(a, b):
        assert a[0] == b[0], "compared configurations must share the strain"
        return a[1] == b[1]


def test_worked_example_of_the_paper():
    kv, cases = load_example()
    P, K, n = int(kv["P"][0]), int(kv["K"][0]), int(kv["n_steps"][0])
    assert [int(x) for x in kv["anchors"]] == [i * K for i in range(P)]
    for c5, c10, q, star in cases:
        wrong = {}
        if c5 == "0":
            wrong[5] = 1
        if c10 == "0":
            wrong[10] = 1
        m = Mock(wrong)
        res = aqs_parallel((0, 0), n, K, P, m.level1, m.level2, m.equal)
        first = res.rounds[0]
        assert first.q == int(q)
        expect_checks = [c == "1" for c in (c5, c10) if c != "-"]
        assert first.checks == expect_checks
        assert res.rounds[0].start == 0
        if len(res.rounds) > 1:
            assert res.rounds[1].start == int(star)
        assert res.r_star == (15, 0) and res.n_current == 15


@pytest.mark.parametrize("P,K,n", [(4, 1, 200), (8, 6, 200), (16, 14, 200), (32, 16, 200), (3, 5, 15)])
def test_best_case_accepts_PK_per_round(P, K, n):
    m = Mock()
    res = aqs_parallel((0, 0), n, K, P, m.level1, m.level2, m.equal)
    assert all(r.q == sum(r.lengths) for r in res.rounds)
    assert len(res.rounds) == math.ceil(n / (P * K))
    assert res.n_current == n and res.computed_steps == n


@pytest.mark.parametrize("P,K,n", [(4, 5, 40), (8, 6, 200), (4, 16, 200)])
def test_worst_case_progresses_K_per_round(P, K, n):
    """Every anchor i >= 1 mispredicts: exactly K steps per round and
    ceil(N_steps / K) rounds (Sec. 3.7)."""
    wrong = {k: 1 for k in range(1, n + P * K + 1)}
    m = Mock(wrong)
    res = aqs_parallel((0, 0), n, K, P, m.level1, m.level2, m.equal)
    assert all(r.q == min(K, r.lengths[0]) for r in res.rounds)
    assert len(res.rounds) == math.ceil(n / K)
    assert res.r_star == (n, 0)


def test_clamped_last_round():
    assert chain_plan(200, 6, 8) == [6] * 8
    assert chain_plan(8, 6, 8) == [6, 2]
    assert chain_plan(4, 6, 8) == [4]
    m = Mock()
    res = aqs_parallel((0, 0), 200, 14, 16, m.level1, m.level2, m.equal)
    assert res.rounds[-1].lengths == [14] * 14 + [4]
    assert res.n_current == 200


def test_adaptive_k_rule():
    assert adaptive_k(4, [True, True], 1, 16) == 8
    assert adaptive_k(12, [True], 1, 16) == 16
    assert adaptive_k(5, [False], 1, 16) == 3
    assert adaptive_k(2, [False], 2, 16) == 2
    assert adaptive_k(1, [False], 1, 16) == 1
    assert adaptive_k(6, [True, False], 1, 16) == 6
    assert adaptive_k(6, [True, True, False], 1, 16) == 6
    assert adaptive_k(6, [], 1, 16) == 6


def test_dynamic_k_doubles_while_every_anchor_agrees():
    """Best case: the rounds' chains grow 2, 4, 8, 16, 16, ...; every step is
    accepted and none is computed twice."""
    m = Mock()
    res = aqs_parallel((0, 0), 200, 2, 4, m.level1, m.level2, m.equal, lambda k, c: adaptive_k(k, c, 1, 16))
    assert [r.K for r in res.rounds][:5] == [2, 4, 8, 16, 16]
    assert [r.q for r in res.rounds][:4] == [8, 16, 32, 64]
    assert res.n_current == 200 and res.computed_steps == 200 and res.r_star == (200, 0)


def test_dynamic_k_halves_while_the_first_anchor_mispredicts():
    """Worst case: K = 8, 4, 2, 1, 1, ...; each round accepts its chain 0."""
    n = 30
    m = Mock({k: 1 for k in range(1, n + 64)})
    res = aqs_parallel((0, 0), n, 8, 4, m.level1, m.level2, m.equal, lambda k, c: adaptive_k(k, c, 1, 16))
    assert [r.K for r in res.rounds][:5] == [8, 4, 2, 1, 1]
    assert all(r.q == r.lengths[0] for r in res.rounds)
    assert res.n_current == n and res.r_star == (n, 0)


def test_dynamic_k_keeps_k_after_a_later_failure():
    """The anchor at strain 12 mispredicts once: round 0 (K = 4) passes its
    first two checks and fails the third, so K stays 4."""
    m = Mock({12: 1})
    res = aqs_parallel((0, 0), 40, 4, 4, m.level1, m.level2, m.equal, lambda k, c: adaptive_k(k, c, 1, 16))
    r0, r1 = res.rounds[:2]
    assert r0.checks == [True, True, False] and r0.q == 12 and r1.K == 4
    assert r1.start == 12 and res.n_current == 40


def test_algorithm_needs_two_threads():
    m = Mock()
    with pytest.raises(ValueError):
        aqs_parallel((0, 0), 10, 5, 1, m.level1, m.level2, m.equal)


@pytest.mark.slow
def test_parallel_equals_sequential_on_a_glass():
    """Accepted parallel trajectory == conventional AQS (Sec. 3.6, Sec. 4)."""
    s = S.uniform_glass_start(2, 256, 1, 0)
    pot = O.kob_andersen()
    fp = O.FireParams(dt0=0.005, dt_max=0.03, f_dec=0.9, alpha0=0.2, f_alpha=0.95, n_delay=5, f_inc=1.2)
    r0 = O.fire(s.pos, s.types, O.box_matrix(2, s.L, 0.0), pot, fp).pos
    dg, K, P, n = 2e-3, 4, 3, 24

    def step(x, k):
        return O.fire(O.affine(x, dg), s.types, O.strain_box(2, s.L, k, dg), pot, fp).pos

    seq = aqs_sequential((0, r0), n, lambda r, k: (k, step(r[1], k)))

    def level1(r_star, m):
        k, x = r_star
        return (k + m, O.affine(x, m * dg))

    def level2(anchors, lengths):
        out = []
        for (k, x), ln in zip(anchors, lengths):
            y = O.fire(x, s.types, O.strain_box(2, s.L, k, dg), pot, fp).pos
            first = (k, y)
            for j in range(1, ln + 1):
                y = step(y, k + j)
            out.append((first, (k + ln, y)))
        return out

    def equal(a, b):
        assert a[0] == b[0]
        return O.equal_configs(a[1], b[1], O.strain_box(2, s.L, a[0], dg))

    res = aqs_parallel((0, r0), n, K, P, level1, level2, equal)
    assert res.n_current == n and res.r_star[0] == n
    H = O.strain_box(2, s.L, n, dg)
    assert O.compare(res.r_star[1], seq[-1][1], H)[0] < 1e-6
    # the same with K chosen anew after every round
    dyn = aqs_parallel((0, r0), n, K, P, level1, level2, equal, lambda k, c: adaptive_k(k, c, 2, 8))
    assert dyn.n_current == n and len({r.K for r in dyn.rounds}) > 1
    assert O.compare(dyn.r_star[1], seq[-1][1], H)[0] < 1e-6
