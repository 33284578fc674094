"""Algorithm 1 (Sec. 3.5) in the oracle: the paper's worked example, the
bounds of Sec. 3.7, the clamped last round, and parallel == sequential on a
real glass (CPU only)."""
import math
import os

import numpy as np
import pytest

import aqs_synth as S
import oracle as O
from oracle.alg1 import adaptive_k, aqs_parallel, aqs_parallel_dyadic, aqs_sequential, chain_plan, has_event

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


class DyadicMock:
    """Configurations are (fine strain index, basin) pairs; the shear stress
    rises by one per fine increment and falls by 1000 at every fine index in
    `events`; an anchor minimisation at a fine index in `wrong` lands in
    basin 1 (a misprediction), fine steps keep the basin."""

    def __init__(self, events=(), wrong=()):
        self.events, self.wrong = tuple(events), set(wrong)
        self.calls = []

    def stress(self, k):
        return k - 1000 * sum(e <= k for e in self.events)

    def level1(self, r, m, h):
        k, b = r
        return (k, b) if m == 0 else (k + m * h, "anchor")

    def level2(self, starts, lengths, h):
        out = []
        for (k, tag), ln in zip(starts, lengths):
            basin = (1 if k in self.wrong else 0) if tag == "anchor" else tag
            out.append(((k, basin), (k + ln * h, basin), [self.stress(k + j * h) for j in range(ln + 1)]))
        self.calls.append((h, list(lengths)))
        return out

    equal = staticmethod(Mock.equal)


def check_ladder(res, n, m_max, events):
    """Invariants of any dyadic run: rounds tile the strain from 0 to n, a
    level-m round starts on a multiple of 2^m and accepts whole increments,
    levels stay in [0, m_max], and every event is accepted in a level-0
    round (stepped through at the finest increment)."""
    assert res.n_current == n and res.r_star[0] == n
    at = 0
    for r in res.rounds:
        assert r.start == at and 0 <= r.level <= m_max
        assert r.start % (1 << r.level) == 0 and r.q % (1 << r.level) == 0
        at += r.q
    assert at == n
    for e in events:
        if e > n:
            continue
        (r,) = [r for r in res.rounds if r.start < e <= r.start + r.q]
        assert r.level == 0, (e, r)


@pytest.mark.parametrize("wrong", [(), (8,), (4, 8), (28, 56, 57, 80)])
def test_dyadic_without_levels_is_algorithm_1(wrong):
    # m_max = 0: every round at the finest increment, the rounds of the plain scheme
    n, K, P = 100, 4, 4
    m = DyadicMock(wrong=wrong)
    dy = aqs_parallel_dyadic((0, 0), n, K, P, 0, m.level1, m.level2, m.equal)
    plain = aqs_parallel((0, 0), n, K, P, lambda r, i: m.level1(r, i, 1),
                         lambda a, ln: [c[:2] for c in m.level2(a, ln, 1)], m.equal)
    assert [(r.start, r.lengths, r.checks, r.q) for r in dy.rounds] == \
        [(r.start, r.lengths, r.checks, r.q) for r in plain.rounds]
    assert all(r.level == 0 and not r.cut for r in dy.rounds)
    assert dy.r_star == plain.r_star and dy.computed_steps == plain.computed_steps


def test_dyadic_climbs_the_ladder_while_elastic():
    n, K, P, m_max = 400, 4, 3, 3
    m = DyadicMock()
    res = aqs_parallel_dyadic((0, 0), n, K, P, m_max, m.level1, m.level2, m.equal)
    check_ladder(res, n, m_max, ())
    lv = [r.level for r in res.rounds]
    assert lv[:4] == [0, 1, 2, 3] and set(lv[3:-2]) == {3}
    # worked by hand: 12 fine steps at level 0, 24 at level 1, then level 2
    # starts at 36 = 9 * 4 and trims its last chain to end at 80 = 10 * 8
    assert [(r.start, r.lengths, r.q) for r in res.rounds[:4]] == \
        [(0, [4, 4, 4], 12), (12, [4, 4, 4], 24), (36, [4, 4, 3], 44), (80, [4, 4, 4], 96)]
    assert res.computed_steps < n // 4


def test_dyadic_cuts_before_an_event_and_steps_through_it_finely():
    n, K, P, m_max = 200, 4, 3, 2
    m = DyadicMock(events=(50,))
    res = aqs_parallel_dyadic((0, 0), n, K, P, m_max, m.level1, m.level2, m.equal)
    check_ladder(res, n, m_max, (50,))
    # level 2 from fine 36: chains [36, 52], [52, 68], [68, 80]; the event at 50
    # lies in chain 0, so nothing is kept, and the level is 0 from 36 until the
    # strain has passed 52 (rounds to 48 and to 60, the second holding the
    # event, so one more level-0 round before level 1)
    cut = [r for r in res.rounds if r.cut]
    assert [(r.start, r.level, r.q) for r in cut] == [(36, 2, 0)]
    i = res.rounds.index(cut[0])
    assert [(r.start, r.level, r.q) for r in res.rounds[i + 1: i + 5]] == \
        [(36, 0, 12), (48, 0, 12), (60, 0, 12), (72, 1, 24)]


@pytest.mark.parametrize("seed", range(6))
def test_dyadic_invariants_under_random_events(seed):
    rng = np.random.default_rng(seed)
    n, K, P, m_max = 300, int(rng.integers(1, 6)), int(rng.integers(2, 6)), int(rng.integers(1, 4))
    events = sorted(rng.choice(np.arange(1, n + 1), size=6, replace=False).tolist())
    wrong = rng.choice(np.arange(1, n + 1), size=10, replace=False).tolist()
    m = DyadicMock(events=events, wrong=wrong)
    res = aqs_parallel_dyadic((0, 0), n, K, P, m_max, m.level1, m.level2, m.equal)
    check_ladder(res, n, m_max, events)
    for a, b in zip(res.rounds, res.rounds[1:]):
        if a.cut:
            assert b.level == 0 and a.level > 0


@pytest.mark.slow
def test_dyadic_equals_sequential_on_a_glass():
    """Through the elastic stretches the coarse steps reach the inherent
    structures of the fine ones, and every plastic event is stepped through
    at the fine increment: the dyadic run ends where conventional AQS does."""
    from gpu_common import fire_pair, load_glass
    pos, types, L, dim = load_glass("glass2d_256")
    fp = fire_pair()[1]
    pot = O.kob_andersen()
    dg, n, K, P, m_max = 2e-4, 96, 4, 3, 2

    def box(k):
        return O.strain_box(dim, L, k, dg)

    def step(x, k, h):   # to fine index k from k - h
        return O.fire(O.affine(x, h * dg), types, box(k), pot, fp).pos

    seq = aqs_sequential((0, pos), n, lambda r, k: (k, step(r[1], k, 1)))

    def level1(r, m, h):
        return (r[0] + m * h, O.affine(r[1], m * h * dg))

    def e_s(y, k):
        E, _, S_, _ = O.energy_forces(y, types, box(k), pot)
        return E, S_[0, 1]

    def level2(starts, lengths, h):
        out = []
        for (k, x), ln in zip(starts, lengths):
            y = O.fire(x, types, box(k), pot, fp).pos
            first = (k, y)
            en, st = [e_s(y, k)[0]], [e_s(y, k)[1]]
            for j in range(1, ln + 1):
                y = step(y, k + j * h, h)
                e, sg = e_s(y, k + j * h)
                en.append(e)
                st.append(sg)
            out.append((first, (k + ln * h, y), st, en))
        return out

    def equal(a, b):
        assert a[0] == b[0]
        return O.compare(a[1], b[1], box(a[0]))[0] < 1e-4

    drops = [k for k in range(1, n + 1) if e_s(seq[k][1], k)[1] < e_s(seq[k - 1][1], k - 1)[1]]
    assert drops                                         # the stretch holds plastic events
    for tol in (None, 1e-2):                             # stress drops alone; and the energy balance
        res = aqs_parallel_dyadic((0, pos), n, K, P, m_max, level1, level2, equal, v_dgamma=L * L * dg,
                                  event_tol=tol)
        check_ladder(res, n, m_max, drops)
        assert {r.level for r in res.rounds} == {0, 1, 2}
        assert any(r.cut for r in res.rounds)
        assert O.compare(res.r_star[1], seq[-1][1], box(n))[0] < 1e-8


def test_energy_balance_marks_released_energy():
    # E(g) = e0 + V (s0 g + c g^2 / 2), s = dE/dg / V: the trapezoid is exact
    # for a quadratic energy, so no step is marked; releasing 2 % of a step's
    # work marks it at tol 1e-2, not at 5e-2
    V, s0, c, h = 400.0, 0.3, 12.0, 1e-3
    g = h * np.arange(6)
    s = list(s0 + c * g)
    e = -1000.0 + V * (s0 * g + c * g * g / 2)
    assert not has_event(s, list(e), V * h, 1e-2)
    e2 = e.copy()
    e2[3:] -= 0.02 * V * h * (s[2] + s[3]) / 2
    assert has_event(s, list(e2), V * h, 1e-2)
    assert not has_event(s, list(e2), V * h, 5e-2)
    assert not has_event(s, list(e2), V * h, None)
    # on a real elastic stretch (the first fine steps of a glass) the balance
    # holds to far better than 1e-2 of the work
    from gpu_common import fire_pair, load_glass
    pos, types, L, dim = load_glass("glass2d_256")
    fp, pot, dg = fire_pair()[1], O.kob_andersen(), 1e-5
    x, en, st = pos, [], []
    for k in range(0, 6):
        H = O.strain_box(dim, L, k, dg)
        x = O.fire(O.affine(x, dg) if k else x, types, H, pot, fp).pos
        E, _, S_, _ = O.energy_forces(x, types, H, pot)
        en.append(E)
        st.append(S_[0, 1])
    assert all(b > a for a, b in zip(st, st[1:]))
    assert not has_event(st, en, L * L * dg, 1e-3)
