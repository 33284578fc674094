"""Host policies of the Algorithm 1 driver, CPU only.  The CU reservation of
live rounds (parallel.reservation_for): unthrottled speculation after rounds
whose checks mostly passed, one batch block per CU after rounds whose
checks mostly failed and for the first round, the default otherwise.  The dynamic
choice of K (parallel.next_k): doubled after a round whose checks all
passed, halved (rounded up) after a failed first check, kept otherwise,
within its bounds.  The dynamic step sizing (parallel.next_level,
parallel.chain_events): level 0 after an event or short of the hold point,
else one level up, within m_max and the alignment of the strain index."""
import pytest

import numpy as np

from paper_2507_20802_amd.parallel import chain_events, next_k, next_level, reservation_for


def test_reservation_follows_the_last_rounds_checks():
    assert reservation_for([]) == 1
    assert reservation_for([True]) == -1
    assert reservation_for([True, True, True, False]) == -1
    assert reservation_for([True, False]) == 0
    assert reservation_for([True, False, False, False]) == 0
    assert reservation_for([False]) == 1
    assert reservation_for([True] + [False] * 4) == 1


@pytest.mark.parametrize("K,checks,bounds,want", [
    (4, [True, True], (1, 16), 8), (12, [True], (1, 16), 16), (5, [False], (1, 16), 3),
    (2, [False, True], (2, 16), 2), (1, [False], (1, 16), 1), (6, [True, False], (1, 16), 6),
    (6, [True, True, False], (1, 16), 6), (6, [], (1, 16), 6), (3, [True, True], (1, 4), 4)])
def test_next_k_follows_the_rounds_checks(K, checks, bounds, want):
    assert next_k(K, checks, *bounds) == want


def test_duty_follows_the_last_rounds_checks():
    """The speculative batch's duty cycle for the next live round: every block
    after a round where speculation paid, one in four after one where it did
    not, one in two in between, the first-round value before any round."""
    from paper_2507_20802_amd import parallel
    assert parallel.duty_for([]) == parallel.FIRST_ROUND_DUTY
    assert parallel.duty_for([True, True, True, False]) == 1
    assert parallel.duty_for([False] * 5) == 4
    assert parallel.duty_for([True, False]) == 2


@pytest.mark.parametrize("level,marked,n,hold,fine,m_max,want", [
    (0, False, 12, 0, 12, 2, 1), (1, False, 36, 0, 36, 2, 2), (2, False, 80, 0, 80, 2, 2),
    (2, False, 84, 0, 84, 3, 2), (2, False, 88, 0, 88, 3, 3), (1, False, 38, 0, 38, 2, 1),
    (0, False, 13, 0, 13, 2, 0), (2, True, 80, 0, 80, 2, 0), (0, False, 48, 52, 48, 2, 0),
    (0, False, 52, 52, 52, 2, 1), (0, False, 12, 0, 12, 0, 0), (0, False, 1012, 0, 1000, 3, 1)])
def test_next_level(level, marked, n, hold, fine, m_max, want):
    assert next_level(level, marked, n, hold, fine, m_max) == want


def test_chain_events_reads_only_the_chains_steps():
    assert not chain_events([0.1, 0.2, 0.3, 0.0], 2)     # entry 3 is past the chain
    assert chain_events([0.1, 0.2, 0.15, 0.3], 3)
    assert chain_events([0.3, 0.2], 1)                   # below the first minimisation
    assert not chain_events([0.2, 0.2, 0.25], 2)         # equal is no drop


def test_chain_events_energy_balance():
    # E(g) = e0 + V (s0 g + c g^2 / 2): s(g) = s0 + c g, and the trapezoid is
    # exact for a quadratic energy, so no step is marked
    V, s0, c, h = 400.0, 0.3, 12.0, 1e-3
    g = h * np.arange(6)
    s = s0 + c * g
    e = -1000.0 + V * (s0 * g + c * g * g / 2)
    assert not chain_events(s, 5, e, V * h, 1e-2)
    # release 2 % of step 3's work: marked at tol 1e-2, not at 5e-2
    e2 = e.copy()
    e2[3:] -= 0.02 * V * h * (s[2] + s[3]) / 2
    assert chain_events(s, 5, e2, V * h, 1e-2)
    assert not chain_events(s, 5, e2, V * h, 5e-2)
    assert not chain_events(s, 5, e2, V * h, None)
    assert not chain_events(s, 2, e2, V * h, 1e-2)       # the release is past the chain
