"""The CU reservation policy of live rounds (parallel.reservation_for), CPU
only: unthrottled speculation after rounds whose checks mostly passed, a
tighter reservation after rounds whose checks mostly failed, the default
otherwise and without history."""
from paper_2507_20802_amd.parallel import reservation_for


def test_reservation_follows_the_last_rounds_checks():
    assert reservation_for([]) == 0
    assert reservation_for([True]) == -1
    assert reservation_for([True, True, True, False]) == -1
    assert reservation_for([True, False]) == 0
    assert reservation_for([True, False, False, False]) == 0
    assert reservation_for([False]) == 2
    assert reservation_for([True] + [False] * 4) == 2
