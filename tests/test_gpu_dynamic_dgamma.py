"""Dynamic step sizing on the GPU against the CPU oracle, through the C ABI
(aqs_set_dgamma): a new increment keeps every slot's strain exactly (box,
energy and forces bit for bit), refuses strains that are not a multiple of
it, and the next steps use it; and the dyadic run of Algorithm 1 takes the
oracle's levels, decisions and accepted steps round by round and ends on its
r_star, which is also conventional AQS at the finest increment."""
import numpy as np
import pytest

import oracle as O
from gpu_common import E_REL_TOL, FTOL, POS_TOL, certified_fmax, fire_pair, load_glass
from oracle.alg1 import aqs_parallel_dyadic, aqs_sequential

pytestmark = pytest.mark.gpu
POT = O.kob_andersen()


def test_new_increment_keeps_the_strain_exactly():
    from paper_2507_20802_amd import Engine
    from paper_2507_20802_amd._lib import AQSError
    pos, types, L, dim = load_glass("glass2d_256")
    eng = Engine(dim, [len(types)] * 3, L, 1e-3)
    for s in (0, 1, 2):
        eng.set_replica(s, types, pos, 0)
    eng.affine_shear([0, 1, 2], [5, 5, 6])
    H5, (E5, F5) = eng.box(0), eng.energy_forces(0)
    eng.set_dgamma([0], 5e-4)                  # finer: 5 -> 10
    assert eng.strain_index(0) == 10 and eng.dgamma[0] == 5e-4
    assert np.array_equal(eng.box(0), H5)
    E, F = eng.energy_forces(0)
    assert E == E5 and np.array_equal(F, F5)
    with pytest.raises(AQSError):              # 10 * 5e-4 is no multiple of 2e-3
        eng.set_dgamma([0], 2e-3)
    assert eng.strain_index(0) == 10 and np.array_equal(eng.box(0), H5)
    eng.set_dgamma([2], 2e-3)                  # coarser: 6 -> 3
    assert eng.strain_index(2) == 3
    assert np.array_equal(eng.box(2), O.strain_box(dim, L, 6, 1e-3))
    with pytest.raises(AQSError):              # slots at different increments
        eng.copy_replica(0, 1)
    eng.set_dgamma([0], 1e-3)                  # back: 10 -> 5
    assert eng.strain_index(0) == 5 and np.array_equal(eng.box(0), H5)
    eng.copy_replica(0, 1)
    eng.set_pure_shear([1], 1e-3)
    with pytest.raises(AQSError):              # a pure shear's box depends on the increment
        eng.set_dgamma([1], 5e-4)


def test_steps_after_a_new_increment_use_it():
    from paper_2507_20802_amd import Engine
    pos, types, L, dim = load_glass("glass2d_256")
    fire, ofire = fire_pair()
    dg = 2e-4
    eng = Engine(dim, [len(types)], L, dg, fire=fire)
    eng.set_replica(0, types, pos, 0)
    eng.affine_shear([0], [4])
    eng.minimize([0])
    x = O.fire(O.affine(pos, 4 * dg), types, O.strain_box(dim, L, 4, dg), POT, ofire).pos
    eng.set_dgamma([0], 4 * dg)                # level 2: fine index 4 is coarse index 1
    recs = eng.minimize([0], n_steps=[3])[0]
    for j in range(1, 4):
        k = 4 + 4 * j
        r = O.fire(O.affine(x, 4 * dg), types, O.strain_box(dim, L, k, dg), POT, ofire)
        x = r.pos
        assert recs[j]["status"] == r.status == 0
        assert abs(recs[j]["energy"] - r.E) <= E_REL_TOL * abs(r.E)
    assert eng.strain_index(0) == 4
    H = O.strain_box(dim, L, 16, dg)
    assert np.array_equal(eng.box(0), H)
    got = eng.positions(0)
    assert O.compare(got, x, H)[0] <= POS_TOL
    assert certified_fmax(got, types, H) < FTOL


_REF = {}


def oracle_dyadic(pos, types, L, dim, dg, n, K, P, m_max, ofire, delta_eq, event_tol):
    key = (dg, n, K, P, m_max, event_tol)
    if key in _REF:
        return _REF[key]

    def box(k):
        return O.strain_box(dim, L, k, dg)

    def step(x, k, h):
        return O.fire(O.affine(x, h * dg), types, box(k), POT, ofire).pos

    def level1(r, m, h):
        return (r[0] + m * h, O.affine(r[1], m * h * dg))

    def e_s(y, k):
        E, _, S_, _ = O.energy_forces(y, types, box(k), POT)
        return E, S_[0, 1]

    def level2(starts, lengths, h):
        out = []
        for (k, x), ln in zip(starts, lengths):
            y = O.fire(x, types, box(k), POT, ofire).pos
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
        return O.compare(a[1], b[1], box(a[0]))[0] < delta_eq

    ref = aqs_parallel_dyadic((0, pos), n, K, P, m_max, level1, level2, equal, v_dgamma=L ** dim * dg,
                              event_tol=event_tol)
    seq = aqs_sequential((0, pos), n, lambda r, k: (k, step(r[1], k, 1)))
    _REF[key] = (ref, seq[-1][1])
    return _REF[key]


@pytest.mark.parametrize("live,event_tol", [(False, 1e-2), (True, 1e-2), (False, None)])
def test_dyadic_run_matches_the_oracle(live, event_tol):
    from paper_2507_20802_amd import Engine, parallel
    pos, types, L, dim = load_glass("glass2d_256")
    fire, ofire = fire_pair()
    dg, n, K, P, m_max = 2e-4, 96, 4, 3, 2
    ref, seq_end = oracle_dyadic(pos, types, L, dim, dg, n, K, P, m_max, ofire, 1e-4, event_tol)
    eng = Engine(dim, [len(types)] * parallel.slots_needed(1, P), L, dg, fire=fire)
    g = parallel.layout(1, P)[0]
    eng.set_replica(g.star, types, pos, 0)
    out = parallel.run(eng, [g], n, K, P, delta_eq=1e-4, live=live, dynamic_dgamma=m_max,
                       event_tol=event_tol)
    got = [(r["start"], r["level"], r["lengths"], r["checks"], r["q"], r["cut"]) for r in g.rounds]
    want = [(r.start, r.level, r.lengths, r.checks, r.q, r.cut) for r in ref.rounds]
    print("levels", [r[1] for r in got], "cuts", [r[5] for r in got])
    assert got == want
    assert {r.level for r in ref.rounds} == {0, 1, 2} and any(r.cut for r in ref.rounds)
    assert out["accepted_steps"] == n and out["statuses_ok"]
    assert g.level == 0 and eng.dgamma[g.star] == dg and eng.strain_index(g.star) == n
    assert g.accepted_strain == sorted(set(g.accepted_strain)) and g.accepted_strain[-1] == n
    H = O.strain_box(dim, L, n, dg)
    x = eng.positions(g.star)
    assert O.compare(x, ref.r_star[1], H)[0] < 1e-8
    assert O.compare(x, seq_end, H)[0] < 1e-8
    assert certified_fmax(x, types, H) < FTOL
