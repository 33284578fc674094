"""Algorithm 1 on the GPU vs the oracle's Algorithm 1 from the same glass:
identical accept/reject decisions, the same accepted steps per round, and
the final r_star equal (Eq. 20) to the oracle's."""
import numpy as np
import pytest

import oracle as O
from gpu_common import fire_pair, load_glass
from oracle.alg1 import adaptive_k, aqs_parallel

pytestmark = pytest.mark.gpu
POT = O.kob_andersen()


def oracle_run(pos, types, L, dim, dg, K, P, n, ofire, delta_eq, k_bounds=None):
    def step(x, k):
        return O.fire(O.affine(x, dg), types, O.strain_box(dim, L, k, dg), POT, ofire).pos

    def level1(r_star, m):
        k, x = r_star
        return (k + m, O.affine(x, m * dg))

    def level2(anchors, lengths):
        out = []
        for (k, x), ln in zip(anchors, lengths):
            y = O.fire(x, types, O.strain_box(dim, L, k, dg), POT, ofire).pos
            first = (k, y)
            for j in range(1, ln + 1):
                y = step(y, k + j)
            out.append((first, (k + ln, y)))
        return out

    margins = []

    def equal(a, b):
        d = O.compare(a[1], b[1], O.strain_box(dim, L, a[0], dg))[0]
        margins.append(d)
        return d < delta_eq

    rule = None if k_bounds is None else (lambda k, c: adaptive_k(k, c, *k_bounds))
    return aqs_parallel((0, pos), n, K, P, level1, level2, equal, rule), margins


@pytest.mark.parametrize("dg,K,P,n", [(4e-3, 5, 4, 20), (1e-3, 3, 3, 12)])
def test_gpu_algorithm1_matches_oracle(dg, K, P, n):
    from paper_2507_20802_amd import Engine, parallel
    pos, types, L, dim = load_glass("glass2d_256")
    fire, ofire = fire_pair()
    delta_eq = 1e-4
    ref, margins = oracle_run(pos, types, L, dim, dg, K, P, n, ofire, delta_eq)
    eng = Engine(dim, [len(types)] * parallel.slots_needed(1, P), L, dg, fire=fire)
    g = parallel.layout(1, P)[0]
    eng.set_replica(g.star, types, pos, 0)
    out = parallel.run(eng, [g], n, K, P, delta_eq=delta_eq)
    gpu_checks = [r["checks"] for r in g.rounds]
    ref_checks = [r.checks for r in ref.rounds]
    print("oracle margins", ["%.2e" % m for m in margins])
    print("gpu margins", ["%.2e" % d.max_disp for d in g.decisions])
    assert gpu_checks == ref_checks
    assert [r["q"] for r in g.rounds] == [r.q for r in ref.rounds]
    assert out["accepted_steps"] == n and out["statuses_ok"]
    H = O.strain_box(dim, L, n, dg)
    star = eng.positions(g.star)
    assert eng.strain_index(g.star) == n
    assert O.compare(star, ref.r_star[1], H)[0] < 1e-8
    # no decision falls in the ambiguous band: "equal" pairs are the same
    # minimum to within 1e-6 sigma, "not equal" pairs differ in energy too
    for d in g.decisions:
        if d.equal:
            assert d.max_disp < 1e-6
        else:
            assert abs(d.de_per_atom) > 1e-10


def test_two_glasses_in_one_batch_match_the_oracle():
    """Two systems (different shear increments) run Algorithm 1 together in
    one batched launch; each matches its own oracle run."""
    from paper_2507_20802_amd import Engine, parallel
    pos, types, L, dim = load_glass("glass2d_256")
    fire, ofire = fire_pair()
    K, P, n = 4, 3, 12
    dgs = [2e-3, 4e-3]
    per = parallel.slots_needed(1, P)
    eng = Engine(dim, [len(types)] * (2 * per), L, [dgs[0]] * per + [dgs[1]] * per, fire=fire)
    gl = parallel.layout(2, P)
    for g in gl:
        eng.set_replica(g.star, types, pos, 0)
    out = parallel.run(eng, gl, n, K, P, delta_eq=1e-4)
    assert out["statuses_ok"] and out["accepted_steps"] == 2 * n
    for g, dg in zip(gl, dgs):
        ref, _ = oracle_run(pos, types, L, dim, dg, K, P, n, ofire, 1e-4)
        assert [r["checks"] for r in g.rounds] == [r.checks for r in ref.rounds]
        H = O.strain_box(dim, L, n, dg)
        assert O.compare(eng.positions(g.star), ref.r_star[1], H)[0] < 1e-8


@pytest.mark.parametrize("dg,K,P,n", [(4e-3, 5, 4, 20), (1e-3, 3, 3, 12)])
def test_live_rounds_match_the_oracle(dg, K, P, n):
    """Algorithm 1 with live checks (checks as soon as their configurations
    exist, the critical chain on its own stream, rejected chains stopped):
    the oracle's decisions, accepted steps per round and final r_star."""
    from paper_2507_20802_amd import Engine, parallel
    pos, types, L, dim = load_glass("glass2d_256")
    fire, ofire = fire_pair()
    ref, _ = oracle_run(pos, types, L, dim, dg, K, P, n, ofire, 1e-4)
    eng = Engine(dim, [len(types)] * parallel.slots_needed(1, P), L, dg, fire=fire)
    g = parallel.layout(1, P)[0]
    eng.set_replica(g.star, types, pos, 0)
    out = parallel.run(eng, [g], n, K, P, delta_eq=1e-4, live=True)
    assert [r["checks"] for r in g.rounds] == [r.checks for r in ref.rounds]
    assert [r["q"] for r in g.rounds] == [r.q for r in ref.rounds]
    assert out["accepted_steps"] == n and out["statuses_ok"]
    H = O.strain_box(dim, L, n, dg)
    assert O.compare(eng.positions(g.star), ref.r_star[1], H)[0] < 1e-8


@pytest.mark.parametrize("live", [False, True])
def test_dynamic_k_matches_the_oracle(live):
    """K chosen anew after every round (halved, doubled and kept on this
    glass, the last round clamped): the oracle's K sequence, decisions and
    accepted steps per round, and its final r_star."""
    from paper_2507_20802_amd import Engine, parallel
    pos, types, L, dim = load_glass("glass2d_256")
    fire, ofire = fire_pair()
    dg, K, P, n, kb = 2e-3, 4, 3, 40, (2, 16)
    ref, _ = oracle_run(pos, types, L, dim, dg, K, P, n, ofire, 1e-4, kb)
    eng = Engine(dim, [len(types)] * parallel.slots_needed(1, P), L, dg, fire=fire)
    g = parallel.layout(1, P)[0]
    eng.set_replica(g.star, types, pos, 0)
    out = parallel.run(eng, [g], n, K, P, delta_eq=1e-4, live=live, dynamic_k=kb)
    print("K per round", [r["K"] for r in g.rounds], "checks", [r["checks"] for r in g.rounds])
    assert [r["K"] for r in g.rounds] == [r.K for r in ref.rounds]
    assert len({r.K for r in ref.rounds}) > 1
    assert [r["checks"] for r in g.rounds] == [r.checks for r in ref.rounds]
    assert [r["q"] for r in g.rounds] == [r.q for r in ref.rounds]
    assert out["accepted_steps"] == n and out["statuses_ok"]
    H = O.strain_box(dim, L, n, dg)
    assert eng.strain_index(g.star) == n
    assert O.compare(eng.positions(g.star), ref.r_star[1], H)[0] < 1e-8


def test_dynamic_k_per_glass_in_one_batch():
    """Two glasses (different shear increments) in one batch, each choosing
    its own K after every round: each matches its own oracle run."""
    from paper_2507_20802_amd import Engine, parallel
    pos, types, L, dim = load_glass("glass2d_256")
    fire, ofire = fire_pair()
    K, P, n, kb = 4, 3, 24, (2, 16)
    dgs = [2e-3, 4e-3]
    per = parallel.slots_needed(1, P)
    eng = Engine(dim, [len(types)] * (2 * per), L, [dgs[0]] * per + [dgs[1]] * per, fire=fire)
    gl = parallel.layout(2, P)
    for g in gl:
        eng.set_replica(g.star, types, pos, 0)
    out = parallel.run(eng, gl, n, K, P, delta_eq=1e-4, dynamic_k=kb)
    assert out["statuses_ok"] and out["accepted_steps"] == 2 * n
    for g, dg in zip(gl, dgs):
        ref, _ = oracle_run(pos, types, L, dim, dg, K, P, n, ofire, 1e-4, kb)
        print(f"dgamma {dg}: K per round", [r["K"] for r in g.rounds])
        assert [r["K"] for r in g.rounds] == [r.K for r in ref.rounds]
        assert [r["checks"] for r in g.rounds] == [r.checks for r in ref.rounds]
        H = O.strain_box(dim, L, n, dg)
        assert O.compare(eng.positions(g.star), ref.r_star[1], H)[0] < 1e-8


def _round(eng, g, P, K, dg_steps, delta_eq, live):
    """Level I from the glass in g.star, then one round through aqs_run_round."""
    for i in range(P):
        eng.copy_replica(g.star, g.chains[i])
    eng.affine_shear(g.chains[1:P], [i * K for i in range(1, P)])
    return eng.run_round(g.chains[:P], [-1] + g.snaps[1:P], [dg_steps] * P, delta_eq=delta_eq, live=live)


@pytest.mark.parametrize("delta_eq", [1e-4, 1e-300, 1e3])
def test_live_round_equals_batched_round(delta_eq):
    """The same round with and without live checks: identical decisions; every
    minimisation the live round finished has bitwise the batched round's
    record; after the first failed check the later chains read CANCELLED
    after their finished minimisations.  delta_eq 1e-300 fails every check
    (all chains after chain 0 are stopped); 1e3 passes every check (the
    critical chain moves through all chains)."""
    from paper_2507_20802_amd import Engine, parallel
    from paper_2507_20802_amd._lib import AQS_CANCELLED
    pos, types, L, dim = load_glass("glass2d_256")
    fire, _ = fire_pair()
    P, K, dg = 4, 6, 2e-3
    eng = Engine(dim, [len(types)] * parallel.slots_needed(1, P), L, dg, fire=fire)
    g = parallel.layout(1, P)[0]
    eng.set_replica(g.star, types, pos, 0)
    rb, cb = _round(eng, g, P, K, K, delta_eq, live=False)
    ends_b = [eng.positions(g.chains[i]) for i in range(P)]
    rl, cl = _round(eng, g, P, K, K, delta_eq, live=True)
    assert [c[:2] for c in cl] == [c[:2] for c in cb]
    decided = [c for c in cb[1:] if c[0]]
    fail = next((i for i, c in enumerate(cb[1:], 1) if c[0] and not c[1]), None)
    if delta_eq == 1e-300:
        assert fail == 1 and len(decided) == 1
    if delta_eq == 1e3:
        assert fail is None and len(decided) == P - 1
    for i in range(P):
        ran = rl[i]["status"] != AQS_CANCELLED
        assert np.array_equal(rl[i][ran], rb[i][ran])
        if fail is None or i < fail:
            assert ran.all()
            assert np.array_equal(eng.positions(g.chains[i]), ends_b[i])
        else:
            # a stopped chain: finished minimisations first, then cancelled ones
            k = int(ran.sum())
            assert not ran[k:].any()


def test_live_cu_reservation_changes_no_result():
    """The batch's force launches yield compute units to the critical chain
    during live rounds (live_batch_blocks), or the two take separate XCDs
    (live_xcds: only the launch tables change); with no limit, the default,
    the tightest limit and two partitions the decisions, every minimisation
    both runs finished and the ends of the chains that ran to completion are
    bitwise the same.  3D slots, so that the force launches fill the GPU."""
    from paper_2507_20802_amd import Engine, Tuning, parallel
    pos, types, L, dim = load_glass("glass3d_1500")
    fire, _ = fire_pair()
    P, K, dg = 4, 5, 1e-3
    out = []
    for blocks, xcds in ((-1, 0), (0, 0), (1, 0), (0, 2), (-1, 4)):
        eng = Engine(dim, [len(types)] * parallel.slots_needed(1, P), L, dg, fire=fire,
                     tuning=Tuning(live_batch_blocks=blocks, live_xcds=xcds))
        g = parallel.layout(1, P)[0]
        eng.set_replica(g.star, types, pos, 0)
        recs, checks = _round(eng, g, P, K, K, 1e-4, live=True)
        out.append((recs, [c[:2] for c in checks], [eng.positions(g.chains[i]) for i in range(P)]))
    from paper_2507_20802_amd._lib import AQS_CANCELLED
    r0, c0, e0 = out[0]
    for recs, checks, ends in out[1:]:
        assert checks == c0
        for i in range(P):
            # a stopped chain's last finished minimisation depends on timing
            both = (recs[i]["status"] != AQS_CANCELLED) & (r0[i]["status"] != AQS_CANCELLED)
            assert np.array_equal(recs[i][both], r0[i][both])
            if both.all():
                assert np.array_equal(ends[i], e0[i])


def test_adaptive_reservation_changes_no_result():
    """parallel.run with live checks, the CU reservation chosen per round from
    the last round's checks, and without: the same rounds and the same r_star
    bit for bit."""
    from paper_2507_20802_amd import Engine, parallel
    pos, types, L, dim = load_glass("glass2d_256")
    fire, _ = fire_pair()
    dg, K, P, n = 4e-3, 5, 4, 20
    res = []
    for adaptive in (True, False):
        eng = Engine(dim, [len(types)] * parallel.slots_needed(1, P), L, dg, fire=fire)
        g = parallel.layout(1, P)[0]
        eng.set_replica(g.star, types, pos, 0)
        out = parallel.run(eng, [g], n, K, P, live=True, adaptive_reservation=adaptive)
        res.append(([(r["checks"], r["q"]) for r in g.rounds], eng.positions(g.star), out["accepted_steps"]))
    assert res[0][0] == res[1][0] and res[0][2] == res[1][2] == n
    assert np.array_equal(res[0][1], res[1][1])


@pytest.mark.parametrize("dg,K", [(4e-3, 6), (1e-5, 3)])
def test_live_round_abandons_after_a_stress_drop(dg, K):
    """live = 2: a fine step of the critical chain whose inherent structure
    carries less shear stress than the step before stops the chains after it
    before their check (decided = 2).  The oracle's chain 0 from the same
    glass says whether such a drop happens (at dgamma = 4e-3 the stress falls
    at step 4, at 1e-5 it only grows); chain 0 is bitwise the batched
    round's; without a drop the round is the live = 1 round."""
    from paper_2507_20802_amd import Engine, parallel
    from paper_2507_20802_amd._lib import AQS_CANCELLED
    pos, types, L, dim = load_glass("glass2d_256")
    fire, ofire = fire_pair()
    x, sig = pos, []
    for k in range(K + 1):
        if k:
            x = O.fire(O.affine(x, dg), types, O.strain_box(dim, L, k, dg), POT, ofire).pos
        sig.append(O.energy_forces(x, types, O.strain_box(dim, L, k, dg), POT)[2][0, 1])
    drop = any(sig[s] < sig[s - 1] for s in range(1, K + 1))
    P = 4
    eng = Engine(dim, [len(types)] * parallel.slots_needed(1, P), L, dg, fire=fire)
    g = parallel.layout(1, P)[0]
    eng.set_replica(g.star, types, pos, 0)
    rb, cb = _round(eng, g, P, K, K, 1e-4, live=False)
    end0 = eng.positions(g.chains[0])
    assert drop == any(rb[0]["sigma_xy"][s] < rb[0]["sigma_xy"][s - 1] for s in range(1, K + 1))
    r1, c1 = _round(eng, g, P, K, K, 1e-4, live=True)
    for i in range(P):
        eng.copy_replica(g.star, g.chains[i])
    eng.affine_shear(g.chains[1:P], [i * K for i in range(1, P)])
    r2, c2 = eng.run_round(g.chains[:P], [-1] + g.snaps[1:P], [K] * P, delta_eq=1e-4, live=True,
                           abandon=True)
    print("oracle stress", ["%.4f" % v for v in sig], "checks", [c[:2] for c in c2])
    assert np.array_equal(r2[0], rb[0]) and np.array_equal(eng.positions(g.chains[0]), end0)
    if drop:
        assert c2[1][0] == 2 and not c2[1][1]
        assert all(c[0] == 0 for c in c2[2:])
        for i in range(1, P):
            ran = r2[i]["status"] != AQS_CANCELLED
            assert np.array_equal(r2[i][ran], rb[i][ran])
            assert not ran[int(ran.sum()):].any()
    else:
        assert [c[:2] for c in c2] == [c[:2] for c in c1]
        for i in range(P):
            ran = (r2[i]["status"] != AQS_CANCELLED) & (r1[i]["status"] != AQS_CANCELLED)
            assert np.array_equal(r2[i][ran], r1[i][ran])
