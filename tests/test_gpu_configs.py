"""GPU against the oracle at the shapes the other parity files do not reach,
through the C ABI: the 2D glass of 4096 atoms (the size of the 2D batch and
of the learned-start workload: two force tiles per cell row), the paper's own
benchmark problem (Sec. 2.2: the potential of Eqs. 14-15, N = 400, shear
increment 1/200), a 3D step at N = 8192 compared position by position, and
the STALLED exits of both minimisers.

Inputs: oracle-quenched glasses (tests/data, tests/data/make_inputs.py).
Bars: energy 1e-10 relative, positions 1e-8 sigma (minimum image),
identical statuses, iteration counts and decisions, end states certified
max|F| < 1e-10 by the oracle's own forces."""
import numpy as np
import pytest

import oracle as O
from gpu_common import E_REL_TOL, FTOL, POS_TOL, fire_pair, load_glass
from oracle.alg1 import aqs_parallel

pytestmark = pytest.mark.gpu
KA = O.kob_andersen()


def _engine(dim, ns, L, dg, pot=None, **kw):
    from paper_2507_20802_amd import Engine
    return Engine(dim, ns, L, dg, pot=pot, **kw)


def _oracle_alg1(pos, types, L, dim, dg, K, P, n, ofire, pot, delta_eq=1e-4):
    """The oracle's Algorithm 1 (oracle/alg1.py) over oracle FIRE."""
    def level1(r_star, m):
        k, x = r_star
        return (k + m, O.affine(x, m * dg))

    def level2(starts, lengths):
        out = []
        for (k, x), ln in zip(starts, lengths):
            y = O.fire(x, types, O.strain_box(dim, L, k, dg), pot, ofire).pos
            first = (k, y)
            for j in range(1, ln + 1):
                y = O.fire(O.affine(y, dg), types, O.strain_box(dim, L, k + j, dg), pot, ofire).pos
            out.append((first, (k + ln, y)))
        return out

    def equal(a, b):
        return O.compare(a[1], b[1], O.strain_box(dim, L, a[0], dg))[0] < delta_eq

    return aqs_parallel((0, pos), n, K, P, level1, level2, equal)


def _step_parity(name, dg, pot, lj=None):
    pos, types, L, dim = load_glass(name)
    fire, ofire = fire_pair()
    H1 = O.strain_box(dim, L, 1, dg)
    ref = O.fire(O.affine(pos, dg), types, H1, pot, ofire)
    eng = _engine(dim, [len(types)], L, dg, pot=lj, fire=fire)
    eng.set_replica(0, types, pos, 0)
    eng.affine_shear([0], [1])
    rec = eng.minimize([0])[0, 0]
    got = eng.positions(0)
    print(f"{name}: iterations gpu {rec['iters']} oracle {ref.iters}, "
          f"distance {O.compare(got, ref.pos, H1)[0]:.2e}")
    assert rec["status"] == ref.status == O.CONVERGED
    assert abs(rec["energy"] - ref.E) <= E_REL_TOL * abs(ref.E)
    assert O.compare(got, ref.pos, H1)[0] <= POS_TOL
    assert O.max_force(got, types, H1, pot) < FTOL


def test_2d_4096_energy_forces_and_stress():
    pos, types, L, dim = load_glass("glass2d_4096")
    k, dg = 3, 1e-4
    x = O.affine(pos, k * dg)
    H = O.strain_box(dim, L, k, dg)
    eng = _engine(dim, [len(types)], L, dg)
    eng.set_replica(0, types, x, k)
    E, F = eng.energy_forces(0)
    Eo, Fo, So, _ = O.energy_forces(x, types, H, KA)
    assert abs(E - Eo) <= 1e-12 * abs(Eo)
    assert np.abs(F - Fo).max() <= 1e-11 * max(1.0, np.abs(Fo).max())
    sig, _ = eng.stress(0)
    assert np.allclose(sig, So, rtol=1e-10, atol=1e-12)


def test_2d_4096_one_aqs_step():
    _step_parity("glass2d_4096", 1e-4, KA)


@pytest.mark.parametrize("live", [False, True])
def test_2d_4096_algorithm1_round(live):
    """One round of Algorithm 1 (P = 2 chains of K = 2 steps at the 2D
    batch's increment 1e-4): the oracle's decision, accepted steps and r_star."""
    from paper_2507_20802_amd import parallel
    pos, types, L, dim = load_glass("glass2d_4096")
    fire, ofire = fire_pair()
    dg, K, P, n = 1e-4, 2, 2, 4
    ref = _oracle_alg1(pos, types, L, dim, dg, K, P, n, ofire, KA)
    eng = _engine(dim, [len(types)] * parallel.slots_needed(1, P), L, dg, fire=fire)
    g = parallel.layout(1, P)[0]
    eng.set_replica(g.star, types, pos, 0)
    out = parallel.run(eng, [g], n, K, P, delta_eq=1e-4, live=live, max_rounds=1)
    assert [r["checks"] for r in g.rounds] == [r.checks for r in ref.rounds[:1]]
    assert [r["q"] for r in g.rounds] == [r.q for r in ref.rounds[:1]]
    assert out["statuses_ok"]
    q = ref.rounds[0].q
    if q == n:   # the oracle's r_star after that round
        H = O.strain_box(dim, L, q, dg)
        assert O.compare(eng.positions(g.star), ref.r_star[1], H)[0] <= POS_TOL


def _paper():
    from paper_2507_20802_amd import speedup
    return speedup.paper_potential()


def test_paper_problem_one_step():
    """The paper's potential and sample (Eqs. 14-15, N = 400, rho = 1) and
    its strain increment 1/200."""
    _step_parity("paper2d_400", 1.0 / 200.0, O.paper_binary(), _paper())


@pytest.mark.parametrize("live", [False, True])
def test_paper_problem_algorithm1(live):
    """Algorithm 1 on the paper's problem (P = 3, K = 2, 12 steps): the
    oracle's decisions, accepted steps per round and final r_star."""
    from paper_2507_20802_amd import parallel
    pos, types, L, dim = load_glass("paper2d_400")
    fire, ofire = fire_pair()
    dg, K, P, n = 1.0 / 200.0, 2, 3, 12
    pot = O.paper_binary()
    ref = _oracle_alg1(pos, types, L, dim, dg, K, P, n, ofire, pot)
    eng = _engine(dim, [len(types)] * parallel.slots_needed(1, P), L, dg, pot=_paper(), fire=fire)
    g = parallel.layout(1, P)[0]
    eng.set_replica(g.star, types, pos, 0)
    out = parallel.run(eng, [g], n, K, P, delta_eq=1e-4, live=live)
    print("checks", [r["checks"] for r in g.rounds])
    assert [r["checks"] for r in g.rounds] == [r.checks for r in ref.rounds]
    assert [r["q"] for r in g.rounds] == [r.q for r in ref.rounds]
    assert out["accepted_steps"] == n and out["statuses_ok"]
    H = O.strain_box(dim, L, n, dg)
    got = eng.positions(g.star)
    assert O.compare(got, ref.r_star[1], H)[0] <= POS_TOL
    assert O.max_force(got, types, H, pot) < FTOL


def test_3d_8192_one_aqs_step():
    """3D, 8192 atoms at the benchmark's increment: positions compared atom by
    atom with the oracle's step."""
    _step_parity("glass3d_8192", 5e-5, KA)


def test_fire_stalled_like_the_oracle():
    """A glass relaxed from a perturbation of its inherent structure with a
    bound of one consecutive P <= 0 step: both stop STALLED at the same
    iteration, with the oracle's energy and positions."""
    pos, types, L, dim = load_glass("glass2d_256")
    import aqs_synth as S
    x = pos + S.rng_for(2507, 20802, 92).normal(0.0, 0.02, size=pos.shape)
    H = O.box_matrix(dim, L, 0.0)
    fire, ofire = fire_pair(n_neg_max=1)
    ref = O.fire(x, types, H, KA, ofire)
    eng = _engine(dim, [len(types)], L, 1e-4, fire=fire)
    eng.set_replica(0, types, x, 0)
    rec = eng.minimize([0])[0, 0]
    print(f"stalled at gpu {rec['iters']} oracle {ref.iters}")
    from paper_2507_20802_amd._lib import AQS_STALLED
    assert ref.status == O.STALLED and rec["status"] == AQS_STALLED
    assert rec["iters"] == ref.iters
    assert abs(rec["energy"] - ref.E) <= E_REL_TOL * abs(ref.E)
    assert O.compare(eng.positions(0), ref.pos, H)[0] <= POS_TOL


def test_cg_stalled_like_the_oracle():
    """Conjugate gradients whose line searches get one evaluation past the
    first trial (ls_max = 1) against a curvature condition no two trials meet
    (sigma = 1e-6): the first failed search with n_fail_max = 0 stops both
    at the same iteration."""
    from paper_2507_20802_amd import Cg
    from paper_2507_20802_amd._lib import AQS_STALLED
    pos, types, L, dim = load_glass("glass2d_256")
    fire, _ = fire_pair()
    dg = 1e-3
    cg = Cg(ls_max=1, n_fail_max=0, sigma=1e-6)
    ocg = O.CgParams(**{k: getattr(cg, k) for k in O.CgParams.__dataclass_fields__})
    H1 = O.strain_box(dim, L, 1, dg)
    ref = O.cg(O.affine(pos, dg), types, H1, KA, ocg)
    eng = _engine(dim, [len(types)], L, dg, fire=fire)
    eng.set_minimizer("cg", cg)
    eng.set_replica(0, types, pos, 0)
    eng.affine_shear([0], [1])
    rec = eng.minimize([0])[0, 0]
    print(f"stalled at gpu {rec['iters']} oracle {ref.iters}")
    assert ref.status == O.STALLED and rec["status"] == AQS_STALLED
    assert rec["iters"] == ref.iters
    assert abs(rec["energy"] - ref.E) <= E_REL_TOL * abs(ref.E)
    assert O.compare(eng.positions(0), ref.pos, H1)[0] <= POS_TOL
