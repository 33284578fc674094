"""The linear-response start (Sec. 2.1, Eqs. 7-8: one Newton step from the
affine start, H u = f(F r), solved by conjugate gradients with Hessian-vector
products from central differences of the forces) on the GPU against the
oracle's solve with the same steps and parameters: the same start decisions
(linear response kept, or the affine start after a rejection or a first
non-positive curvature) at every fine step, energies within 1e-10 relative,
the final configuration within 1e-8 sigma, every inherent structure
certified; also with the solve stopped by its tolerance, and for two slots
solved in one batch."""
import numpy as np
import pytest

import oracle as O
from gpu_common import E_REL_TOL, FTOL, POS_TOL, certified_fmax, fire_pair, load_glass
from oracle.linear_response import linear_response_start

pytestmark = pytest.mark.gpu
POT = O.kob_andersen()


def oracle_chain(pos, types, L, dim, dg, nst, ofire, max_cg=50, tol=1e-3):
    out, x = [], pos
    for k in range(1, nst + 1):
        H = O.strain_box(dim, L, k, dg)
        start, iters, ok, _ = linear_response_start(O.affine(x, dg), types, H, POT, max_cg=max_cg, tol=tol)
        r = O.fire(start, types, H, POT, ofire)
        assert r.status == O.CONVERGED
        out.append((r.E, ok, iters, r.pos))
        x = r.pos
    return out


@pytest.mark.parametrize("name,dg,nst,tol", [("glass2d_256", 1e-4, 4, 1e-3), ("glass2d_1000", 1e-4, 3, 1e-3),
                                             ("glass3d_1500", 2e-5, 2, 1e-3), ("glass2d_256", 1e-4, 3, 0.3)])
def test_linear_response_chain_matches_the_oracle(name, dg, nst, tol):
    from paper_2507_20802_amd import AQS_START_FALLBACK, AQS_START_LINEAR, Engine
    pos, types, L, dim = load_glass(name)
    fire, ofire = fire_pair()
    ref = oracle_chain(pos, types, L, dim, dg, nst, ofire, tol=tol)
    eng = Engine(dim, [len(types), len(types)], L, dg, fire=fire)
    eng.set_linear_start(50, tol, 1e-5)
    eng.set_replica(0, types, pos, 0)
    eng.set_replica(1, types, pos, 0)
    eng.counters(reset=True)
    rec = eng.minimize([0, 1], n_steps=[nst, nst], start=AQS_START_LINEAR)
    evals = eng.counters()["atom_evals"]
    print(name, dg, tol, "oracle CG updates", [it for _, _, it, _ in ref], "kept", [bool(ok) for _, ok, _, _ in ref],
          "gpu FIRE iterations", rec[0]["iters"][1:])
    for r in range(2):
        recs = rec[r]
        for k in range(1, nst + 1):
            E, ok, _, _ = ref[k - 1]
            assert recs[k]["status"] == 0
            assert recs[k]["start"] == (AQS_START_LINEAR if ok else AQS_START_FALLBACK), (r, k)
            assert abs(recs[k]["energy"] - E) <= E_REL_TOL * abs(E)
        H = O.strain_box(dim, L, nst, dg)
        got = eng.positions(r)
        assert O.compare(got, ref[-1][3], H)[0] <= POS_TOL
        assert certified_fmax(got, types, H) < FTOL
    # the solve's evaluations are counted: at least f(x0) and one probe pair per update
    n = len(types)
    assert evals >= 2 * n * sum(1 + 2 * it for _, _, it, _ in ref)
    if tol >= 0.1:
        assert all(it < 50 for _, _, it, _ in ref)     # stopped by the tolerance


def test_linear_response_start_saves_fire_iterations():
    from paper_2507_20802_amd import AQS_START_LINEAR, AQS_START_PLAIN, Engine
    pos, types, L, dim = load_glass("glass2d_256")
    fire, _ = fire_pair()
    nst, dg = 6, 1e-5
    eng = Engine(dim, [len(types), len(types)], L, dg, fire=fire)
    for s in (0, 1):
        eng.set_replica(s, types, pos, 0)
    plain = eng.minimize([0], n_steps=[nst], start=AQS_START_PLAIN)[0]
    lin = eng.minimize([1], n_steps=[nst], start=AQS_START_LINEAR)[0]
    assert np.all(lin["start"][1:] == AQS_START_LINEAR)
    assert lin["iters"][1:].sum() < plain["iters"][1:].sum()
    H = O.strain_box(dim, L, nst, dg)
    assert O.compare(eng.positions(0), eng.positions(1), H)[0] < 1e-8


def test_linear_start_parameters_are_checked():
    from paper_2507_20802_amd import Engine
    from paper_2507_20802_amd._lib import AQSError
    pos, types, L, dim = load_glass("glass2d_256")
    eng = Engine(dim, [len(types)], L, 1e-4)
    for bad in [(0, 1e-3, 1e-5), (50, 0.0, 1e-5), (50, 1.0, 1e-5), (50, 1e-3, 0.0), (50, 1e-3, 0.5)]:
        with pytest.raises(AQSError):
            eng.set_linear_start(*bad)
    eng.set_linear_start(10, 1e-2, 1e-6)


@pytest.mark.parametrize("live", [False, True])
def test_algorithm1_with_the_linear_start_matches_the_oracle(live):
    """Algorithm 1 whose every fine step starts from the linear response
    (batched, and live: the critical chain's solves on its own stream beside
    the batch's): the oracle's decisions, q per round and final r_star."""
    from paper_2507_20802_amd import AQS_START_LINEAR, Engine, parallel
    from oracle.alg1 import aqs_parallel
    pos, types, L, dim = load_glass("glass2d_256")
    fire, ofire = fire_pair()
    dg, K, P, n = 1e-4, 4, 3, 12

    def box(k):
        return O.strain_box(dim, L, k, dg)

    def step(x, k):
        start = linear_response_start(O.affine(x, dg), types, box(k), POT)[0]
        return O.fire(start, types, box(k), POT, ofire).pos

    def level1(r, m):
        return (r[0] + m, O.affine(r[1], m * dg))

    def level2(anchors, lengths):
        out = []
        for (k, x), ln in zip(anchors, lengths):
            y = O.fire(x, types, box(k), POT, ofire).pos
            first = (k, y)
            for j in range(1, ln + 1):
                y = step(y, k + j)
            out.append((first, (k + ln, y)))
        return out

    def equal(a, b):
        return O.compare(a[1], b[1], box(a[0]))[0] < 1e-4

    ref = aqs_parallel((0, pos), n, K, P, level1, level2, equal)
    eng = Engine(dim, [len(types)] * parallel.slots_needed(1, P), L, dg, fire=fire)
    g = parallel.layout(1, P)[0]
    eng.set_replica(g.star, types, pos, 0)
    out = parallel.run(eng, [g], n, K, P, delta_eq=1e-4, start=AQS_START_LINEAR, live=live)
    assert [r["checks"] for r in g.rounds] == [r.checks for r in ref.rounds]
    assert [r["q"] for r in g.rounds] == [r.q for r in ref.rounds]
    assert out["accepted_steps"] == n and out["statuses_ok"]
    assert AQS_START_LINEAR in g.step_starts
    assert O.compare(eng.positions(g.star), ref.r_star[1], box(n))[0] < 1e-8


@pytest.mark.parametrize("kind", ["pure_shear", "cg"])
def test_linear_response_start_under_pure_shear_and_with_cg(kind):
    """The same solve for a pure-sheared slot (Eq. 17: the plain start and
    the list test of the general box) and under the conjugate-gradient
    minimiser: the oracle's start decisions, energies and end state."""
    from paper_2507_20802_amd import AQS_START_FALLBACK, AQS_START_LINEAR, Cg, Engine
    pos, types, L, dim = load_glass("glass2d_256")
    fire, ofire = fire_pair()
    dg, nst = 1e-4, 3
    dgy = 5e-5 if kind == "pure_shear" else 0.0
    cg = Cg()
    ocg = O.CgParams(**{k: getattr(cg, k) for k in O.CgParams.__dataclass_fields__})
    out, x = [], pos
    for k in range(1, nst + 1):
        H = O.strain_box(dim, L, k, dg, dgy)
        start, iters, ok, _ = linear_response_start(O.affine(x, dg, dgy), types, H, POT)
        r = O.cg(start, types, H, POT, ocg) if kind == "cg" else O.fire(start, types, H, POT, ofire)
        assert r.status == O.CONVERGED
        out.append((r.E, ok, r.pos))
        x = r.pos
    eng = Engine(dim, [len(types)], L, dg, fire=fire)
    if kind == "cg":
        eng.set_minimizer("cg", cg)
    else:
        eng.set_pure_shear([0], dgy)
    eng.set_replica(0, types, pos, 0)
    recs = eng.minimize([0], n_steps=[nst], start=AQS_START_LINEAR)[0]
    for k in range(1, nst + 1):
        E, ok, _ = out[k - 1]
        assert recs[k]["status"] == 0
        assert recs[k]["start"] == (AQS_START_LINEAR if ok else AQS_START_FALLBACK), k
        assert abs(recs[k]["energy"] - E) <= E_REL_TOL * abs(E)
    H = O.strain_box(dim, L, nst, dg, dgy)
    got = eng.positions(0)
    assert O.compare(got, out[-1][2], H)[0] <= POS_TOL
    assert certified_fmax(got, types, H) < FTOL
