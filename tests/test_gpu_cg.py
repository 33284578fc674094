"""Conjugate gradients (the paper's own minimiser, Sec. 2.1) on the GPU
against the oracle's, through the C ABI.  Bars as for FIRE: relative energy
1e-10, positions 1e-8 sigma (minimum image), identical statuses, every
inherent structure certified max|F| < 1e-10 by the oracle's own forces;
Algorithm 1 with identical decisions.  Also: the iteration limit, list
rebuilds inside a minimisation, graph replay, and CG and FIRE on the GPU
reaching the same inherent structure (Eq. 20)."""
import numpy as np
import pytest

import oracle as O
from gpu_common import E_REL_TOL, FTOL, POS_TOL, certified_fmax, fire_pair, load_glass
from oracle.alg1 import aqs_parallel

pytestmark = pytest.mark.gpu
POT = O.kob_andersen()


def cg_pair(**kw):
    """The same conjugate-gradient constants for the engine and the oracle."""
    from paper_2507_20802_amd import Cg
    g = Cg(**kw)
    return g, O.CgParams(**{k: getattr(g, k) for k in O.CgParams.__dataclass_fields__})


def cg_engine(dim, ns, L, dg, cg=None, **kw):
    from paper_2507_20802_amd import Engine, Tuning
    eng = Engine(dim, ns, L, dg, tuning=kw.pop("tuning", None) or Tuning(), **kw)
    eng.set_minimizer("cg", cg or cg_pair()[0])
    return eng


@pytest.mark.parametrize("name,dg", [("glass2d_1000", 1e-4), ("glass3d_1500", 5e-5), ("glass2d_256", 1e-3)])
def test_one_aqs_step_parity(name, dg):
    pos, types, L, dim = load_glass(name)
    cg, ocg = cg_pair()
    H1 = O.strain_box(dim, L, 1, dg)
    ref = O.cg(O.affine(pos, dg), types, H1, POT, ocg)
    eng = cg_engine(dim, [len(types)], L, dg, cg)
    eng.set_replica(0, types, pos, 0)
    eng.affine_shear([0], [1])
    rec = eng.minimize([0])[0, 0]
    got = eng.positions(0)
    print(f"{name}: gpu {rec['iters']} oracle {ref.iters} CG iterations ({ref.dirs} directions)")
    assert rec["status"] == ref.status == O.CONVERGED
    assert abs(rec["energy"] - ref.E) <= E_REL_TOL * abs(ref.E)
    assert O.compare(got, ref.pos, H1)[0] <= POS_TOL
    assert certified_fmax(got, types, H1) < FTOL


def test_device_chain_matches_sequential_oracle():
    pos, types, L, dim = load_glass("glass2d_256")
    dg, nst = 1e-4, 8
    cg, ocg = cg_pair()
    eng = cg_engine(dim, [len(types)], L, dg, cg)
    eng.set_replica(0, types, pos, 0)
    recs = eng.minimize([0], n_steps=[nst])[0]
    x = pos
    for k in range(0, nst + 1):
        H = O.strain_box(dim, L, k, dg)
        r = O.cg(O.affine(x, dg) if k else x, types, H, POT, ocg)
        x = r.pos
        assert recs[k]["status"] == r.status == 0
        assert abs(recs[k]["energy"] - r.E) <= E_REL_TOL * abs(r.E)
    assert recs[0]["iters"] == 0
    H = O.strain_box(dim, L, nst, dg)
    got = eng.positions(0)
    assert O.compare(got, x, H)[0] <= POS_TOL
    assert certified_fmax(got, types, H) < FTOL


def test_maxiter_stops_like_the_oracle():
    pos, types, L, dim = load_glass("glass2d_256")
    cg, ocg = cg_pair(max_iter=7)
    H = O.strain_box(dim, L, 1, 1e-2)
    ref = O.cg(O.affine(pos, 1e-2), types, H, POT, ocg)
    eng = cg_engine(dim, [len(types)], L, 1e-2, cg)
    eng.set_replica(0, types, pos, 0)
    eng.affine_shear([0], [1])
    rec = eng.minimize([0])[0, 0]
    assert rec["status"] == ref.status == O.MAXITER and rec["iters"] == ref.iters == 7
    assert O.compare(eng.positions(0), ref.pos, H)[0] <= 1e-12


def test_rebuilds_during_minimisation_keep_parity():
    """A tiny skin forces neighbour-list rebuilds (which re-sort the atoms and
    their search directions and origin forces) inside the minimisation."""
    from paper_2507_20802_amd import Tuning
    pos, types, L, dim = load_glass("glass3d_1500")
    cg, ocg = cg_pair()
    dg = 2e-3
    H = O.strain_box(dim, L, 1, dg)
    ref = O.cg(O.affine(pos, dg), types, H, POT, ocg)
    eng = cg_engine(dim, [len(types)], L, dg, cg, tuning=Tuning(skin=0.002))
    eng.set_replica(0, types, pos, 0)
    eng.affine_shear([0], [1])
    rec = eng.minimize([0])[0, 0]
    assert eng.counters()["rebuilds"] > 3
    assert rec["status"] == ref.status == 0
    assert abs(rec["energy"] - ref.E) <= E_REL_TOL * abs(ref.E)
    assert O.compare(eng.positions(0), ref.pos, H)[0] <= POS_TOL


def test_graph_replay_and_uneven_batch():
    """Three slots of different size in one launch, with and without graph
    replay: bitwise the same records and positions; each slot equals its own
    oracle run."""
    from paper_2507_20802_amd import Tuning
    cg, ocg = cg_pair()
    names = ["glass2d_1000", "glass2d_256", "glass2d_1000b"]
    glasses = [load_glass(n) for n in names]
    dg = 2e-4
    out = []
    for use_graph in (0, 1):
        eng = cg_engine(2, [len(g[1]) for g in glasses], np.array([[g[2]] * 2 for g in glasses]), dg, cg,
                        tuning=Tuning(use_graph=use_graph, block_iters=16))
        for r, (pos, types, _, _) in enumerate(glasses):
            eng.set_replica(r, types, pos, 0)
        rec = eng.minimize([0, 1, 2], n_steps=[2, 2, 2])
        out.append((rec, [eng.positions(r) for r in range(3)]))
    (ra, pa), (rb, pb) = out
    assert np.array_equal(ra, rb) and all(np.array_equal(x, y) for x, y in zip(pa, pb))
    for r, (pos, types, L, dim) in enumerate(glasses):
        x = pos
        for k in (1, 2):
            x = O.cg(O.affine(x, dg), types, O.strain_box(dim, L, k, dg), POT, ocg).pos
        assert O.compare(pa[r], x, O.strain_box(dim, L, 2, dg))[0] <= POS_TOL


def test_cg_and_fire_reach_the_same_inherent_structures():
    """Both minimisers on the GPU, the same AQS steps: the same inherent
    structures (Eq. 20 at 1e-8 sigma) and energies."""
    pos, types, L, dim = load_glass("glass3d_1500")
    from paper_2507_20802_amd import Engine
    dg, nst = 5e-5, 4
    fire, _ = fire_pair()
    ends, recs = [], []
    for kind in ("fire", "cg"):
        eng = Engine(dim, [len(types)], L, dg, fire=fire)
        if kind == "cg":
            eng.set_minimizer("cg", cg_pair()[0])
        eng.set_replica(0, types, pos, 0)
        recs.append(eng.minimize([0], n_steps=[nst])[0])
        ends.append(eng.positions(0))
    H = O.strain_box(dim, L, nst, dg)
    assert O.compare(ends[0], ends[1], H)[0] < 1e-8
    assert np.all(recs[0]["status"] == 0) and np.all(recs[1]["status"] == 0)
    assert np.allclose(recs[0]["energy"], recs[1]["energy"], rtol=1e-12, atol=0)
    print("FIRE iterations", recs[0]["iters"][1:], "CG iterations", recs[1]["iters"][1:])


def test_bad_parameters_are_rejected():
    from paper_2507_20802_amd import Cg, Engine
    from paper_2507_20802_amd._lib import AQSError
    pos, types, L, dim = load_glass("glass2d_256")
    eng = Engine(dim, [len(types)], L, 1e-4)
    for bad in (Cg(sigma=0.0), Cg(sigma=1.0), Cg(grow=1.05), Cg(dmax=0.0), Cg(ls_max=0), Cg(a_init=-1.0)):
        with pytest.raises(AQSError):
            eng.set_minimizer("cg", bad)
    eng.set_minimizer("fire")


def oracle_run_cg(pos, types, L, dim, dg, K, P, n, ocg, delta_eq):
    def level1(r_star, m):
        k, x = r_star
        return (k + m, O.affine(x, m * dg))

    def level2(anchors, lengths):
        out = []
        for (k, x), ln in zip(anchors, lengths):
            y = O.cg(x, types, O.strain_box(dim, L, k, dg), POT, ocg).pos
            first = (k, y)
            for j in range(1, ln + 1):
                y = O.cg(O.affine(y, dg), types, O.strain_box(dim, L, k + j, dg), POT, ocg).pos
            out.append((first, (k + ln, y)))
        return out

    def equal(a, b):
        return O.compare(a[1], b[1], O.strain_box(dim, L, a[0], dg))[0] < delta_eq

    return aqs_parallel((0, pos), n, K, P, level1, level2, equal)


@pytest.mark.parametrize("live", [False, True])
def test_algorithm1_with_cg_matches_oracle(live):
    from paper_2507_20802_amd import parallel
    pos, types, L, dim = load_glass("glass2d_256")
    cg, ocg = cg_pair()
    dg, K, P, n, delta_eq = 4e-3, 5, 4, 20, 1e-4
    ref = oracle_run_cg(pos, types, L, dim, dg, K, P, n, ocg, delta_eq)
    eng = cg_engine(dim, [len(types)] * parallel.slots_needed(1, P), L, dg, cg)
    g = parallel.layout(1, P)[0]
    eng.set_replica(g.star, types, pos, 0)
    out = parallel.run(eng, [g], n, K, P, delta_eq=delta_eq, live=live)
    assert [r["checks"] for r in g.rounds] == [r.checks for r in ref.rounds]
    assert [r["q"] for r in g.rounds] == [r.q for r in ref.rounds]
    assert out["accepted_steps"] == n and out["statuses_ok"]
    H = O.strain_box(dim, L, n, dg)
    assert eng.strain_index(g.star) == n
    assert O.compare(eng.positions(g.star), ref.r_star[1], H)[0] < 1e-8


def test_full_size_cg_and_extrapolated_chains_are_certified():
    """The benchmark's replica size (3D, 32768 atoms), four slots: two AQS
    steps with conjugate gradients, and three with FIRE from the
    extrapolated start.  Every end state is certified by the oracle's own
    forces (max|F| < 1e-10) with the oracle's energy at those positions.
    (Whether the two minimisers' first inherent structures agree is only
    reported: these glasses rearrange at almost every step at this size.)"""
    import aqs_synth as S
    from paper_2507_20802_amd import AQS_START_EXTRAPOLATED, Engine
    n, dg = 32768, 5e-5
    s = S.uniform_glass_start(3, n, 3, 0)
    fire, _ = fire_pair()
    eng = Engine(3, [n] * 4, s.L, dg, fire=fire)
    eng.set_replica(0, s.types, s.pos, 0)
    assert eng.minimize([0])[0, 0]["status"] == 0
    for r in (1, 2, 3):
        eng.copy_replica(0, r)
    eng.set_minimizer("cg", cg_pair()[0])
    rc = eng.minimize([0, 1], n_steps=[2, 1])
    eng.set_minimizer("fire")
    rf = eng.minimize([2, 3], n_steps=[3, 1], start=AQS_START_EXTRAPOLATED)
    assert np.all(rc["status"][:, :2] == 0) and np.all(rf["status"][0] == 0) and np.all(rf["status"][1, :2] == 0)
    for r, k, E in ((0, 2, rc[0, 2]["energy"]), (2, 3, rf[0, 3]["energy"])):
        H = O.strain_box(3, s.L, k, dg)
        got = eng.positions(r)
        Eo, Fo, _, _ = O.energy_forces(got, s.types, H, POT)
        assert np.sqrt((Fo * Fo).sum(1)).max() < FTOL
        assert abs(E - Eo) <= E_REL_TOL * abs(Eo)
    # after one step: the CG slot 1 and the plain-started FIRE slot 3 (step 1
    # has no history, so it starts from F r)
    assert rf[1, 1]["start"] == 2
    eq, md, _ = eng.compare(1, 3, 1e-4)
    print("CG vs FIRE after one step: max displacement", md, "equal (Eq. 20):", bool(eq))
