"""The extrapolated start (the extrapolation the paper's conclusion, Sec. 5,
proposes: the last step's non-affine displacement predicts the next one) on
the GPU against the oracle's chain with the same rules: the same start
decisions (extrapolated or fallback) at every fine step, energies within
1e-10 relative, the final configuration within 1e-8 sigma, and every
inherent structure equal (Eq. 20) to the plain-start chain's."""
import numpy as np
import pytest

import oracle as O
from gpu_common import E_REL_TOL, FTOL, POS_TOL, certified_fmax, fire_pair, load_glass
from oracle import learned as Lr

pytestmark = pytest.mark.gpu
POT = O.kob_andersen()


def oracle_chain(pos, types, L, dim, dg, nst, minimise):
    """Fine steps 1..nst from the inherent structure pos; step 1 has no
    history and starts from F r.  Returns per step (E, start code, IS)."""
    out, prev, x = [], None, pos
    for k in range(1, nst + 1):
        H = O.strain_box(dim, L, k, dg)
        if prev is None:
            x0, which = O.affine(x, dg), Lr.FALLBACK
        else:
            uh = Lr.extrapolated_uhat(prev, x, O.strain_box(dim, L, k - 1, dg), dg)
            plain, start, ok = Lr.learned_start(x, uh, dg)
            x0, which = Lr.choose_start(plain, start, ok, types, H, POT, O.energy_forces)
        r = minimise(x0, types, H)
        assert r.status == O.CONVERGED
        out.append((r.E, which, r.pos))
        prev, x = x, r.pos
    return out


def _codes(which):
    from paper_2507_20802_amd import AQS_START_EXTRAPOLATED, AQS_START_FALLBACK
    return AQS_START_EXTRAPOLATED if which == Lr.LEARNED else AQS_START_FALLBACK


@pytest.mark.parametrize("name,dg,nst,kind", [("glass2d_256", 1e-5, 8, "fire"), ("glass3d_1500", 2e-5, 5, "fire"),
                                              ("glass2d_1000", 1e-5, 5, "cg")])
def test_extrapolated_chain_matches_the_oracle(name, dg, nst, kind):
    from paper_2507_20802_amd import AQS_START_EXTRAPOLATED, Cg, Engine
    pos, types, L, dim = load_glass(name)
    fire, ofire = fire_pair()
    cg = Cg()
    ocg = O.CgParams(**{k: getattr(cg, k) for k in O.CgParams.__dataclass_fields__})
    if kind == "fire":
        def minimise(x0, t, H):
            return O.fire(x0, t, H, POT, ofire)
    else:
        def minimise(x0, t, H):
            return O.cg(x0, t, H, POT, ocg)
    ref = oracle_chain(pos, types, L, dim, dg, nst, minimise)
    eng = Engine(dim, [len(types), len(types)], L, dg, fire=fire)
    if kind == "cg":
        eng.set_minimizer("cg", cg)
    eng.set_replica(0, types, pos, 0)
    eng.set_replica(1, types, pos, 0)
    rec = eng.minimize([0, 1], n_steps=[nst, nst], start=AQS_START_EXTRAPOLATED)
    for r in range(2):
        recs = rec[r]
        assert recs[0]["iters"] == 0 and recs[0]["status"] == 0
        for k in range(1, nst + 1):
            E, which, _ = ref[k - 1]
            assert recs[k]["status"] == 0
            assert recs[k]["start"] == _codes(which), (r, k)
            assert abs(recs[k]["energy"] - E) <= E_REL_TOL * abs(E)
        H = O.strain_box(dim, L, nst, dg)
        got = eng.positions(r)
        assert O.compare(got, ref[-1][2], H)[0] <= POS_TOL
        assert certified_fmax(got, types, H) < FTOL
    starts = [w for _, w, _ in ref]
    print(name, kind, "oracle starts", starts, "gpu iterations", rec[0]["iters"][1:])
    assert starts[0] == Lr.FALLBACK and Lr.LEARNED in starts[1:]


def test_extrapolated_start_saves_iterations_and_keeps_the_plain_chain():
    """The plain and the extrapolated chain side by side in one batch: the
    same inherent structure after every step (Eq. 20), fewer FIRE
    iterations for the extrapolated one."""
    from paper_2507_20802_amd import AQS_START_EXTRAPOLATED, AQS_START_PLAIN, Engine
    pos, types, L, dim = load_glass("glass2d_256")
    fire, _ = fire_pair()
    dg, nst = 1e-5, 10
    its, ends = {}, {}
    for mode in (AQS_START_PLAIN, AQS_START_EXTRAPOLATED):
        eng = Engine(dim, [len(types)], L, dg, fire=fire)
        eng.set_replica(0, types, pos, 0)
        rec = eng.minimize([0], n_steps=[nst], start=mode)[0]
        assert np.all(rec["status"] == 0)
        its[mode] = int(rec["iters"][1:].sum())
        ends[mode] = eng.positions(0)
    H = O.strain_box(dim, L, nst, dg)
    assert O.compare(ends[AQS_START_PLAIN], ends[AQS_START_EXTRAPOLATED], H)[0] < 1e-6
    print("FIRE iterations: plain", its[AQS_START_PLAIN], "extrapolated", its[AQS_START_EXTRAPOLATED])
    assert its[AQS_START_EXTRAPOLATED] < its[AQS_START_PLAIN]
