"""Edge cases at the C ABI on the GPU: closed forms (a dimer relaxes to the
pair minimum 2^(1/6) sigma with the shifted pair energy of Eq. (13); a
perfect lattice, sheared or not, is at rest by inversion symmetry), an empty
selection, and the host checks' error codes on a live context, which keeps
working after them."""
import math

import numpy as np
import pytest

import oracle as O
from gpu_common import load_glass

pytestmark = pytest.mark.gpu

# shifted Lennard-Jones pair energy at its minimum r = 2^(1/6): -1 - U(2.5)
E_DIMER = -1.0 - 4.0 * (2.5 ** -12 - 2.5 ** -6)


@pytest.mark.parametrize("dim,r0", [(2, 1.3), (3, 1.02), (3, 1.9)])
def test_dimer_relaxes_to_the_pair_minimum(dim, r0):
    from paper_2507_20802_amd import Engine
    x = np.full((2, dim), 4.0)
    x[1, 0] += r0
    x[1, 1] += 0.25 * r0
    eng = Engine(dim, [2], 12.0, 1e-4)
    eng.set_replica(0, np.zeros(2, np.uint8), x, 0)
    rec = eng.minimize([0])[0, 0]
    y = eng.positions(0)
    r = float(np.linalg.norm(y[1] - y[0]))
    print(f"dim {dim} r0 {r0}: iters {rec['iters']} r - 2^(1/6) {r - 2 ** (1 / 6):.2e}")
    assert rec["status"] == 0 and rec["iters"] > 0 and rec["max_f"] < 1e-10
    assert abs(r - 2.0 ** (1.0 / 6.0)) < 1e-10
    assert abs(rec["energy"] - E_DIMER) < 1e-13
    # equal and opposite forces from rest: the centre of mass stays, and the
    # bond keeps its direction
    assert np.abs(y.mean(0) - x.mean(0)).max() < 1e-12
    d0 = (x[1] - x[0]) / np.linalg.norm(x[1] - x[0])
    assert np.abs((y[1] - y[0]) / r - d0).max() < 1e-12


def _triangular(nx, ny, a):
    pos = np.array([((i + 0.5 * (j % 2)) * a, j * a * math.sqrt(3) / 2) for j in range(ny) for i in range(nx)])
    return pos, np.array([nx * a, ny * a * math.sqrt(3) / 2])


def test_perfect_lattice_is_at_rest_sheared_or_not():
    """Every atom of a Bravais lattice is a centre of inversion, also after
    the affine shear of positions and box together: zero iterations, the
    oracle's energy, positions kept (up to the periodic images)."""
    from paper_2507_20802_amd import Engine
    pos, L = _triangular(8, 10, 1.08)
    n = len(pos)
    types = np.zeros(n, np.uint8)
    dg = 1e-2
    eng = Engine(2, [n], L[None, :], dg)
    eng.set_replica(0, types, pos, 0)
    for k in (0, 3):
        if k:
            eng.affine_shear([0], [k])
        x = eng.positions(0)
        rec = eng.minimize([0])[0, 0]
        H = O.box_matrix(2, list(L), k * dg)
        e_ref = O.energy_forces(x, types, H, O.kob_andersen())[0]
        assert rec["status"] == 0 and rec["iters"] == 0 and rec["max_f"] < 1e-11
        assert abs(rec["energy"] - e_ref) <= 1e-12 * abs(e_ref)
        # kept up to a lattice vector of the box (sheared atoms past x = Lx
        # come back wrapped)
        assert O.compare(eng.positions(0), x, H)[0] < 1e-12
    # the sheared lattice carries a shear stress (the box is strained)
    s, _ = eng.stress(0)
    assert abs(s[0, 1]) > 1e-3


def test_empty_selection_changes_nothing():
    from paper_2507_20802_amd import Engine
    pos, types, L, dim = load_glass("glass2d_256")
    eng = Engine(dim, [len(types)], L, 1e-4)
    eng.set_replica(0, types, pos, 0)
    rec = eng.minimize([])
    assert rec.shape[0] == 0
    assert np.array_equal(eng.positions(0), pos) or np.abs(eng.positions(0) - pos).max() < 1e-12
    assert eng.strain_index(0) == 0


def test_host_checks_reject_bad_calls_and_the_context_keeps_working():
    from paper_2507_20802_amd import Engine
    from paper_2507_20802_amd._lib import (AQS_ECAPACITY, AQS_EINVAL, AQS_ESTATE, AQS_START_LEARNED,
                                           AQSError)
    pos, types, L, dim = load_glass("glass2d_256")
    n = len(types)
    dg = 1e-3
    eng = Engine(dim, [n] * 3, L, dg)
    eng.set_replica(0, types, pos, 0)

    def code(fn, *a, **kw):
        with pytest.raises(AQSError) as e:
            fn(*a, **kw)
        print(e.value)
        return e.value.code

    assert code(eng.minimize, [1]) == AQS_ESTATE                       # slot 1 holds nothing
    assert code(eng.minimize, [3]) == AQS_EINVAL                       # no slot 3
    assert code(eng.minimize, [-1]) == AQS_EINVAL
    assert code(eng.minimize, [0, 0]) == AQS_EINVAL                    # selected twice
    assert code(eng.minimize, [0], n_steps=[1025]) == AQS_ECAPACITY     # default log holds 1024 steps
    assert code(eng.minimize, [0], n_steps=[-1]) == AQS_ECAPACITY
    assert code(eng.minimize, [0], start=7) == AQS_EINVAL
    assert code(eng.minimize, [0], start=AQS_START_LEARNED) == AQS_ESTATE   # no network loaded
    assert code(eng.minimize, [0], snap_dst=[5]) == AQS_EINVAL
    bad = types.copy()
    bad[5] = 2
    assert code(eng.set_replica, 1, bad, pos, 0) == AQS_EINVAL
    eng.set_replica(1, types, pos, 0)
    assert code(eng.minimize, [0, 1], snap_dst=[1, -1]) == AQS_EINVAL   # snapshot slot also minimised
    # a slot listed twice in one affine shear is refused and nothing moves
    before = [eng.positions(r) for r in (0, 1)]
    assert code(eng.affine_shear, [1, 1], [1, 1]) == AQS_EINVAL
    assert code(eng.affine_shear, [0, 1, 0], [2, 1, 3]) == AQS_EINVAL
    assert eng.strain_index(0) == 0 and eng.strain_index(1) == 0
    assert all(np.array_equal(eng.positions(r), b) for r, b in zip((0, 1), before))
    eng.affine_shear([1], [2])
    assert code(eng.compare, 0, 1) == AQS_EINVAL                       # different strain indices
    assert code(eng.copy_replica, 0, 5) == AQS_EINVAL
    assert code(eng.stress, 4) == AQS_EINVAL
    assert eng._lib.aqs_set_minimizer(eng._ctx, 7, None) == AQS_EINVAL
    # after all of that, slot 0 runs exactly as in a fresh context
    rec = eng.minimize([0], n_steps=[2])
    ref = Engine(dim, [n], L, dg)
    ref.set_replica(0, types, pos, 0)
    want = ref.minimize([0], n_steps=[2])
    assert np.array_equal(rec["iters"], want["iters"]) and np.array_equal(rec["energy"], want["energy"])
    assert np.array_equal(eng.positions(0), ref.positions(0))
    assert (rec["status"] == 0).all()
