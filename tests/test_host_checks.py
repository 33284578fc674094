"""Host-side shape checks of the library, CPU only: aqs_workspace_bytes
(no device call) rejects shapes the kernels cannot take, with the reason in
aqs_last_error, and sizes the workspace of valid ones."""
import ctypes

import numpy as np
import pytest

from paper_2507_20802_amd import _lib
from paper_2507_20802_amd.engine import LJParams, Tuning


def _ws(dim, n_atoms, box):
    lib = _lib.load()
    pot = LJParams().to_c(dim)
    tn = Tuning().to_c()
    n = np.ascontiguousarray(n_atoms, dtype=np.int32)
    b = np.ascontiguousarray(box, dtype=np.float64).reshape(-1)
    nbytes = lib.aqs_workspace_bytes(ctypes.byref(pot), ctypes.byref(tn), int(n.size),
                                     n.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                     b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return int(nbytes), lib.aqs_last_error().decode()


@pytest.mark.parametrize("dim,n_atoms,box,reason", [
    (4, [100], [[12.0] * 4], "dim must be 2 or 3"),
    (3, [], [], "n_rep must be positive"),
    (3, [0], [[12.0] * 3], "bad atom count"),
    (3, [100, -5], [[12.0] * 3] * 2, "bad atom count"),
    (3, [100], [[8.0] * 3], "too small"),
    (2, [100], [[20.0, 8.0]], "too small"),
])
def test_bad_shapes_are_rejected_with_a_reason(dim, n_atoms, box, reason):
    nbytes, msg = _ws(dim, n_atoms, box)
    assert nbytes == 0 and reason in msg


def test_workspace_grows_with_the_slots():
    one, _ = _ws(3, [1000], [[12.0] * 3])
    two, _ = _ws(3, [1000, 1000], [[12.0] * 3] * 2)
    big, _ = _ws(3, [2000], [[12.0] * 3])
    assert 0 < one < two and one < big
    assert one % 256 == 0 and two % 256 == 0


def test_workspace_of_the_benchmark_shape():
    """33 slots of the 3D N = 32768 glass (sixteen chains, their snapshots and
    r_star): about 2.1 GB (the word and packed neighbour lists, 6 bytes per
    entry, are 1.25 GB of it; the compact halos of force tiles sized for the
    smallest tile fill, 0.36 GB), 0.7 % of the GPU's 288 GB."""
    L = (32768 / 1.2) ** (1.0 / 3.0)
    nbytes, _ = _ws(3, [32768] * 33, [[L] * 3] * 33)
    lists = 33 * 32768 * 192 * 6
    assert lists < nbytes < lists + 1.0e9
