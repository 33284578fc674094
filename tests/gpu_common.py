"""Helpers shared by the GPU tests: stored oracle-quenched glasses, the
engine/oracle parameter mapping and the parity measures."""
from __future__ import annotations

import os

import numpy as np

import oracle as O

DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")

# parity bars of the hot path (per call, from the same input state)
E_REL_TOL = 1e-10      # |E_gpu - E_oracle| / |E_oracle|
POS_TOL = 1e-8         # max minimum-image position difference (sigma_AA)
FTOL = 1e-10           # certified max |F_i| of an inherent structure


def load_glass(name: str):
    z = np.load(os.path.join(DATA, name + ".npz"))
    return z["pos"], z["types"], float(z["L"]), int(z["dim"])


def fire_pair(**kw):
    """The same FIRE constants for the engine and the oracle."""
    from paper_2507_20802_amd import Fire
    f = Fire(**kw)
    o = O.FireParams(**{k: getattr(f, k) for k in O.FireParams.__dataclass_fields__})
    return f, o


def certified_fmax(pos, types, H) -> float:
    return O.max_force(pos, types, H, O.kob_andersen())
