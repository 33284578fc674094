"""Autotuner of the engine's launch knobs for a workload shape.

The knobs change how the work is laid out, never what is computed beyond
the rounding order of one atom's force sum: lanes per atom of the force
kernel (which also sets the force-tile length), the Verlet skin (list length
against rebuild frequency) and the FIRE iterations launched between state
read-backs.  For a shape (dim, atoms per slot, slots) the tuner times short
device chains of AQS steps of a seeded glass on the GPU (coordinate descent
from the defaults), re-checks that the winner reaches the same inherent structure
as the defaults, and caches the result as JSON keyed by the shape bucket and
the device name.

Everything it times runs in libaqs.so; this module only chooses arguments.
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import asdict

import numpy as np

from .engine import Engine, Fire, Tuning

KNOBS = {
    "threads_per_atom": (2, 1, 4),
    "skin": (0.3, 0.25, 0.35, 0.2, 0.15),
    "block_iters": (32, 16, 64),
}
DEFAULT = {k: v[0] for k, v in KNOBS.items()}


def bucket_key(dim: int, n_atoms: int, n_rep: int, device: str = "") -> str:
    """Shape bucket: dimension, atoms per slot to the nearest power of two,
    slots to the nearest power of two, device name."""
    nb = int(round(math.log2(max(int(n_atoms), 1))))
    rb = int(round(math.log2(max(int(n_rep), 1))))
    return f"d{int(dim)}_n2^{nb}_r2^{rb}_{device.replace(' ', '_')}"


def cache_path() -> str:
    return os.environ.get("AQS_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "aqs_mi355x", "tune.json"))


# results of tuning runs on MI355X shipped with the package; a user cache
# (cache_path()) takes precedence entry by entry
PACKAGED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_mi355x.json")


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def lookup(key: str, cache: str | None = None):
    entry = load_cache(cache).get(key)
    if entry is None and cache is None:
        entry = load_cache(PACKAGED).get(key)
    return entry


def save_cache(entries: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(entries, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuning_of(knobs: dict, base: Tuning | None = None) -> Tuning:
    t = Tuning(**asdict(base)) if base is not None else Tuning()
    for k, v in knobs.items():
        setattr(t, k, v)
    return t


def coordinate_order(start: dict | None = None):
    """Candidates of one coordinate-descent pass: each knob in turn over its
    values, the others at the current best (the caller updates the best)."""
    for name, values in KNOBS.items():
        yield name, values


def device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"


def _glass(dim: int, n: int, seed: int):
    import aqs_synth as S
    s = S.uniform_glass_start(dim, n, 3, seed)
    eng = Engine(dim, [n], s.L, 1e-4)
    eng.set_replica(0, s.types, s.pos, 0)
    rec = eng.minimize([0])[0, 0]
    if rec["status"] != 0:
        raise RuntimeError("the tuner's glass did not converge")
    return s, eng.positions(0)


def _trial(dim, n, n_rep, s, is_pos, knobs, iters, dg, steps=3):
    """Wall time of a short device chain of every copy: one shear increment
    dg from the inherent structure, minimised, then `steps` more AQS steps
    (the batched loop's tail, rebuilds and polls included); `iters` caps
    each minimisation."""
    import torch
    eng = Engine(dim, [n] * n_rep, s.L, dg, fire=Fire(max_iter=iters), tuning=tuning_of(knobs))
    for r in range(n_rep):
        eng.set_replica(r, s.types, is_pos, 0)
    eng.affine_shear(list(range(n_rep)), [1] * n_rep)
    torch.cuda.synchronize()
    t = time.perf_counter()
    eng.minimize(list(range(n_rep)), n_steps=[steps] * n_rep)
    torch.cuda.synchronize()
    return time.perf_counter() - t


def _same_inherent_structure(dim, n, s, is_pos, knobs, dg) -> dict:
    """One AQS step of the glass with the defaults and with `knobs`: energies
    within 1e-10 relative and positions within 1e-8 (minimum image)."""
    recs, pos = [], []
    for kn in (DEFAULT, knobs):
        eng = Engine(dim, [n, n], s.L, dg, tuning=tuning_of(kn))
        eng.set_replica(0, s.types, is_pos, 0)
        eng.affine_shear([0], [1])
        recs.append(eng.minimize([0])[0, 0])
        pos.append(eng.positions(0))
    eng.set_replica(1, s.types, pos[0], 1)          # the defaults' result beside the winner's
    _, d, _ = eng.compare(0, 1)
    rel = abs(recs[0]["energy"] - recs[1]["energy"]) / abs(recs[0]["energy"])
    ok = recs[0]["status"] == 0 and recs[1]["status"] == 0 and rel <= 1e-10 and d <= 1e-8
    return {"ok": bool(ok), "energy_rel": float(rel), "max_disp": float(d)}


def tune(dim: int, n_atoms: int, n_rep: int, iters: int = 5000, repeats: int = 2, passes: int = 1,
         dg: float = 5e-5, seed: int = 11, cache: str | None = None, log=None) -> dict:
    """Tune the knobs for the shape, store and return the cache entry."""
    s, is_pos = _glass(dim, n_atoms, seed)
    best = dict(DEFAULT)
    timed = {}

    def run(kn):
        key = json.dumps(kn, sort_keys=True)
        if key not in timed:
            timed[key] = min(_trial(dim, n_atoms, n_rep, s, is_pos, kn, iters, dg) for _ in range(repeats))
            if log:
                log(f"{kn}: {timed[key] * 1e3:.1f} ms")
        return timed[key]

    best_t = run(best)
    for _ in range(passes):
        for name, values in coordinate_order():
            for v in values:
                kn = dict(best, **{name: v})
                t = run(kn)
                if t < best_t:
                    best, best_t = kn, t
    check = _same_inherent_structure(dim, n_atoms, s, is_pos, best, dg)
    if not check["ok"]:
        best, best_t = dict(DEFAULT), run(DEFAULT)
    entry = {"knobs": best, "ms": best_t * 1e3, "default_ms": run(DEFAULT) * 1e3,
             "trials": len(timed), "max_iter": iters, "parity": check}
    key = bucket_key(dim, n_atoms, n_rep, device_name())
    entries = load_cache(cache)
    entries[key] = entry
    save_cache(entries, cache)
    return entry


def tuned(dim: int, n_atoms, n_rep: int, cache: str | None = None, run_if_missing: bool = False,
          log=None) -> Tuning:
    """The cached tuning of the shape (largest slot), the tuner's result if
    run_if_missing, else the defaults."""
    n = int(np.max(np.atleast_1d(n_atoms)))
    key = bucket_key(dim, n, n_rep, device_name())
    entry = lookup(key, cache)
    if entry is None and run_if_missing:
        entry = tune(dim, n, n_rep, cache=cache, log=log)
    return tuning_of(entry["knobs"]) if entry else Tuning()
