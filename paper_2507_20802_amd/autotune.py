"""Autotuner of the engine's launch knobs for a workload shape.

The knobs change how the work is laid out, never what is computed beyond
the rounding order of one atom's force sum: lanes per atom of the force
kernel (which also sets the force-tile length), the force tiles' fill of a
block, the force kernel's occupancy hint (waves per SIMD), the Verlet skin
(list length against rebuild frequency), the FIRE iterations launched
between state read-backs and their replay as a hipGraph; for live rounds of Algorithm 1 also the compute units left to the
critical chain (XCDs reserved for it, batch force blocks per CU).  Graph
replay is chosen twice: first on the batch, then, for shapes that hold live
rounds, on one replica alone -- the critical chain, which sets a live
round's time and runs bound by launch latency, so replay can pay there when
it does not in the batch.  For a
shape (dim, atoms per slot, slots) the tuner times short device chains of
AQS steps of a seeded glass on the GPU (coordinate descent from the
defaults), then, with enough slots for two chains and their snapshots,
short live rounds; it re-checks that the winner reaches the same inherent
structure as the defaults (and the live winner the same round, bit for
bit), and caches the result as JSON keyed by the shape bucket and the
device name.

Compile-time shapes are not knobs: the 256-thread block (four wavefronts)
is fixed by the force kernel's LDS halo (31 KB, five blocks per CU) and its
register budget; of the occupancy hint only the two instantiations built
(five and four waves per SIMD) are candidates.

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
    "tile_fill": (0.9, 0.7, 1.2),
    "use_graph": (0, 1),
    "force_waves": (5, 4),
}
DEFAULT = {k: v[0] for k, v in KNOBS.items()}
# knobs of live rounds only (aqs_run_round with live checks)
LIVE_KNOBS = {
    "live_xcds": (0, 2, 4),
    "live_batch_blocks": (0, -1, 2),
}
LIVE_DEFAULT = {k: v[0] for k, v in LIVE_KNOBS.items()}


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


def _live_trial(dim, n, n_rep, s, is_pos, knobs, dg, steps):
    """Wall time and outcome of one live round: P = (n_rep - 1) // 2 chains
    of `steps` fine steps from the inherent structure (level-I anchors
    steps * dg apart), checked and cancelled live."""
    import torch
    from . import parallel
    P = (n_rep - 1) // 2
    eng = Engine(dim, [n] * parallel.slots_needed(1, P), s.L, dg, fire=Fire(), tuning=tuning_of(knobs))
    g = parallel.layout(1, P)[0]
    eng.set_replica(g.star, s.types, is_pos, 0)
    for i in range(P):
        eng.copy_replica(g.star, g.chains[i])
    eng.affine_shear(g.chains[1:], [i * steps for i in range(1, P)])
    torch.cuda.synchronize()
    t = time.perf_counter()
    recs, checks = eng.run_round(g.chains, [-1] + g.snaps[1:], [steps] * P, live=True)
    torch.cuda.synchronize()
    return time.perf_counter() - t, (recs, checks)


def _same_round(a, b) -> bool:
    """Two live rounds of the same chains: the same decisions and bitwise the
    same records of every minimisation both finished."""
    from ._lib import AQS_CANCELLED
    (ra, ca), (rb, cb) = a, b
    if [c[:2] for c in ca] != [c[:2] for c in cb]:
        return False
    for x, y in zip(ra, rb):
        both = (x["status"] != AQS_CANCELLED) & (y["status"] != AQS_CANCELLED)
        if not np.array_equal(x[both], y[both]):
            return False
    return True


def tune(dim: int, n_atoms: int, n_rep: int, iters: int = 5000, repeats: int = 2, passes: int = 1,
         dg: float = 5e-5, seed: int = 11, cache: str | None = None, log=None,
         live_steps: int = 20, crit_steps: int = 10) -> dict:
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
    crit = None
    if n_rep >= 5:
        # the critical chain of a live round: one replica alone; graph replay
        # leaves every result bitwise unchanged, so only time decides
        crit = {}
        for g in KNOBS["use_graph"]:
            crit[g] = min(_trial(dim, n_atoms, 1, s, is_pos, dict(best, use_graph=g), iters, dg,
                                 steps=crit_steps) for _ in range(repeats))
            if log:
                log(f"critical chain use_graph={g}: {crit[g] * 1e3:.1f} ms")
        g = min(crit, key=crit.get)
        if g != best["use_graph"]:
            best = dict(best, use_graph=g)
            best_t = run(best)
    entry = {"knobs": best, "ms": best_t * 1e3, "default_ms": run(DEFAULT) * 1e3,
             "trials": len(timed), "max_iter": iters, "parity": check}
    if crit is not None:
        entry["critical_chain"] = {"steps": crit_steps,
                                   "ms_by_use_graph": {str(k): v * 1e3 for k, v in crit.items()}}
    if n_rep >= 5:
        # live rounds: the critical chain's share of the GPU, on top of the
        # batched winner
        live, ltimed, outcome = dict(LIVE_DEFAULT), {}, {}

        def run_live(kn):
            key = json.dumps(kn, sort_keys=True)
            if key not in ltimed:
                res = [_live_trial(dim, n_atoms, n_rep, s, is_pos, dict(best, **kn), dg, live_steps)
                       for _ in range(repeats)]
                ltimed[key] = min(r[0] for r in res)
                outcome[key] = res[0][1]
                if log:
                    log(f"live {kn}: {ltimed[key] * 1e3:.1f} ms")
            return ltimed[key]

        live_t = run_live(live)
        for name, values in LIVE_KNOBS.items():
            for v in values:
                kn = dict(live, **{name: v})
                t = run_live(kn)
                if t < live_t:
                    live, live_t = kn, t
        same = _same_round(outcome[json.dumps(live, sort_keys=True)],
                           outcome[json.dumps(LIVE_DEFAULT, sort_keys=True)])
        if not same:
            live, live_t = dict(LIVE_DEFAULT), run_live(LIVE_DEFAULT)
        entry["knobs"] = dict(best, **live)
        entry["live"] = {"ms": live_t * 1e3, "default_ms": run_live(LIVE_DEFAULT) * 1e3,
                         "trials": len(ltimed), "steps": live_steps, "same_round_as_default": bool(same)}
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


# shapes of the shipped tuning: the benchmark's batch (3D, 16 chains of 32768
# atoms with their snapshots and r_star), the 2D batch of four glasses, one
# small 2D replica, the uneven 3D batch (largest replica) and the paper's
# problem batched over samples
SHIPPED_SHAPES = ((3, 32768, 33), (3, 32768, 16), (2, 4096, 32), (2, 256, 1), (3, 131072, 24), (2, 400, 256))


def main(argv=None) -> int:
    """Tune shapes on the GPU and store them (default: the shipped shapes
    into the packaged file)."""
    import argparse
    import torch
    ap = argparse.ArgumentParser(description="tune the engine's knobs for workload shapes")
    ap.add_argument("--shape", action="append", default=[], metavar="DIM,N,SLOTS")
    ap.add_argument("--cache", default=PACKAGED)
    ap.add_argument("--repeats", type=int, default=2)
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    shapes = [tuple(int(v) for v in s.split(",")) for s in args.shape] or SHIPPED_SHAPES
    for dim, n, reps in shapes:
        entry = tune(dim, n, reps, repeats=args.repeats, cache=args.cache,
                     log=lambda m: print(f"[tune {dim}D n={n} x{reps}] {m}", flush=True))
        print(json.dumps({"shape": [dim, n, reps], **entry}), flush=True)
    return 0


if __name__ == "__main__":
    import sys
    sys.exit(main())
