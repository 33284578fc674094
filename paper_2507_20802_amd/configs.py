"""Throughput of the engine on the workloads beside the benchmark's
(3D, N = 32768, one round of P = 16 x K = 200, in bench.py):

* small   2D binary LJ glass, N = 256, 50 sequential AQS steps of 1e-4
          (one replica: launch-latency bound);
* batch2d four 2D N = 4096 glasses, each one round of Algorithm 1 with
          P = 8 chains of K = 100 steps of 1e-4 (level-I anchors 1e-2 apart),
          all 32 chains in one batched launch sequence;
* uneven  24 3D replicas, N log-uniform in [2048, 131072] and dgamma in
          {1e-5, 1e-4} (seeded), 100 sequential AQS steps each, all in one
          batch with graph-replayed iteration blocks and tuned knobs;
* paper   the paper's benchmark problem (Sec. 2.2: 2D, N = 400, Eqs. 14-15,
          dgamma = 1/200, 200 steps) for many samples at once: every sample's
          sequential AQS in one batch, against one sample alone;
* learned4 the learned start on 2D N = 4096 glasses: trained on 49 plain
          steps of one glass, evaluated on another (iterations, accepted
          starts, inherent-structure mismatches against the plain start).

Every glass is a seeded uniform random start quenched on the device (the
paper's samples are not available; the paper's problem uses its cell,
composition and potential); FIRE to max|F| < 1e-10.  Run as
python -m paper_2507_20802_amd.configs [small batch2d uneven paper]
[--paper-samples S --paper-steps K] (one JSON line each).  Times are wall-clock around the timed call, inputs resident on the
device.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import autotune, parallel
from .engine import Engine, Fire


def _sync():
    import torch
    torch.cuda.synchronize()


def _quenched(eng, slot, smp):
    eng.set_replica(slot, smp.types, smp.pos, 0)
    rec = eng.minimize([slot])[0, 0]
    if rec["status"] != 0:
        raise RuntimeError(f"quench of slot {slot} failed (status {rec['status']})")


def small(steps: int = 50, dgamma: float = 1e-4) -> dict:
    import aqs_synth as S
    smp = S.uniform_glass_start(2, 256, 1, 0)
    eng = Engine(2, [256], smp.L, dgamma, fire=Fire(), tuning="auto")
    _quenched(eng, 0, smp)
    is_pos = eng.positions(0)
    eng.minimize([0], n_steps=[3])                       # warm-up
    eng.set_replica(0, smp.types, is_pos, 0)
    _sync()
    t = time.perf_counter()
    rec = eng.minimize([0], n_steps=[steps])[0]
    _sync()
    dt = time.perf_counter() - t
    it = rec["iters"][1:]
    return {"config": "small", "workload": f"2D N=256, {steps} sequential AQS steps, dgamma={dgamma:g}",
            "aqs_steps_per_s": steps / dt, "wall_s": dt, "fire_iters_per_step": float(it.mean()),
            "us_per_iteration": 1e6 * dt / float(it.sum()), "all_converged": bool(np.all(rec["status"] == 0))}


def batch2d(glasses: int = 4, P: int = 8, K: int = 100, dgamma: float = 1e-4) -> dict:
    import aqs_synth as S
    n = 4096
    smps = [S.uniform_glass_start(2, n, 2, r) for r in range(glasses)]
    per = parallel.slots_needed(1, P)
    eng = Engine(2, [n] * (glasses * per), smps[0].L, dgamma, fire=Fire(), tuning="auto")
    gl = parallel.layout(glasses, P)
    pos = []
    for g, smp in zip(gl, smps):
        _quenched(eng, g.star, smp)
        pos.append(eng.positions(g.star))
    # warm-up round of short chains
    parallel.run(eng, gl, P * 5, 5, P, max_rounds=1)
    for g, smp, x in zip(gl, smps, pos):
        eng.set_replica(g.star, smp.types, x, 0)
    gl = parallel.layout(glasses, P)
    _sync()
    t = time.perf_counter()
    out = parallel.run(eng, gl, P * K, K, P, max_rounds=1)
    _sync()
    dt = time.perf_counter() - t
    return {"config": "batch2d", "workload": f"{glasses} x 2D N={n}, one round of P={P} x K={K}, "
            f"dgamma={dgamma:g}, dgamma_c={K * dgamma:g}, {glasses * P} chains batched",
            "accepted_steps_per_s": out["accepted_steps"] / dt, "computed_steps_per_s": out["computed_steps"] / dt,
            "wall_s": dt, "accepted": out["accepted_steps"], "computed": out["computed_steps"],
            "fire_iters_per_step": out["iters_mean"], "all_converged": out["statuses_ok"],
            "checks": [r["checks"] for g in gl for r in g.rounds]}


def uneven(steps: int = 100, reps: int = 24) -> dict:
    import aqs_synth as S
    rng = S.rng_for(5)
    ns = [int(round(np.exp(rng.uniform(np.log(2048), np.log(131072))))) for _ in range(reps)]
    dgs = [float(rng.choice([1e-5, 1e-4])) for _ in range(reps)]
    smps = [S.uniform_glass_start(3, n, 5, r) for r, n in enumerate(ns)]
    tn = autotune.tuned(3, ns, reps)
    tn.use_graph = 1
    eng = Engine(3, ns, np.array([[s.L] * 3 for s in smps]), dgs, fire=Fire(), tuning=tn)
    for r, s in enumerate(smps):
        eng.set_replica(r, s.types, s.pos, 0)
    q = eng.minimize(list(range(reps)))
    if np.any(q[:, 0]["status"] != 0):
        raise RuntimeError("quench failed")
    is_pos = [eng.positions(r) for r in range(reps)]
    eng.minimize(list(range(reps)), n_steps=[2] * reps)    # warm-up
    for r, s in enumerate(smps):
        eng.set_replica(r, s.types, is_pos[r], 0)
    _sync()
    t = time.perf_counter()
    rec = eng.minimize(list(range(reps)), n_steps=[steps] * reps)
    _sync()
    dt = time.perf_counter() - t
    it = rec["iters"][:, 1:]
    atoms = int(sum(ns))
    return {"config": "uneven", "workload": f"{reps} 3D replicas, N log-uniform in [2048, 131072] "
            f"({atoms} atoms), dgamma in {{1e-5, 1e-4}}, {steps} sequential AQS steps each",
            "aqs_steps_per_s": reps * steps / dt, "atom_steps_per_s": atoms * steps / dt, "wall_s": dt,
            "fire_iters_per_step": float(it.mean()), "all_converged": bool(np.all(rec["status"] == 0)),
            "n_atoms": ns, "dgamma": dgs}


def paper(samples: int = 256, steps: int = 200) -> dict:
    import aqs_synth as S
    from . import speedup as SP
    smps = [S.paper_sample_start(21, j) for j in range(samples)]
    n = smps[0].n
    eng = Engine(2, [n] * samples, smps[0].L, SP.DGAMMA, pot=SP.paper_potential(), fire=Fire())
    for j, smp in enumerate(smps):
        eng.set_replica(j, smp.types, smp.pos, 0)
    q = eng.minimize(list(range(samples)))
    if np.any(q[:, 0]["status"] != 0):
        raise RuntimeError("quench failed")
    is_pos = [eng.positions(j) for j in range(samples)]
    # one sample alone
    eng.set_replica(0, smps[0].types, is_pos[0], 0)
    _sync()
    t = time.perf_counter()
    r1 = eng.minimize([0], n_steps=[steps])[0]
    _sync()
    t_one = time.perf_counter() - t
    for j, smp in enumerate(smps):
        eng.set_replica(j, smp.types, is_pos[j], 0)
    _sync()
    t = time.perf_counter()
    rec = eng.minimize(list(range(samples)), n_steps=[steps] * samples)
    _sync()
    dt = time.perf_counter() - t
    same0 = bool(np.array_equal(rec[0]["energy"], r1["energy"]))
    return {"config": "paper", "workload": f"{samples} samples of the paper's 2D N={n} problem, "
            f"{steps} sequential AQS steps of dgamma={SP.DGAMMA:g} each, in one batch",
            "aqs_steps_per_s": samples * steps / dt, "wall_s": dt, "one_sample_wall_s": t_one,
            "one_sample_aqs_steps_per_s": steps / t_one, "gain_over_one_at_a_time": samples * t_one / dt,
            "fire_iters_per_step": float(rec["iters"][:, 1:].mean()),
            "all_converged": bool(np.all(rec["status"] == 0)), "sample0_same_as_alone": same0}


def learned4(train_steps: int = 49, eval_steps: int = 50, epochs: int = 50, dgamma: float = 1e-4) -> dict:
    """The learned start on 2D N = 4096 glasses: the network is trained on
    the GPU on train_steps plain AQS steps of one glass (49 x 4096 = 200 704
    samples), then a second glass runs eval_steps steps from its inherent
    structure with the plain, the learned and the extrapolated start (whole
    chains, timed), and step by step: from every inherent structure of the
    plain chain one learned step, compared with the plain step (Eq. 20)."""
    import aqs_synth as S
    import torch
    from . import learned
    from ._lib import AQS_START_EXTRAPOLATED, AQS_START_FALLBACK, AQS_START_LEARNED, AQS_START_PLAIN
    n = 4096
    tr, ev = S.uniform_glass_start(2, n, 4, 0), S.uniform_glass_start(2, n, 4, 1)
    eng = Engine(2, [n] * 3, tr.L, dgamma, fire=Fire(), tuning="auto")
    _quenched(eng, 0, tr)
    _sync()
    t = time.perf_counter()
    feat, tgt, _ = learned.collect_samples(eng, 0, 1, train_steps)
    orders = torch.from_numpy(S.epoch_orders(feat.shape[0], epochs, 4, 2)).cuda()
    model = learned.make_mlp(2, S.mlp_init(2, 4, 3))
    hist = learned.train(model, feat, tgt, orders, learned.TrainParams(batch=4096, epochs=epochs))
    _sync()
    t_train = time.perf_counter() - t
    eng.learned_load(model)
    _quenched(eng, 0, ev)
    x0 = eng.positions(0)
    chains = {}
    for name, mode in (("plain", AQS_START_PLAIN), ("learned", AQS_START_LEARNED),
                       ("extrapolated", AQS_START_EXTRAPOLATED)):
        eng.set_replica(0, ev.types, x0, 0)
        _sync()
        t = time.perf_counter()
        rec = eng.minimize([0], n_steps=[eval_steps], start=mode)[0]
        _sync()
        dt = time.perf_counter() - t
        st = rec["start"][1:]
        chains[name] = {"wall_s": dt, "aqs_steps_per_s": eval_steps / dt,
                        "fire_iters_per_step": float(rec["iters"][1:].mean()),
                        "predicted_starts_accepted": int(np.sum((st == AQS_START_LEARNED) |
                                                                (st == AQS_START_EXTRAPOLATED))),
                        "fallbacks": int(np.sum(st == AQS_START_FALLBACK)),
                        "all_converged": bool(np.all(rec["status"] == 0)),
                        "final": eng.positions(0)}
    # step by step from the plain chain's inherent structures
    eng.set_replica(0, ev.types, x0, 0)
    mism, accepted, dists, it_p, it_l = 0, 0, [], 0, 0
    for k in range(eval_steps):
        eng.copy_replica(0, 1)
        rp = eng.minimize([0], n_steps=[1])[0, 1]
        rl = eng.minimize([1], n_steps=[1], start=AQS_START_LEARNED)[0, 1]
        eq, md, _ = eng.compare(0, 1, 1e-4)
        mism += int(not eq)
        accepted += int(rl["start"] == AQS_START_LEARNED)
        dists.append(md)
        it_p += int(rp["iters"])
        it_l += int(rl["iters"])
    same = {}
    for name in ("learned", "extrapolated"):
        eng.set_replica(1, ev.types, chains[name].pop("final"), eval_steps)
        eng.set_replica(2, ev.types, chains["plain"]["final"], eval_steps)
        same[name] = bool(eng.compare(1, 2, 1e-4)[0])
    chains["plain"].pop("final")
    return {"config": "learned4", "workload": f"2D N={n}: network trained on {train_steps} plain AQS steps "
            f"({feat.shape[0]} samples, {epochs} epochs) of one glass, evaluated on {eval_steps} steps of "
            f"another, dgamma={dgamma:g}, FIRE to max|F|<1e-10",
            "train_s": t_train, "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
            "chains": chains, "final_is_equal_to_plain": same,
            "stepwise": {"steps": eval_steps, "learned_accepted": accepted, "is_mismatches": mism,
                         "fire_iters_plain": it_p, "fire_iters_learned": it_l,
                         "max_distance": float(max(dists))}}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("configs", nargs="*", default=["small", "batch2d", "uneven", "paper"])
    ap.add_argument("--paper-samples", type=int, default=256)
    ap.add_argument("--paper-steps", type=int, default=200)
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    runs = {"small": small, "batch2d": batch2d, "uneven": uneven,
            "paper": lambda: paper(args.paper_samples, args.paper_steps), "learned4": learned4}
    for name in args.configs:
        print(json.dumps(runs[name]()), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
