#!/usr/bin/env python3
"""Benchmark of the batched AQS hot path on one MI355X.

Workload (default): a 3D binary Lennard-Jones glass, N = 32768 atoms
(Kob-Andersen-type parameters, 80:20, density 1.2, cutoff 2.5 sigma_ab),
quenched on the GPU from seeded uniform random positions.  One "step" is
one round of Algorithm 1 (Sec. 3.5) with P = 16 level-II chains of K = 200
fine AQS steps at dgamma = 5e-5 (level-I anchors at i * 1e-2), every
minimisation run by FIRE to max|F| < 1e-10, all chains batched on the GPU.
Each step starts from the same inherent structure (already in HBM); the
accepted steps of a round are q of Algorithm 1 (at least K), the computed
ones P * K plus the anchor minimisations.

Prints one JSON line: accepted AQS steps/s (value), FIRE iterations per AQS
step, the roofline of the dominant kernel (the FP64 force kernel, timed with
HIP events on its stream inside the timed region) and the CPU oracle timed
on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "AQS steps/s & FIRE iters/step at N=32k, learned-start vs plain, max|F|<1e-10"
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector
HBM_PEAK_GBS = 8000.0
# algorithmic FP64 work of one in-cutoff pair, counted once (Newton's third
# law): the separation and r^2, the reciprocal, the LJ powers, U'(r)/r, the
# shifted energy and the force components
FLOPS_PER_PAIR = 29
# algorithmic bytes per atom of the force kernel: positions (d doubles) and
# the type (one byte) in, velocities in for F.v and forces out (d doubles
# each): 24 d + 1
FORCE_BYTES_PER_ATOM = {2: 49, 3: 73}


TRAFFIC_SOURCES = ("md_kernels.hip", "cells.hip", "tiles.h", "engine.h")


def kernel_sources_sha256() -> str:
    """Hash of the sources that decide the force kernel's memory traffic."""
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2507_20802_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def force_traffic(dim: int, atoms_per_launch: float):
    """HBM bytes per force launch from the committed FETCH_SIZE / WRITE_SIZE
    counter summary (bytes per atom, copy-calibrated), or None when there is
    none or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"k_force_{dim}d_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic_json:"):
                t = json.loads(line.split(":", 1)[1])
                if t.get("sources_sha256") != kernel_sources_sha256():
                    return None
                return (t["fetch_bytes_per_atom"] + t["write_bytes_per_atom"]) * atoms_per_launch
    return None


def in_cutoff_neighbours(pos, types, L, pot) -> float:
    """Mean number of neighbours within rc_ab (directed pairs per atom) of
    an orthogonal periodic box, counted with a k-d tree (host tooling)."""
    from scipy.spatial import cKDTree
    n, dim = pos.shape
    x = np.mod(pos, L)
    tree = cKDTree(x, boxsize=L)
    rcm = pot.rc_factor * max(max(r) for r in pot.sigma)
    pairs = tree.query_pairs(rcm, output_type="ndarray")
    d = x[pairs[:, 0]] - x[pairs[:, 1]]
    d -= L * np.round(d / L)
    r = np.sqrt((d * d).sum(1))
    sig = np.asarray(pot.sigma)[types[pairs[:, 0]], types[pairs[:, 1]]]
    inside = r < pot.rc_factor * sig
    return 2.0 * inside.sum() / n


def cpu_baseline(dim, n, dg, iters_per_step, seconds=20.0):
    """Time the CPU oracle (sequential AQS, O(N^2) pair sums, all host
    threads) on a bounded sample: a few force evaluations of the same
    workload size; AQS steps/s = 1 / (t_eval * (iterations per step + 1))."""
    import oracle as O
    import aqs_synth as S
    s = S.jittered_lattice_start(dim, round(n ** (1 / dim)), 3, 9) if round(n ** (1 / dim)) ** dim == n \
        else S.uniform_glass_start(dim, n, 3, 9)
    H = O.strain_box(dim, s.L, 1, dg)
    x = O.affine(s.pos, dg)
    pot = O.kob_andersen()
    O.energy_forces(x[:64], s.types[:64], O.box_matrix(dim, 50.0, 0.0), pot)  # load
    t0 = time.perf_counter()
    evals = 0
    while True:
        O.energy_forces(x, s.types, H, pot)
        evals += 1
        if time.perf_counter() - t0 > seconds / 2 or evals >= 50:
            break
    t_eval = (time.perf_counter() - t0) / evals
    rate = 1.0 / (t_eval * (iters_per_step + 1.0))
    return {"value": rate, "unit": "AQS steps/s", "cores": O.get_threads(), "kind": "oracle",
            "sample": f"{evals} O(N^2) force evaluations of the N={n} {dim}D workload "
                      f"({t_eval:.3f} s each) x (GPU-measured {iters_per_step:.1f} FIRE iterations + 1) "
                      f"per sequential AQS step",
            "t_eval_s": t_eval}


def copy_calibration(mib: int) -> int:
    """Plain streaming kernels of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters: three device copies and three negations of MIB MiB
    (each reads and writes MIB MiB)."""
    import torch
    torch.cuda.set_device(0)
    n = mib * (1 << 20) // 8
    src = torch.rand(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 8, "bytes_written": n * 8}), flush=True)
    return 0


def train_network(eng, dim, n, dg, slot_a, slot_b, steps, epochs, seed):
    """Learned start: descriptors and non-affine targets from `steps` plain
    AQS steps of a separately seeded glass, then the network trained on the
    GPU (Adam, Huber loss, batch 4096).  Returns the model and a summary."""
    import torch
    import aqs_synth as S
    from paper_2507_20802_amd import learned
    s = S.uniform_glass_start(dim, n, 3, seed)
    eng.set_replica(slot_a, s.types, s.pos, 0)
    t0 = time.perf_counter()
    q = eng.minimize([slot_a])[0, 0]
    if q["status"] != 0:
        raise RuntimeError("quench of the training glass failed")
    feat, tgt, recs = learned.collect_samples(eng, slot_a, slot_b, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    orders = torch.from_numpy(S.epoch_orders(feat.shape[0], epochs, 3, seed, 7)).cuda()
    model = learned.make_mlp(dim, S.mlp_init(dim, 3, seed, 8))
    hist = learned.train(model, feat, tgt, orders, learned.TrainParams(batch=4096, epochs=epochs))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return model, {"samples": int(feat.shape[0]), "plain_steps": steps, "epochs": epochs,
                   "data_s": t1 - t0, "train_s": t2 - t1, "loss_first": float(hist[0]),
                   "loss_last": float(hist[-1])}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dim", type=int, default=3)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--P", type=int, default=16)
    ap.add_argument("--K", type=int, default=200)
    ap.add_argument("--dgamma", type=float, default=5e-5)
    ap.add_argument("--warmup-K", type=int, default=20, help="fine steps per chain in warmup rounds")
    ap.add_argument("--profile-every", type=int, default=4)
    ap.add_argument("--train-steps", type=int, default=7, help="plain AQS steps of training data")
    ap.add_argument("--epochs", type=int, default=50)
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-start reference rounds")
    ap.add_argument("--only-plain", action="store_true", help="time the plain start only (no network)")
    ap.add_argument("--skin", type=float, default=0.3, help="Verlet skin (sigma_AA)")
    ap.add_argument("--graph", type=int, default=0, help="replay iteration blocks as hipGraphs (1/0)")
    ap.add_argument("--live", type=int, default=1,
                    help="live checks (1/0): checks as soon as possible, the critical chain on a stream of "
                         "its own, rejected chains stopped; the learned form is also timed without them")
    ap.add_argument("--tuning", choices=("default", "auto", "autotune"), default="auto",
                    help="launch knobs: the defaults, the autotuner's cache, or tune when not cached")
    ap.add_argument("--extrap", type=int, default=1,
                    help="also time the extrapolated start (previous step's non-affine displacement) (1/0)")
    ap.add_argument("--cg", type=int, default=1,
                    help="also time the plain start with the conjugate-gradient minimiser (1/0)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only stream MIB MiB device-to-device (counter calibration) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported by this build "
              f"(the multi-GPU sharding is design only).", file=sys.stderr)
        return 2

    import torch
    import aqs_synth as S
    from paper_2507_20802_amd import (AQS_START_EXTRAPOLATED, AQS_START_LEARNED, AQS_START_PLAIN, Cg, Engine,
                                      Fire, LJParams, Tuning, parallel)

    torch.cuda.set_device(0)
    dim, n, P, K, dg = args.dim, args.n, args.P, args.K, args.dgamma
    pot = LJParams()
    s = S.uniform_glass_start(dim, n, 3, 0)
    nslots = parallel.slots_needed(1, P)
    ref_slot = nslots              # final r_star of the plain round, for the IS comparison
    tuning = Tuning(skin=args.skin, use_graph=args.graph) if args.tuning == "default" else args.tuning
    eng = Engine(dim, [n] * (nslots + 1), s.L, dg, pot=pot, fire=Fire(), tuning=tuning)
    glass = parallel.layout(1, P)[0]
    t0 = time.perf_counter()
    eng.set_replica(glass.star, s.types, s.pos, 0)
    q = eng.minimize([glass.star])[0, 0]
    quench_s = time.perf_counter() - t0
    if q["status"] != 0:
        print(f"quench failed: status {q['status']}", file=sys.stderr)
        return 1
    is_pos = eng.positions(glass.star)
    nb = in_cutoff_neighbours(is_pos, s.types, s.L, pot)
    train_info = None
    if not args.only_plain:
        model, train_info = train_network(eng, dim, n, dg, glass.chains[0], glass.chains[1],
                                          args.train_steps, args.epochs, 1)
        eng.learned_load(model)

    def one_round(Kr, start, live):
        eng.set_replica(glass.star, s.types, is_pos, 0)
        g = parallel.layout(1, P)[0]
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = parallel.run(eng, [g], P * Kr, Kr, P, start=start, max_rounds=1, live=live)
        torch.cuda.synchronize()
        return time.perf_counter() - t, out, g

    live = bool(args.live)
    forms = ([] if args.no_plain else [("plain", AQS_START_PLAIN, live, "fire")]) + \
        ([] if args.only_plain else [("learned", AQS_START_LEARNED, live, "fire")])
    # the extrapolated start and the paper's own minimiser on the same round
    if args.extrap and not args.no_plain:
        forms.append(("extrapolated", AQS_START_EXTRAPOLATED, live, "fire"))
    if args.cg and not args.no_plain:
        forms.append(("cg", AQS_START_PLAIN, live, "cg"))
    # the batched round without live checks, timed last: the force-kernel
    # roofline is taken there (one stream, every chain in each launch)
    main_form = "plain" if args.only_plain else "learned"
    roof_form = main_form + "_batched" if live else main_form
    if live:
        forms.append((roof_form, AQS_START_PLAIN if args.only_plain else AQS_START_LEARNED, False, "fire"))
    for _ in range(args.warmup):
        for _, st, lv, mz in forms:
            eng.set_minimizer(mz, Cg() if mz == "cg" else None)
            one_round(args.warmup_K, st, lv)
    res_forms = {}
    for name, st, lv, mz in forms:
        eng.set_minimizer(mz, Cg() if mz == "cg" else None)
        eng.counters(reset=True)
        eng.set_profiling(args.profile_every)
        tot_t, acc, comp, iters, ok, rounds, starts = 0.0, 0, 0, [], True, [], []
        for _ in range(args.steps):
            dt, out, g = one_round(K, st, lv)
            tot_t += dt
            acc += out["accepted_steps"]
            comp += out["computed_steps"]
            iters.extend(g.step_iters)
            starts.extend(g.step_starts)
            ok = ok and out["statuses_ok"]
            rounds.append({"wall_s": dt, "accepted": out["accepted_steps"], "computed": out["computed_steps"],
                           "rounds_of_alg1": out["rounds"], "decisions": [d.equal for d in g.decisions],
                           "anchor_iters": g.anchor_iters})
        eng.set_profiling(0)
        star_vs_plain = None
        if name == "plain":
            eng.copy_replica(glass.star, ref_slot)
        elif "plain" in res_forms:
            eq, md, de = eng.compare(glass.star, ref_slot, 1e-4)   # r_star after the last round (Eq. 20)
            star_vs_plain = {"equal": bool(eq), "max_disp": md, "de_per_atom": de}
        it = np.asarray(iters, dtype=np.float64)
        res_forms[name] = {"value": acc / tot_t, "ms_per_step": 1e3 * tot_t / args.steps,
                           "computed_steps_per_s": comp / tot_t,
                           "fire_iters_per_step": {"mean": float(it.mean()), "median": float(np.median(it)),
                                                   "p95": float(np.percentile(it, 95))},
                           "all_converged": bool(ok), "rounds": rounds, "counters": eng.counters(),
                           "starts": {"plain": starts.count(0), "learned": starts.count(1),
                                      "fallback": starts.count(2), "extrapolated": starts.count(3)},
                           "live_checks": bool(lv), "minimizer": mz, "final_star_vs_plain": star_vs_plain}
    eng.set_minimizer("fire")
    cg_form = res_forms.pop("cg", None)
    ex_form = res_forms.pop("extrapolated", None)
    lr = res_forms[main_form]
    cnt = res_forms[roof_form]["counters"]
    # inherent-structure agreement of the two forms: same decisions, same final r_star (Eq. 20)
    comparison = None
    if "plain" in res_forms and "learned" in res_forms:
        pl = res_forms["plain"]
        same_dec = [r["decisions"] for r in lr["rounds"]] == [r["decisions"] for r in pl["rounds"]]
        fs = lr["final_star_vs_plain"]
        eq = all(f["final_star_vs_plain"]["equal"] for k, f in res_forms.items() if k != "plain")
        same_all = all([r["decisions"] for r in f["rounds"]] == [r["decisions"] for r in pl["rounds"]]
                       for f in res_forms.values())
        comparison = {"same_decisions": bool(same_dec), "final_star_equal": bool(fs["equal"]),
                      "final_star_max_disp": fs["max_disp"], "final_star_de_per_atom": fs["de_per_atom"],
                      "every_form_same_decisions_and_final_star": bool(eq and same_all),
                      "is_mismatches": int((not fs["equal"]) + (not same_dec)),
                      "iters_ratio_learned_over_plain": lr["fire_iters_per_step"]["mean"]
                      / pl["fire_iters_per_step"]["mean"],
                      "wall_ratio_learned_over_plain": lr["ms_per_step"] / pl["ms_per_step"]}
    # roofline of the force kernel in the batched round (one stream)
    flops_per_atom = 0.5 * nb * FLOPS_PER_PAIR
    avg_ms = cnt["force_ms"] / max(cnt["force_timed"], 1)
    evals = cnt.get("atom_evals", 0)
    atom_evals_per_launch = evals / cnt["force_launches"] if evals and cnt["force_launches"] else P * n
    # no HIP-event samples (--profile-every 0): no achieved rate
    achieved_tflops = flops_per_atom * atom_evals_per_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else None
    achieved_gbs = FORCE_BYTES_PER_ATOM[dim] * atom_evals_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None
    res = {
        "metric": METRIC,
        "value": lr["value"],
        "unit": "accepted AQS steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": lr["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{dim}D binary LJ glass N={n}, Algorithm 1 round: P={P} chains x K={K} "
                               f"fine AQS steps, dgamma={dg:g}, dgamma_c={K * dg:g}, FIRE to max|F|<1e-10, "
                               + ("plain start" if args.only_plain else
                                  "learned start (plain start timed alongside)")
                               + (", live checks" if live else ""),
                   "dim": dim, "n_atoms": n, "P": P, "K": K, "dgamma": dg, "live_checks": live,
                   "knobs": {"threads_per_atom": eng.tuning.threads_per_atom, "skin": eng.tuning.skin,
                             "block_iters": eng.tuning.block_iters, "use_graph": eng.tuning.use_graph,
                             "source": args.tuning}},
        "computed_steps_per_s": lr["computed_steps_per_s"],
        "fire_iters_per_step": lr["fire_iters_per_step"],
        "all_converged": lr["all_converged"],
        "learned_start": {"starts": lr["starts"], "training": train_info},
        "plain": None if args.only_plain else
        {k: v for k, v in res_forms.get("plain", {}).items() if k != "counters"},
        "batched": None if not live else
        {k: v for k, v in res_forms[roof_form].items() if k != "counters"},
        "learned_vs_plain": comparison,
        "extrapolated": None if ex_form is None else
        {"value": ex_form["value"], "ms_per_step": ex_form["ms_per_step"],
         "computed_steps_per_s": ex_form["computed_steps_per_s"],
         "fire_iters_per_step": ex_form["fire_iters_per_step"], "starts": ex_form["starts"],
         "all_converged": ex_form["all_converged"], "final_star_vs_plain": ex_form["final_star_vs_plain"],
         "same_decisions_as_plain": [r["decisions"] for r in ex_form["rounds"]]
         == [r["decisions"] for r in res_forms["plain"]["rounds"]],
         "iters_ratio_over_plain": ex_form["fire_iters_per_step"]["mean"]
         / res_forms["plain"]["fire_iters_per_step"]["mean"],
         "wall_ratio_over_plain": ex_form["ms_per_step"] / res_forms["plain"]["ms_per_step"],
         "rounds": ex_form["rounds"]},
        "cg": None if cg_form is None else
        {"value": cg_form["value"], "ms_per_step": cg_form["ms_per_step"],
         "computed_steps_per_s": cg_form["computed_steps_per_s"],
         "iters_per_step": cg_form["fire_iters_per_step"], "all_converged": cg_form["all_converged"],
         "final_star_vs_plain_fire": cg_form["final_star_vs_plain"],
         "same_decisions_as_plain_fire": [r["decisions"] for r in cg_form["rounds"]]
         == [r["decisions"] for r in res_forms["plain"]["rounds"]],
         "iters_ratio_cg_over_fire": cg_form["fire_iters_per_step"]["mean"]
         / res_forms["plain"]["fire_iters_per_step"]["mean"],
         "wall_ratio_cg_over_fire": cg_form["ms_per_step"] / res_forms["plain"]["ms_per_step"],
         "params": vars(Cg()),
         "rounds": cg_form["rounds"]},
        "quench_s": quench_s,
        "mean_neighbours_in_cutoff": nb,
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tflops / FP64_PEAK_TFLOPS if achieved_tflops else None,
                     "traffic": force_traffic(dim, atom_evals_per_launch),
                     "kernel": f"k_force<{dim}>", "avg_launch_ms": avg_ms,
                     "atoms_per_launch": atom_evals_per_launch,
                     "algorithmic_flops_per_atom": flops_per_atom,
                     "hbm_gbs_algorithmic": achieved_gbs,
                     "hbm_frac": achieved_gbs / HBM_PEAK_GBS if achieved_gbs else None},
        "counters": cnt,
        "rounds": lr["rounds"],
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(dim, n, dg, float(lr["fire_iters_per_step"]["mean"]), args.cpu_seconds)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
