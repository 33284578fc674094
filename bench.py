#!/usr/bin/env python3
"""Benchmark of the batched AQS hot path on one MI355X.

Workload (default): a 3D binary Lennard-Jones glass, N = 32768 atoms
(Kob-Andersen-type parameters, 80:20, density 1.2, cutoff 2.5 sigma_ab),
quenched on the GPU from seeded uniform random positions; its first plain
AQS steps train the learned start.  One "step" is one round of Algorithm 1
(Sec. 3.5) with P = 16 level-II chains of K = 200 fine AQS steps at
dgamma = 5e-5 (level-I anchors at i * 1e-2), every minimisation run by FIRE
to max|F| < 1e-10, the learned start with live checks (the headline form).
A stress drop in the chain a check waits on (a plastic event) stops the
chains after it before that check, which then counts as failed (--abandon).
Each step starts from the same inherent structure (already in HBM); the
accepted steps of a round are q of Algorithm 1 (at least K), the computed
ones P * K plus the anchor minimisations.

Beside the timed steps: a few rounds of the plain start (learned vs plain),
conventional sequential AQS of the same K steps from the same structure (the
C^(S) of Eq. 21, for the speed-up S), one round with live checks but no
abandonment, and on request the extrapolated start, conjugate gradients and
the batched round without live checks.

Prints one JSON line: accepted AQS steps/s (value), FIRE iterations per AQS
step, the roofline of the dominant kernel (the FP64 force kernel, its own
start and end recorded by HIP events with the dispatches of every 64th block
of iterations inside the timed steps, on each launch's stream) and the CPU
oracle timed on a bounded sample on the host cores.
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
# law): the separation (3), r^2 (5), the reciprocal (about 8), the LJ powers
# and U'(r)/r (8), the shifted energy (3), the force components on both atoms
# (6): 33 flops
FLOPS_PER_PAIR = 33
# algorithmic bytes per atom of the force kernel: positions (d doubles) and
# the type (one byte) in, forces out (d doubles): 16 d + 1
FORCE_BYTES_PER_ATOM = {2: 33, 3: 49}


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


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pos, types, L, dg, iters_per_step, seconds=15.0):
    """Time the CPU oracle (sequential AQS: O(N^2) pair sums over all host
    threads) on a bounded sample of the same workload: force evaluations of
    the benchmark's own inherent structure after one affine increment, until
    `seconds`/2 have passed (at least one); AQS steps/s = 1 / (t_eval x
    (iterations per step + 1)), with the GPU-measured iterations."""
    import oracle as O
    dim = pos.shape[1]
    H = O.strain_box(dim, L, 1, dg)
    x = O.affine(pos, dg)
    pot = O.kob_andersen()
    O.energy_forces(x[:64], types[:64], O.box_matrix(dim, 50.0, 0.0), pot)  # load the library
    t0 = time.perf_counter()
    evals = 0
    while True:
        O.energy_forces(x, types, H, pot)
        evals += 1
        if time.perf_counter() - t0 > seconds / 2 or evals >= 50:
            break
    t_eval = (time.perf_counter() - t0) / evals
    rate = 1.0 / (t_eval * (iters_per_step + 1.0))
    return {"value": rate, "unit": "AQS steps/s", "cores": O.get_threads(), "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"{evals} O(N^2) force evaluations of the benchmark's N={len(types)} {dim}D inherent "
                      f"structure after one increment ({t_eval:.3f} s each) x (GPU-measured "
                      f"{iters_per_step:.1f} FIRE iterations + 1) per sequential AQS step",
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


def train_on_history(eng, star, spare, steps, epochs, seed, dim):
    """Learned start trained online on the benchmark glass's own history:
    `steps` plain AQS steps of the inherent structure in `star` (left at the
    last one) give the descriptors and non-affine targets, then the network
    is trained on the GPU (Adam, Huber loss, batch 4096).  Returns the model
    and a summary."""
    import torch
    import aqs_synth as S
    from paper_2507_20802_amd import learned
    t0 = time.perf_counter()
    feat, tgt, recs = learned.collect_samples(eng, star, spare, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    orders = torch.from_numpy(S.epoch_orders(feat.shape[0], epochs, 3, seed, 7)).cuda()
    model = learned.make_mlp(dim, S.mlp_init(dim, 3, seed, 8))
    hist = learned.train(model, feat, tgt, orders, learned.TrainParams(batch=4096, epochs=epochs))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return model, {"samples": int(feat.shape[0]), "plain_steps": steps, "epochs": epochs,
                   "history_iters": [int(r["iters"]) for r in recs],
                   "data_s": t1 - t0, "train_s": t2 - t1, "loss_first": float(hist[0]),
                   "loss_last": float(hist[-1])}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3,
                    help="timed steps: rounds of Algorithm 1 of the headline form")
    ap.add_argument("--warmup", type=int, default=1, help="untimed rounds (of --warmup-K steps) first")
    ap.add_argument("--dim", type=int, default=3)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--P", type=int, default=16)
    ap.add_argument("--K", type=int, default=200)
    ap.add_argument("--dgamma", type=float, default=5e-5)
    ap.add_argument("--warmup-K", type=int, default=20, help="fine steps per chain in warmup rounds")
    ap.add_argument("--profile-every", type=int, default=64,
                    help="time every n-th block of iterations with HIP events (force-kernel roofline); "
                         "a timed kernel costs the critical chain about 5 us, so the headline samples sparsely")
    ap.add_argument("--train-steps", type=int, default=7,
                    help="plain AQS steps of the glass's own history that train the network")
    ap.add_argument("--epochs", type=int, default=50)
    ap.add_argument("--plain-rounds", type=int, default=2,
                    help="rounds of the plain-start form timed beside the headline (0: none)")
    ap.add_argument("--sequential", type=int, default=1,
                    help="time conventional sequential AQS of the same K steps (1/0), Eq. 21's C^(S)")
    ap.add_argument("--kernel-K", type=int, default=5,
                    help="fine steps per chain of the kernel form's batched round")
    ap.add_argument("--abandon", type=int, default=1,
                    help="live rounds: a stress drop (plastic event) in the critical chain stops the chains "
                         "after it before their check (1/0)")
    ap.add_argument("--forms", default="live1,kernel",
                    help="extra forms, comma-separated: live1 (live checks without abandonment), kernel "
                         "(a short batched round, every force launch timed: the force kernel on all "
                         "chains at once), extrapolated, cg, batched (one round each)")
    ap.add_argument("--only-plain", action="store_true", help="headline with the plain start (no network)")
    ap.add_argument("--graph", type=int, default=0, help="replay iteration blocks as hipGraphs (1/0)")
    ap.add_argument("--live", type=int, default=1,
                    help="live checks (1/0): checks as soon as possible, the critical chain on a stream of "
                         "its own, rejected chains stopped")
    ap.add_argument("--live-xcds", type=int, default=None,
                    help="live rounds: XCDs (of 8) reserved for the critical chain (0: none; default: the tuning's)")
    ap.add_argument("--live-duty", type=int, default=None,
                    help="duty cycle of the speculative batch in live rounds (default: the first-round policy)")
    ap.add_argument("--live-blocks", type=int, default=None,
                    help="live rounds: batch force blocks per CU beside the critical chain (0: 3; < 0: no limit)")
    ap.add_argument("--tuning", choices=("default", "auto", "autotune"), default="auto",
                    help="launch knobs: the defaults, the autotuner's cache, or tune when not cached")
    ap.add_argument("--skin", type=float, default=0.3, help="Verlet skin with --tuning default")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only stream MIB MiB device-to-device (counter calibration) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the engine "
              f"drives one GPU; sharding over several is described, not implemented).", file=sys.stderr)
        return 2
    extra = [f for f in args.forms.split(",") if f]
    for f in extra:
        if f not in ("live1", "kernel", "extrapolated", "cg", "batched"):
            print(f"unknown form {f}", file=sys.stderr)
            return 2

    import torch
    import aqs_synth as S
    from paper_2507_20802_amd import (AQS_START_EXTRAPOLATED, AQS_START_LEARNED, AQS_START_PLAIN, Cg, Engine,
                                      Fire, LJParams, Tuning, parallel)

    t_job = time.perf_counter()
    torch.cuda.set_device(0)
    dim, n, P, K, dg = args.dim, args.n, args.P, args.K, args.dgamma
    pot = LJParams()
    s = S.uniform_glass_start(dim, n, 3, 0)
    nslots = parallel.slots_needed(1, P)
    ref_slot = nslots              # final r_star of the plain round, for the IS comparison
    tuning = Tuning(skin=args.skin, use_graph=args.graph) if args.tuning == "default" else args.tuning
    eng = Engine(dim, [n] * (nslots + 1), s.L, dg, pot=pot, fire=Fire(), tuning=tuning)
    if args.live_xcds is not None:
        eng.set_live_xcds(args.live_xcds)
        eng.tuning.live_xcds = args.live_xcds
    if args.live_blocks is not None:
        eng.tuning.live_batch_blocks = args.live_blocks
        eng.set_live_batch_blocks(args.live_blocks)
    glass = parallel.layout(1, P)[0]
    t0 = time.perf_counter()
    eng.set_replica(glass.star, s.types, s.pos, 0)
    q = eng.minimize([glass.star])[0, 0]
    quench_s = time.perf_counter() - t0
    if q["status"] != 0:
        print(f"quench failed: status {q['status']}", file=sys.stderr)
        return 1
    log(f"quenched N={n} {dim}D glass in {quench_s:.1f} s ({int(q['iters'])} iterations)")
    train_info, k0 = None, 0
    if not args.only_plain:
        # the glass's own first plain steps train the network; the timed rounds start after them
        model, train_info = train_on_history(eng, glass.star, glass.chains[0], args.train_steps,
                                             args.epochs, 0, dim)
        eng.learned_load(model)
        k0 = eng.strain_index(glass.star)
        log(f"trained on {args.train_steps} plain steps of the glass ({train_info['samples']} samples): "
            f"loss {train_info['loss_first']:.3f} -> {train_info['loss_last']:.3f}")
    is_pos = eng.positions(glass.star)
    nb = in_cutoff_neighbours(is_pos, s.types, s.L, pot)   # the box is still orthogonal to 1e-3

    def one_round(Kr, start, live, abandon):
        eng.set_replica(glass.star, s.types, is_pos, k0)
        g = parallel.layout(1, P)[0]
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = parallel.run(eng, [g], P * Kr, Kr, P, start=start, max_rounds=1, live=live, abandon=abandon,
                           live_duty=args.live_duty)
        torch.cuda.synchronize()
        return time.perf_counter() - t, out, g

    def timed_form(name, start, live, mz, rounds, abandon, k=None, every=None):
        eng.set_minimizer(mz, Cg() if mz == "cg" else None)
        eng.counters(reset=True)
        eng.set_profiling(args.profile_every if every is None else every)
        tot_t, acc, comp, iters, ok, rr, starts = 0.0, 0, 0, [], True, [], []
        for _ in range(rounds):
            dt, out, g = one_round(K if k is None else k, start, live, abandon)
            tot_t += dt
            acc += out["accepted_steps"]
            comp += out["computed_steps"]
            iters.extend(g.step_iters)
            starts.extend(g.step_starts)
            ok = ok and out["statuses_ok"]
            rr.append({"wall_s": dt, "accepted": out["accepted_steps"], "computed": out["computed_steps"],
                       "decisions": [d.equal for d in g.decisions],
                       "predicted": [bool(np.isnan(d.max_disp)) for d in g.decisions],
                       "anchor_iters": g.anchor_iters})
            log(f"{name} round {len(rr)}/{rounds}: {dt:.2f} s, {out['accepted_steps']} accepted")
        eng.set_profiling(0)
        eng.set_minimizer("fire")
        it = np.asarray(iters, dtype=np.float64)
        res = {"value": acc / tot_t, "ms_per_step": 1e3 * tot_t / rounds, "rounds": rounds,
               "computed_steps_per_s": comp / tot_t,
               "fire_iters_per_step": {"mean": float(it.mean()), "median": float(np.median(it)),
                                       "p95": float(np.percentile(it, 95))},
               "all_converged": bool(ok), "per_round": rr, "counters": eng.counters(),
               "starts": {"plain": starts.count(0), "learned": starts.count(1),
                          "fallback": starts.count(2), "extrapolated": starts.count(3)},
               "live_checks": bool(live), "abandon": bool(abandon and live), "minimizer": mz}
        log(f"{name}: {res['value']:.2f} accepted AQS steps/s, {res['ms_per_step']:.0f} ms per round, "
            f"{res['fire_iters_per_step']['mean']:.0f} iterations per step")
        return res

    live = bool(args.live)
    abandon = bool(args.abandon) and live
    head_start = AQS_START_PLAIN if args.only_plain else AQS_START_LEARNED
    # warmup: short rounds of the headline form
    for w in range(args.warmup):
        dt, _, _ = one_round(args.warmup_K, head_start, live, abandon)
        log(f"warmup round {w + 1}/{args.warmup} (K={args.warmup_K}): {dt:.2f} s")
    head = timed_form("headline", head_start, live, "fire", args.steps, abandon)
    eng.copy_replica(glass.star, ref_slot)                       # r_star after the headline round

    def star_vs_headline():
        """The configuration in the star slot against the headline's r_star
        (Eq. 20), when both are at the same strain index."""
        if eng.strain_index(glass.star) != eng.strain_index(ref_slot):
            return {"equal": None, "strain_indices": [eng.strain_index(glass.star), eng.strain_index(ref_slot)]}
        eq, md, de = eng.compare(glass.star, ref_slot, 1e-4)
        return {"equal": bool(eq), "max_disp": md, "de_per_atom": de}
    forms = {}
    if args.plain_rounds > 0 and not args.only_plain:
        forms["plain"] = timed_form("plain", AQS_START_PLAIN, live, "fire", args.plain_rounds, abandon)
        forms["plain"]["final_star_vs_headline"] = star_vs_headline()
    for f in extra:
        if f == "kernel":
            forms[f] = timed_form(f, AQS_START_PLAIN, False, "fire", 1, False, k=args.kernel_K, every=1)
            continue
        st = {"live1": head_start, "extrapolated": AQS_START_EXTRAPOLATED, "cg": AQS_START_PLAIN,
              "batched": head_start}[f]
        forms[f] = timed_form(f, st, live and f != "batched", "cg" if f == "cg" else "fire", 1,
                              abandon and f not in ("live1", "batched"))
        forms[f]["final_star_vs_headline"] = star_vs_headline()
    seq = None
    if args.sequential:
        # conventional AQS (Eq. 12) of the same K steps from the same inherent
        # structure: one replica alone on the GPU, plain start (C^(S) of Eq. 21)
        eng.set_replica(glass.star, s.types, is_pos, k0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        rec = eng.minimize([glass.star], n_steps=[K])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        it = rec["iters"][0, 1:].astype(np.float64)
        seq = {"steps": K, "wall_s": dt, "value": K / dt,
               "fire_iters_per_step": {"mean": float(it.mean()), "median": float(np.median(it))},
               "all_converged": bool((rec["status"][0] == 0).all()),
               "end_vs_headline_r_star": star_vs_headline()}
        log(f"sequential: {seq['value']:.2f} AQS steps/s")

    # roofline of the force kernel over the headline's timed launches (HIP
    # events recorded with the dispatches, on the stream of each launch; both
    # driver lanes with live checks)
    cnt = head["counters"]
    flops_per_atom = 0.5 * nb * FLOPS_PER_PAIR
    n_timed = cnt["force_timed"]
    avg_ms = cnt["force_ms"] / n_timed if n_timed else 0.0
    atoms_per_launch = cnt["timed_atom_evals"] / n_timed if n_timed else 0.0
    achieved_tflops = flops_per_atom * atoms_per_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else None
    achieved_gbs = FORCE_BYTES_PER_ATOM[dim] * atoms_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None
    traffic = force_traffic(dim, atoms_per_launch)
    kernel_form = None
    if "kernel" in forms:
        kc = forms["kernel"]["counters"]
        kms = kc["force_ms"] / kc["force_timed"]
        katoms = kc["timed_atom_evals"] / kc["force_timed"]
        ktf = flops_per_atom * katoms / (kms * 1e-3) / 1e12
        kernel_form = {"kernel": f"k_force<{dim}>", "avg_launch_ms": kms, "timed_launches": kc["force_timed"],
                       "atoms_per_launch": katoms, "achieved_tflops": ktf, "frac_fp64": ktf / FP64_PEAK_TFLOPS,
                       "hbm_gbs_algorithmic": FORCE_BYTES_PER_ATOM[dim] * katoms / (kms * 1e-3) / 1e9,
                       "traffic_bytes_per_atom": (force_traffic(dim, katoms) / katoms)
                       if force_traffic(dim, katoms) else None,
                       "update_avg_ms": kc["update_ms"] / kc["update_timed"],
                       "round": f"plain start, batched (no live checks), P={P} x K={args.kernel_K}, "
                                f"every force launch timed"}
    comparison = None
    if "plain" in forms:
        pl = forms["plain"]
        same_dec = [r["decisions"] for r in head["per_round"][:pl["rounds"]]] == \
            [r["decisions"] for r in pl["per_round"]]
        fs = pl["final_star_vs_headline"]
        comparison = {"same_decisions": bool(same_dec), "final_star_equal": fs["equal"],
                      "final_star_max_disp": fs.get("max_disp"), "final_star_de_per_atom": fs.get("de_per_atom"),
                      "is_mismatches": int((fs["equal"] is not True) + (not same_dec)),
                      "iters_ratio_headline_over_plain": head["fire_iters_per_step"]["mean"]
                      / pl["fire_iters_per_step"]["mean"],
                      "wall_ratio_headline_over_plain": head["ms_per_step"] / pl["ms_per_step"]}
    res = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "accepted AQS steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{dim}D binary LJ glass N={n}, one round of Algorithm 1 per step: P={P} chains x "
                               f"K={K} fine AQS steps, dgamma={dg:g}, dgamma_c={K * dg:g}, FIRE to max|F|<1e-10, "
                               + ("plain start" if args.only_plain else
                                  f"learned start trained on the glass's first {args.train_steps} plain steps")
                               + (", live checks" if live else ", batched checks")
                               + (", speculation stopped at a stress drop of the critical chain" if abandon else ""),
                   "dim": dim, "n_atoms": n, "P": P, "K": K, "dgamma": dg, "live_checks": live,
                   "abandon_on_stress_drop": abandon,
                   "start_strain_index": k0,
                   "knobs": {"threads_per_atom": eng.tuning.threads_per_atom, "skin": eng.tuning.skin,
                             "block_iters": eng.tuning.block_iters, "use_graph": eng.tuning.use_graph,
                             "live_batch_blocks": eng.tuning.live_batch_blocks,
                             "live_xcds": eng.tuning.live_xcds, "source": args.tuning}},
        "computed_steps_per_s": head["computed_steps_per_s"],
        "fire_iters_per_step": head["fire_iters_per_step"],
        "all_converged": head["all_converged"],
        "starts": head["starts"],
        "learned_start": {"training": train_info},
        "per_round": head["per_round"],
        "plain": None if "plain" not in forms else
        {k: v for k, v in forms["plain"].items() if k not in ("counters",)},
        "learned_vs_plain": comparison,
        "sequential": seq,
        "speedup_vs_sequential": None if seq is None else head["value"] / seq["value"],
        "speedup_vs_sequential_live1": None if seq is None or "live1" not in forms
        else forms["live1"]["value"] / seq["value"],
        "extra_forms": {f: {k: v for k, v in forms[f].items() if k != "counters"} for f in extra if f != "kernel"},
        "quench_s": quench_s,
        "mean_neighbours_in_cutoff": nb,
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tflops / FP64_PEAK_TFLOPS if achieved_tflops else None,
                     "traffic": traffic,
                     "kernel": f"k_force<{dim}>", "avg_launch_ms": avg_ms, "timed_launches": n_timed,
                     "atoms_per_launch": atoms_per_launch,
                     "algorithmic_flops_per_atom": flops_per_atom,
                     "algorithmic_bytes_per_atom": FORCE_BYTES_PER_ATOM[dim],
                     "hbm_gbs_algorithmic": achieved_gbs,
                     "hbm_frac_algorithmic": achieved_gbs / HBM_PEAK_GBS if achieved_gbs else None,
                     "traffic_bytes_per_atom": traffic / atoms_per_launch if traffic and atoms_per_launch else None},
        "counters": cnt,
        "force_kernel_all_chains": kernel_form,
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(is_pos, s.types, s.L, dg, float(head["fire_iters_per_step"]["mean"]),
                                           args.cpu_seconds)
    res["job_wall_s"] = time.perf_counter() - t_job
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
