"""Algorithm 1 of the paper (Sec. 3.5, "Parallel calculation scheme") on the
GPU engine, for one or many independent glasses at once.

Per round and glass, with r_star in its slot:
  level I   copy r_star into P' chain slots; chain i gets the affine map
            F_N^(i K dgamma) in one multiplication (Eq. 18)
  level II  one batched aqs_minimize_batch over every chain of every glass:
            the anchor minimisation F(r^c_iK) (its result is copied on the
            device into a snapshot slot: the "outgoing" configuration of
            Sec. 3.3) followed by the chain's fine AQS steps (Eq. 19), each
            chain advancing on its own on the device
  check     for i = 1..P'-1 in order: end of chain i-1 ("incoming") vs the
            snapshot of chain i ("outgoing"), Eq. (20); first failure stops
  update    q accepted steps; r_star <- r_q (Algorithm 1)

Readings (the paper is silent): the last round is clamped to the remaining
steps (P' = ceil(R / K) chains, the last with R - (P'-1) K steps); a round
with a single chain accepts it; r_q is the end of chain q/K - 1.

dynamic_k=(k_min, k_max) chooses each glass's K anew after every round (the
dynamic choice of K of the paper's outlook, Sec. 5; the rule, next_k, is a
reading).  Chain 0 of a round always starts from the verified r_star and
every accepted step is checked, so the accepted trajectory does not depend
on the K sequence; only rounds and computed steps do.

dynamic_dgamma=m_max sizes the strain increment per glass and round (the
dynamic step sizing of the same outlook; the rule, a reading, is
next_level): a round runs at level m with increment 2^m dgamma (dgamma the
slots' increment when the run starts, the finest), steps are counted in
fine increments, and a level-m round starts on a multiple of 2^m of them.
A plastic event shows as a shear stress below the step before's, as
energy released within a step (chain_events: on an elastic branch
dE/dgamma = V sigma_xy, so a step's energy change is the trapezoidal work of
the stress up to third order in the step), or as a failed check; a round at
level m > 0 keeps its chains only up to the first
that holds one, and the glass stays at level 0 until its strain has passed
the end of that chain, so every event is stepped through at the finest
increment; rounds without an event climb one level at a time.  Levels
change through aqs_set_dgamma, which keeps each slot's strain exactly; at
the end of run() every slot is back at the finest increment.

live=True runs each glass's round through aqs_run_round with live checks
(the improvement the paper proposes in Sec. 4): a check is taken as soon as
both of its configurations exist, the chain the next check waits on runs on a
stream of its own, and the chains after a failed check are stopped.  The
decisions, q and r_star are those of the batched round; glasses are then
processed one after another.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

from ._lib import AQS_CANCELLED, AQS_START_PLAIN


def chain_plan(remaining: int, K: int, P: int) -> List[int]:
    """Fine-step counts of the chains of one round (last round clamped)."""
    if remaining >= P * K:
        return [K] * P
    p = math.ceil(remaining / K)
    return [K] * (p - 1) + [remaining - (p - 1) * K]


@dataclass
class Decision:
    round: int
    index: int          # i of the check (compares end of chain i-1 with outgoing of chain i)
    strain_index: int   # k of both configurations
    equal: bool
    max_disp: float
    de_per_atom: float


@dataclass
class GlassRun:
    star: int                   # slot of r_star
    chains: List[int]           # P chain slots
    snaps: List[int]            # P snapshot slots (entry 0 unused)
    n_current: int = 0
    rounds: List[dict] = field(default_factory=list)
    decisions: List[Decision] = field(default_factory=list)
    step_iters: List[int] = field(default_factory=list)     # FIRE iterations of every fine step computed
    step_starts: List[int] = field(default_factory=list)    # start used by every fine step (AQS_START_*)
    accepted_iters: List[int] = field(default_factory=list)  # ... of the accepted fine steps
    anchor_iters: List[int] = field(default_factory=list)    # anchor minimisations
    energies: List[float] = field(default_factory=list)      # accepted trajectory E (per accepted step)
    sigma_xy: List[float] = field(default_factory=list)
    statuses_ok: bool = True
    computed_steps: int = 0
    accepted_strain: List[int] = field(default_factory=list)  # fine strain index of every accepted step
    level: int = 0              # the slots' increment is dgamma0 2^level (dynamic_dgamma)
    dgamma0: float = 0.0        # the finest increment (dynamic_dgamma)
    hold: int = 0               # level 0 until n_current reaches this (dynamic_dgamma)


def slots_needed(n_glasses: int, P: int) -> int:
    return n_glasses * (1 + 2 * P)


def layout(n_glasses: int, P: int, first: int = 0) -> List[GlassRun]:
    """Slot assignment: per glass, [star, chain_0..chain_{P-1}, snap_0..snap_{P-1}]."""
    out = []
    s = first
    for _ in range(n_glasses):
        star = s
        chains = list(range(s + 1, s + 1 + P))
        snaps = list(range(s + 1 + P, s + 1 + 2 * P))
        out.append(GlassRun(star, chains, snaps))
        s += 1 + 2 * P
    return out


def next_k(K: int, checks: List[bool], k_min: int, k_max: int) -> int:
    """A glass's chain length for its next round: 2K when every check of the
    round passed, ceil(K / 2) when its first check failed, else K; within
    [k_min, k_max].  A round without checks (one chain) keeps K."""
    if len(checks) == 0:
        return K
    if all(checks):
        k = K * 2
    elif checks[0]:
        k = K
    else:
        k = -(-K // 2)
    return max(k_min, min(k, k_max))


def chain_events(sigma_xy, length: int, energy=None, work: float = 0.0, tol: Optional[float] = None) -> bool:
    """A plastic event in a chain (entry 0 is the chain's first
    minimisation, entry j its step j): a step ends at a shear stress below
    the one before; or, with energies, `work` = volume x the step's strain
    and `tol`, a step's energy change falls short of the trapezoidal work
    work (s_(j-1) + s_j) / 2 by more than tol work (|s_(j-1)| + |s_j|) / 2."""
    s = np.asarray(sigma_xy[: length + 1], dtype=np.float64)
    if np.any(s[1:] < s[:-1]):
        return True
    if energy is None or tol is None:
        return False
    e = np.asarray(energy[: length + 1], dtype=np.float64)
    lo = work * (s[1:] + s[:-1]) / 2.0 - tol * work * (np.abs(s[1:]) + np.abs(s[:-1])) / 2.0
    return bool(np.any(e[1:] - e[:-1] < lo))


def next_level(level: int, marked: bool, n_current: int, hold: int, fine_index: int, m_max: int) -> int:
    """A glass's level for its next round (dynamic_dgamma): 0 when the round
    marked an event or the strain is still short of the hold point; else one
    higher, at most m_max, and lowered until the fine strain index reached is
    a multiple of its increment."""
    lv = 0 if marked or n_current < hold else min(level + 1, m_max)
    while lv > 0 and fine_index % (1 << lv):
        lv -= 1
    return lv


def reservation_for(last_checks: List[bool]) -> int:
    """Batch force blocks per CU for the next live round (aqs_tuning
    live_batch_blocks) from the decided checks of the last round: speculation
    that paid (at least three quarters passed) runs unthrottled (-1); checks
    that mostly failed (under a quarter passed), and the first round, leave
    one block per CU to the batch, so that the critical chain keeps most of
    its own speed; otherwise the default (0, i.e. 3)."""
    if not last_checks:
        return 1
    f = sum(bool(c) for c in last_checks) / len(last_checks)
    if f >= 0.75:
        return -1
    if f < 0.25:
        return 1
    return 0


# duty cycle of the speculative batch in the first live round, before any
# check has been seen (aqs_set_live_duty)
FIRST_ROUND_DUTY = 1


def duty_for(last_checks: List[bool]) -> int:
    """Duty cycle of the speculative batch for the next live round (the batch
    runs one block of iterations in this many while a critical chain runs):
    every block when at least three quarters of the last round's decided
    checks passed; one in four when under a quarter passed; one in two
    otherwise; FIRST_ROUND_DUTY before any round."""
    if not last_checks:
        return FIRST_ROUND_DUTY
    f = sum(bool(c) for c in last_checks) / len(last_checks)
    if f >= 0.75:
        return 1
    if f < 0.25:
        return 4
    return 2


def set_level(engine, g: GlassRun, level: int) -> None:
    """Every slot of the glass to the increment dgamma0 2^level, strains kept:
    the chains and snapshots first take r_star's configuration (their
    leftover strain indices need not convert)."""
    for s in g.chains + g.snaps[1:]:
        engine.copy_replica(g.star, s)
    slots = [g.star] + g.chains + g.snaps[1:]
    engine.set_dgamma(slots, g.dgamma0 * float(1 << level))
    g.level = level


def run(engine, glasses: List[GlassRun], n_steps: int, K: int, P: int, delta_eq: float = 1e-4,
        start: int = AQS_START_PLAIN, max_rounds: int | None = None, log=None, live: bool = False,
        adaptive_reservation: bool = True, dynamic_k: Optional[Tuple[int, int]] = None,
        abandon: bool = False, live_duty: Optional[int] = None,
        dynamic_dgamma: Optional[int] = None, event_tol: Optional[float] = 1e-2) -> dict:
    """Run Algorithm 1 to n_steps accepted fine steps for every glass (each
    glass's r_star must be loaded in its star slot as an inherent structure).
    With live checks and adaptive_reservation, each round's CU reservation
    for the critical chain follows the previous round's checks
    (reservation_for).  dynamic_k=(k_min, k_max): every glass starts with K
    and takes next_k after each round.  Returns timing and counts; per-glass
    details (each round's K among them) are filled into glasses.
    abandon (with live): a stress drop in the critical chain stops the chains
    after it before their check, which counts as failed (predicted, not
    evaluated: the decision's max_disp is NaN).
    dynamic_dgamma=m_max (simple shear only): increments dgamma 2^m, m in
    [0, m_max], chosen per glass and round (next_level); n_steps, N_current,
    q and the decisions' strain indices count fine increments; event_tol:
    tolerance of the energy balance that marks events (chain_events; None:
    stress drops and failed checks only)."""
    if P < 2:
        raise ValueError("Algorithm 1 needs P >= 2 (Sec. 3.2)")
    if K < 1:
        raise ValueError("K must be >= 1")
    if dynamic_k is not None and not 1 <= dynamic_k[0] <= dynamic_k[1]:
        raise ValueError("dynamic_k needs 1 <= k_min <= k_max")
    m_max = int(dynamic_dgamma or 0)
    if m_max < 0:
        raise ValueError("dynamic_dgamma needs m_max >= 0")
    for g in glasses:
        if m_max and g.level == 0:
            g.dgamma0 = float(engine.dgamma[g.star])
    kg = [K] * len(glasses)
    t0 = time.perf_counter()
    rnd = 0
    t_min = 0.0
    t_check = 0.0
    last_checks: List[bool] = []
    while any(g.n_current < n_steps for g in glasses):
        if max_rounds is not None and rnd >= max_rounds:
            break
        sel, nst, snp, plans = [], [], [], {}
        dks, aff = [], []
        for gi, g in enumerate(glasses):
            if g.n_current >= n_steps:
                continue
            rem = n_steps - g.n_current
            lv = g.level
            while rem < (1 << lv):                  # no overshoot of the target strain
                lv -= 1
            if lv != g.level:
                set_level(engine, g, lv)
            h = 1 << lv
            lengths = chain_plan(rem // h, kg[gi], P)
            k_lv = engine.strain_index(g.star)
            if lv < m_max and (k_lv + sum(lengths)) % 2 and sum(lengths) * h < rem:
                # end on an even index so that the next round can climb
                if lengths[-1] > 1:
                    lengths[-1] -= 1
                elif len(lengths) > 1:
                    lengths.pop()
            plans[gi] = lengths
            for i, ln in enumerate(lengths):
                engine.copy_replica(g.star, g.chains[i])
                if i > 0:
                    aff.append(g.chains[i])
                    dks.append(i * kg[gi])
                sel.append(g.chains[i])
                nst.append(ln)
                snp.append(g.snaps[i] if i > 0 else -1)
        if aff:
            engine.affine_shear(aff, dks)           # level I (Eq. 18)
        t1 = time.perf_counter()
        rows, outcomes = {}, {}
        if live and adaptive_reservation:
            engine.set_live_batch_blocks(reservation_for(last_checks))
        if live:
            engine.set_live_duty(live_duty if live_duty is not None
                                 else (duty_for(last_checks) if adaptive_reservation else 1))
        last_checks = []
        if live:
            for gi, lengths in plans.items():        # level II + live checks, glass by glass
                g = glasses[gi]
                p = len(lengths)
                recs, chk = engine.run_round(g.chains[:p], [-1] + g.snaps[1:p], lengths, start=start,
                                             delta_eq=delta_eq, live=True, abandon=abandon)
                for i in range(p):
                    rows[g.chains[i]] = recs[i]
                outcomes[gi] = [(c[1], c[2] if c[0] == 1 else float("nan"), c[3] if c[0] == 1 else float("nan"))
                                for c in chk[1:] if c[0]]
        else:
            recs = engine.minimize(sel, n_steps=nst, snap_dst=snp, start=start)   # level II
            rows = {s: recs[j] for j, s in enumerate(sel)}
        t2 = time.perf_counter()
        t_min += t2 - t1
        for gi, lengths in plans.items():
            g = glasses[gi]
            Kr = kg[gi]
            lv = g.level
            h = 1 << lv
            k0 = engine.strain_index(g.star)         # in increments of the round's level
            q = lengths[0]
            last = 0
            checks = []
            for i in range(1, len(lengths)):
                if live:
                    if i - 1 >= len(outcomes[gi]):
                        break
                    eq, md, de = outcomes[gi][i - 1]
                else:
                    eq, md, de = engine.compare(g.chains[i - 1], g.snaps[i], delta_eq)   # Eq. (20)
                k = (k0 + i * Kr) << lv     # fine index of both configurations of check i
                d = Decision(rnd, i, k, eq, md, de)
                g.decisions.append(d)
                checks.append(eq)
                if eq:
                    q = i * Kr + lengths[i]
                    last = i
                else:
                    q = i * Kr
                    last = i - 1
                    break
            cut = False
            if m_max:
                # chains of the accepted prefix holding an event; a failed
                # check after chain c means chain c crossed one
                work = float(np.prod(engine.box_len[g.star])) * float(engine.dgamma[g.star])
                marked = [c for c in range(last + 1)
                          if chain_events(rows[g.chains[c]]["sigma_xy"], lengths[c], rows[g.chains[c]]["energy"],
                                          work, event_tol)]
                if last + 1 < len(lengths) and checks and not checks[-1]:
                    marked.append(last)
                if lv > 0 and marked:
                    cut = True
                    last = min(marked) - 1
                    q = sum(lengths[: last + 1])
                    g.hold = g.n_current + sum(lengths[: last + 2]) * h
            # bookkeeping of iterations (fine steps are records 1..len of each
            # chain; a chain stopped after a failed check keeps its finished ones)
            for i, ln in enumerate(lengths):
                r = rows[g.chains[i]]
                ran = r["status"][: ln + 1] != AQS_CANCELLED
                if np.any(r["status"][: ln + 1][ran] != 0):
                    g.statuses_ok = False
                if not ran[0]:
                    continue
                g.anchor_iters.append(int(r["iters"][0]))
                fine = np.nonzero(ran[1:])[0] + 1
                g.step_iters.extend(int(r["iters"][s]) for s in fine)
                g.step_starts.extend(int(r["start"][s]) for s in fine)
                g.computed_steps += int(fine.size)
                if i <= last:
                    g.accepted_strain.extend(((k0 + i * Kr + j) << lv) for j in range(1, ln + 1))
                    g.accepted_iters.extend(int(x) for x in r["iters"][1: ln + 1])
                    g.energies.extend(float(x) for x in r["energy"][1: ln + 1])
                    g.sigma_xy.extend(float(x) for x in r["sigma_xy"][1: ln + 1])
            if last >= 0:
                engine.copy_replica(g.chains[last], g.star)   # r_star <- r_q
            q *= h
            g.rounds.append({"round": rnd, "start": g.n_current, "lengths": lengths,
                             "checks": checks, "q": q, "K": Kr, "level": lv, "cut": cut})
            if dynamic_k is not None:
                kg[gi] = next_k(Kr, checks, dynamic_k[0], dynamic_k[1])
            last_checks.extend(checks)
            g.n_current += q
            if m_max:
                nl = next_level(lv, bool(marked), g.n_current, g.hold, (k0 << lv) + q, m_max)
                if nl != lv:
                    set_level(engine, g, nl)
            if log:
                log(f"round {rnd} glass {gi}: checks {checks} q {q} -> N_current {g.n_current}")
        t_check += time.perf_counter() - t2
        rnd += 1
    if live and adaptive_reservation:
        engine.set_live_batch_blocks(engine.tuning.live_batch_blocks)
    for g in glasses:
        if g.level:
            set_level(engine, g, 0)
    wall = time.perf_counter() - t0
    acc = sum(g.n_current for g in glasses)
    comp = sum(g.computed_steps for g in glasses)
    it = np.array([x for g in glasses for x in g.step_iters], dtype=np.int64)
    return {"wall_s": wall, "minimize_s": t_min, "check_s": t_check, "rounds": rnd,
            "accepted_steps": acc, "computed_steps": comp,
            "iters_mean": float(it.mean()) if it.size else 0.0,
            "iters_median": float(np.median(it)) if it.size else 0.0,
            "iters_p95": float(np.percentile(it, 95)) if it.size else 0.0,
            "statuses_ok": all(g.statuses_ok for g in glasses)}
