"""Algorithm 1 of the paper (Sec. 3.5, "Parallel calculation scheme") in plain
Python -- TEST INFRASTRUCTURE ONLY.

The procedure aqs_parallel(r0, H, F_N, dgamma, dgamma_c, N_steps, K, P):

    N_current <- 0;  r_star <- r0
    while N_current < N_steps:
        level I:  r^c_{iK} <- F_N^(i dgamma_c) r_star,  i = 0..P-1      (Eq. 18)
        level II, every i in parallel:
            outgoing_i <- F(r^c_{iK})                                   (Eq. 10)
            end_i      <- (F o F_N^(dgamma))^K (outgoing_i)              (Eq. 19)
        sequential check, i = 1..P-1:
            if end_{i-1} ~= outgoing_i (Eq. 20):  q <- (i+1) K, continue
            else:                                  q <- i K,     stop
        r_star <- r_q;  N_current <- N_current + q

Readings where the paper is silent:
  * the last round is clamped: with R = N_steps - N_current < P K remaining
    steps, only P' = ceil(R / K) chains run and the last one takes
    K' = R - (P' - 1) K steps (N_steps need not be a multiple of K);
  * with a single chain in a round (P' = 1) its K' steps are accepted
    (chain 0 starts from the verified r_star, Sec. 3.7 worst case);
  * r_q is the end of chain q/K - 1: the incoming configuration at the first
    failed check, or the end of the last chain when every check passes.

The dynamic choice of K that the paper's outlook proposes (Sec. 5) is an
optional rule next_k(K, checks) -> K for the next round; adaptive_k is the
one read here.  Every round's chains still start from the verified r_star
and every accepted step is checked, so the accepted trajectory is the same
for any K sequence; only the number of rounds and computed steps change.

The operators are passed in, so the same procedure serves mocked equality
outcomes (index arithmetic tests) and real minimisations (oracle FIRE).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Any, Callable, List


@dataclass
class Round:
    start: int               # N_current at the start of the round
    chains: int              # P' chains run
    lengths: List[int]       # fine steps of each chain
    checks: List[bool]       # outcomes of the checks at i = 1 .. evaluated
    q: int                   # accepted steps
    K: int = 0               # chain length of the round


@dataclass
class Result:
    r_star: Any
    n_current: int
    rounds: List[Round] = field(default_factory=list)
    computed_steps: int = 0  # fine steps computed over all chains (accepted or not)


def chain_plan(remaining: int, K: int, P: int) -> List[int]:
    """Fine-step counts of the chains of one round (last round clamped)."""
    if remaining >= P * K:
        return [K] * P
    p = math.ceil(remaining / K)
    return [K] * (p - 1) + [remaining - (p - 1) * K]


def adaptive_k(K: int, checks: List[bool], k_min: int, k_max: int) -> int:
    """Chain length of the next round (the reading of the dynamic choice of
    K): twice K after a round whose every check passed (longer chains lose
    nothing while the anchors keep agreeing), half of K rounded up after a
    round whose first check failed (anchors closer together), K otherwise;
    then clamped to [k_min, k_max].  A round with one chain made no check
    and keeps K."""
    if not checks:
        return K
    if all(checks):
        nxt = 2 * K
    elif not checks[0]:
        nxt = (K + 1) // 2
    else:
        nxt = K
    return min(k_max, max(k_min, nxt))


def aqs_parallel(r0: Any, n_steps: int, K: int, P: int,
                 level1: Callable[[Any, int], Any],
                 level2: Callable[[List[Any], List[int]], List[tuple]],
                 equal: Callable[[Any, Any], bool],
                 next_k: Callable[[int, List[bool]], int] | None = None) -> Result:
    """Algorithm 1 (with next_k: K chosen anew after every round).

    level1(r_star, m)       -> anchor F_N^(m dgamma) r_star (m = i K fine steps)
    level2(anchors, lengths)-> for each anchor i, (outgoing_i, end_i): the
                               minimised anchor and the end of its chain of
                               lengths[i] fine AQS steps (run "in parallel")
    equal(a, b)             -> the equality test of Eq. (20)
    """
    if P < 2:
        raise ValueError("Algorithm 1 needs P >= 2 threads (Sec. 3.2)")
    if K < 1:
        raise ValueError("K must be >= 1")
    n_cur = 0
    r_star = r0
    res = Result(r_star, 0)
    while n_cur < n_steps:
        lengths = chain_plan(n_steps - n_cur, K, P)
        anchors = [level1(r_star, i * K) for i in range(len(lengths))]
        out = level2(anchors, lengths)
        res.computed_steps += sum(lengths)
        q = lengths[0]
        r_q = out[0][1]
        checks = []
        for i in range(1, len(lengths)):
            ok = bool(equal(out[i - 1][1], out[i][0]))
            checks.append(ok)
            if ok:
                q = i * K + lengths[i]
                r_q = out[i][1]
            else:
                q = i * K
                r_q = out[i - 1][1]
                break
        res.rounds.append(Round(n_cur, len(lengths), lengths, checks, q, K))
        r_star = r_q
        n_cur += q
        if next_k is not None:
            K = next_k(K, checks)
            if K < 1:
                raise ValueError("K must be >= 1")
    res.r_star = r_star
    res.n_current = n_cur
    return res


def aqs_sequential(r0: Any, n_steps: int, step: Callable[[Any, int], Any]) -> list:
    """Conventional AQS, Eq. (12): r_k = (F o F_N^(dgamma))(r_{k-1});
    step(r, k) returns r_k from r_{k-1}.  Returns [r_0, r_1, ..., r_n]."""
    traj = [r0]
    r = r0
    for k in range(1, n_steps + 1):
        r = step(r, k)
        traj.append(r)
    return traj
