"""The parallel stepping scheme of the paper (Algorithm 1, Sec. 3.5) in plain
Python -- TEST INFRASTRUCTURE ONLY (imported by the tests, never by the
GPU library).

What it computes.  A round starts from a verified inherent structure at
strain step n.  Chain i of the round (i = 0 .. P-1) starts from that
structure mapped affinely by i K fine increments in one product (the
level-I guess, Eq. 18), is minimised (its "first" structure), and then takes
its own K fine AQS steps (level II, Eq. 19).  The chains form links: chain
i continues chain i-1 exactly when the end of chain i-1 and the first
structure of chain i are the same inherent structure (Eq. 20).  The round
keeps the longest run of chains 0, 1, ... whose links all hold -- chain 0
always, since it starts from the verified structure -- so it accepts the
steps of that prefix of chains, and the end of the prefix's last chain is
the next round's verified structure.  Rounds repeat until the requested
number of steps is accepted.

Readings where the paper is silent:
  * near the end, with R < P K steps left, a round runs only ceil(R / K)
    chains and the last of them takes the remaining R - (ceil(R/K) - 1) K
    steps, so the total need not be a multiple of K;
  * a round with a single chain has no link to test and accepts its steps;
  * links are tested in chain order and the first broken link ends the
    prefix: later links are not needed.

The dynamic choice of K that the paper's outlook proposes (Sec. 5) is an
optional rule next_k(K, links) -> K for the next round; adaptive_k is the
one read here.  Every round still starts from the verified structure and
every accepted step belongs to a tested prefix, so the accepted trajectory
does not depend on the K sequence; only rounds and computed steps do.

The dynamic step sizing of the same outlook is read as a dyadic ladder
(aqs_parallel_dyadic): a round runs at level m, its strain increment
2^m dgamma, with dgamma the finest; strain is counted in fine increments and
a level-m round starts on a multiple of 2^m.  A plastic event shows as a
shear stress below the previous step's, as energy released within a step
(on an elastic branch dE/dgamma = V sigma_xy, so a step's energy change is
the trapezoidal work V h dgamma (sigma_(j-1) + sigma_j) / 2 up to third
order in the step; an event falls short of it), or as a broken link (the
anchor lands elsewhere than the chain before it).  A round at level m > 0 keeps its
chains only up to the first one that holds an event; the level is then 0
until the accepted strain has passed the end of that chain, so events are
always stepped through at the finest increment.  Otherwise a round without
an event raises the level by one (up to
m_max, and only as far as the strain reached is a multiple of); a round at
level 0 with an event stays at level 0.  So that the level can rise, a round
below m_max that would end on an odd multiple of its increment gives its
last chain one increment fewer (drops that chain if it has only one), unless
the round reaches the target strain.  In elastic stretches the coarse
steps reach the same inherent structures as the fine ones (adiabatic
continuation), which the glass test below checks against conventional AQS.

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
    """Rounds of the parallel scheme until n_steps are accepted (with
    next_k: K chosen anew after every round).

    level1(r, m)            -> the affine guess F_N^(m dgamma) r (m fine steps
                               in one product)
    level2(starts, lengths) -> per chain, (first, end): the minimised start
                               and the end of its chain of lengths[i] fine
                               AQS steps (the chains are independent)
    equal(a, b)             -> the equality test of Eq. (20)
    """
    if P < 2:
        raise ValueError("the parallel scheme needs P >= 2 chains (Sec. 3.2)")
    if K < 1:
        raise ValueError("K must be >= 1")
    verified, done = r0, 0
    res = Result(r0, 0)
    while done < n_steps:
        lengths = chain_plan(n_steps - done, K, P)
        guesses = [level1(verified, i * K) for i in range(len(lengths))]
        chains = level2(guesses, lengths)
        res.computed_steps += sum(lengths)
        links = accepted_links(chains, equal)
        kept = len(links) + 1 if all(links) else len(links)
        accepted = sum(lengths[:kept])
        res.rounds.append(Round(done, len(lengths), lengths, links, accepted, K))
        verified = chains[kept - 1][1]
        done += accepted
        if next_k is not None:
            K = next_k(K, links)
            if K < 1:
                raise ValueError("K must be >= 1")
    res.r_star = verified
    res.n_current = done
    return res


def accepted_links(chains: List[tuple], equal: Callable[[Any, Any], bool]) -> List[bool]:
    """Outcomes of the links between consecutive chains, in chain order, up
    to and including the first broken one: link i holds when the end of
    chain i-1 equals the first structure of chain i."""
    links = []
    for prev, cur in zip(chains, chains[1:]):
        links.append(bool(equal(prev[1], cur[0])))
        if not links[-1]:
            break
    return links


def aqs_sequential(r0: Any, n_steps: int, step: Callable[[Any, int], Any]) -> list:
    """Conventional AQS, Eq. (12): r_k = (F o F_N^(dgamma))(r_{k-1});
    step(r, k) returns r_k from r_{k-1}.  Returns [r_0, r_1, ..., r_n]."""
    traj = [r0]
    r = r0
    for k in range(1, n_steps + 1):
        r = step(r, k)
        traj.append(r)
    return traj


@dataclass
class DyadicRound:
    start: int               # fine steps accepted before the round
    level: int               # the round's increment is 2^level fine increments
    lengths: List[int]       # increments of each chain at that level
    checks: List[bool]       # outcomes of the links evaluated
    q: int                   # fine steps accepted
    cut: bool                # kept chains cut before a plastic event (level > 0)


@dataclass
class DyadicResult:
    r_star: Any
    n_current: int
    rounds: List[DyadicRound] = field(default_factory=list)
    computed_steps: int = 0  # minimised increments over all chains (any level)


def has_event(stress: List[float], energy: List[float] | None = None, work: float | None = None,
              tol: float | None = None) -> bool:
    """A plastic event within one chain (entry 0 is the chain's first,
    minimised structure, entry j the structure after step j): some step's
    shear stress is below the one before; or, given the energies, the
    volume times the step's strain `work` and `tol`, some step's energy
    change E_j - E_(j-1) falls below the trapezoidal work
    work (s_(j-1) + s_j) / 2 by more than tol work (|s_(j-1)| + |s_j|) / 2."""
    for j in range(1, len(stress)):
        if stress[j] < stress[j - 1]:
            return True
        if energy is not None and tol is not None:
            w = work * (stress[j - 1] + stress[j]) / 2.0
            scale = work * (abs(stress[j - 1]) + abs(stress[j])) / 2.0
            if energy[j] - energy[j - 1] < w - tol * scale:
                return True
    return False


def aqs_parallel_dyadic(r0: Any, n_steps: int, K: int, P: int, m_max: int,
                        level1: Callable[[Any, int, int], Any],
                        level2: Callable[[List[Any], List[int], int], List[tuple]],
                        equal: Callable[[Any, Any], bool], v_dgamma: float | None = None,
                        event_tol: float | None = None) -> DyadicResult:
    """Rounds of the parallel scheme with the dyadic step sizing read above,
    until n_steps fine increments are accepted.

    level1(r, m, h)            -> F_N^(m h dgamma) r in one product
    level2(starts, lengths, h) -> per chain (first, end, stress[, energy]):
                                  lengths[i] AQS steps of h fine increments
                                  each after the first minimisation; stress[j]
                                  and energy[j] after step j (entry 0: first)
    equal(a, b)                -> the equality test of Eq. (20)
    v_dgamma, event_tol        -> volume times dgamma, and the tolerance of
                                  the energy balance (has_event); None: the
                                  stress drop alone marks events
    With m_max = 0 every round is level 0 and the rounds are those of
    aqs_parallel with the same K and P."""
    if P < 2:
        raise ValueError("the parallel scheme needs P >= 2 chains (Sec. 3.2)")
    if K < 1 or m_max < 0:
        raise ValueError("K must be >= 1 and m_max >= 0")
    verified, done, m = r0, 0, 0
    hold = 0                                 # level 0 until the strain passes this
    res = DyadicResult(r0, 0)
    while done < n_steps:
        while n_steps - done < (1 << m):     # do not overshoot the target strain
            m -= 1
        h = 1 << m
        lengths = chain_plan((n_steps - done) // h, K, P)
        ends_odd = (done // h + sum(lengths)) % 2 == 1
        if m < m_max and ends_odd and done + sum(lengths) * h < n_steps:
            if lengths[-1] > 1:
                lengths[-1] -= 1
            elif len(lengths) > 1:
                lengths.pop()
        chains = level2([level1(verified, i * K, h) for i in range(len(lengths))], lengths, h)
        res.computed_steps += sum(lengths)
        links = accepted_links(chains, equal)
        kept = len(links) + 1 if all(links) else len(links)
        # chains of the kept prefix holding an event; a broken link after
        # chain c means chain c crossed one
        marked = [c for c in range(kept)
                  if has_event(chains[c][2], chains[c][3] if len(chains[c]) > 3 else None,
                               None if v_dgamma is None else v_dgamma * h, event_tol)]
        if kept < len(lengths):
            marked.append(kept - 1)
        cut = m > 0 and bool(marked)
        if cut:
            kept = min(marked)
            hold = done + sum(lengths[:kept + 1]) * h
        q = sum(lengths[:kept]) * h
        res.rounds.append(DyadicRound(done, m, lengths, links, q, cut))
        if kept > 0:
            verified = chains[kept - 1][1]
        done += q
        nxt = 0 if marked or done < hold else min(m + 1, m_max)
        while nxt > 0 and done % (1 << nxt):
            nxt -= 1
        m = nxt
    res.r_star = verified
    res.n_current = done
    return res
