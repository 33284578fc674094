"""The paper's benchmark problem (Sec. 2.2) as set up for the speed-up runs:
potential and sample composition against the values the paper prints
(tests/golden/paper_values.txt); a short speed-up run on the GPU."""
import math
import os

import numpy as np
import pytest

import aqs_synth as S

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    out = {}
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, *v = line.split()
            out[k] = v
    return out


def _num(expr: str) -> float:
    return float(eval(expr, {"sin": math.sin, "sqrt": math.sqrt, "pi": math.pi}))


def test_paper_potential_and_sample_match_the_printed_values():
    from paper_2507_20802_amd import speedup
    g = golden("paper_values.txt")
    p = speedup.paper_potential()
    assert p.sigma[0][0] == pytest.approx(_num(g["sigma_SS"][0]), rel=1e-15)
    assert p.sigma[1][1] == pytest.approx(_num(g["sigma_LL"][0]), rel=1e-15)
    assert p.sigma[0][1] == p.sigma[1][0] == _num(g["sigma_SL"][0])
    assert p.eps[0][0] == _num(g["eps_SS"][0]) and p.eps[1][1] == _num(g["eps_LL"][0])
    assert p.eps[0][1] == p.eps[1][0] == _num(g["eps_SL"][0])
    assert speedup.DGAMMA == _num(g["dgamma"][0]) and speedup.N_STEPS == int(g["n_steps"][0])
    s = S.paper_sample_start(21, 0)
    n_s, n_l = int((s.types == 0).sum()), int((s.types == 1).sum())
    assert s.n == int(g["n_atoms"][0]) and s.L == pytest.approx(float(g["box_side"][0]))
    # the integer split closest to the golden-mean ratio
    r = _num(g["ratio_LS"][0])
    best = min(range(1, s.n), key=lambda k: abs(k / (s.n - k) - r))
    assert n_l == best and n_s == s.n - best
    assert np.all((s.pos >= 0) & (s.pos < s.L))


@pytest.mark.gpu
def test_short_speedup_run_keeps_the_sequential_trajectory():
    """Two samples, 12 steps: Algorithm 1 with live checks and without ends in
    the configuration of the sequential AQS run (Eq. 20) for every (P, K)."""
    from paper_2507_20802_amd import speedup
    for live in (True, False):
        res = speedup.speedups(range(2), [4], [2, 3], n_steps=12, live=live)
        for row in res["table"]:
            assert row["final_equal"] == row["samples"] == 2
            assert row["mu"] > 0.0 and math.isfinite(row["sigma"])


@pytest.mark.gpu
def test_short_speedup_run_with_the_papers_minimiser():
    """The same protocol with conjugate gradients (the paper's minimiser):
    Algorithm 1 still ends in the sequential run's configuration."""
    from paper_2507_20802_amd import speedup
    res = speedup.speedups(range(2), [4], [3], n_steps=12, live=True, minimizer="cg")
    assert res["minimizer"] == "cg"
    for row in res["table"]:
        assert row["final_equal"] == row["samples"] == 2


@pytest.mark.gpu
def test_small_workload_runner():
    """The runner of the other workloads, on its smallest one (a few steps)."""
    from paper_2507_20802_amd import configs
    out = configs.small(steps=5)
    assert out["all_converged"] and out["aqs_steps_per_s"] > 0.0


@pytest.mark.gpu
def test_paper_problem_batched_over_samples():
    """Samples of the paper's problem in one batch: each converges, and the
    first one's record equals its run alone bit for bit."""
    from paper_2507_20802_amd import configs
    out = configs.paper(samples=8, steps=4)
    assert out["all_converged"] and out["sample0_same_as_alone"]
