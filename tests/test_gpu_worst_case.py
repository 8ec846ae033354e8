"""Worst-case aliasing experiments of Section 4.1 (Table 4.1) on the GPU.

The HIP path (bucket sampler, lattice DFTs, extraction with Remark 2.9 and the
PFP/PFN count, through the C ABI) is compared with the oracle's classification,
which counts aliases directly: exact integer counts per function, on small
configurations with heavy aliasing, on a truncated detected list, and at the full
sizes of the paper's two experiments.  The success rates of a few hundred
repetitions are compared with the rates the paper prints, within binomial
tolerances.
"""
import json
import math
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def m():
    import paper_2006_13053_amd as mod
    mod.lib()
    torch.cuda.set_device(0)
    return mod


@pytest.fixture(scope="module")
def wc(m):
    from paper_2006_13053_amd import worst_case
    return worst_case


def dev():
    return torch.device("cuda", 0)


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def _batch_inputs(sets, na):
    """Concatenate F candidate sets (support first) into the run's device arguments."""
    F = len(sets)
    cand = np.concatenate(sets, axis=1)
    off = np.concatenate([[0], np.cumsum([s.shape[1] for s in sets])]).astype(np.int64)
    terms = np.concatenate([s[:, :k] for s, k in zip(sets, na)], axis=1)
    toff = np.concatenate([[0], np.cumsum(na)]).astype(np.int64)
    return T(cand), T(off), T(np.asarray(na, np.int64)), T(terms), T(toff), F


@pytest.mark.parametrize("seed,L,F", [(1, 5, 3), (2, 6, 2), (3, 7, 4), (4, 9, 1), (5, 4, 3)])
def test_counts_match_oracle_heavy_aliasing(m, wc, seed, L, F):
    say("worst case small", seed, L, F)
    rng = np.random.default_rng(seed)
    d, M = 3, int(rng.choice(synth.primes_in(41, 97)))
    sets, na = [], []
    for f in range(F):
        n = int(rng.integers(150, 400))
        sets.append(synth.distinct_uniform_points(rng, n, d, -20, 20))
        na.append(int(rng.integers(5, 30)))
    z = rng.integers(0, M, size=(F * L, d))
    run = wc.CountingRun(d, F, L, M, z, cap=1024)
    cand, off, n_act, terms, toff, _ = _batch_inputs(sets, na)
    got = run.run(cand, off, n_act, terms, toff).cpu().numpy()
    run.close()
    for f in range(F):
        cls = oracle.pfpn(sets[f], na[f], np.full(L, M), z[f * L:(f + 1) * L])
        want = oracle.pfpn_counts(cls)
        assert tuple(int(v) for v in got[f, :3]) == want, (f, got[f], want)
        assert int(got[f, 3]) == 0


def test_truncated_list_keeps_exact_pfp(m, wc):
    say("worst case truncated")
    rng = np.random.default_rng(8)
    d, L, M = 3, 5, 43
    s = synth.distinct_uniform_points(rng, 600, d, -20, 20)
    z = rng.integers(0, M, size=(L, d))
    cls = oracle.pfpn(s, 30, np.full(L, M), z)
    pfp, pfn, _ = oracle.pfpn_counts(cls)
    assert 30 + pfp > 60
    run = wc.CountingRun(d, 1, L, M, z, cap=60)
    cand, off, n_act, terms, toff, _ = _batch_inputs([s], [30])
    got = run.run(cand, off, n_act, terms, toff).cpu().numpy()[0]
    run.close()
    # the kept entries are a subset of the detected set: PFP stays exact, PFN a lower bound
    assert int(got[0]) == pfp and int(got[1]) <= pfn and int(got[3]) == 1


@pytest.mark.parametrize("L", [21, 13])
def test_full_size_random_3d_matches_oracle(m, wc, L):
    """Section 4.1.2 at full size: |Gamma| = 10^7 in [-1000, 1000]^3, |I| = 1000,
    M = 10331; two repetitions, exact counts against the oracle."""
    import bench
    say("worst case random 3d full size", L)
    res, _, _ = bench.worst_case_random_3d(m, torch, Ls=(L,), reps=2, batch=2, seed=77)
    import synth.counter as sc
    rng = np.random.default_rng(77)
    z = rng.integers(0, 10331, size=(L, 3))
    for rep in range(2):
        g = sc.distinct_grid_points(77 * 1_000_003 + rep, 10_000_000, 3, 1000).numpy()
        want = oracle.pfpn_counts(oracle.pfpn(g, 1000, np.full(L, 10331), z))
        say("rep", rep, "gpu", res[L][rep].tolist(), "oracle", want)
        assert tuple(int(v) for v in res[L][rep, :3]) == want
        assert int(res[L][rep, 3]) == 0


def test_full_size_hyperbolic_cross_matches_oracle(m, wc):
    """Section 4.1.3 at full size: the 8-d hyperbolic cross (|Gamma| = 10,665,297)
    with the weighted cross I (|I| = 1069) first, M = 11047, one lattice draw at
    L = 15, exact counts against the oracle."""
    import bench
    say("worst case hyperbolic cross full size")
    g, na = bench.cross_8d_set()
    assert g.shape[1] == 10_665_297 and na == 1069
    L = 15
    res, _, _ = bench.worst_case_cross_8d(m, torch, Ls=(L,), reps=1, batch=1, seed=91, gamma=(g, na))
    rng = np.random.default_rng(91)
    z = rng.integers(0, 11047, size=(L, 8))
    want = oracle.pfpn_counts(oracle.pfpn(g, na, np.full(L, 11047), z))
    say("gpu", res[L][0].tolist(), "oracle", want)
    assert tuple(int(v) for v in res[L][0, :3]) == want


def _gold():
    with open(os.path.join(ROOT, "tests", "golden", "worst_case_success_rates.json")) as fh:
        return json.load(fh)


def _within(rate, printed, reps):
    """Binomial band: 4.5 standard deviations of a rate near the printed one, plus
    the printed values' rounding and the spread between lattice draws (0.03)."""
    p = min(max(printed, 0.02), 0.98)
    return abs(rate - printed) <= 4.5 * math.sqrt(p * (1 - p) / reps) + 0.03


def test_success_rates_random_3d_match_paper(m, wc):
    """Success rates of Figures 4.1/4.2 at L where they change fastest."""
    import bench
    g = _gold()["random_3d"]
    reps = 160
    Ls = (11, 13, 23, 25, 27)
    res, gen_ms, run_ms = bench.worst_case_random_3d(m, torch, Ls=Ls, reps=reps, batch=16, seed=5)
    say("random 3d", reps, "reps", f"generation {gen_ms:.0f} ms, method {run_ms:.0f} ms")
    for L in Ls:
        s = wc.summarize(res[L])
        say("L", L, s)
        for key in ("median", "median_r1l", "pfp_le10", "pfp_le100"):
            if str(L) in g[key]:
                assert _within(s[key], g[key][str(L)], reps), (L, key, s[key], g[key][str(L)])


def test_success_rates_hyperbolic_cross_match_paper(m, wc):
    """Success rates of Figures 4.3/4.4 at L where they change fastest."""
    import bench
    g = _gold()["hyperbolic_cross_8d"]
    reps = 160
    Ls = (11, 21, 23, 25)
    res, gen_ms, run_ms = bench.worst_case_cross_8d(m, torch, Ls=Ls, reps=reps, batch=8, seed=7)
    say("cross 8d", reps, "reps", f"setup {gen_ms:.0f} ms, method {run_ms:.0f} ms")
    for L in Ls:
        s = wc.summarize(res[L])
        say("L", L, s)
        for key in ("median", "median_r1l", "pfp_le10", "pfp_le100"):
            if str(L) in g[key]:
                assert _within(s[key], g[key][str(L)], reps), (L, key, s[key], g[key][str(L)])
