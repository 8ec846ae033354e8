"""The seeded input generators behind the Section 4.1 workloads: distinct random
points of a grid (Gamma uniformly at random, I uniformly at random inside it)."""
import itertools
import math

import numpy as np
import torch

import synth
import synth.counter as sc


def _keys(g, box):
    base = 2 * box + 1
    k = torch.zeros(g.shape[1], dtype=torch.int64)
    for u in range(g.shape[0]):
        k = k * base + (g[u] + box)
    return k


def test_distinct_grid_points_are_distinct_in_range_and_deterministic():
    g = sc.distinct_grid_points(5, 200_000, 3, 1000)
    assert g.shape == (3, 200_000) and g.dtype == torch.int64
    assert int(g.min()) >= -1000 and int(g.max()) <= 1000
    assert torch.unique(_keys(g, 1000)).numel() == 200_000
    assert torch.equal(g, sc.distinct_grid_points(5, 200_000, 3, 1000))
    assert not torch.equal(g, sc.distinct_grid_points(6, 200_000, 3, 1000))
    # a prefix of the draw is the draw of the prefix (I = first |I| of Gamma)
    assert torch.equal(g[:, :1000], sc.distinct_grid_points(5, 1000, 3, 1000))


def test_distinct_grid_points_cover_the_whole_grid():
    for d, box in [(1, 50), (2, 30), (3, 6)]:
        n = (2 * box + 1) ** d
        g = sc.distinct_grid_points(11, n, d, box)
        assert torch.unique(_keys(g, box)).numel() == n


def test_distinct_grid_points_look_uniform():
    """Marginals and the first-position distribution of a uniform random subset:
    chi-square statistics per degree of freedom near 1."""
    g = sc.distinct_grid_points(3, 400_000, 3, 100)
    for u in range(3):
        h = torch.bincount(g[u] + 100, minlength=201).double()
        chi = float(((h - h.mean()) ** 2 / h.mean()).sum()) / 200
        assert 0.7 < chi < 1.35, (u, chi)
    # first point over many seeds: uniform over a small grid
    firsts = torch.stack([sc.distinct_grid_points(s, 1, 2, 3)[:, 0] for s in range(3000)], 1)
    h = torch.bincount(_keys(firsts, 3), minlength=49).double()
    chi = float(((h - h.mean()) ** 2 / h.mean()).sum()) / 48
    assert 0.6 < chi < 1.5


def test_support_first_reorders_stably():
    g = np.arange(20, dtype=np.int64).reshape(2, 10)
    member = np.array([0, 1, 0, 0, 1, 0, 1, 0, 0, 0], bool)
    r, n = synth.support_first(g, member)
    assert n == 3
    assert r[0].tolist() == [1, 4, 6, 0, 2, 3, 5, 7, 8, 9]


def test_hyperbolic_cross_sizes_printed_in_paper():
    """Section 4.1.3: |Gamma| = 10,665,297 for the unweighted cross (d = 8, bound 32) and
    |I| = 1069 for the weighted one (weights t^1.08); small cases by brute force."""
    g = synth.hyperbolic_cross(8, 32)
    assert g.shape == (8, 10_665_297)
    assert np.abs(g).max() == 32
    w = synth.hyperbolic_cross(8, 32, 1.08)
    assert w.shape == (8, 1069)
    assert synth.weighted_cross_member(g, 32, 1.08).sum() == 1069
    for d, N in [(1, 7), (2, 9), (3, 6)]:
        h = synth.hyperbolic_cross(d, N)
        brute = [k for k in itertools.product(range(-N, N + 1), repeat=d)
                 if math.prod(max(1, abs(v)) for v in k) <= N]
        assert sorted(map(tuple, h.T.tolist())) == sorted(brute)
