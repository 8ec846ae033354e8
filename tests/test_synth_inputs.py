"""The seeded input generators behind the Section 4.1 workloads: distinct random
points of a grid (Gamma uniformly at random, I uniformly at random inside it)."""
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
