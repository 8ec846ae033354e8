"""Counter-based input generator for large candidate sets.

SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): output n >= 1 from seed S is
mix(S + n * 0x9E3779B97F4A7C15) with the published 64-bit finaliser.  Written with
torch int64 tensor ops (wrap-around multiply, emulated logical shifts), so the same
function runs on the device (generating tens of GB in milliseconds) and on the host
(regenerating any candidate on its own).  Pure input generation: no arithmetic of
the method lives here.
"""
from __future__ import annotations

import math

import numpy as np
import torch

_GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_MASK64 = (1 << 64) - 1


def _s64(x: int) -> int:
    """Two's complement reinterpretation of a 64-bit unsigned constant."""
    x &= _MASK64
    return x - (1 << 64) if x >= (1 << 63) else x


def _lsr(x: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of an int64 tensor."""
    return (x >> k) & ((1 << (64 - k)) - 1)


def splitmix64(seed: int, n: torch.Tensor) -> torch.Tensor:
    """SplitMix64 outputs for counters n (int64 tensor), as int64 bit patterns."""
    x = n * _s64(_GAMMA) + _s64(seed)
    x = (x ^ _lsr(x, 30)) * _s64(_M1)
    x = (x ^ _lsr(x, 27)) * _s64(_M2)
    return x ^ _lsr(x, 31)


def splitmix64_py(seed: int, n: int) -> int:
    """Big-integer statement of the same function (for checking the tensor version)."""
    x = (seed + n * _GAMMA) & _MASK64
    x = ((x ^ (x >> 30)) * _M1) & _MASK64
    x = ((x ^ (x >> 27)) * _M2) & _MASK64
    return x ^ (x >> 31)


def uniform_int(seed: int, n: torch.Tensor, lo: int, hi: int) -> torch.Tensor:
    """Integer in [lo, hi] from the top 53 bits of the counter's output."""
    x = _lsr(splitmix64(seed, n), 11)
    return x % (hi - lo + 1) + lo


def candidates(seed: int, func: int, d: int, n: int, box: int, device="cpu",
               start: int = 0, count: int | None = None) -> torch.Tensor:
    """Candidates start..start+count-1 of function ``func``: SoA int64 [d, count] uniform
    in [-box, box]^d.  Candidate i, coordinate u uses counter
    ((func * 64 + u) << 36) + i + 1."""
    count = n - start if count is None else count
    i = torch.arange(start, start + count, dtype=torch.int64, device=device)
    rows = []
    for u in range(d):
        base = ((func * 64 + u) << 36) + 1
        rows.append(uniform_int(seed, i + base, -box, box))
    return torch.stack(rows)


_PHASE_BITS = 16


def phase_table(device="cpu") -> torch.Tensor:
    """Unit phases e^{2 pi i m / 2^16}, m < 2^16, complex128 (built in numpy on the host,
    so device and host use bit-identical values)."""
    m = np.arange(1 << _PHASE_BITS, dtype=np.float64)
    ang = 2.0 * math.pi * m / float(1 << _PHASE_BITS)
    tab = np.cos(ang) + 1j * np.sin(ang)
    return torch.from_numpy(tab).to(device)


def compressible_coefs(seed: int, func: int, cand: torch.Tensor, table: torch.Tensor,
                       start: int = 0) -> torch.Tensor:
    """c_k = (1 + ||k||_1)^-2 times a unit phase drawn from the phase table.  The
    magnitude uses only exact integer work and one correctly rounded division, so host
    and device agree bit for bit."""
    n = cand.shape[1]
    i = torch.arange(start, start + n, dtype=torch.int64, device=cand.device)
    base = ((func * 64 + 63) << 36) + 1
    m = _lsr(splitmix64(seed, i + base), 64 - _PHASE_BITS)
    l1 = cand.abs().sum(0) + 1
    mag = 1.0 / (l1 * l1).to(torch.float64)
    return mag * table[m]


def dominant_indices(seed: int, func: int, n: int, count: int) -> np.ndarray:
    """``count`` distinct indices uniform in [0, n) (ascending)."""
    rng = np.random.default_rng([seed & 0xFFFFFFFF, func, 17])
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)


def dominant_phases(seed: int, func: int, count: int) -> np.ndarray:
    rng = np.random.default_rng([seed & 0xFFFFFFFF, func, 18])
    m = rng.integers(0, 1 << _PHASE_BITS, size=count)
    ang = 2.0 * math.pi * m.astype(np.float64) / float(1 << _PHASE_BITS)
    return np.cos(ang) + 1j * np.sin(ang)


# ----------------------------------------------------------------------------- distinct points
def _feistel(x: torch.Tensor, keys, h: int) -> torch.Tensor:
    """Balanced Feistel network on 2h-bit integers (a bijection of [0, 2^(2h)))."""
    mask = (1 << h) - 1
    lo, hi = x & mask, _lsr(x, h) & mask
    for k in keys:
        lo, hi = hi ^ (splitmix64(k, lo + 1) & mask), lo
    return (hi << h) | lo


def distinct_grid_points(seed: int, n: int, d: int, box: int, device="cpu") -> torch.Tensor:
    """n distinct points of {-box..box}^d, uniformly at random and in random order (so
    the first s of them are a uniform s-subset), SoA int64 [d, n].  Point i is the
    image of i under a keyed Feistel permutation of [0, 2^(2h)) (cycle-walked into
    [0, (2 box + 1)^d)), written in base 2 box + 1."""
    base = 2 * box + 1
    D = base ** d
    if n > D:
        raise ValueError("more points than the grid holds")
    h = 1
    while (1 << (2 * h)) < D:
        h += 1
    if 2 * h > 62:
        raise ValueError("grid too large for the 62-bit permutation")
    keys = [splitmix64_py(seed, 1000 + r) & ((1 << 63) - 1) for r in range(4)]
    y = _feistel(torch.arange(n, dtype=torch.int64, device=device), keys, h)
    idx = torch.nonzero(y >= D).squeeze(1)
    while idx.numel():   # cycle-walking: iterate the permutation until the value is in range
        v = _feistel(y[idx], keys, h)
        y[idx] = v
        idx = idx[v >= D]
    rows = []
    for _ in range(d):
        rows.append(y % base - box)
        y = y // base
    return torch.stack(rows[::-1])
