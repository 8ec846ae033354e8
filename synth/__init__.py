"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the method: it only draws candidate sets,
supports, coefficients, lattice sizes, generating vectors and sample noise, with
the shapes and distributions of the paper's synthetic workloads (Section 4:
random candidate sets, random sparse polynomials on the cube [-N, N]^d, random
lattices with prime sizes).  Every workload is seed-driven.

Large candidate sets are drawn with a counter-based generator (``counter``), so a
sampled candidate can be regenerated on its own on the host while the full set is
generated on the device.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import counter  # noqa: F401


def primes_in(lo: int, hi: int) -> np.ndarray:
    """All primes p with lo <= p <= hi (sieve)."""
    hi = int(hi)
    sieve = np.ones(hi + 1, bool)
    sieve[:2] = False
    for q in range(2, int(math.isqrt(hi)) + 1):
        if sieve[q]:
            sieve[q * q::q] = False
    p = np.nonzero(sieve)[0]
    return p[p >= lo].astype(np.int64)


def next_prime_above(x: float) -> int:
    """Smallest prime strictly greater than x."""
    n = int(math.floor(x)) + 1
    while True:
        if n >= 2 and all(n % q for q in range(2, int(math.isqrt(n)) + 1)):
            return n
        n += 1


def distinct_uniform_points(rng, n: int, d: int, lo: int, hi: int) -> np.ndarray:
    """n distinct points uniform in [lo, hi]^d, returned SoA [d, n] int64 (draw order)."""
    span = hi - lo + 1
    out = np.empty((0, d), np.int64)
    seen = set()
    while out.shape[0] < n:
        need = n - out.shape[0]
        cand = rng.integers(lo, hi + 1, size=(need + need // 8 + 16, d), dtype=np.int64)
        keep = []
        for row in cand:
            key = row.tobytes()
            if key not in seen:
                seen.add(key)
                keep.append(row)
                if len(keep) == need:
                    break
        out = np.concatenate([out, np.array(keep, np.int64).reshape(-1, d)])
    assert span ** d >= n
    return np.ascontiguousarray(out.T)


@dataclass
class Problem:
    """One function instance: candidates, true support, coefficients, lattices."""
    d: int
    cand: np.ndarray          # [d, n] int64 candidate set Gamma
    supp_idx: np.ndarray      # indices of the true support I inside Gamma
    coef: np.ndarray          # complex128 [s] coefficients of the support
    M: np.ndarray             # [L] int64 prime lattice sizes
    z: np.ndarray             # [L, d] int64 generating vectors
    theta: float
    noise: np.ndarray | None = None   # complex128 [sum M] additive sample noise or None
    meta: dict = field(default_factory=dict)

    @property
    def supp(self) -> np.ndarray:
        return np.ascontiguousarray(self.cand[:, self.supp_idx])

    @property
    def L(self) -> int:
        return int(self.M.shape[0])

    @property
    def n(self) -> int:
        return int(self.cand.shape[1])


def draw_lattices(rng, L: int, d: int, plo: int, phi: int, distinct: bool = True):
    """L primes uniform over the primes in [plo, phi] (distinct when possible) and
    generating vectors z_l uniform in [0, M_l)^d."""
    P = primes_in(plo, phi)
    if distinct and P.shape[0] >= L:
        M = rng.choice(P, size=L, replace=False)
    else:
        M = rng.choice(P, size=L, replace=True)
    M = M.astype(np.int64)
    z = np.stack([rng.integers(0, m, size=d, dtype=np.int64) for m in M])
    return M, z


def small_config(seed: int, d=5, n=2000, s=20, box=32, L=5, mlo=None, mhi=None) -> Problem:
    """Plain method, small: d = 5, 2000 distinct candidates in [-32, 32]^5, s = 20
    support drawn from the candidates, N(0,1) complex coefficients, L = 5 lattices with
    distinct primes in [8s, 16s], noise-free, theta = 1e-12."""
    rng = np.random.default_rng(1_000_003 * 1 + seed)
    cand = distinct_uniform_points(rng, n, d, -box, box)
    supp_idx = np.sort(rng.choice(n, size=s, replace=False)).astype(np.int64)
    coef = rng.standard_normal(s) + 1j * rng.standard_normal(s)
    M, z = draw_lattices(rng, L, d, mlo or 8 * s, mhi or 16 * s)
    return Problem(d, cand, supp_idx, coef, M, z, theta=1e-12,
                   meta=dict(workload="small", seed=seed))


def mid_config(seed: int, d=10, n=100_000, s=100, box=64, L=10) -> Problem:
    """Plain method, mid: d = 10, 1e5 candidates uniform in [-64, 64]^10, s = 100,
    |c| ~ U[1, 10] with uniform phase, L = 10 primes in [8s, 16s], complex Gaussian
    sample noise at 40 dB SNR per lattice, theta = 1/3."""
    rng = np.random.default_rng(1_000_003 * 2 + seed)
    cand = distinct_uniform_points(rng, n, d, -box, box)
    supp_idx = np.sort(rng.choice(n, size=s, replace=False)).astype(np.int64)
    mag = rng.uniform(1.0, 10.0, s)
    ph = rng.uniform(0.0, 2 * np.pi, s)
    coef = mag * np.exp(1j * ph)
    M, z = draw_lattices(rng, L, d, 8 * s, 16 * s)
    return Problem(d, cand, supp_idx, coef, M, z, theta=1.0 / 3.0,
                   meta=dict(workload="mid", seed=seed, snr_db=40.0,
                             noise_seed=1_000_003 * 2 + seed + 7))


def noise_for(samples_clean: np.ndarray, M: np.ndarray, snr_db: float, seed: int) -> np.ndarray:
    """Additive complex Gaussian noise per lattice with E|eta|^2 = ||f_l||^2 / (M_l 10^(snr/10)),
    split equally between real and imaginary parts."""
    rng = np.random.default_rng(seed)
    out = np.zeros_like(samples_clean)
    off = 0
    for m in M:
        m = int(m)
        fl = samples_clean[off:off + m]
        p = float(np.sum(np.abs(fl) ** 2)) / m / (10.0 ** (snr_db / 10.0))
        sd = math.sqrt(p / 2.0)
        out[off:off + m] = sd * rng.standard_normal(m) + 1j * sd * rng.standard_normal(m)
        off += m
    return out


def batch_config(seed: int, nfunc=512, d=10, box=128, L=8, slo=10, shi=1000, nlo=1000,
                 nhi=1_000_000, scale=1.0):
    """Batched workload: nfunc functions with s log-uniform in [10, 1000] and |Gamma|
    log-uniform in [1e3, 1e6] from [-128, 128]^10, L = 8 lattices with distinct primes
    in [8s, 16s], N(0,1) complex coefficients, noise-free, theta = 1e-12.  ``scale``
    shrinks |Gamma| (for tests)."""
    rng = np.random.default_rng(1_000_003 * 4 + seed)
    probs = []
    for f in range(nfunc):
        s = int(round(math.exp(rng.uniform(math.log(slo), math.log(shi)))))
        n = int(round(math.exp(rng.uniform(math.log(nlo), math.log(nhi))) * scale))
        n = max(n, s)
        cand = rng.integers(-box, box + 1, size=(d, n), dtype=np.int64)
        supp_idx = np.sort(rng.choice(n, size=s, replace=False)).astype(np.int64)
        coef = rng.standard_normal(s) + 1j * rng.standard_normal(s)
        M, z = draw_lattices(rng, L, d, 8 * s, 16 * s)
        probs.append(Problem(d, cand, supp_idx, coef, M, z, theta=1e-12,
                             meta=dict(workload="batch", seed=seed, func=f)))
    return probs


def sparse_poly_box(seed: int, d=25, s=200, box=32):
    """Random sparse polynomial on [-N, N]^d: s distinct frequencies uniform in the box,
    complex N(0,1) coefficients (the dimension-incremental workload; the box is never
    enumerated)."""
    rng = np.random.default_rng(1_000_003 * 3 + seed)
    freq = distinct_uniform_points(rng, s, d, -box, box)
    coef = rng.standard_normal(s) + 1j * rng.standard_normal(s)
    return freq, coef


def dirichlet(problem: Problem) -> Problem:
    """The same candidates and support with all-ones coefficients (eq. (4.1))."""
    return Problem(problem.d, problem.cand, problem.supp_idx,
                   np.ones(problem.supp_idx.shape[0], np.complex128), problem.M, problem.z,
                   theta=0.5, meta=dict(problem.meta, dirichlet=True))


# ----------------------------------------------------------------------------- Section 4.1 sets
def hyperbolic_cross(d: int, bound: float, weight_exp: float | None = None) -> np.ndarray:
    """{k in Z^d : prod_t max(1, w_t |k_t|) <= bound} as SoA int64 [d, n], with
    w_t = t^weight_exp (t = 1..d) for the weighted cross and w_t = 1 without
    weights (the sets of Section 4.1.3).  The product is accumulated left to
    right in float64; every factor is >= 1, so a partial product above the bound
    can be pruned."""
    prod = np.ones(1)
    rows = np.zeros((1, 0), np.int64)
    for t in range(1, d + 1):
        w = 1.0 if weight_exp is None else float(t) ** weight_exp
        # a superset of the admissible |k_t| per partial product, filtered exactly below
        kmax = np.floor(bound / (prod * w)).astype(np.int64) + 1
        nopt = 2 * kmax + 1
        rep = np.repeat(np.arange(prod.shape[0]), nopt)
        start = np.repeat(np.cumsum(nopt) - nopt, nopt)
        k = np.arange(rep.shape[0], dtype=np.int64) - start - np.repeat(kmax, nopt)
        p = prod[rep] * np.maximum(1.0, w * np.abs(k))
        ok = p <= bound
        rep, k, prod = rep[ok], k[ok], p[ok]
        rows = np.concatenate([rows[rep], k[:, None]], axis=1)
    return np.ascontiguousarray(rows.T)


def support_first(gamma: np.ndarray, member: np.ndarray) -> tuple[np.ndarray, int]:
    """Reorder a candidate set so that the members of the support come first (in their
    original order) -> (reordered set, support size)."""
    member = np.asarray(member, bool)
    order = np.concatenate([np.nonzero(member)[0], np.nonzero(~member)[0]])
    return np.ascontiguousarray(gamma[:, order]), int(member.sum())


def weighted_cross_member(gamma: np.ndarray, bound: float, weight_exp: float) -> np.ndarray:
    """Membership of the columns of gamma in the weighted hyperbolic cross (same product
    order as hyperbolic_cross)."""
    prod = np.ones(gamma.shape[1])
    for t in range(1, gamma.shape[0] + 1):
        prod = prod * np.maximum(1.0, float(t) ** weight_exp * np.abs(gamma[t - 1]))
    return prod <= bound
