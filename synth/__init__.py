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


@dataclass
class BatchWorkload:
    """The batched workload at full size: F functions, function f with s[f] support
    terms among n[f] candidates (``candidates(f)``), L lattices of distinct primes in
    [8 s, 16 s].  Candidates come from the counter generator (uniform in the box, no
    de-duplication: two equal candidates in one set have probability < 1e-13)."""
    seed: int
    d: int
    L: int
    box: int
    s: np.ndarray             # [F] support sizes
    n: np.ndarray             # [F] candidate-set sizes
    M: np.ndarray             # [F*L] lattice sizes
    z: np.ndarray             # [F*L, d] generating vectors
    supp_idx: list            # F arrays of support positions inside each candidate set
    coef: list                # F complex128 coefficient arrays

    @property
    def F(self) -> int:
        return int(self.s.shape[0])

    @property
    def set_off(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.n)]).astype(np.int64)

    @property
    def term_off(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.s)]).astype(np.int64)

    def candidates(self, f: int, device="cpu"):
        """Candidate set of function f, SoA int64 [d, n[f]] (a torch tensor)."""
        return counter.candidates(self.seed, f, self.d, int(self.n[f]), self.box, device=device)


def batch_workload(seed: int = 2027, F: int = 512, d: int = 10, L: int = 8, box: int = 128,
                   slo: int = 10, shi: int = 1000, nlo: int = 1000, nhi: int = 1_000_000) -> BatchWorkload:
    """Batched workload: F functions, s log-uniform in [10, 1000], |Gamma| log-uniform in
    [1e3, 1e6] uniform in [-128, 128]^10, support at uniform random positions of the
    set, L = 8 distinct primes uniform in [8 s, 16 s] with uniform generating vectors,
    complex N(0,1) coefficients (noise-free)."""
    rng = np.random.default_rng(seed)
    s = np.rint(np.exp(rng.uniform(math.log(slo), math.log(shi), F))).astype(np.int64)
    n = np.rint(np.exp(rng.uniform(math.log(nlo), math.log(nhi), F))).astype(np.int64)
    n = np.maximum(n, s)
    Ms, zs, supp_idx = [], [], []
    for f in range(F):
        M, z = draw_lattices(rng, L, d, 8 * int(s[f]), 16 * int(s[f]))
        Ms.append(M)
        zs.append(z)
        supp_idx.append(np.sort(rng.choice(int(n[f]), size=int(s[f]), replace=False)))
    coef = [rng.standard_normal(int(s[f])) + 1j * rng.standard_normal(int(s[f])) for f in range(F)]
    return BatchWorkload(seed, d, L, box, s, n, np.concatenate(Ms), np.concatenate(zs), supp_idx, coef)


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


# ----------------------------------------------------------------------------- Section 4.2.3
# eq. (4.3): products over the coordinates {1,3,8}, {2,5,6,10}, {4,7,9} (1-based) of the
# B-splines N_2, N_4, N_6.
EQ43_ORDERS = (2, 4, 6)
EQ43_SETS = ((1, 3, 8), (2, 5, 6, 10), (4, 7, 9))


def eq43_function():
    """(orders, coordinate bit masks) of the test function eq. (4.3), d = 10."""
    masks = [sum(1 << (u - 1) for u in S) for S in EQ43_SETS]
    return list(EQ43_ORDERS), masks


def bspline_const(m: int) -> float:
    """C_m of N_m(x) = C_m sum_k sinc(pi k/m)^m (-1)^k e^{2 pi i k x} with unit L2 norm:
    C_m^-2 = sum_k sinc(pi k/m)^{2m} (Parseval), summed to |k| <= 2*10^5."""
    k = np.arange(1, 200001, dtype=np.float64)
    x = np.pi * k / m
    return float(1.0 / math.sqrt(1.0 + 2.0 * np.sum((np.sin(x) / x) ** (2 * m))))


def bspline_coefficients(freq, orders, masks) -> np.ndarray:
    """Fourier coefficients of sum_j prod_{u in S_j} N_{m_j}(x_u) at the frequencies
    freq [n, d]: product j contributes prod_{u in S_j} C_m sinc(pi k_u/m)^m (-1)^{k_u}
    when k_u = 0 outside S_j."""
    freq = np.asarray(freq, np.int64)
    n, d = freq.shape
    out = np.zeros(n, np.float64)
    for m, mask in zip(orders, masks):
        inside = np.array([(mask >> u) & 1 for u in range(d)], bool)
        ok = np.all(freq[:, ~inside] == 0, axis=1)
        c = bspline_const(m)
        val = np.ones(n)
        for u in np.nonzero(inside)[0]:
            k = freq[:, u].astype(np.float64)
            x = np.pi * k / m
            sinc = np.where(k == 0, 1.0, np.sin(x) / np.where(k == 0, 1.0, x))
            val = val * c * sinc ** m * np.where(freq[:, u] % 2 == 0, 1.0, -1.0)
        out += np.where(ok, val, 0.0)
    return out.astype(np.complex128)


def bspline_norm2(orders, masks) -> float:
    """||f||_2^2 for products on pairwise disjoint coordinate sets: each product has
    unit norm, and two products on disjoint sets overlap only through their means
    C_m^{|S|}."""
    sets = [int(mk) for mk in masks]
    for a in range(len(sets)):
        for b in range(a + 1, len(sets)):
            if sets[a] & sets[b]:
                raise ValueError("coordinate sets must be disjoint")
    means = [bspline_const(m) ** bin(mk).count("1") for m, mk in zip(orders, sets)]
    return float(len(sets) + 2 * sum(means[a] * means[b] for a in range(len(sets)) for b in range(a + 1, len(sets))))


def bspline_rel_l2_error(freq, coef, orders, masks) -> float:
    """Relative L2 error of the trigonometric polynomial (freq, coef) as an
    approximation of the test function (Section 4.2.3): sqrt(||f||^2 - sum_I |f_k|^2 +
    sum_I |p_k - f_k|^2) / ||f||."""
    fk = bspline_coefficients(freq, orders, masks)
    nf2 = bspline_norm2(orders, masks)
    e2 = nf2 - float(np.sum(np.abs(fk) ** 2)) + float(np.sum(np.abs(np.asarray(coef) - fk) ** 2))
    return math.sqrt(max(e2, 0.0) / nf2)
