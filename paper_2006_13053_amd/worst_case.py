"""Worst-case aliasing experiments of Section 4.1 on the GPU (PFP/PFN, Table 4.1).

The method is run on the counting polynomial of eq. (4.1): all-ones coefficients
on the support I.  By the aliasing formula eq. (2.4) the lattice value at the
bucket of a candidate k counts the members of I in that bucket, so one pass of
sampling, lattice DFTs and extraction tells, for every k in Gamma, whether it is
a potential false positive (k outside I, median > 0) or a potential false
negative (k in I, median > 1), and which potential false positives survive the
singleton post-processing of Remark 2.9.  Every step runs in the HIP library:
mr1l_sample (bucket mode), mr1l_fft, mr1l_extract and mr1l_pfpn_count.

Candidate sets must list the support first: candidates [0, |I|) of each
function's set are I.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import Plan, _dev, extract_buffers, mr1l_extract, mr1l_fft, mr1l_pfpn_count, mr1l_sample

# The lattice values are integer counts (up to rounding), so any threshold in (0, 1)
# gives the same non-zero test; 1/4 also separates a zero post-processed coefficient
# from a median of at least 1/2 (even L).
THETA = 0.25
CAP = 8192


def cor27_failure_bound(n_gamma: int, c: float, L: int) -> float:
    """Failure probability bound of Corollary 2.7 solved for delta (lattice size
    M > c |I|): |Gamma| (c - 1)^(-(c - 2) L / (4 c)), the dashed lines of
    Figures 4.1 and 4.3 (c = 10.33)."""
    return float(n_gamma * math.exp(-(c - 2.0) * L * math.log(c - 1.0) / (4.0 * c)))


class CountingRun:
    """A plan of F functions with L lattices of size M each plus its buffers.

    run() classifies F candidate sets at once (one function per set), each with
    the support first; the generating vectors can be replaced between runs
    (set_z) for experiments that draw new lattices per repetition.
    """

    def __init__(self, d: int, F: int, L: int, M: int, z, cap: int = CAP, dtype=torch.complex128,
                 profile: bool = False):
        z = np.asarray(z, np.int64).reshape(F * L, d)
        self.d, self.F, self.L, self.M, self.cap = d, F, L, int(M), int(cap)
        self.plan = Plan(d, np.full(F * L, int(M), np.int64), z, F=F, dtype=dtype)
        if profile:
            self.plan.profile(True)
        self.f = torch.empty(self.plan.nodes, dtype=dtype, device=_dev())
        self.ghat = torch.empty_like(self.f)
        self.bitmap = torch.empty((self.plan.nodes + 31) // 32, dtype=torch.int32, device=_dev())
        self.counts = torch.empty((F, 4), dtype=torch.int64, device=_dev())
        self._ex = None
        self._coef = None

    def set_z(self, z):
        self.plan.set_z(np.asarray(z, np.int64).reshape(self.F * self.L, self.d))

    def run(self, cand, set_off, n_active, terms, term_off):
        """cand dev int64 [d, n_total]; set_off dev int64 [F+1]; n_active dev int64 [F];
        terms dev int64 [d, sum |I_f|] (the supports, function by function) with
        term_off dev int64 [F+1] -> counts dev int64 [F, 4] (#PFP, #PFN, #PFP after
        Remark 2.9, flags; see mr1l_pfpn_count)."""
        n_terms = int(terms.shape[1])
        if self._coef is None or self._coef.shape[0] < n_terms:
            self._coef = torch.ones(n_terms, dtype=self.plan.dtype, device=_dev())
        mr1l_sample(self.plan, terms, self._coef[:n_terms], f=self.f, term_off=term_off, mode=2)
        mr1l_fft(self.plan, self.f, THETA, ghat=self.ghat, bitmap=self.bitmap)
        if self._ex is None:
            self._ex = extract_buffers(self.plan, self.cap, 1, 0, want_votes=False, want_w=False)
            self._ex["det_mask"] = None
            self._ex["det_hash"] = None
        ex = mr1l_extract(self.plan, cand, self.ghat, self.bitmap, THETA, s_cap=1, cap=self.cap,
                          postproc=True, set_off=set_off, want_w=False, out=self._ex)
        return mr1l_pfpn_count(self.plan, ex, n_active, counts=self.counts)

    def close(self):
        self.plan.close()


def summarize(counts) -> dict:
    """Success statistics of repetitions (rows #PFP, #PFN, #PFP after Remark 2.9,
    flags) in the senses of Section 4.1: no PFP and no PFN (median), no PFN and
    at most 10 or 100 PFPs, and no PFN with no PFP left after the post-processing
    (median + R1L; a truncated detected list counts as a failure there).  A
    truncated list (more than CAP detected candidates, so more than 100 PFPs) keeps
    the PFP count exact but not the PFN count: max_pfn covers the complete lists."""
    c = np.asarray(counts, np.int64).reshape(-1, 4)
    if np.any(c[:, 3] & 2):
        raise RuntimeError("support not detected whole: the candidate sets must list the support first")
    pfp, pfn, post, trunc = c[:, 0], c[:, 1], c[:, 2], (c[:, 3] & 1) != 0
    r = max(1, c.shape[0])
    return dict(
        reps=int(c.shape[0]),
        median=float(((pfp == 0) & (pfn == 0)).sum() / r),
        median_r1l=float(((pfn == 0) & (post == 0) & ~trunc).sum() / r),
        pfp_le10=float(((pfn == 0) & (pfp <= 10)).sum() / r),
        pfp_le100=float(((pfn == 0) & (pfp <= 100)).sum() / r),
        max_pfp=int(pfp.max(initial=0)),
        max_pfn=int(pfn[~trunc].max(initial=0)),
        truncated=int(trunc.sum()),
    )
