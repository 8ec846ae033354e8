"""CPU reference oracle for the multiple-rank-1-lattice sparse FFT (test infrastructure).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  The GPU library never
imports, links or executes anything here, and this package never imports the GPU
library.  The arithmetic lives in ``mr1l_oracle.c`` (plain C, long-double sums,
direct DFTs, no FFT); this module only marshals numpy arrays through ctypes.

Every function cites the passage of arXiv:2006.13053 it follows; see the C file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mr1l_oracle.c")
_LIB_DEFAULT = os.path.join(_HERE, "liboracle.so")
# A test that plants a mistake in the oracle points this at a mutated build.
_LIB = os.environ.get("MR1L_ORACLE_LIB", _LIB_DEFAULT)
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP on).  Returns the library path."""
    return build_from(_SRC, _LIB_DEFAULT, force)


def build_from(src: str, out: str, force: bool = True) -> str:
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_from(_SRC, _LIB, force=True)
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


_i32, _i64, _u64, _d = C.c_int32, C.c_int64, C.c_uint64, C.c_double
_p = C.c_void_p


def _declare(L):
    L.orc_is_prime.argtypes = [_i64]
    L.orc_is_prime.restype = C.c_int
    L.orc_num_threads.restype = C.c_int
    L.orc_hash_one.argtypes = [_i32, _p, _i64, _p, _i64]
    L.orc_hash_one.restype = _i64
    L.orc_hash.argtypes = [_i32, _i64, _p, _i32, _p, _p, _p]
    L.orc_counts.argtypes = [_i32, _i64, _p, _i32, _p, _p, _p]
    L.orc_sample.argtypes = [_i32, _i32, _i64, _p, _p, _p, _i32, _p, _p, _p]
    L.orc_sample_nodes.argtypes = [_i32, _i32, _i64, _p, _p, _p, _p, _i64, _i64, _p, _p]
    L.orc_dft.argtypes = [_i32, _p, _p, _p, _i32]
    L.orc_bucket_sums.argtypes = [_i32, _i64, _p, _p, _i32, _p, _p, _p]
    L.orc_dft_bins.argtypes = [_i64, _p, _i64, _p, _p, _i32]
    L.orc_extract.argtypes = [_i32, _i64, _p, _i32, _p, _p, _p, _d, _i32, _i32, _i64, _i64,
                              _p, _p, _p, _p, _p, _p, _p, _p, _p]
    L.orc_extract.restype = _i64
    L.orc_weights.argtypes = [_i32, _i64, _p, _i32, _p, _p, _p, _i64, _p, _p, _i32, _p]
    L.orc_adjoint.argtypes = [_i32, _i64, _p, _i32, _p, _p, _i64, _p, _p, _p, _p]
    L.orc_splitmix64.argtypes = [_u64, _u64]
    L.orc_splitmix64.restype = _u64
    L.orc_num_lattices_eq42.argtypes = [_i64, _d, _d]
    L.orc_num_lattices_eq42.restype = _i32
    L.orc_dimincr.argtypes = [_i32, _i64, _i64, _p, _p, _i32, _p, _p, _i64, _i64, _i32, _d, _d, _d, _i64,
                              _i32, _u64, _i64, _i32, _p, _p, _p]
    L.orc_sample_bspline.argtypes = [_i32, _i32, _i32, _p, _p, _p, _i32, _p, _p, _p]
    L.orc_bspline_periodic.argtypes = [_i32, C.c_longdouble]
    L.orc_bspline_periodic.restype = C.c_longdouble
    L.orc_dimincr.restype = _i64
    L.orc_pfpn.argtypes = [_i32, _i64, _p, _i64, _i32, _p, _p, _p]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _cplx(a):
    """complex array -> interleaved float64 view (copy)."""
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a.view(np.float64)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def is_prime(n: int) -> bool:
    return bool(lib().orc_is_prime(int(n)))


def hash_buckets(freq, M, z):
    """h[l, i] = (k_i . z_l) mod M_l  (freq: [d, n] int64, z: [L, d])."""
    freq, M, z = _c(freq, np.int64), _c(M, np.int64), _c(z, np.int64)
    d, n = freq.shape
    L = M.shape[0]
    out = np.zeros((L, n), np.int32)
    lib().orc_hash(d, n, _ptr(freq), L, _ptr(M), _ptr(z), _ptr(out))
    return out


def counts(freq, M, z):
    """Bucket occupancy over all lattices, concatenated: int32 [sum M]."""
    freq, M, z = _c(freq, np.int64), _c(M, np.int64), _c(z, np.int64)
    d, n = freq.shape
    out = np.zeros(int(M.sum()), np.int32)
    lib().orc_counts(d, n, _ptr(freq), M.shape[0], _ptr(M), _ptr(z), _ptr(out))
    return out


def sample(freq, coef, M, z, anchor=None, t=None):
    """Samples of sum_k c_k e^{2 pi i k.x} on the lattices (complex128 [sum M])."""
    freq, M, z = _c(freq, np.int64), _c(M, np.int64), _c(z, np.int64)
    d, s = freq.shape
    t = d if t is None else int(t)
    co = _cplx(coef)
    anc = None if anchor is None else _c(anchor, np.uint32)
    out = np.zeros(2 * int(M.sum()), np.float64)
    lib().orc_sample(d, t, s, _ptr(freq), _ptr(co), _ptr(anc), M.shape[0], _ptr(M), _ptr(z),
                     _ptr(out))
    return out.view(np.complex128)


def sample_nodes(freq, coef, zl, Ml, j_list, anchor=None, t=None):
    """Sample values at nodes j of one lattice (complex128 [len(j_list)])."""
    freq, zl = _c(freq, np.int64), _c(zl, np.int64)
    d, s = freq.shape
    t = d if t is None else int(t)
    co = _cplx(coef)
    anc = None if anchor is None else _c(anchor, np.uint32)
    j = _c(j_list, np.int64)
    out = np.zeros(2 * j.shape[0], np.float64)
    lib().orc_sample_nodes(d, t, s, _ptr(freq), _ptr(co), _ptr(anc), _ptr(zl), int(Ml),
                           j.shape[0], _ptr(j), _ptr(out))
    return out.view(np.complex128)


def dft(f, M, sign=-1):
    """ghat_l[h] = (1/M_l) sum_j f_l[j] e^{sign 2 pi i j h / M_l}, direct."""
    M = _c(M, np.int64)
    fi = _cplx(f)
    out = np.zeros_like(fi)
    lib().orc_dft(M.shape[0], _ptr(M), _ptr(fi), _ptr(out), int(sign))
    return out.view(np.complex128)


def bucket_sums(freq, coef, M, z):
    """Aliasing formula eq. (2.4): per-bucket coefficient sums, complex128 [sum M]."""
    freq, M, z = _c(freq, np.int64), _c(M, np.int64), _c(z, np.int64)
    d, n = freq.shape
    co = _cplx(coef)
    out = np.zeros(2 * int(M.sum()), np.float64)
    lib().orc_bucket_sums(d, n, _ptr(freq), _ptr(co), M.shape[0], _ptr(M), _ptr(z), _ptr(out))
    return out.view(np.complex128)


def dft_bins(fl, Ml, bins, sign=-1):
    fi = _cplx(fl)
    b = _c(bins, np.int64)
    out = np.zeros(2 * b.shape[0], np.float64)
    lib().orc_dft_bins(int(Ml), _ptr(fi), b.shape[0], _ptr(b), _ptr(out), int(sign))
    return out.view(np.complex128)


def extract(freq, M, z, ghat, theta, s_cap, vote_min=None, postproc=True, cap=None):
    """Algorithm 2 (+ Remark 2.9 post-processing) + Algorithm 4 for fixed lattices.

    Returns a dict of numpy arrays: votes, det_idx, det_med, det_mask, det_coef,
    out_idx, out_coef, out_pos, n_det.
    """
    freq, M, z = _c(freq, np.int64), _c(M, np.int64), _c(z, np.int64)
    d, n = freq.shape
    L = M.shape[0]
    vote_min = (L + 1) // 2 if vote_min is None else int(vote_min)
    cap = n if cap is None else int(cap)
    g = _cplx(ghat)
    votes = np.zeros(n, np.uint8)
    det_idx = np.zeros(max(cap, 1), np.int64)
    det_med = np.zeros(2 * max(cap, 1), np.float64)
    det_mask = np.zeros(max(cap, 1), np.uint64)
    det_coef = np.zeros(2 * max(cap, 1), np.float64)
    sc = max(int(s_cap), 1)
    out_idx = np.zeros(sc, np.int64)
    out_coef = np.zeros(2 * sc, np.float64)
    out_pos = np.zeros(sc, np.int64)
    n_out = C.c_int64(0)
    nd = lib().orc_extract(d, n, _ptr(freq), L, _ptr(M), _ptr(z), _ptr(g), float(theta), vote_min,
                           int(bool(postproc)), int(s_cap), cap, _ptr(votes), _ptr(det_idx),
                           _ptr(det_med), _ptr(det_mask), _ptr(det_coef), C.byref(n_out),
                           _ptr(out_idx), _ptr(out_coef), _ptr(out_pos))
    k = min(nd, cap)
    no = n_out.value
    return dict(n_det=int(nd), votes=votes, det_idx=det_idx[:k],
                det_med=det_med.view(np.complex128)[:k], det_mask=det_mask[:k],
                det_coef=det_coef.view(np.complex128)[:k], out_idx=out_idx[:no],
                out_coef=out_coef.view(np.complex128)[:no], out_pos=out_pos[:no])


def weights(freq, M, z, ghat, det_idx, det_mask, postproc=True):
    """Real weights [n_det, L, 2] of the fixed-selection linear map (see C file)."""
    freq, M, z = _c(freq, np.int64), _c(M, np.int64), _c(z, np.int64)
    d, n = freq.shape
    L = M.shape[0]
    di, dm = _c(det_idx, np.int64), _c(det_mask, np.uint64)
    nd = di.shape[0]
    w = np.zeros((max(nd, 1), L, 2), np.float64)
    lib().orc_weights(d, n, _ptr(freq), L, _ptr(M), _ptr(z), _ptr(_cplx(ghat)), nd, _ptr(di),
                      _ptr(dm), int(bool(postproc)), _ptr(w))
    return w[:nd]


def adjoint(freq, M, z, det_idx, w, grad):
    """Dense transpose of the fixed-selection map: grad wrt samples [sum M] complex."""
    freq, M, z = _c(freq, np.int64), _c(M, np.int64), _c(z, np.int64)
    d, n = freq.shape
    L = M.shape[0]
    di = _c(det_idx, np.int64)
    w = _c(w, np.float64)
    g = _cplx(grad)
    out = np.zeros(2 * int(M.sum()), np.float64)
    lib().orc_adjoint(d, n, _ptr(freq), L, _ptr(M), _ptr(z), di.shape[0], _ptr(di), _ptr(w),
                      _ptr(g), _ptr(out))
    return out.view(np.complex128)


def splitmix64(seed: int, n: int) -> int:
    return int(lib().orc_splitmix64(C.c_uint64(seed & (2**64 - 1)), C.c_uint64(n)))


def num_lattices_eq42(nJ: int, c: float = 10.33, delta: float = 0.9) -> int:
    return int(lib().orc_num_lattices_eq42(int(nJ), float(c), float(delta)))


def dimincr(poly_freq, poly_coef, N, s, s_local, r, theta, c, delta, Mlat, seed,
            postproc=True, cap_set=1 << 20, step1=False, bspline=None, d=None):
    """Algorithm 3 Step 2 with Algorithm 4; the single-coordinate sets come from Step 1
    (step1) or are the full range [-N, N].  The function is the sparse polynomial
    (poly_freq, poly_coef), or with bspline = (orders, coordinate masks) the test
    function of eq. (4.3) in d coordinates.

    Returns (freq [n, d] int64 lexicographically sorted, coef [n] complex, samples).
    """
    if bspline is None:
        pf = _c(poly_freq, np.int64)
        d, sp = pf.shape
        pc = _cplx(poly_coef)
        bn, bo, bd = 0, None, None
    else:
        pf, pc, sp = None, None, 0
        bo = _c(bspline[0], np.int32)
        bd = _c(bspline[1], np.uint64)
        bn = int(bo.shape[0])
    out_f = np.zeros((max(int(s), 1), d), np.int64)
    out_c = np.zeros(2 * max(int(s), 1), np.float64)
    tot = C.c_int64(0)
    n = lib().orc_dimincr(d, int(N), sp, _ptr(pf), _ptr(pc), bn, _ptr(bo), _ptr(bd), int(s), int(s_local),
                          int(r), float(theta), float(c), float(delta), int(Mlat), int(bool(postproc)),
                          C.c_uint64(seed & (2**64 - 1)), int(cap_set), int(bool(step1)), _ptr(out_f),
                          _ptr(out_c), C.byref(tot))
    if n < 0:
        raise RuntimeError("oracle dimincr: capacity exceeded")
    return out_f[:n], out_c.view(np.complex128)[:n], int(tot.value)


def bspline_periodic(m, x):
    """N_m(x) of eq. (4.3) (unit L2 norm, period 1), long double, returned as float."""
    return float(lib().orc_bspline_periodic(int(m), C.c_longdouble(float(x))))


def sample_bspline(order, dims, M, z, anchor=None, t=None):
    """Samples of sum_j prod_{u in S_j} N_{m_j}(x_u) at the lattice nodes (coordinates
    u < t from the lattices, u >= t anchors a_u / 2^32); dims[j] = bit mask of S_j."""
    order = _c(order, np.int32)
    dims = _c(dims, np.uint64)
    M = _c(M, np.int64)
    z = _c(z, np.int64).reshape(len(M), -1)
    t = z.shape[1] if t is None else int(t)
    d_poly = t + (0 if anchor is None else len(anchor))
    anc = None if anchor is None else _c(anchor, np.uint32)
    f = np.zeros(2 * int(M.sum()), np.float64)
    lib().orc_sample_bspline(t, d_poly, len(order), _ptr(order), _ptr(dims), _ptr(anc), len(M), _ptr(M), _ptr(z),
                             _ptr(f))
    return f.view(np.complex128)


def pfpn(freq, n_active, M, z):
    """Table 4.1 classification for the counting polynomial eq. (4.1) with support
    freq[:, :n_active] -> uint8 [n]: bit 0 PFP, bit 1 PFN, bit 2 PFP kept by the
    Remark 2.9 post-processing (see the C file)."""
    freq = _c(freq, np.int64)
    d, n = freq.shape
    M = _c(M, np.int64)
    z = _c(z, np.int64).reshape(len(M), d)
    cls = np.zeros(n, np.uint8)
    lib().orc_pfpn(d, n, _ptr(freq), int(n_active), len(M), _ptr(M), _ptr(z), _ptr(cls))
    return cls


def pfpn_counts(cls):
    """(#PFP, #PFN, #PFP kept by post-processing) of a pfpn classification."""
    cls = np.asarray(cls)
    return int(((cls & 1) != 0).sum()), int(((cls & 2) != 0).sum()), int(((cls & 4) != 0).sum())


def lsq_matrix(freq, M, z):
    """Sampling matrix of the trigonometric polynomials with frequencies freq on the
    concatenated lattice nodes: A[(l, j), q] = e^{2 pi i j h_l(k_q) / M_l}, since
    k . x_j = j (k . z_l) / M_l mod 1 (eq. (2.1)); the phase j h mod M is reduced in
    integers.  Dense, for small cases."""
    h = hash_buckets(freq, M, z)
    rows = []
    for l, m in enumerate(np.asarray(M, np.int64)):
        j = np.arange(int(m), dtype=np.int64)[:, None]
        ph = (j * h[l][None, :]) % int(m)
        rows.append(np.exp(2j * np.pi * ph / float(m)))
    return np.vstack(rows)


def lsq(freq, M, z, f, det_idx):
    """Remark 2.9, least-squares variant: coefficients on the candidates det_idx that
    minimise the sum over all lattice nodes of |sum_k c_k e^{2 pi i k.x_j} - f(x_j)|^2
    (numpy's least squares on the dense sampling matrix; minimum norm if singular)."""
    A = lsq_matrix(np.asarray(freq)[:, np.asarray(det_idx, np.int64)], M, z)
    c, *_ = np.linalg.lstsq(A, np.asarray(f, np.complex128), rcond=None)
    return c
