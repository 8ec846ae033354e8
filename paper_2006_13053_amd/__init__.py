"""MI355X (gfx950) multiple-rank-1-lattice sparse FFT (arXiv:2006.13053).

Thin Python binding of the C ABI in ``include/mr1l.h``: every function here only
marshals torch tensors (device memory) and the current HIP stream into the library
``_lib/libmr1l.so``; all arithmetic runs in the library's HIP kernels.  There is no
CPU fallback: if the library is missing or no GPU is present the calls raise.

Names follow the ABI: ``mr1l_sample``, ``mr1l_fft``, ``mr1l_hash_count``,
``mr1l_extract``, ``mr1l_adjoint``, ``mr1l_dimincr``, plus ``Plan`` (plan
create/destroy), ``Graph`` (HIP graph capture of a plan's calls) and
``LatticeCoefficients`` (torch.autograd.Function: forward = DFT + extract,
backward = adjoint).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libmr1l.so")

MR1L_C64, MR1L_C128 = 1, 2
MAX_CAP = 8192
_lib = None


class Mr1lError(RuntimeError):
    """A library call returned an error status."""


class ExtractOpts(C.Structure):
    _fields_ = [("theta", C.c_double), ("vote_min", C.c_int32), ("postproc", C.c_int32),
                ("s_cap", C.c_int64), ("cap", C.c_int64)]


class ExtractOut(C.Structure):
    _fields_ = [(name, C.c_void_p) for name in
                ("n_det", "det_idx", "det_coef", "det_med", "det_mask", "det_hash", "det_w",
                 "n_out", "out_idx", "out_coef", "out_pos", "votes")]


class DimincrParams(C.Structure):
    _fields_ = [("d", C.c_int32), ("N", C.c_int64), ("s", C.c_int64), ("s_local", C.c_int64),
                ("r", C.c_int32), ("theta", C.c_double), ("c", C.c_double), ("delta", C.c_double),
                ("M", C.c_int64), ("postproc", C.c_int32), ("seed", C.c_uint64), ("dtype", C.c_int32),
                ("step1", C.c_int32), ("bs_n", C.c_int32), ("bs_order", C.c_int32 * 16),
                ("bs_dims", C.c_uint64 * 16), ("lsq_iters", C.c_int32)]


SAMPLE_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int64),
                        C.POINTER(C.c_int64), C.POINTER(C.c_uint32), C.c_void_p, C.c_void_p)

_P, _I32, _I64, _D, _U64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint64

# exported symbols and their argument types (kept in the order of include/mr1l.h)
SIGNATURES = {
    "mr1l_version": ([], C.c_int),
    "mr1l_last_error": ([], C.c_char_p),
    "mr1l_plan_create": ([C.POINTER(_P), _I32, _I32, _I32, _P, _P, _I32, _P], C.c_int),
    "mr1l_plan_destroy": ([_P], C.c_int),
    "mr1l_release_cache": ([], C.c_int),
    "mr1l_plan_nodes": ([_P], _I64),
    "mr1l_plan_set_stream": ([_P, _P], C.c_int),
    "mr1l_plan_set_z": ([_P, _P], C.c_int),
    "mr1l_sample": ([_P, _I32, _P, _I64, _P, _P, _P, _P, _I32], C.c_int),
    "mr1l_sample_noalloc": ([_P, _I32, _P, _I64, _P, _P, _P, _P, _I32], C.c_int),
    "mr1l_fft": ([_P, _P, _P, _D, _P], C.c_int),
    "mr1l_hash_count": ([_P, _I64, _P, _P, _P, _P], C.c_int),
    "mr1l_extract": ([_P, _I64, _P, _P, _P, _P, C.POINTER(ExtractOpts), C.POINTER(ExtractOut)], C.c_int),
    "mr1l_adjoint": ([_P, _I64, _I64, _P, _P, _P, _P, _P, _P], C.c_int),
    "mr1l_graph_begin": ([_P], C.c_int),
    "mr1l_graph_end": ([_P, C.POINTER(_P)], C.c_int),
    "mr1l_graph_launch": ([_P, _P], C.c_int),
    "mr1l_graph_destroy": ([_P], C.c_int),
    "mr1l_dimincr": ([C.POINTER(DimincrParams), SAMPLE_FN, _P, _P, _P, _I64, _I64, C.POINTER(_I64), _P, _P,
                      C.POINTER(_I64), _P], C.c_int),
    "mr1l_profile": ([_P, _I32], C.c_int),
    "mr1l_profile_read": ([_P, _P, _P], C.c_int),
    "mr1l_num_lattices": ([_I64, _D, _D], _I32),
    "mr1l_check_injective": ([_P, _I64, _P, _P, _P], C.c_int),
    "mr1l_fft_schedule_count": ([], C.c_int),
    "mr1l_fft_schedule_name": ([_I32], C.c_char_p),
    "mr1l_plan_fft_schedule": ([_P, _I64, _I32], C.c_int),
    "mr1l_fft_tune": ([_P, _I32, _I32, _P, _P], C.c_int),
    "mr1l_sample_bspline": ([_P, _I32, _I32, _P, _P, _P, _P], C.c_int),
    "mr1l_lsq": ([_P, _I64, _P, _P, _P, _P, _P, _I32, C.c_double, _P, _P, _P, C.c_double, _I64, _P, _P, _P],
                 C.c_int),
    "mr1l_pfpn_count": ([_P, _I64, _P, _P, _P, _P, _P, C.c_double, _P], C.c_int),
}

STAGES = ("fft", "vote", "tail", "sample")


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"mr1l HIP library not built: {LIB_PATH} missing "
                              "(run __graft_entry__.build() or paper_2006_13053_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        msg = lib().mr1l_last_error()
        raise Mr1lError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise Mr1lError("device tensor expected")
    if not t.is_contiguous():
        # the library reads row-major arrays through a raw pointer
        raise Mr1lError("contiguous (row-major) tensor expected")
    return C.c_void_p(t.data_ptr())


def _stream_handle(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


class _PlanStream:
    """Orders one library call with torch's current stream when the plan runs on another
    stream: the plan's stream first waits for the work queued so far on the current
    stream (which made the inputs), every tensor passed to ``keep`` is marked as used on
    the plan's stream (so the caching allocator does not hand its memory out again
    before the library has finished with it), and afterwards the current stream waits
    for the plan's stream (which makes the outputs).  Nothing is done while the plan
    records a graph, or when both streams are the same."""

    def __init__(self, plan):
        self.plan = plan
        self.ps = None
        self.held = []

    def __enter__(self):
        ps = self.plan._stream
        cur = torch.cuda.current_stream()
        if ps is not None and ps != cur and not self.plan._capturing:
            ps.wait_stream(cur)
            self.ps, self.cur = ps, cur
        return self.keep

    def keep(self, *ts):
        if self.ps is not None:
            self.held.extend(t for t in ts if isinstance(t, torch.Tensor) and t.is_cuda)

    def __exit__(self, et, ev, tb):
        if self.ps is not None:
            for t in self.held:
                t.record_stream(self.ps)
            self.cur.wait_stream(self.ps)
        return False


def _ctype(dtype):
    if dtype == torch.complex128:
        return MR1L_C128
    if dtype == torch.complex64:
        return MR1L_C64
    raise Mr1lError("dtype must be torch.complex128 or torch.complex64")


class Plan:
    """Multiple rank-1 lattice configuration of F functions (mr1l_plan_create)."""

    def __init__(self, d: int, M, z, F: int = 1, dtype=torch.complex128, stream=None):
        M = np.ascontiguousarray(np.asarray(M, dtype=np.int64).reshape(-1))
        if M.shape[0] % F:
            raise Mr1lError("len(M) must be a multiple of F")
        L = M.shape[0] // F
        z = np.ascontiguousarray(np.asarray(z, dtype=np.int64).reshape(F * L * d))
        self.d, self.F, self.L, self.dtype = int(d), int(F), int(L), dtype
        self.M = M.copy()
        # the stream the library orders this plan's calls on
        self._stream = torch.cuda.current_stream() if stream is None else stream
        self._capturing = False
        h = _P()
        _check(lib().mr1l_plan_create(C.byref(h), self.d, self.F, self.L, M.ctypes.data_as(_P),
                                      z.ctypes.data_as(_P), _ctype(dtype), _stream_handle(stream)),
               "mr1l_plan_create")
        self.handle = h
        self.nodes = int(lib().mr1l_plan_nodes(h))
        self.offsets = np.concatenate([[0], np.cumsum(M)]).astype(np.int64)

    def set_stream(self, stream=None):
        self._stream = torch.cuda.current_stream() if stream is None else stream
        _check(lib().mr1l_plan_set_stream(self.handle, _stream_handle(stream)), "mr1l_plan_set_stream")

    def set_z(self, z):
        z = np.ascontiguousarray(np.asarray(z, dtype=np.int64).reshape(-1))
        _check(lib().mr1l_plan_set_z(self.handle, z.ctypes.data_as(_P)), "mr1l_plan_set_z")

    def profile(self, enable: bool = True):
        """Record HIP events around every stage of the following calls."""
        _check(lib().mr1l_profile(self.handle, int(bool(enable))), "mr1l_profile")

    def profile_read(self):
        """{stage: (total ms, launches)} of the recorded calls (synchronises)."""
        ms = np.zeros(len(STAGES), np.float64)
        cnt = np.zeros(len(STAGES), np.int64)
        _check(lib().mr1l_profile_read(self.handle, ms.ctypes.data_as(_P), cnt.ctypes.data_as(_P)),
               "mr1l_profile_read")
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(STAGES)}

    def fft_schedule(self, M: int, sched: int | None = None) -> int:
        """DFT schedule of lattice size M (set it when sched is given)."""
        rc = lib().mr1l_plan_fft_schedule(self.handle, int(M), -1 if sched is None else int(sched))
        if rc < 0:
            _check(rc, "mr1l_plan_fft_schedule")
        return int(rc)

    def fft_tune(self, reps: int = 5):
        """Autotune the DFT schedule of every distinct size -> {M: {schedule name: ms}}."""
        nm = len(np.unique(self.M))
        ns = fft_schedule_count()
        sizes = np.zeros(nm, np.int64)
        times = np.zeros((nm, ns), np.float32)
        _check(lib().mr1l_fft_tune(self.handle, int(reps), nm, sizes.ctypes.data_as(_P), times.ctypes.data_as(_P)),
               "mr1l_fft_tune")
        names = fft_schedule_names()
        return {int(sizes[i]): {names[j]: float(times[i, j]) for j in range(ns) if times[i, j] >= 0}
                for i in range(nm)}

    def close(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.mr1l_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mr1l_release_cache():
    """Free the library's cached device blocks of the current device."""
    _check(lib().mr1l_release_cache(), "mr1l_release_cache")


def mr1l_check_injective(plan: Plan, freq, set_off=None):
    """Whether each function's candidates stay distinct modulo each of its lattice
    sizes (M in P^Gamma) -> (all injective, per-function flags)."""
    ok = np.zeros(plan.F, np.int32)
    rc = lib().mr1l_check_injective(plan.handle, int(freq.shape[1]), _ptr(set_off), _ptr(freq),
                                    ok.ctypes.data_as(_P))
    if rc not in (0, -4):   # -4: MR1L_E_NOT_INJECTIVE
        _check(rc, "mr1l_check_injective")
    return rc == 0, ok.astype(bool)


def mr1l_lsq(plan: Plan, ex: "Extracted", ghat, max_iter: int = 100, tol: float = 1e-14, theta: float | None = None,
             s_cap: int | None = None, coef=None):
    """Least-squares coefficients on the detected set of an extract call (Remark 2.9)
    and Algorithm 4 on them -> dict(coef, resid, iters, n_out, out_idx, out_coef).
    The extract call must have kept det_hash and det_mask."""
    if ex.get("det_hash") is None or ex.get("det_mask") is None:
        raise Mr1lError("mr1l_lsq needs the extract call's det_hash and det_mask")
    dev = _dev()
    F = plan.F
    s_cap = ex.s_cap if s_cap is None else int(s_cap)
    theta = ex.theta if theta is None else float(theta)
    coef = ex["det_coef"].clone() if coef is None else coef
    out = dict(coef=coef, resid=torch.zeros(F, dtype=torch.float64, device=dev),
               iters=torch.zeros(F, dtype=torch.int32, device=dev),
               n_out=torch.zeros(F, dtype=torch.int64, device=dev),
               out_idx=torch.zeros((F, s_cap), dtype=torch.int64, device=dev),
               out_coef=torch.zeros((F, s_cap), dtype=plan.dtype, device=dev))
    with _PlanStream(plan) as keep:
        _check(lib().mr1l_lsq(plan.handle, ex.cap, _ptr(ex["n_det"]), _ptr(ex["det_idx"]), _ptr(ex["det_hash"]),
                              _ptr(ex["det_mask"]), _ptr(ghat), int(max_iter), float(tol), _ptr(coef),
                              _ptr(out["resid"]), _ptr(out["iters"]), theta, s_cap, _ptr(out["n_out"]),
                              _ptr(out["out_idx"]), _ptr(out["out_coef"])), "mr1l_lsq")
        keep(ghat, *out.values(), *[v for v in ex.values() if v is not None])
    return out


def mr1l_pfpn_count(plan: Plan, ex: "Extracted", n_active, counts=None):
    """Per-function worst-case counts of one extract pass over the counting polynomial
    (support listed first in each set) -> int64 [F, 4]: #PFP, #PFN, #PFP left after
    the singleton post-processing, flags."""
    if counts is None:
        counts = torch.empty((plan.F, 4), dtype=torch.int64, device=_dev())
    with _PlanStream(plan) as keep:
        _check(lib().mr1l_pfpn_count(plan.handle, ex.cap, _ptr(n_active), _ptr(ex["n_det"]), _ptr(ex["det_idx"]),
                                     _ptr(ex["det_med"]), _ptr(ex["det_coef"]), float(ex.theta), _ptr(counts)),
               "mr1l_pfpn_count")
        keep(n_active, counts, ex["n_det"], ex["det_idx"], ex["det_med"], ex["det_coef"])
    return counts


def fft_schedule_count() -> int:
    return int(lib().mr1l_fft_schedule_count())


def fft_schedule_names():
    return [lib().mr1l_fft_schedule_name(i).decode() for i in range(fft_schedule_count())]


def _dev():
    return torch.device("cuda", torch.cuda.current_device())


def mr1l_sample(plan: Plan, freq, coef, f=None, term_off=None, anchor=None, mode: int = 0):
    """Samples of sum_k c_k e^{2 pi i k.x} at the plan's lattice nodes -> complex [nodes]."""
    d_poly = int(freq.shape[0])
    n_terms = int(freq.shape[1])
    if f is None:
        f = torch.empty(plan.nodes, dtype=plan.dtype, device=_dev())
    with _PlanStream(plan) as keep:
        _check(lib().mr1l_sample(plan.handle, d_poly, _ptr(term_off), n_terms, _ptr(freq), _ptr(coef),
                                 _ptr(anchor), _ptr(f), int(mode)), "mr1l_sample")
        keep(term_off, freq, coef, anchor, f)
    return f


def mr1l_sample_noalloc(plan: Plan, freq, coef, f, term_off, anchor=None, mode: int = 0):
    """mr1l_sample with the term scratch in the library's static array (no allocation in
    the call; the caller passes every buffer, term_off included)."""
    if f is None or term_off is None:
        raise Mr1lError("f and term_off are required")
    d_poly = int(freq.shape[0])
    n_terms = int(freq.shape[1])
    with _PlanStream(plan) as keep:
        _check(lib().mr1l_sample_noalloc(plan.handle, d_poly, _ptr(term_off), n_terms, _ptr(freq), _ptr(coef),
                                         _ptr(anchor), _ptr(f), int(mode)), "mr1l_sample_noalloc")
        keep(term_off, freq, coef, anchor, f)
    return f


def mr1l_sample_bspline(plan: Plan, d_poly: int, order, dims, anchor=None, f=None):
    """Samples of sum_j prod_{u in S_j} N_{m_j}(x_u) (eq. (4.3)) at the plan's nodes.
    order: [n_prod] ints; dims: [F, n_prod] (or [n_prod], all functions alike) bit masks
    of the coordinates of each product."""
    order = np.ascontiguousarray(np.asarray(order, dtype=np.int32).reshape(-1))
    dims = np.asarray(dims, dtype=np.uint64)
    if dims.ndim == 1:
        dims = np.tile(dims, (plan.F, 1))
    dims = np.ascontiguousarray(dims.reshape(plan.F, order.shape[0]))
    if f is None:
        f = torch.empty(plan.nodes, dtype=plan.dtype, device=_dev())
    with _PlanStream(plan) as keep:
        _check(lib().mr1l_sample_bspline(plan.handle, int(d_poly), int(order.shape[0]), order.ctypes.data_as(_P),
                                         dims.ctypes.data_as(_P), _ptr(anchor), _ptr(f)), "mr1l_sample_bspline")
        keep(anchor, f)
    return f


def mr1l_fft(plan: Plan, f, theta: float, ghat=None, bitmap=None, want_bitmap: bool = True):
    """Normalised lattice DFTs and the non-zero bitmap -> (ghat, bitmap)."""
    if ghat is None:
        ghat = torch.empty(plan.nodes, dtype=plan.dtype, device=_dev())
    if bitmap is None and want_bitmap:
        bitmap = torch.empty((plan.nodes + 31) // 32, dtype=torch.int32, device=_dev())
    with _PlanStream(plan) as keep:
        _check(lib().mr1l_fft(plan.handle, _ptr(f), _ptr(ghat), float(theta), _ptr(bitmap)), "mr1l_fft")
        keep(f, ghat, bitmap)
    return ghat, bitmap


def mr1l_hash_count(plan: Plan, freq, set_off=None, want_hash: bool = True, want_counts: bool = True):
    """Buckets [L, n] (int32) and occupancy counts [nodes] (int32)."""
    n = int(freq.shape[1])
    h = torch.empty((plan.L, n), dtype=torch.int32, device=_dev()) if want_hash else None
    c = torch.empty(plan.nodes, dtype=torch.int32, device=_dev()) if want_counts else None
    with _PlanStream(plan) as keep:
        _check(lib().mr1l_hash_count(plan.handle, n, _ptr(set_off), _ptr(freq), _ptr(h), _ptr(c)),
               "mr1l_hash_count")
        keep(set_off, freq, h, c)
    return h, c


class Extracted(dict):
    """Device outputs of mr1l_extract (dict of tensors + the options used)."""


def extract_buffers(plan: Plan, cap: int, s_cap: int, n_total: int, want_votes=False, want_w=True):
    dev = _dev()
    F, L = plan.F, plan.L
    e = Extracted(
        n_det=torch.zeros(F, dtype=torch.int64, device=dev),
        det_idx=torch.zeros((F, cap), dtype=torch.int64, device=dev),
        det_coef=torch.zeros((F, cap), dtype=plan.dtype, device=dev),
        det_med=torch.zeros((F, cap), dtype=plan.dtype, device=dev),
        det_mask=torch.zeros((F, cap) if L <= 32 else (F, cap, (L + 31) // 32), dtype=torch.int32, device=dev),
        det_hash=torch.zeros((F, cap, L), dtype=torch.int32, device=dev),
        det_w=torch.zeros((F, cap, L, 2), dtype=torch.float64, device=dev) if want_w else None,
        n_out=torch.zeros(F, dtype=torch.int64, device=dev),
        out_idx=torch.zeros((F, s_cap), dtype=torch.int64, device=dev),
        out_coef=torch.zeros((F, s_cap), dtype=plan.dtype, device=dev),
        out_pos=torch.zeros((F, s_cap), dtype=torch.int32, device=dev),
        votes=torch.zeros(n_total, dtype=torch.uint8, device=dev) if want_votes else None,
    )
    e.cap, e.s_cap = int(cap), int(s_cap)
    return e


def mr1l_extract(plan: Plan, freq, ghat, bitmap, theta: float, s_cap: int, cap: int | None = None,
                 vote_min: int = 0, postproc: bool = True, set_off=None, want_votes: bool = False,
                 want_w: bool = True, out: Extracted | None = None):
    """Algorithm 2 (+ Remark 2.9) + Algorithm 4 over the candidate sets -> Extracted."""
    n = int(freq.shape[1])
    cap = MAX_CAP if cap is None else int(cap)
    if out is None:
        out = extract_buffers(plan, cap, s_cap, n, want_votes, want_w)
    o = ExtractOpts(float(theta), int(vote_min), int(bool(postproc)), int(s_cap), int(cap))
    x = ExtractOut(*[None if out.get(k) is None else out[k].data_ptr() for k, _ in ExtractOut._fields_])
    with _PlanStream(plan) as keep:
        _check(lib().mr1l_extract(plan.handle, n, _ptr(set_off), _ptr(freq), _ptr(ghat), _ptr(bitmap),
                                  C.byref(o), C.byref(x)), "mr1l_extract")
        keep(set_off, freq, ghat, bitmap, *[v for v in out.values() if v is not None])
    out.theta, out.postproc = float(theta), bool(postproc)
    return out


def mr1l_adjoint(plan: Plan, ex: Extracted, grad_out, grad_f=None):
    """Transpose of samples -> out_coef for the support/selection of ``ex``."""
    if grad_f is None:
        grad_f = torch.empty(plan.nodes, dtype=plan.dtype, device=_dev())
    g = grad_out.contiguous().to(plan.dtype)
    with _PlanStream(plan) as keep:
        _check(lib().mr1l_adjoint(plan.handle, ex.cap, ex.s_cap, _ptr(ex["n_out"]), _ptr(ex["out_pos"]),
                                  _ptr(ex["det_hash"]), _ptr(ex["det_w"]), _ptr(g), _ptr(grad_f)),
               "mr1l_adjoint")
        keep(g, grad_f, ex["n_out"], ex["out_pos"], ex["det_hash"], ex["det_w"])
    return grad_f


class Graph:
    """HIP graph of a plan's calls: ``with Graph(plan) as g: ...`` then ``g.launch()``."""

    def __init__(self, plan: Plan):
        self.plan, self.handle = plan, None

    def __enter__(self):
        _check(lib().mr1l_graph_begin(self.plan.handle), "mr1l_graph_begin")
        self.plan._capturing = True
        return self

    def __exit__(self, et, ev, tb):
        h = _P()
        self.plan._capturing = False
        rc = lib().mr1l_graph_end(self.plan.handle, C.byref(h))
        if et is None:
            _check(rc, "mr1l_graph_end")
            self.handle = h
        return False

    def launch(self, stream=None):
        _check(lib().mr1l_graph_launch(self.handle, _stream_handle(stream)), "mr1l_graph_launch")

    def __del__(self):
        try:
            if self.handle is not None and _lib is not None:
                _lib.mr1l_graph_destroy(self.handle)
        except Exception:
            pass


def mr1l_num_lattices(nJ: int, c: float = 10.33, delta: float = 0.9) -> int:
    return int(lib().mr1l_num_lattices(int(nJ), float(c), float(delta)))


def mr1l_dimincr(d: int, N: int, s: int, s_local: int, r: int, theta: float, M: int, seed: int,
                 poly_freq=None, poly_coef=None, c: float = 10.33, delta: float = 0.9,
                 postproc: bool = True, dtype=torch.complex128, cap: int = 1 << 16, sample_fn=None,
                 step1: bool = False, bspline=None, lsq_iters: int = 0):
    """Algorithm 3 driver (Step 2, and Step 1 when step1) -> (freq [n, d] int64 numpy,
    coef [n] numpy, total samples).  bspline = (orders, coordinate masks) selects the
    built-in B-spline test function (eq. (4.3)) instead of the polynomial."""
    prm = DimincrParams(int(d), int(N), int(s), int(s_local), int(r), float(theta), float(c), float(delta),
                        int(M), int(bool(postproc)), int(seed) & (2**64 - 1), _ctype(dtype), int(bool(step1)))
    prm.lsq_iters = int(lsq_iters)
    if bspline is not None:
        orders, masks = list(bspline[0]), list(bspline[1])
        prm.bs_n = len(orders)
        for q, (mq, dq) in enumerate(zip(orders, masks)):
            prm.bs_order[q] = int(mq)
            prm.bs_dims[q] = int(dq)
    fo = np.zeros((cap, d), np.int64)
    co = np.zeros(cap, np.complex128 if dtype == torch.complex128 else np.complex64)
    n_out, tot = C.c_int64(0), C.c_int64(0)
    cb = SAMPLE_FN(0) if sample_fn is None else SAMPLE_FN(sample_fn)
    ps = 0 if poly_freq is None else int(poly_freq.shape[1])
    _check(lib().mr1l_dimincr(C.byref(prm), cb, None, _ptr(poly_freq), _ptr(poly_coef), ps, int(cap),
                              C.byref(n_out), fo.ctypes.data_as(_P), co.ctypes.data_as(_P), C.byref(tot),
                              _stream_handle()), "mr1l_dimincr")
    n = n_out.value
    return fo[:n], co[:n], int(tot.value)


class LatticeCoefficients(torch.autograd.Function):
    """Coefficients of Algorithm 4 as a function of the samples.

    forward(f) runs mr1l_fft + mr1l_extract and returns out_coef [F, s_cap]; the
    support and the selections (singleton masks, median order statistics) are held
    fixed, so the map is real-linear and backward is mr1l_adjoint.
    """

    @staticmethod
    def forward(ctx, f, plan, freq, theta, s_cap, cap, postproc, set_off=None):
        ghat, bitmap = mr1l_fft(plan, f.detach(), theta)
        ex = mr1l_extract(plan, freq, ghat, bitmap, theta, s_cap, cap, postproc=postproc, set_off=set_off)
        ctx.plan, ctx.ex = plan, ex
        ctx.mark_non_differentiable(ex["n_out"], ex["out_idx"])
        return ex["out_coef"].clone(), ex["n_out"], ex["out_idx"]

    @staticmethod
    def backward(ctx, grad_coef, _g_nout=None, _g_idx=None):
        gf = mr1l_adjoint(ctx.plan, ctx.ex, grad_coef)
        return gf, None, None, None, None, None, None, None
