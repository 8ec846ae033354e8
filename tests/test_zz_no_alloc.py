"""The allocation-free sampler (mr1l_sample_noalloc) against mr1l_sample: the same
kernels with the term scratch in the library's static per-device array.  Two calls in a
row on one device, the second with fewer terms (the array keeps the first call's
contents), in both sampling modes and both precisions; results equal mr1l_sample's
(bit-exact for the direct sum, whose order of operations is fixed; within the
precision's tolerance for the bucket sums, whose atomics add in any order) and the
oracle's samples.  Sizes beyond the array are refused before anything runs."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = {torch.complex128: 1e-11, torch.complex64: 1e-5}


@pytest.fixture(scope="module")
def m():
    import paper_2006_13053_amd as mod
    mod.lib()
    torch.cuda.set_device(0)
    return mod


def dev():
    return torch.device("cuda", 0)


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(1e-300, float(np.abs(b).max())))


def say(*a):
    print("[gpu-case]", *a, flush=True)


def batch_problem(F, seed):
    """F functions of the batched kind (d = 10, L = 8, s in [10, 1000]) as one batch."""
    probs = synth.batch_config(seed, nfunc=F, scale=0.01)
    d = probs[0].d
    M = np.concatenate([q.M for q in probs])
    z = np.concatenate([q.z for q in probs])
    supp = np.concatenate([q.supp for q in probs], axis=1)
    coef = np.concatenate([q.coef for q in probs])
    toff = np.concatenate([[0], np.cumsum([len(q.coef) for q in probs])]).astype(np.int64)
    return d, M, z, supp, coef, toff, probs


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("mode", [1, 2])
def test_noalloc_sample_matches_allocating_sample(m, dtype, mode):
    say("noalloc sample", dtype, "mode", mode)
    d, M, z, supp, coef, toff, probs = batch_problem(6, 11)
    L = probs[0].L
    plan = m.Plan(d, M, z, F=len(probs), dtype=dtype)
    cf = T(coef).to(dtype)
    # call 1: every term; call 2: the first half of each function's terms
    half = [np.arange(toff[i], toff[i] + max(1, (toff[i + 1] - toff[i]) // 2)) for i in range(len(probs))]
    sel = np.concatenate(half)
    toff2 = np.concatenate([[0], np.cumsum([len(h) for h in half])]).astype(np.int64)
    for sp, co, to in ((supp, coef, toff), (supp[:, sel], coef[sel], toff2)):
        fs, cs, ts = T(sp), T(co).to(dtype), T(to)
        f_ref = m.mr1l_sample(plan, fs, cs, term_off=ts, mode=mode)
        f_na = torch.full_like(f_ref, float("nan"))
        m.mr1l_sample_noalloc(plan, fs, cs, f_na, ts, mode=mode)
        torch.cuda.synchronize()
        a, b = f_na.cpu().numpy(), f_ref.cpu().numpy()
        if mode == 1:
            assert np.array_equal(a, b)
        else:
            assert rel(a, b) <= TOL[dtype]
        off = 0
        for i, q in enumerate(probs):
            lo, hi = int(to[i]), int(to[i + 1])
            fo = oracle.sample(np.ascontiguousarray(sp[:, lo:hi]), co[lo:hi], q.M, q.z)
            assert rel(a[off:off + fo.shape[0]].astype(np.complex128), fo) <= TOL[dtype], i
            off += fo.shape[0]
    assert plan.nodes == int(M.sum()) and L == 8


def test_noalloc_sample_refuses_sizes_beyond_the_static_array(m):
    say("noalloc sample capacity")
    p = synth.small_config(0)
    plan = m.Plan(p.d, p.M, p.z)
    # 64 MiB / (16 + 4 L) terms fit in complex128 with L = 5: 36 B per term
    n = (64 << 20) // 36 + 1024
    freq = torch.zeros((p.d, n), dtype=torch.int64, device=dev())
    coef = torch.zeros(n, dtype=torch.complex128, device=dev())
    f = torch.empty(plan.nodes, dtype=torch.complex128, device=dev())
    toff = T(np.array([0, n], np.int64))
    with pytest.raises(m.Mr1lError, match="static term scratch"):
        m.mr1l_sample_noalloc(plan, freq, coef, f, toff)
    with pytest.raises(m.Mr1lError):
        m.mr1l_sample_noalloc(plan, freq[:, :10], coef[:10], f, None)
