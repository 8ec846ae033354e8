"""The batched workload at full size against the oracle, function by function.

512 functions in one plan (d = 10, s log-uniform in [10, 1000], |Gamma| log-uniform in
[1e3, 1e6] from [-128, 128]^10, L = 8 distinct primes in [8s, 16s], 7.58e7 candidates
in all), run as one launch per stage, in complex128 and complex64.  This is the regime
where a vote workgroup walks many tiles and crosses function boundaries.

The oracle's lattice values are the bucket sums of eq. (2.4) (the normalised lattice
DFT of noise-free samples of a sparse polynomial equals them exactly), computed in
double precision per function; its Algorithm 2 + Remark 2.9 + Algorithm 4 run over
every candidate of every function.  Compared per function: lattice values (1e-11 /
1e-5 of the function's largest modulus), the non-zero bitmap, the detected count and
indices, the singleton masks (bit-exact), the median and post-processed coefficients
(tolerance), Algorithm 4's entries and order (up to rounding ties).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from test_gpu_parity import EPS, TOL, check_limit, close, fragile, mask64, say, unpack_bits

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m():
    import paper_2006_13053_amd as mod
    mod.lib()
    torch.cuda.set_device(0)
    return mod


@pytest.fixture(scope="module")
def workload():
    """Inputs shared by both precisions: the draws and every candidate set on the host."""
    wl = synth.batch_workload(2027, 512)
    dev = torch.device("cuda", 0)
    off = wl.set_off
    cand_dev = torch.empty((wl.d, int(off[-1])), dtype=torch.int64, device=dev)
    for f in range(wl.F):
        cand_dev[:, off[f]:off[f + 1]] = wl.candidates(f, device=dev)
    cand = cand_dev.cpu().numpy()
    supp = np.ascontiguousarray(np.concatenate([cand[:, off[f] + wl.supp_idx[f]] for f in range(wl.F)], axis=1))
    yield wl, cand_dev, cand, supp
    del cand_dev


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_batched_workload_full_size_matches_oracle(m, workload, dtype):
    wl, cand_dev, cand, supp = workload
    F, L, d = wl.F, wl.L, wl.d
    theta = 1e-3 if dtype == torch.complex64 else 1e-12
    cap, s_cap = 4096, 2048
    tol, eps = TOL[dtype], EPS[dtype]
    say("full batched workload", dtype, "candidates", int(wl.n.sum()))
    dev = torch.device("cuda", 0)
    plan = m.Plan(d, wl.M, wl.z, F=F, dtype=dtype)
    f = m.mr1l_sample(plan, torch.from_numpy(supp).to(dev),
                      torch.from_numpy(np.concatenate(wl.coef)).to(dev).to(dtype),
                      term_off=torch.from_numpy(wl.term_off).to(dev), mode=1)
    g, bm = m.mr1l_fft(plan, f, theta)
    so = torch.from_numpy(wl.set_off).to(dev)
    ex = m.mr1l_extract(plan, cand_dev, g, bm, theta, s_cap=s_cap, cap=cap, set_off=so, want_w=False)
    torch.cuda.synchronize()
    gh = g.cpu().numpy().astype(np.complex128)
    bits = unpack_bits(bm.cpu().numpy(), plan.nodes)
    r = {k: ex[k].cpu() for k in ("n_det", "det_idx", "det_coef", "det_med", "det_mask", "n_out", "out_idx",
                                  "out_coef", "out_pos")}
    node_off = np.concatenate([[0], np.cumsum(wl.M)]).astype(np.int64)
    soff, toff = wl.set_off, wl.term_off
    n_fragile, n_checked, n_det_total = 0, 0, 0
    for fi in range(F):
        Mf = wl.M[fi * L:(fi + 1) * L]
        zf = wl.z[fi * L:(fi + 1) * L]
        a, b = node_off[fi * L], node_off[(fi + 1) * L]
        go = oracle.bucket_sums(np.ascontiguousarray(supp[:, toff[fi]:toff[fi + 1]]), wl.coef[fi], Mf, zf)
        close(gh[a:b], go, tol, f"function {fi} lattice values")
        band = fragile(go, theta, eps)
        assert np.array_equal(bits[a:b][~band], ((go.real ** 2 + go.imag ** 2) >= theta * theta)[~band]), fi
        if band.any():
            n_fragile += 1
            continue
        cf = np.ascontiguousarray(cand[:, soff[fi]:soff[fi + 1]])
        ro = oracle.extract(cf, Mf, zf, go, theta, s_cap=s_cap, cap=cap)
        nd = int(r["n_det"][fi])
        assert nd == ro["n_det"], (fi, nd, ro["n_det"])
        k = min(nd, cap)
        det_idx = r["det_idx"][fi, :k].numpy()
        assert np.array_equal(det_idx, ro["det_idx"]), fi
        assert np.array_equal(mask64(r["det_mask"][fi, :k]), ro["det_mask"]), fi
        close(r["det_med"][fi, :k].numpy(), ro["det_med"], tol, f"function {fi} medians")
        close(r["det_coef"][fi, :k].numpy(), ro["det_coef"], tol, f"function {fi} post-processed coefficients")
        no = int(r["n_out"][fi])
        rr = dict(out_idx=r["out_idx"][fi, :no].numpy(), out_coef=r["out_coef"][fi, :no].numpy())
        check_limit(rr, ro, eps, tol)
        assert np.array_equal(det_idx[r["out_pos"][fi, :no].numpy()], rr["out_idx"]), fi
        # every true support member is found: the method recovers these polynomials
        assert np.isin(wl.supp_idx[fi], det_idx).all(), fi
        n_checked += 1
        n_det_total += nd
    say(f"{n_checked} functions equal to the oracle ({n_det_total} detected), {n_fragile} with a threshold "
        f"decision inside the rounding band")
    assert n_fragile == 0
    assert n_checked == F
