"""Least-squares coefficients on the detected set (Remark 2.9) through the C ABI,
against the oracle's dense least squares on the same samples and detected set."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


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


def run(m, d, M, z, F, sets, f, theta, cap, s_cap):
    plan = m.Plan(d, M, z, F=F)
    g, bm = m.mr1l_fft(plan, T(f), theta)
    off = np.concatenate([[0], np.cumsum([s.shape[1] for s in sets])]).astype(np.int64)
    ex = m.mr1l_extract(plan, T(np.concatenate(sets, axis=1)), g, bm, theta, s_cap=s_cap, cap=cap,
                        set_off=T(off) if F > 1 else None)
    ls = m.mr1l_lsq(plan, ex, g, max_iter=400, tol=1e-15)
    torch.cuda.synchronize()
    return plan, ex, ls


def full_rank(cand, M, z, det):
    A = oracle.lsq_matrix(cand[:, det], M, z)
    return np.linalg.matrix_rank(A) == len(det)


@pytest.mark.parametrize("seed", list(range(8)))
def test_lsq_matches_oracle_noisy(m, seed):
    """Noisy samples (40 dB): the least-squares fit on the detected set equals the
    oracle's dense solution; Algorithm 4 keeps the same candidates."""
    say("lsq noisy", seed)
    p = synth.small_config(seed, L=6)
    fo = oracle.sample(p.supp, p.coef, p.M, p.z)
    f = fo + synth.noise_for(fo, p.M, 40.0, seed)
    plan, ex, ls = run(m, p.d, p.M, p.z, 1, [p.cand], f, 0.1, 2000, 64)
    nd = int(ex["n_det"][0])
    det = ex["det_idx"][0, :nd].cpu().numpy()
    if not full_rank(p.cand, p.M, p.z, det):
        pytest.skip("detected set not determined by the lattices")
    want = oracle.lsq(p.cand, p.M, p.z, f, det)
    got = ls["coef"][0, :nd].cpu().numpy()
    err = np.abs(got - want).max() / np.abs(want).max()
    say("n_det", nd, "iters", int(ls["iters"][0]), "resid", float(ls["resid"][0]), "err", err)
    assert err < 1e-9
    keep = np.abs(want) >= 0.1
    assert not np.any(np.abs(np.abs(want) - 0.1) < 1e-8)
    no = int(ls["n_out"][0])
    assert sorted(ls["out_idx"][0, :no].cpu().numpy().tolist()) == sorted(det[keep].tolist())


@pytest.mark.parametrize("seed", list(range(6)))
def test_lsq_zeroes_false_positives(m, seed):
    """Noise-free with heavy aliasing: the detected set holds false positives, the
    least-squares coefficients are exact on the support and zero elsewhere, and
    Algorithm 4 returns exactly the support."""
    say("lsq false positives", seed)
    p = synth.small_config(seed, L=5, mlo=60, mhi=110)
    f = oracle.sample(p.supp, p.coef, p.M, p.z)
    plan, ex, ls = run(m, p.d, p.M, p.z, 1, [p.cand], f, 1e-9, 2000, 200)
    nd = int(ex["n_det"][0])
    det = ex["det_idx"][0, :nd].cpu().numpy()
    if not set(p.supp_idx.tolist()) <= set(det.tolist()) or not full_rank(p.cand, p.M, p.z, det):
        pytest.skip("support not detected or not determined")
    say("n_det", nd, "support", len(p.supp_idx), "iters", int(ls["iters"][0]))
    want = np.zeros(nd, np.complex128)
    want[np.searchsorted(det, p.supp_idx)] = p.coef
    got = ls["coef"][0, :nd].cpu().numpy()
    assert np.abs(got - want).max() < 1e-9 * np.abs(p.coef).max()
    no = int(ls["n_out"][0])
    assert sorted(ls["out_idx"][0, :no].cpu().numpy().tolist()) == sorted(p.supp_idx.tolist())


def test_lsq_batched_many_lattices_and_empty(m):
    """Three functions (one with an empty candidate set) with 37 lattices each."""
    say("lsq batched L=37")
    rng = np.random.default_rng(17)
    L, d = 37, 4
    sets, Ms, zs, fs, supps = [], [], [], [], []
    for fi, (n, s) in enumerate([(800, 12), (0, 0), (1500, 30)]):
        cand = synth.distinct_uniform_points(rng, max(n, 1), d, -40, 40)[:, :n]
        supp = np.sort(rng.choice(n, size=s, replace=False)) if n else np.zeros(0, np.int64)
        coef = rng.standard_normal(s) + 1j * rng.standard_normal(s)
        M, z = synth.draw_lattices(rng, L, d, 40, 400)
        fo = oracle.sample(cand[:, supp], coef, M, z)
        fs.append(fo + (synth.noise_for(fo, M, 30.0, fi) if s else 0))
        sets.append(cand)
        Ms.append(M)
        zs.append(z)
        supps.append(supp)
    M = np.concatenate(Ms)
    z = np.concatenate(zs)
    plan, ex, ls = run(m, d, M, z, 3, sets, np.concatenate(fs), 0.05, 4096, 256)
    for fi in range(3):
        nd = int(ex["n_det"][fi])
        if fi == 1:
            assert nd == 0 and int(ls["iters"][1]) == 0 and int(ls["n_out"][1]) == 0
            continue
        det = ex["det_idx"][fi, :nd].cpu().numpy()
        Ml, zl = Ms[fi], zs[fi]
        assert full_rank(sets[fi], Ml, zl, det)
        want = oracle.lsq(sets[fi], Ml, zl, fs[fi], det)
        got = ls["coef"][fi, :nd].cpu().numpy()
        err = np.abs(got - want).max() / np.abs(want).max()
        say("function", fi, "n_det", nd, "iters", int(ls["iters"][fi]), "err", err)
        assert err < 1e-9


def test_lsq_long_list_normal_equations(m):
    """A 9,000-entry detected list (cap > 8192: the CG's group sums in global memory,
    Algorithm 4 by the global sort): the solution satisfies the normal equations
    G c = b rebuilt on the host from the oracle's buckets and the lattice values (the
    DFT itself is checked elsewhere), and the kept s~ = 100 are its largest entries."""
    say("lsq long list")
    rng = np.random.default_rng(23)
    d, n, L = 3, 9000, 5
    cand = synth.distinct_uniform_points(rng, n, d, -400, 400)
    M, z = synth.draw_lattices(rng, L, d, 40000, 60000)
    f = rng.standard_normal(int(M.sum())) + 1j * rng.standard_normal(int(M.sum()))
    plan = m.Plan(d, M, z)
    g, bm = m.mr1l_fft(plan, T(f), 1e-9)
    ex = m.mr1l_extract(plan, T(cand), g, bm, 1e-9, s_cap=100, cap=n, want_w=False)
    torch.cuda.synchronize()
    assert int(ex["n_det"][0]) == n
    ls = m.mr1l_lsq(plan, ex, g, max_iter=300, tol=1e-13)
    torch.cuda.synchronize()
    say("iters", int(ls["iters"][0]), "resid", float(ls["resid"][0]))
    assert float(ls["resid"][0]) <= 1e-13
    # normal equations checked on the host: G c = b, G and b from the bucket structure
    c = ls["coef"][0, :n].cpu().numpy()
    h = oracle.hash_buckets(cand, M, z)
    go = g.cpu().numpy()
    offs = np.concatenate([[0], np.cumsum(M)])
    Gc = np.zeros(n, np.complex128)
    b = np.zeros(n, np.complex128)
    for l in range(L):
        sums = np.zeros(int(M[l]), np.complex128)
        np.add.at(sums, h[l], c)
        Gc += M[l] * sums[h[l]]
        b += M[l] * go[offs[l] + h[l]]
    assert np.linalg.norm(Gc - b) <= 1e-10 * np.linalg.norm(b)
    # Algorithm 4 on the solution: the 100 largest magnitudes (theta is far below them)
    c_dev = ls["coef"][0, :n].cpu().numpy()
    want = set(cand_idx for cand_idx in np.asarray(ex["det_idx"][0, :n].cpu())[np.argsort(-np.abs(c_dev))[:100]])
    assert int(ls["n_out"][0]) == 100
    assert set(ls["out_idx"][0].cpu().numpy().tolist()) == want
