"""Parity of the HIP path (through the C ABI) with the CPU oracle on the same seeded inputs.

Integer results (buckets, counts, votes, detected sets, singleton masks, output order)
must be bit-exact; floating point within 1e-11 (complex128) or 1e-5 (complex64)
relative to the scale of the compared vector.  A threshold decision whose oracle
modulus lies within a rounding band of theta is reported and excluded from the exact
comparison (expected: none).
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = {torch.complex128: 1e-11, torch.complex64: 1e-5}


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


def close(a, b, tol, what):
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    if a.size == 0:
        return
    scale = max(1e-300, float(np.abs(b).max()))
    err = float(np.abs(a - b).max()) / scale
    assert err <= tol, f"{what}: rel err {err:.3e} > {tol:.0e}"


def unpack_bits(words, nodes):
    w = np.asarray(words).view(np.uint32)
    bits = ((w[:, None] >> np.arange(32, dtype=np.uint32)[None, :]) & 1).reshape(-1)
    return bits[:nodes].astype(bool)


def oracle_bitmap(g, theta):
    return (g.real ** 2 + g.imag ** 2) >= theta * theta


EPS = {torch.complex128: 2.0 ** -53, torch.complex64: 2.0 ** -24}


def fragile(g, theta, eps):
    """Threshold decisions whose oracle modulus lies within the DFT's rounding error of
    theta (unit roundoff of the working precision times 16 log2 of the largest
    Bluestein length, relative to the largest modulus)."""
    mag = np.abs(g)
    return np.abs(mag - theta) <= 16 * 16 * eps * max(1e-300, mag.max())


def check_limit(r, ro, eps, tol):
    """Algorithm 4 output: same entries and the same order except among entries whose
    moduli are equal within rounding (their order is not unique)."""
    gi, go_ = r["out_idx"], ro["out_idx"]
    gc, oc = r["out_coef"], ro["out_coef"]
    assert gi.shape == go_.shape, (gi.shape, go_.shape)
    if gi.size == 0:
        return
    scale = max(1e-300, float(np.abs(oc).max()))
    delta = 256 * eps * scale
    omag = dict(zip(go_.tolist(), np.abs(oc).tolist()))
    mag_min = float(np.abs(oc).min())
    boundary = {i for i, mg in omag.items() if abs(mg - mag_min) <= delta}
    missing = set(go_.tolist()) - set(gi.tolist())
    assert missing <= boundary, f"outputs differ beyond boundary ties: {sorted(missing)[:10]}"
    close(np.sort(np.abs(gc))[::-1], np.sort(np.abs(oc))[::-1], tol, "output moduli")
    seq = [omag.get(i, mag_min) for i in gi.tolist()]
    assert all(seq[o] >= seq[o + 1] - delta for o in range(len(seq) - 1)), "order differs beyond ties"
    ocd = dict(zip(go_.tolist(), oc.tolist()))
    for i, c in zip(gi.tolist(), gc.tolist()):
        if i in ocd:
            assert abs(c - ocd[i]) <= tol * scale


# ------------------------------------------------------------------ hashing
@pytest.mark.parametrize("d,n,box,L,mlo,mhi", [
    (5, 2000, 32, 5, 160, 320),
    (10, 20000, 64, 10, 800, 1600),
    (25, 5000, 32, 7, 4133, 4133),
    (3, 3000, 2**40, 6, 10000, 16000),      # beyond the 24-bit bound: exact 64-bit path
    (10, 4000, 512, 20, 16001, 16001),
    (13, 3000, 40, 6, 500, 900),            # dimensions without a kernel of their own:
    (23, 3000, 20, 6, 2000, 3000),          # coordinate registers for d <= 16, <= 32
    (40, 2000, 10, 5, 3000, 4000),          # and any d
])
def test_hash_count_bit_exact(m, d, n, box, L, mlo, mhi):
    say("hash_count", d, n, box, L)
    rng = np.random.default_rng(d * 7 + L)
    freq = rng.integers(-box, box + 1, size=(d, n), dtype=np.int64)
    freq[:, 0] = box
    freq[:, 1] = -box
    if box < 2**20:
        freq[0, 2] = 2**45            # one candidate outside the fast bound
    M, z = synth.draw_lattices(rng, L, d, mlo, mhi, distinct=mlo != mhi)
    plan = m.Plan(d, M, z)
    h, c = m.mr1l_hash_count(plan, T(freq))
    torch.cuda.synchronize()
    assert np.array_equal(h.cpu().numpy(), oracle.hash_buckets(freq, M, z))
    assert np.array_equal(c.cpu().numpy(), oracle.counts(freq, M, z))


def test_hash_count_batched_functions(m):
    say("hash_count batched F=3")
    rng = np.random.default_rng(3)
    d, L = 6, 4
    sizes = [100, 1, 777]
    sets = [rng.integers(-100, 101, size=(d, n), dtype=np.int64) for n in sizes]
    Ms, zs = [], []
    for f in range(3):
        M, z = synth.draw_lattices(rng, L, d, 200, 600)
        Ms.append(M)
        zs.append(z)
    plan = m.Plan(d, np.concatenate(Ms), np.concatenate(zs), F=3)
    allf = np.concatenate(sets, axis=1)
    off = T(np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64))
    h, c = m.mr1l_hash_count(plan, T(allf), set_off=off)
    torch.cuda.synchronize()
    h, c = h.cpu().numpy(), c.cpu().numpy()
    pos, nodes = 0, 0
    for f in range(3):
        ho = oracle.hash_buckets(sets[f], Ms[f], zs[f])
        assert np.array_equal(h[:, pos:pos + sizes[f]], ho)
        co = oracle.counts(sets[f], Ms[f], zs[f])
        assert np.array_equal(c[nodes:nodes + co.shape[0]], co)
        pos += sizes[f]
        nodes += co.shape[0]


# ------------------------------------------------------------------ DFT
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("Ms", [[2, 3, 5, 7], [163, 211, 317], [1009, 4133], [5113, 5119], [16001], [15991, 12007],
                                [40009], [131071]])
def test_fft_matches_direct_dft(m, Ms, dtype):
    say("fft", Ms, dtype)
    rng = np.random.default_rng(sum(Ms))
    M = np.array(Ms, np.int64)
    z = rng.integers(0, 2, size=(len(Ms), 1)).astype(np.int64)
    f = rng.standard_normal(int(M.sum())) + 1j * rng.standard_normal(int(M.sum()))
    plan = m.Plan(1, M, z % M[:, None], dtype=dtype)
    g, bm = m.mr1l_fft(plan, T(f.astype(np.complex128)).to(dtype), theta=0.05)
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.complex128)
    off = 0
    for mm in M:
        mm = int(mm)
        if mm <= 5200:
            go = oracle.dft(f[off:off + mm], np.array([mm]))
            bins = np.arange(mm)
        else:   # large prime: direct DFT on sampled bins (O(M) each)
            bins = np.unique(np.concatenate([[0, 1, mm - 1], rng.integers(0, mm, 400)]))
            go = oracle.dft_bins(f[off:off + mm], mm, bins)
        scale = np.abs(go).max()
        err = np.abs(g[off + bins] - go).max() / scale
        assert err <= TOL[dtype], f"M={mm} err {err:.2e}"
        off += mm


def test_plan_created_on_one_stream_runs_on_another(m):
    """A plan's tables are uploaded and its spectra computed on the creation stream
    without a host wait; moving the plan to another stream orders that stream after the
    creation work, so the first transform on it already sees the tables (same values as a
    plan created and run on the current stream)."""
    say("plan stream switch")
    rng = np.random.default_rng(77)
    M = np.array([16001, 12007, 4133, 211, 7], np.int64)
    z = np.stack([rng.integers(0, mm, size=3) for mm in M])
    f = T(rng.standard_normal(int(M.sum())) + 1j * rng.standard_normal(int(M.sum())))
    ref = m.Plan(3, M, z)
    g0, _ = m.mr1l_fft(ref, f, 1e-9)
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    for rep in range(3):
        with torch.cuda.stream(sa):
            p = m.Plan(3, M, z)
        p.set_stream(sb)
        with torch.cuda.stream(sb):
            g1, _ = m.mr1l_fft(p, f, 1e-9)
        torch.cuda.synchronize()
        assert torch.equal(g0, g1), rep
        p.close()


def test_plans_reuse_cached_device_blocks(m):
    """Plans destroyed and created in turn reuse the library's cached device blocks (also
    the long-list scratch, which grows inside the call): every repetition gives the first
    one's results, before and after the cache is emptied."""
    say("device block cache")
    rng = np.random.default_rng(91)
    d, L = 3, 7
    cand = synth.distinct_uniform_points(rng, 12000, d, -100, 100)
    M, z = synth.draw_lattices(rng, L, d, 3000, 4000)
    g_np = rng.standard_normal(int(M.sum())) + 1j * rng.standard_normal(int(M.sum()))

    def run():
        plan = m.Plan(d, M, z)
        g = T(g_np)
        bm = torch.full(((plan.nodes + 31) // 32,), -1, dtype=torch.int32, device=dev())
        ex = m.mr1l_extract(plan, T(cand), g, bm, 1e-9, s_cap=500, cap=16384, want_w=False)
        torch.cuda.synchronize()
        out = [ex[k].clone() for k in ("n_det", "det_idx", "det_coef", "det_mask", "n_out", "out_idx", "out_coef")]
        plan.close()
        return out

    ref = run()
    assert int(ref[0][0]) == 12000
    for rep in range(4):
        if rep == 2:
            m.mr1l_release_cache()
        got = run()
        for a, b in zip(ref, got):
            assert torch.equal(a, b), rep


def _fft_check(m, plan, f, dtype, rng):
    g, _ = m.mr1l_fft(plan, T(f.astype(np.complex128)).to(dtype), theta=0.05)
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.complex128)
    off = 0
    for mm in plan.M:
        mm = int(mm)
        if mm <= 5200:
            go = oracle.dft(f[off:off + mm], np.array([mm]))
            bins = np.arange(mm)
        else:
            bins = np.unique(np.concatenate([[0, 1, mm - 1], rng.integers(0, mm, 300)]))
            go = oracle.dft_bins(f[off:off + mm], mm, bins)
        err = np.abs(g[off + bins] - go).max() / np.abs(go).max()
        assert err <= TOL[dtype], f"M={mm} err {err:.2e}"
        off += mm
    # the non-zero bitmap, dense for the small sizes and about half full for the largest
    # (|ghat|^2 has mean 2/M here), against the threshold test on the returned values
    # taken in the kernel's precision
    th = float(np.sqrt(2.0 / max(int(mm) for mm in plan.M)))
    g2, bm = m.mr1l_fft(plan, T(f.astype(np.complex128)).to(dtype), theta=th)
    torch.cuda.synchronize()
    gv = g2.cpu().numpy()
    rt = np.float64 if dtype == torch.complex128 else np.float32
    want = gv.real.astype(rt) * gv.real.astype(rt) + gv.imag.astype(rt) * gv.imag.astype(rt) >= rt(th * th)
    assert np.array_equal(unpack_bits(bm.cpu().numpy(), plan.nodes), want)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("Ms", [[2, 3, 5, 7, 163], [1009, 4133], [16001], [20011, 32749], [40009]])
def test_fft_every_schedule(m, Ms, dtype):
    """Every DFT schedule that applies to a size computes the same transform (the
    sizes 20011 and 32749 sit where the two-level chirp table outgrows its LDS copy)."""
    rng = np.random.default_rng(7 + sum(Ms))
    M = np.array(Ms, np.int64)
    f = rng.standard_normal(int(M.sum())) + 1j * rng.standard_normal(int(M.sum()))
    plan = m.Plan(1, M, np.ones((len(Ms), 1), np.int64), dtype=dtype)
    names = m.fft_schedule_names()
    for s, name in enumerate(names):
        if name in ("reg", "split"):
            ok = [reg_ok(int(mm), dtype) if name == "reg" else split_ok(int(mm), dtype) for mm in M]
            for mm, o in zip(M, ok):
                if o:
                    assert plan.fft_schedule(int(mm), s) == s
                else:
                    with pytest.raises(m.Mr1lError):
                        plan.fft_schedule(int(mm), s)
            if not any(ok):
                continue
        elif name.startswith("rader"):
            if not any(rader_ok(int(mm), dtype) for mm in M):
                with pytest.raises(m.Mr1lError):
                    plan.fft_schedule(int(M[0]), s)
                continue
            for mm in np.unique(M):
                if rader_ok(int(mm), dtype):
                    assert plan.fft_schedule(int(mm), s) == s
        elif s == 0 and max(Ms) > 5000:
            with pytest.raises(m.Mr1lError):
                plan.fft_schedule(int(M[0]), s)
            continue
        else:
            for mm in np.unique(M):
                assert plan.fft_schedule(int(mm), s) == s
        say("fft schedule", name, Ms, dtype)
        _fft_check(m, plan, f, dtype, rng)


def reg_ok(M, dtype):
    """Sizes the reg schedule takes: the power of two N >= 2M - 1 (at least 64) is at
    most 16384 in complex128 and 32768 in complex64."""
    n = 64
    while n < 2 * M - 1:
        n *= 2
    return n <= (16384 if dtype == torch.complex128 else 32768)


def split_ok(M, dtype):
    """Sizes the split schedule takes: complex128, too large for reg, M <= 4 * 8192."""
    return dtype == torch.complex128 and not reg_ok(M, dtype) and M <= 32768


def rader_ok(M, dtype):
    """Sizes the Rader schedule takes: prime M, M - 1 = 2^a 5^b, a multiple of the
    20 values per thread, within one workgroup (1024 threads) and its LDS."""
    P = M - 1
    if M < 3 or any(M % q == 0 for q in range(2, int(M ** 0.5) + 1)):
        return False
    q = P
    while q % 2 == 0:
        q //= 2
    while q % 5 == 0:
        q //= 5
    e, th, w = (20, 1024, 8) if dtype == torch.complex128 else (20, 1024, 4)
    return q == 1 and P % e == 0 and P // e <= th and P * w + 2048 <= 163840


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_rader_schedule_forward_and_inverse(m, dtype):
    """Prime sizes with M - 1 = 2^a 5^b under the Rader schedule (with sizes of other
    schedules in the same plan): the forward DFT against the oracle, and the inverse
    DFT through the bucket sampler (eq. (2.4) then an inverse lattice DFT times M)."""
    Ms = [41, 101, 401, 641, 1601, 4001, 16001, 211, 4133]
    rng = np.random.default_rng(3)
    M = np.array(Ms, np.int64)
    z = rng.integers(1, 40, size=(len(Ms), 2)) % M[:, None]
    plan = m.Plan(2, M, z, dtype=dtype)
    rs = m.fft_schedule_names().index("rader-20")
    took = [mm for mm in Ms if rader_ok(mm, dtype)]
    assert 16001 in took
    for mm in took:
        assert plan.fft_schedule(mm, rs) == rs
    say("rader", dtype, took)
    f = rng.standard_normal(int(M.sum())) + 1j * rng.standard_normal(int(M.sum()))
    _fft_check(m, plan, f, dtype, rng)
    freq = synth.distinct_uniform_points(rng, 300, 2, -500, 500)
    coef = rng.standard_normal(300) + 1j * rng.standard_normal(300)
    got = m.mr1l_sample(plan, T(freq), T(coef).to(dtype), mode=2)
    torch.cuda.synchronize()
    want = oracle.sample(freq, coef, M, z)
    err = np.abs(got.cpu().numpy().astype(np.complex128) - want).max() / np.abs(want).max()
    assert err <= 10 * TOL[dtype], err


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_register_schedules_every_length_forward_and_inverse(m, dtype):
    """The reg schedule on every transform length it has (one prime size per power of
    two N from 64 to its largest, several lattices of the small sizes sharing a
    workgroup) and the split schedule on 2, 3 and 4 blocks (complex128): forward DFTs
    against the oracle, the non-zero bitmap, and the inverse DFT through the bucket
    sampler."""
    Ms = [2, 3, 31, 61, 127, 251, 509, 1021, 2039, 4093, 8191]
    if dtype == torch.complex64:
        Ms += [16381]
    else:
        Ms += [8209, 16001, 16411, 24571, 24593, 32749]
    # more lattices of one size than one workgroup holds (32 of size 37 per workgroup)
    Ms += [37] * 40 + [211] * (64 - 40 - len(Ms))
    rng = np.random.default_rng(11)
    M = np.array(Ms, np.int64)
    z = rng.integers(1, 1000, size=(len(Ms), 2)) % M[:, None]
    plan = m.Plan(2, M, z, dtype=dtype)
    names = m.fft_schedule_names()
    for mm in sorted(set(Ms)):
        want = "reg" if reg_ok(mm, dtype) else "split"
        assert split_ok(mm, dtype) or want == "reg", mm
        assert plan.fft_schedule(mm, names.index(want)) == names.index(want)
    say("register schedules", dtype)
    f = rng.standard_normal(int(M.sum())) + 1j * rng.standard_normal(int(M.sum()))
    _fft_check(m, plan, f, dtype, rng)
    freq = synth.distinct_uniform_points(rng, 400, 2, -500, 500)
    coef = rng.standard_normal(400) + 1j * rng.standard_normal(400)
    got = m.mr1l_sample(plan, T(freq), T(coef).to(dtype), mode=2)
    torch.cuda.synchronize()
    want = oracle.sample(freq, coef, M, z)
    err = np.abs(got.cpu().numpy().astype(np.complex128) - want).max() / np.abs(want).max()
    assert err <= 10 * TOL[dtype], err


def test_fft_tuner_picks_fastest_and_stays_exact(m):
    rng = np.random.default_rng(99)
    M = np.array([211] * 8 + [4133] * 8 + [16001] * 8, np.int64)
    z = rng.integers(1, 200, size=(len(M), 2)).astype(np.int64)
    plan = m.Plan(2, M, z)
    say("fft tune")
    res = plan.fft_tune(reps=2)
    assert sorted(res) == [211, 4133, 16001]
    for mm, times in res.items():
        assert times and all(t > 0 for t in times.values())
        assert ("lds" in times) == (mm != 16001)
        best = min(times, key=times.get)
        assert m.fft_schedule_names()[plan.fft_schedule(mm)] == best
        # a later plan of the same size starts on the tuned schedule
        assert m.Plan(2, np.array([mm]), z[:1]).fft_schedule(mm) == plan.fft_schedule(mm)
    f = rng.standard_normal(int(M.sum())) + 1j * rng.standard_normal(int(M.sum()))
    _fft_check(m, plan, f, torch.complex128, rng)


def test_fft_bitmap_and_aliasing_formula(m):
    """Sample -> DFT on a sparse polynomial equals the bucket sums (eq. (2.4)); the
    bitmap is exactly the set of occupied buckets."""
    say("fft bitmap eq. 2.4")
    p = synth.small_config(4)
    plan = m.Plan(p.d, p.M, p.z)
    f = oracle.sample(p.supp, p.coef, p.M, p.z)
    g, bm = m.mr1l_fft(plan, T(f), p.theta)
    torch.cuda.synchronize()
    b = oracle.bucket_sums(p.supp, p.coef, p.M, p.z)
    close(g.cpu().numpy(), b, 1e-11, "ghat vs bucket sums")
    occupied = oracle.counts(p.supp, p.M, p.z) > 0
    assert np.array_equal(unpack_bits(bm.cpu().numpy(), plan.nodes), occupied)


def test_inverse_dft_via_sampler_bucket_mode(m):
    say("sample bucket mode")
    p = synth.small_config(5)
    plan = m.Plan(p.d, p.M, p.z)
    fb = m.mr1l_sample(plan, T(p.supp), T(p.coef), mode=2)
    fd = m.mr1l_sample(plan, T(p.supp), T(p.coef), mode=1)
    torch.cuda.synchronize()
    fo = oracle.sample(p.supp, p.coef, p.M, p.z)
    close(fd.cpu().numpy(), fo, 1e-11, "direct samples")
    close(fb.cpu().numpy(), fo, 1e-11, "bucket-mode samples")


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("anchored", [False, True])
def test_sample_bucket_mode_lds_sums(m, dtype, anchored):
    """Bucket-mode sampling of functions with many terms per bucket (the buckets of a
    lattice summed in LDS per chunk of terms): three functions of uneven length, against
    the oracle's direct evaluation of eq. (2.2)."""
    say("sample bucket mode lds", dtype, anchored)
    rng = np.random.default_rng(21 + anchored)
    d_poly, t, F, L = 5, (3 if anchored else 5), 4, 4
    counts = [5000, 12000, 0, 700]   # one function without terms
    freqs = [rng.integers(-60, 61, size=(d_poly, n), dtype=np.int64) for n in counts]
    coefs = [rng.standard_normal(n) + 1j * rng.standard_normal(n) for n in counts]
    Ms, zs = [], []
    for f in range(F):
        M, z = synth.draw_lattices(rng, L, t, 150, 400)
        Ms.append(M)
        zs.append(z)
    anc = rng.integers(0, 2**32, size=(F, d_poly - t), dtype=np.uint64).astype(np.uint32)
    plan = m.Plan(t, np.concatenate(Ms), np.concatenate(zs), F=F, dtype=dtype)
    toff = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    kw = dict(anchor=T(anc.reshape(-1).view(np.int32))) if anchored else {}
    got = m.mr1l_sample(plan, T(np.concatenate(freqs, axis=1)), T(np.concatenate(coefs)).to(dtype),
                        term_off=T(toff), mode=2, **kw)
    torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.complex128)
    off = 0
    for f in range(F):
        n = int(Ms[f].sum())
        if counts[f] == 0:
            assert np.all(got[off:off + n] == 0), f
            off += n
            continue
        want = oracle.sample(freqs[f], coefs[f], Ms[f], zs[f], anchor=anc[f] if anchored else None,
                             t=t if anchored else None)
        err = np.abs(got[off:off + n] - want).max() / np.abs(want).max()
        assert err <= TOL[dtype], (f, err)
        off += n


@pytest.mark.parametrize("mode", [1, 2])
def test_sample_more_than_16_dimensions(m, mode):
    """Lattices of dimension 20 (beyond the register-held coordinate path of the term
    preparation), direct and bucket modes, against the oracle."""
    say("sample d=20", mode)
    rng = np.random.default_rng(31)
    d, n = 20, 3000
    freq = rng.integers(-40, 41, size=(d, n), dtype=np.int64)
    coef = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    M, z = synth.draw_lattices(rng, 3, d, 200, 300)
    plan = m.Plan(d, M, z)
    got = m.mr1l_sample(plan, T(freq), T(coef), mode=mode)
    torch.cuda.synchronize()
    close(got.cpu().numpy(), oracle.sample(freq, coef, M, z), 1e-11, f"d=20 mode {mode}")


def test_sample_with_anchors(m):
    say("sample anchors")
    rng = np.random.default_rng(8)
    d, t, s = 8, 3, 40
    freq = rng.integers(-32, 33, size=(d, s), dtype=np.int64)
    coef = rng.standard_normal(s) + 1j * rng.standard_normal(s)
    anc = rng.integers(0, 2**32, size=d - t, dtype=np.uint64).astype(np.uint32)
    M, z = synth.draw_lattices(rng, 5, t, 300, 700)
    plan = m.Plan(t, M, z)
    for mode in (1, 2):
        f = m.mr1l_sample(plan, T(freq), T(coef), anchor=T(anc.view(np.int32)), mode=mode)
        torch.cuda.synchronize()
        close(f.cpu().numpy(), oracle.sample(freq, coef, M, z, anchor=anc, t=t), 1e-11, f"anchored mode {mode}")


# ------------------------------------------------------------------ full pass
def mask64(dm):
    """Singleton masks ([n] or [n][2] uint32 words) as uint64 values."""
    w = dm.cpu().numpy().view(np.uint32).astype(np.uint64)
    return w if w.ndim == 1 else w[:, 0] | (w[:, 1] << np.uint64(32))


def gpu_pass(m, p, f_np=None, dtype=torch.complex128, s_cap=None, cap=4096, postproc=True, vote_min=0,
             want_votes=True):
    plan = m.Plan(p.d, p.M, p.z, dtype=dtype)
    if f_np is None:
        f = m.mr1l_sample(plan, T(p.supp), T(p.coef.astype(np.complex128)).to(dtype))
    else:
        f = T(f_np).to(dtype)
    g, bm = m.mr1l_fft(plan, f, p.theta)
    s_cap = s_cap or min(cap, p.n)
    ex = m.mr1l_extract(plan, T(p.cand), g, bm, p.theta, s_cap=s_cap, cap=cap, postproc=postproc,
                        vote_min=vote_min, want_votes=want_votes)
    torch.cuda.synchronize()
    nd = int(ex["n_det"][0])
    k = min(nd, cap)
    no = int(ex["n_out"][0])
    r = dict(n_det=nd, ghat=g.cpu().numpy(), bitmap=unpack_bits(bm.cpu().numpy(), plan.nodes),
             det_idx=ex["det_idx"][0, :k].cpu().numpy(), det_mask=mask64(ex["det_mask"][0, :k]),
             det_coef=ex["det_coef"][0, :k].cpu().numpy(), det_med=ex["det_med"][0, :k].cpu().numpy(),
             out_idx=ex["out_idx"][0, :no].cpu().numpy(), out_coef=ex["out_coef"][0, :no].cpu().numpy(),
             out_pos=ex["out_pos"][0, :no].cpu().numpy())
    if want_votes:
        r["votes"] = ex["votes"].cpu().numpy()
    return r, plan, ex, f


def compare_pass(r, ro, go, theta, tol, s_cap, eps=EPS[torch.complex128]):
    band = fragile(go, theta, eps)
    exact = ~band
    assert np.array_equal(r["bitmap"][exact], oracle_bitmap(go, theta)[exact])
    if band.any():
        pytest.skip(f"{int(band.sum())} threshold decisions inside the rounding band")
    if "votes" in r:
        assert np.array_equal(r["votes"], ro["votes"])
    assert r["n_det"] == ro["n_det"]
    assert np.array_equal(r["det_idx"], ro["det_idx"])
    assert np.array_equal(r["det_mask"], ro["det_mask"])
    close(r["det_med"], ro["det_med"], tol, "median coefficients")
    close(r["det_coef"], ro["det_coef"], tol, "post-processed coefficients")
    check_limit(r, ro, eps, tol)
    # out_pos points into the detected list at the output's candidate
    assert np.array_equal(r["det_idx"][r["out_pos"]], r["out_idx"])


@pytest.mark.parametrize("L,seed", [(33, 1), (37, 2), (40, 3), (48, 4), (64, 5)])
def test_full_pass_beyond_32_lattices(m, L, seed):
    """More than 32 lattices per function: two-word singleton masks, wider median
    selection (odd and even L); plus the Dirichlet counts of eq. (4.1)."""
    say("full pass L", L, "seed", seed)
    p = synth.small_config(seed, L=L, mlo=200, mhi=900)
    r, *_ = gpu_pass(m, p, s_cap=40, cap=2000)
    fo = oracle.sample(p.supp, p.coef, p.M, p.z)
    go = oracle.dft(fo, p.M)
    ro = oracle.extract(p.cand, p.M, p.z, go, p.theta, s_cap=40, cap=2000)
    compare_pass(r, ro, go, p.theta, 1e-11, 40)
    pd = synth.dirichlet(synth.small_config(seed, L=L, mlo=31, mhi=400))
    r, *_ = gpu_pass(m, pd, s_cap=2000, cap=2000)
    god = oracle.dft(oracle.sample(pd.supp, pd.coef, pd.M, pd.z), pd.M)
    rod = oracle.extract(pd.cand, pd.M, pd.z, god, pd.theta, s_cap=2000, cap=2000)
    assert np.any(rod["det_mask"] >> np.uint64(32))   # masks use the second word
    compare_pass(r, rod, god, pd.theta, 1e-11, 2000)


@pytest.mark.parametrize("seed", list(range(100)))
def test_small_config_full_pass(m, seed):
    """d = 5, 2000 candidates, s = 20, L = 5, noise-free complex128 (the small plain case)."""
    say("small full pass seed", seed)
    p = synth.small_config(seed)
    r, *_ = gpu_pass(m, p, s_cap=40, cap=2000)
    fo = oracle.sample(p.supp, p.coef, p.M, p.z)
    go = oracle.dft(fo, p.M)
    close(r["ghat"], go, 1e-11, "ghat")
    ro = oracle.extract(p.cand, p.M, p.z, go, p.theta, s_cap=40, cap=2000)
    compare_pass(r, ro, go, p.theta, 1e-11, 40)


@pytest.mark.parametrize("postproc", [True, False])
def test_small_config_complex64(m, postproc):
    say("small full pass c64", postproc)
    p = synth.small_config(11)
    p.theta = 1e-3
    fo = oracle.sample(p.supp, p.coef, p.M, p.z)
    r, *_ = gpu_pass(m, p, f_np=fo, dtype=torch.complex64, s_cap=40, cap=2000, postproc=postproc)
    go = oracle.dft(fo, p.M)
    ro = oracle.extract(p.cand, p.M, p.z, go, p.theta, s_cap=40, cap=2000, postproc=postproc)
    compare_pass(r, ro, go, p.theta, 1e-5, 40, eps=EPS[torch.complex64])


@pytest.mark.parametrize("seed", list(range(20)))
def test_mid_config_full_pass_with_noise(m, seed):
    """d = 10, 1e5 candidates in [-64,64]^10, s = 100, L = 10, 40 dB noise, theta = 1/3."""
    say("mid full pass seed", seed)
    p = synth.mid_config(seed)
    fo = oracle.sample(p.supp, p.coef, p.M, p.z)
    f = fo + synth.noise_for(fo, p.M, 40.0, p.meta["noise_seed"])
    r, *_ = gpu_pass(m, p, f_np=f, s_cap=200, cap=4096)
    go = oracle.dft(f, p.M)
    ro = oracle.extract(p.cand, p.M, p.z, go, p.theta, s_cap=200, cap=4096)
    compare_pass(r, ro, go, p.theta, 1e-11, 200)
    # the support is found and its coefficients are within the noise of the truth
    assert set(p.supp_idx.tolist()) <= set(r["out_idx"].tolist())


def test_long_list_mode_with_empty_and_undetected_functions(m):
    """cap > 8192 (global-memory paths) with a function whose set is empty, one whose
    lattice values are all zero (nothing detected) and one that detects 12,000
    candidates: counts, order, masks and coefficients against the oracle."""
    say("long lists, empty functions")
    rng = np.random.default_rng(77)
    d, L = 3, 6
    sizes = [0, 3000, 12000]
    sets = [synth.distinct_uniform_points(rng, n, d, -80, 80) if n else np.zeros((d, 0), np.int64) for n in sizes]
    Ms, zs, fs = [], [], []
    for fi, n in enumerate(sizes):
        M, z = synth.draw_lattices(rng, L, d, 1500, 2500)
        Ms.append(M)
        zs.append(z)
        f = rng.standard_normal(int(M.sum())) + 1j * rng.standard_normal(int(M.sum()))
        fs.append(f if fi != 1 else np.zeros_like(f))
    plan = m.Plan(d, np.concatenate(Ms), np.concatenate(zs), F=3)
    g, bm = m.mr1l_fft(plan, T(np.concatenate(fs)), 1e-9)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    ex = m.mr1l_extract(plan, T(np.concatenate(sets, axis=1)), g, bm, 1e-9, s_cap=5000, cap=16384,
                        set_off=T(off), want_w=False)
    torch.cuda.synchronize()
    assert [int(v) for v in ex["n_det"].cpu()] == [0, 0, 12000]
    assert [int(v) for v in ex["n_out"].cpu()] == [0, 0, 5000]
    go = oracle.dft(fs[2], Ms[2])
    ro = oracle.extract(sets[2], Ms[2], zs[2], go, 1e-9, s_cap=5000, cap=16384)
    assert np.array_equal(ex["det_idx"][2, :12000].cpu().numpy(), ro["det_idx"])
    assert np.array_equal(mask64(ex["det_mask"][2, :12000]), ro["det_mask"])
    close(ex["det_coef"][2, :12000].cpu().numpy(), ro["det_coef"], 1e-11, "coefficients")
    r = dict(out_idx=ex["out_idx"][2, :5000].cpu().numpy(), out_coef=ex["out_coef"][2, :5000].cpu().numpy())
    check_limit(r, ro, EPS[torch.complex128], 1e-11)


@pytest.mark.parametrize("d", [13, 23, 40])
def test_full_pass_dimensions_without_own_kernel(m, d):
    """The vote kernel for dimensions that have no instance of their own (registers
    sized for d <= 16, d <= 32 and any d): full pass against the oracle."""
    say("full pass d", d)
    p = synth.small_config(40 + d, d=d, n=3000, box=12, L=7, mlo=300, mhi=600)
    r, *_ = gpu_pass(m, p, s_cap=40, cap=2000)
    go = oracle.dft(oracle.sample(p.supp, p.coef, p.M, p.z), p.M)
    ro = oracle.extract(p.cand, p.M, p.z, go, p.theta, s_cap=40, cap=2000)
    compare_pass(r, ro, go, p.theta, 1e-11, 40)


def test_vote_exact_path_edge_coordinates(m):
    """Candidates whose coordinates straddle the fast hash's bound wherever it lies
    (2^k - 1, 2^k, 2^k + 1 for k = 8..40, both signs) and 64-bit values whose low word
    alone would pass (2^32 + 5, -2^32 + 5): the vote pass's range test and its exact
    64-bit path, against the oracle; part of the support sits on such candidates."""
    say("vote exact path edges")
    rng = np.random.default_rng(57)
    d, L = 3, 7
    small = synth.distinct_uniform_points(rng, 1500, d, -30, 30)
    special = []
    for k in range(8, 41):
        for v in (2**k - 1, 2**k, 2**k + 1):
            for sgn in (1, -1):
                special.append([sgn * v, int(rng.integers(-5, 6)), int(rng.integers(-5, 6))])
    for v in (2**32 + 5, -2**32 + 5, 2**31, -2**31, 2**45 + 3):
        special.append([int(rng.integers(-5, 6)), v, int(rng.integers(-5, 6))])
    special = np.unique(np.array(special, np.int64), axis=0).T
    cand = np.concatenate([small, special], axis=1)
    cand = np.unique(cand, axis=1)
    n = cand.shape[1]
    supp_idx = np.sort(np.concatenate([rng.choice(n, 12, replace=False),
                                       np.flatnonzero(np.abs(cand).max(axis=0) > 2**20)[:8]]))
    supp_idx = np.unique(supp_idx)
    coef = rng.standard_normal(supp_idx.size) + 1j * rng.standard_normal(supp_idx.size)
    M, z = synth.draw_lattices(rng, L, d, 300, 900)
    f = oracle.sample(cand[:, supp_idx], coef, M, z)
    p = synth.Problem(d, cand, supp_idx, coef, M, z, theta=1e-12, meta=dict(workload="edges"))
    r, *_ = gpu_pass(m, p, f_np=f, s_cap=64, cap=4096)
    go = oracle.dft(f, M)
    ro = oracle.extract(cand, M, z, go, 1e-12, s_cap=64, cap=4096)
    compare_pass(r, ro, go, 1e-12, 1e-11, 64)


def test_vote_min_general_nu(m):
    say("vote_min")
    p = synth.small_config(6, mlo=40, mhi=90)
    fo = oracle.sample(p.supp, p.coef, p.M, p.z)
    go = oracle.dft(fo, p.M)
    for vm in (1, 2, 4, 5):
        r, *_ = gpu_pass(m, p, f_np=fo, s_cap=64, cap=2000, vote_min=vm)
        ro = oracle.extract(p.cand, p.M, p.z, go, p.theta, s_cap=64, cap=2000, vote_min=vm)
        compare_pass(r, ro, go, p.theta, 1e-11, 64)


def test_dirichlet_counting_polynomial(m):
    """eq. (4.1): all-ones coefficients on I; the lattice values are the integer alias
    counts and the median classification of Table 4.1 follows."""
    say("dirichlet")
    p = synth.dirichlet(synth.small_config(7, mlo=30, mhi=60))
    r, *_ = gpu_pass(m, p, s_cap=2000, cap=2000, postproc=False)
    cnt = oracle.counts(p.supp, p.M, p.z)
    assert np.abs(r["ghat"] - cnt).max() < 1e-11
    go = oracle.dft(oracle.sample(p.supp, p.coef, p.M, p.z), p.M)
    ro = oracle.extract(p.cand, p.M, p.z, go, p.theta, s_cap=2000, cap=2000, postproc=False)
    compare_pass(r, ro, go, p.theta, 1e-11, 2000)


def test_injectivity_check_matches_definition(m):
    """|Gamma mod M| = |Gamma| (Section 2.1), for sizes above and below the expansion
    of the set, single and batched."""
    rng = np.random.default_rng(11)
    d = 3
    cases = []
    for n, box, Ms in [(400, 20, [41, 43]), (30, 20, [7, 11]), (60, 20, [13, 17]), (200, 3, [5, 7]),
                       (1000, 40, [83, 89, 97]), (30, 20, [31, 37])]:
        cand = synth.distinct_uniform_points(rng, n, d, -box, box)
        M = np.array(Ms, np.int64)
        z = rng.integers(0, M.min(), size=(len(Ms), d)).astype(np.int64)
        want = all(np.unique(np.mod(cand, int(mm)), axis=1).shape[1] == n for mm in M)
        plan = m.Plan(d, M, z)
        ok_all, ok = m.mr1l_check_injective(plan, T(cand))
        say("injective", n, box, Ms, want)
        assert ok_all == want and bool(ok[0]) == want
        cases.append((cand, M, z, want))
    # a duplicate modulo M planted in a set whose range exceeds M
    cand = synth.distinct_uniform_points(rng, 50, d, -20, 20)
    cand[:, 7] = cand[:, 3] + np.array([13, -26, 0])
    if np.unique(cand, axis=1).shape[1] == 50:
        ok_all, _ = m.mr1l_check_injective(m.Plan(d, np.array([13]), np.ones((1, d), np.int64)), T(cand))
        assert not ok_all
    # batched: one plan over all cases with the same number of lattices
    sel = [c for c in cases if len(c[1]) == 2]
    plan = m.Plan(d, np.concatenate([c[1] for c in sel]), np.concatenate([c[2] for c in sel]), F=len(sel))
    soff = np.concatenate([[0], np.cumsum([c[0].shape[1] for c in sel])]).astype(np.int64)
    ok_all, ok = m.mr1l_check_injective(plan, T(np.concatenate([c[0] for c in sel], axis=1)), T(soff))
    assert list(ok) == [c[3] for c in sel] and ok_all == all(c[3] for c in sel)


@pytest.mark.parametrize("cap", [1, 2, 63, 1024, 1025, 4096, 8192])
def test_detected_order_and_limit_at_sort_sizes(m, cap):
    """The block sorts of the detected set and of Algorithm 4 at list lengths around
    their size boundaries (one value per thread up to 1024 entries, then 2, 4 and 8;
    lane-shuffle stages up to 64 values apart, LDS beyond): noise samples make every
    bucket non-zero, so every candidate of a function is detected and its sorted list is
    0, 1, ..., n - 1; Algorithm 4 against the oracle."""
    say("sort sizes", cap)
    rng = np.random.default_rng(7000 + cap)
    d, L = 3, 5
    sizes = sorted({n for n in (1, 2, 3, 63, 64, 65, 255, 256, 257, 1023, 1024, 1025, 2047, 2048, 4095,
                                4096, 4097, 8191, 8192) if n <= cap})
    F = len(sizes)
    sets, Ms, zs, fs = [], [], [], []
    for n in sizes:
        sets.append(synth.distinct_uniform_points(rng, n, d, -60, 60))
        M, z = synth.draw_lattices(rng, L, d, 1500, 2500)
        Ms.append(M)
        zs.append(z)
        fs.append(rng.standard_normal(int(M.sum())) + 1j * rng.standard_normal(int(M.sum())))
    plan = m.Plan(d, np.concatenate(Ms), np.concatenate(zs), F=F)
    g, bm = m.mr1l_fft(plan, T(np.concatenate(fs)), 1e-9)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    s_cap = max(1, cap // 2)
    ex = m.mr1l_extract(plan, T(np.concatenate(sets, axis=1)), g, bm, 1e-9, s_cap=s_cap, cap=cap,
                        set_off=T(off), want_w=False)
    torch.cuda.synchronize()
    for fi, n in enumerate(sizes):
        assert int(ex["n_det"][fi]) == n
        assert np.array_equal(ex["det_idx"][fi, :n].cpu().numpy(), np.arange(n))
        go = oracle.dft(fs[fi], Ms[fi])
        ro = oracle.extract(sets[fi], Ms[fi], zs[fi], go, 1e-9, s_cap=s_cap, cap=cap)
        no = int(ex["n_out"][fi])
        assert no == len(ro["out_idx"])
        r = dict(out_idx=ex["out_idx"][fi, :no].cpu().numpy(), out_coef=ex["out_coef"][fi, :no].cpu().numpy())
        check_limit(r, ro, EPS[torch.complex128], 1e-11)
        assert np.array_equal(ex["out_pos"][fi, :no].long().cpu().numpy(), r["out_idx"])


@pytest.mark.parametrize("seed,F,L", [(1, 1, 7), (2, 2, 7), (3, 1, 40)])
def test_long_detected_lists_match_oracle(m, seed, F, L):
    """Detected lists longer than 8192 (global-memory compaction and selection): noise
    samples make every bucket non-zero, so every candidate is detected; Algorithm 4
    keeps the 10000 (the kept pairs take the global sort) or 2500 (one workgroup's
    sort) largest medians.  Against the oracle per function, and against the LDS path
    on the same pass truncated to fit."""
    say("long lists", seed, F, L)
    rng = np.random.default_rng(100 + seed)
    d = 4
    sets, Ms, zs, fs = [], [], [], []
    for fi in range(F):
        n = 30000 - 7000 * fi
        sets.append(synth.distinct_uniform_points(rng, n, d, -60, 60))
        M, z = synth.draw_lattices(rng, L, d, 1500, 2500)
        Ms.append(M)
        zs.append(z)
        fs.append(rng.standard_normal(int(M.sum())) + 1j * rng.standard_normal(int(M.sum())))
    plan = m.Plan(d, np.concatenate(Ms), np.concatenate(zs), F=F)
    g, bm = m.mr1l_fft(plan, T(np.concatenate(fs)), 1e-9)
    off = np.concatenate([[0], np.cumsum([x.shape[1] for x in sets])]).astype(np.int64)
    cand = T(np.concatenate(sets, axis=1))
    # s~ above one workgroup's sort (the kept pairs take the global sort) and below it
    for s_cap in (10000, 2500):
        ex = m.mr1l_extract(plan, cand, g, bm, 1e-9, s_cap=s_cap, cap=32768, set_off=T(off), want_w=False)
        torch.cuda.synchronize()
        for fi in range(F):
            go = oracle.dft(fs[fi], Ms[fi])
            ro = oracle.extract(sets[fi], Ms[fi], zs[fi], go, 1e-9, s_cap=s_cap, cap=32768)
            nd = int(ex["n_det"][fi])
            assert nd == ro["n_det"] == sets[fi].shape[1]
            assert np.array_equal(ex["det_idx"][fi, :nd].cpu().numpy(), ro["det_idx"])
            assert np.array_equal(mask64(ex["det_mask"][fi, :nd]), ro["det_mask"])
            close(ex["det_coef"][fi, :nd].cpu().numpy(), ro["det_coef"], 1e-11, "coefficients")
            no = int(ex["n_out"][fi])
            r = dict(out_idx=ex["out_idx"][fi, :no].cpu().numpy(), out_coef=ex["out_coef"][fi, :no].cpu().numpy())
            check_limit(r, ro, EPS[torch.complex128], 1e-11)
            assert np.array_equal(ex["det_idx"][fi, ex["out_pos"][fi, :no].long()].cpu().numpy(), r["out_idx"])
    # a list that fits one workgroup's sort: the LDS path (cap 8192) and the global
    # path (cap 9000) give identical results
    sub = [x[:, :6000] for x in sets]
    off2 = T(np.arange(F + 1, dtype=np.int64) * 6000)
    cs = T(np.concatenate(sub, axis=1))
    outs = [m.mr1l_extract(plan, cs, g, bm, 1e-9, s_cap=3000, cap=c, set_off=off2, want_w=False) for c in (8192, 9000)]
    torch.cuda.synchronize()
    a, b = outs
    for fi in range(F):
        assert int(a["n_det"][fi]) == int(b["n_det"][fi]) == 6000
        assert torch.equal(a["det_idx"][fi, :6000], b["det_idx"][fi, :6000])
        assert torch.equal(a["det_coef"][fi, :6000], b["det_coef"][fi, :6000])
        assert int(a["n_out"][fi]) == int(b["n_out"][fi])
        assert torch.equal(a["out_idx"][fi], b["out_idx"][fi]) and torch.equal(a["out_coef"][fi], b["out_coef"][fi])


@pytest.mark.parametrize("L,mlo,mhi,F", [(20, 39000, 41000, 2), (3, 700000, 720000, 1), (48, 2500, 3500, 1)])
def test_long_lists_lattice_groups_match_oracle(m, L, mlo, mhi, F):
    """Long detected lists whose bucket bitmaps need several LDS passes: 20 lattices of
    M ~ 40000 (the occupancy count takes the lattices in two groups), 3 lattices of
    M ~ 700000 (one lattice exceeds the LDS: per-lattice passes over bucket spans), and
    48 lattices (the LDS-column combine with a separate mask pass).  The lattice values
    are random and every bit of the non-zero bitmap is set, so every candidate is
    detected; against the oracle on the same values."""
    say("long lists, lattice groups", L, mlo, F)
    rng = np.random.default_rng(7000 + L)
    d = 3
    sets, Ms, zs, gs = [], [], [], []
    for fi in range(F):
        sets.append(synth.distinct_uniform_points(rng, 20000 - 3000 * fi, d, -200, 200))
        M, z = synth.draw_lattices(rng, L, d, mlo, mhi)
        Ms.append(M)
        zs.append(z)
        gs.append(rng.standard_normal(int(M.sum())) + 1j * rng.standard_normal(int(M.sum())))
    plan = m.Plan(d, np.concatenate(Ms), np.concatenate(zs), F=F)
    g = T(np.concatenate(gs))
    bm = torch.full(((plan.nodes + 31) // 32,), -1, dtype=torch.int32, device=dev())
    off = np.concatenate([[0], np.cumsum([x.shape[1] for x in sets])]).astype(np.int64)
    ex = m.mr1l_extract(plan, T(np.concatenate(sets, axis=1)), g, bm, 1e-9, s_cap=2500, cap=32768,
                        set_off=T(off), want_w=False)
    torch.cuda.synchronize()
    for fi in range(F):
        ro = oracle.extract(sets[fi], Ms[fi], zs[fi], gs[fi], 1e-9, s_cap=2500, cap=32768)
        nd = int(ex["n_det"][fi])
        assert nd == ro["n_det"] == sets[fi].shape[1]
        assert np.array_equal(ex["det_idx"][fi, :nd].cpu().numpy(), ro["det_idx"])
        assert np.array_equal(mask64(ex["det_mask"][fi, :nd]), ro["det_mask"])
        close(ex["det_coef"][fi, :nd].cpu().numpy(), ro["det_coef"], 1e-11, "coefficients")
        no = int(ex["n_out"][fi])
        r = dict(out_idx=ex["out_idx"][fi, :no].cpu().numpy(), out_coef=ex["out_coef"][fi, :no].cpu().numpy())
        check_limit(r, ro, EPS[torch.complex128], 1e-11)


@pytest.mark.parametrize("mlo,mhi", [(2000, 3000), (40000, 50000)])
def test_short_lists_staged_coordinates_match_oracle(m, mlo, mhi):
    """Short detected lists take their buckets from the coordinates the vote pass staged:
    packed 16-bit pairs when every M <= 2^15 (first case), 32-bit words otherwise (second),
    and for candidates beyond the fast bound (|k| near 2^40 here) the exact path from the
    candidate set.  Random lattice values with every bitmap bit set, so that every
    candidate is detected; against the oracle, two functions of unequal size."""
    say("short lists, staged coordinates", mlo)
    rng = np.random.default_rng(mlo)
    d, L = 3, 7
    sets, Ms, zs, gs = [], [], [], []
    for fi in range(2):
        c = synth.distinct_uniform_points(rng, 3000 - 700 * fi, d, -200, 200)
        big = np.array([[(1 << 40) + 7 * j + fi, -(1 << 40) - j, 3 * j] for j in range(5)], np.int64).T
        sets.append(np.concatenate([c[:, :1000], big, c[:, 1000:]], axis=1))
        M, z = synth.draw_lattices(rng, L, d, mlo, mhi)
        Ms.append(M)
        zs.append(z)
        gs.append(rng.standard_normal(int(M.sum())) + 1j * rng.standard_normal(int(M.sum())))
    plan = m.Plan(d, np.concatenate(Ms), np.concatenate(zs), F=2)
    bm = torch.full(((plan.nodes + 31) // 32,), -1, dtype=torch.int32, device=dev())
    off = np.concatenate([[0], np.cumsum([x.shape[1] for x in sets])]).astype(np.int64)
    ex = m.mr1l_extract(plan, T(np.concatenate(sets, axis=1)), T(np.concatenate(gs)), bm, 1e-9, s_cap=500,
                        cap=4096, set_off=T(off), want_w=False)
    torch.cuda.synchronize()
    for fi in range(2):
        ro = oracle.extract(sets[fi], Ms[fi], zs[fi], gs[fi], 1e-9, s_cap=500, cap=4096)
        nd = int(ex["n_det"][fi])
        assert nd == ro["n_det"] == sets[fi].shape[1]
        assert np.array_equal(ex["det_idx"][fi, :nd].cpu().numpy(), ro["det_idx"])
        assert np.array_equal(mask64(ex["det_mask"][fi, :nd]), ro["det_mask"])
        close(ex["det_coef"][fi, :nd].cpu().numpy(), ro["det_coef"], 1e-11, "coefficients")
        no = int(ex["n_out"][fi])
        r = dict(out_idx=ex["out_idx"][fi, :no].cpu().numpy(), out_coef=ex["out_coef"][fi, :no].cpu().numpy())
        check_limit(r, ro, EPS[torch.complex128], 1e-11)


def test_empty_and_ragged_inputs(m):
    say("empty/ragged")
    p = synth.small_config(8)
    plan = m.Plan(p.d, p.M, p.z)
    f = m.mr1l_sample(plan, T(p.supp), T(p.coef))
    g, bm = m.mr1l_fft(plan, f, p.theta)
    empty = torch.zeros((p.d, 0), dtype=torch.int64, device=dev())
    ex = m.mr1l_extract(plan, empty, g, bm, p.theta, s_cap=4, cap=16)
    torch.cuda.synchronize()
    assert int(ex["n_det"][0]) == 0 and int(ex["n_out"][0]) == 0
    for n in (1, 63, 65, 257, 1999):
        sub = p.cand[:, :n]
        ex = m.mr1l_extract(plan, T(sub), g, bm, p.theta, s_cap=min(8, n), cap=n)
        torch.cuda.synchronize()
        go = oracle.dft(oracle.sample(p.supp, p.coef, p.M, p.z), p.M)
        ro = oracle.extract(sub, p.M, p.z, go, p.theta, s_cap=min(8, n), cap=n)
        assert int(ex["n_det"][0]) == ro["n_det"]
        assert np.array_equal(ex["det_idx"][0, :ro["n_det"]].cpu().numpy(), ro["det_idx"])
        no = int(ex["n_out"][0])
        assert np.array_equal(ex["out_idx"][0, :no].cpu().numpy(), ro["out_idx"])


def test_capacity_overflow_reports_required_size(m):
    say("capacity")
    p = synth.dirichlet(synth.small_config(9, mlo=20, mhi=30))
    plan = m.Plan(p.d, p.M, p.z)
    f = m.mr1l_sample(plan, T(p.supp), T(p.coef))
    g, bm = m.mr1l_fft(plan, f, p.theta)
    ex = m.mr1l_extract(plan, T(p.cand), g, bm, p.theta, s_cap=4, cap=8)
    torch.cuda.synchronize()
    go = oracle.dft(oracle.sample(p.supp, p.coef, p.M, p.z), p.M)
    ro = oracle.extract(p.cand, p.M, p.z, go, p.theta, s_cap=4, cap=p.n)
    assert ro["n_det"] > 8
    assert int(ex["n_det"][0]) == ro["n_det"]


# ------------------------------------------------------------------ adjoint / autograd
def test_adjoint_dense_transpose_and_dot_product(m):
    say("adjoint")
    p = synth.mid_config(1, n=3000, s=15, L=5)
    fo = oracle.sample(p.supp, p.coef, p.M, p.z)
    f = fo + synth.noise_for(fo, p.M, 40.0, 5)
    r, plan, ex, fdev = gpu_pass(m, p, f_np=f, s_cap=30, cap=512)
    no = int(ex["n_out"][0])
    rng = np.random.default_rng(1)
    y = np.zeros((1, 30), np.complex128)
    y[0, :no] = rng.standard_normal(no) + 1j * rng.standard_normal(no)
    gf = m.mr1l_adjoint(plan, ex, T(y)).cpu().numpy()
    # oracle dense transpose with the oracle's own selection
    go = oracle.dft(f, p.M)
    ro = oracle.extract(p.cand, p.M, p.z, go, p.theta, s_cap=30, cap=512)
    w = oracle.weights(p.cand, p.M, p.z, go, ro["det_idx"], ro["det_mask"])
    yd = np.zeros(len(ro["det_idx"]), np.complex128)
    yd[ro["out_pos"]] = y[0, :no]
    ga = oracle.adjoint(p.cand, p.M, p.z, ro["det_idx"], w, yd)
    close(gf, ga, 1e-11, "adjoint vs dense transpose")
    # dot-product identity against the forward map of the library
    x = rng.standard_normal(f.shape[0]) + 1j * rng.standard_normal(f.shape[0])
    eps = 1e-4

    def coef_of(ff):
        rr, *_ = gpu_pass(m, p, f_np=ff, s_cap=30, cap=512)
        assert np.array_equal(rr["out_idx"], r["out_idx"])
        return rr["out_coef"]
    lin = (coef_of(f + eps * x) - coef_of(f - eps * x)) / (2 * eps)
    lhs = float(np.real(np.vdot(y[0, :no], lin)))
    rhs = float(np.real(np.vdot(gf, x)))
    assert abs(lhs - rhs) <= 1e-7 * max(1.0, abs(rhs))


def test_autograd_function_finite_differences(m):
    say("autograd FD")
    p = synth.mid_config(2, n=2000, s=10, L=5)
    fo = oracle.sample(p.supp, p.coef, p.M, p.z)
    f0 = fo + synth.noise_for(fo, p.M, 40.0, 9)
    plan = m.Plan(p.d, p.M, p.z)
    freq = T(p.cand)
    f = T(f0).requires_grad_(True)
    out, n_out, idx = m.LatticeCoefficients.apply(f, plan, freq, p.theta, 20, 512, True)
    rng = np.random.default_rng(2)
    wv = T(rng.standard_normal(20) + 1j * rng.standard_normal(20))
    loss = torch.real(torch.sum(torch.conj(wv) * out[0]))
    loss.backward()
    g = f.grad.cpu().numpy()

    def L_of(ff):
        o, _, ii = m.LatticeCoefficients.apply(T(ff), plan, freq, p.theta, 20, 512, True)
        assert torch.equal(ii, idx)
        return float(torch.real(torch.sum(torch.conj(wv) * o[0])).item())
    h = 1e-6
    # rounding noise of the central difference ~ u ||w o out||_2 / h, 8 times that allowed
    noise = 8 * np.finfo(np.float64).eps * float(torch.linalg.norm(torch.abs(wv) * torch.abs(out[0].detach()))) / h
    for j in rng.integers(0, f0.shape[0], 16):
        for unit in (1.0, 1j):
            e = np.zeros_like(f0)
            e[j] = unit
            fd = (L_of(f0 + h * e) - L_of(f0 - h * e)) / (2 * h)
            an = g[j].real if unit == 1.0 else g[j].imag
            assert fd == pytest.approx(an, rel=1e-5, abs=max(1e-8, noise))


# ------------------------------------------------------------------ batched and graphs
def test_batched_plan_equals_plain_calls(m):
    say("batched vs plain")
    probs = synth.batch_config(0, nfunc=5, scale=0.01)
    d, L = probs[0].d, probs[0].L
    Ms = np.concatenate([q.M for q in probs])
    zs = np.concatenate([q.z for q in probs])
    plan = m.Plan(d, Ms, zs, F=len(probs))
    toff = T(np.concatenate([[0], np.cumsum([q.supp.shape[1] for q in probs])]).astype(np.int64))
    soff = T(np.concatenate([[0], np.cumsum([q.n for q in probs])]).astype(np.int64))
    supp = T(np.concatenate([q.supp for q in probs], axis=1))
    coef = T(np.concatenate([q.coef for q in probs]))
    cand = T(np.concatenate([q.cand for q in probs], axis=1))
    f = m.mr1l_sample(plan, supp, coef, term_off=toff)
    g, bm = m.mr1l_fft(plan, f, 1e-12)
    exb = m.mr1l_extract(plan, cand, g, bm, 1e-12, s_cap=512, cap=2048, set_off=soff)
    torch.cuda.synchronize()
    for fi, q in enumerate(probs):
        r, *_ = gpu_pass(m, q, s_cap=512, cap=2048, want_votes=False)
        nd = int(exb["n_det"][fi])
        assert nd == r["n_det"]
        assert np.array_equal(exb["det_idx"][fi, :nd].cpu().numpy(), r["det_idx"])
        no = int(exb["n_out"][fi])
        assert np.array_equal(exb["out_idx"][fi, :no].cpu().numpy(), r["out_idx"])
        close(exb["out_coef"][fi, :no].cpu().numpy(), r["out_coef"], 1e-11, "batched coef")
        # and both equal the oracle
        go = oracle.dft(oracle.sample(q.supp, q.coef, q.M, q.z), q.M)
        ro = oracle.extract(q.cand, q.M, q.z, go, 1e-12, s_cap=512, cap=2048)
        assert np.array_equal(r["out_idx"], ro["out_idx"])


def test_batched_autograd_finite_differences_and_dot_product(m):
    """Backward of the batched coefficient map (8 functions of the batched workload,
    reduced |Gamma|, 40 dB noise, theta = 0.05): central differences with h = 1e-6 on 16
    sample coordinates per function, and the dot-product identity over all samples."""
    say("batched autograd")
    probs = synth.batch_config(3, nfunc=8, scale=0.004, shi=200)
    d = probs[0].d
    F = len(probs)
    Ms = np.concatenate([q.M for q in probs])
    zs = np.concatenate([q.z for q in probs])
    plan = m.Plan(d, Ms, zs, F=F)
    soff = T(np.concatenate([[0], np.cumsum([q.n for q in probs])]).astype(np.int64))
    cand = T(np.concatenate([q.cand for q in probs], axis=1))
    parts = []
    for i, q in enumerate(probs):
        fo = oracle.sample(q.supp, q.coef, q.M, q.z)
        parts.append(fo + synth.noise_for(fo, q.M, 40.0, 100 + i))
    f0 = np.concatenate(parts)
    theta, s_cap, cap = 0.05, 256, 1024
    f = T(f0).requires_grad_(True)
    out, n_out, idx = m.LatticeCoefficients.apply(f, plan, cand, theta, s_cap, cap, True, soff)
    rng = np.random.default_rng(4)
    wv = T(rng.standard_normal((F, s_cap)) + 1j * rng.standard_normal((F, s_cap)))
    loss = torch.real(torch.sum(torch.conj(wv) * out))
    loss.backward()
    g = f.grad.cpu().numpy()

    def coefs(ff):
        o, _, ii = m.LatticeCoefficients.apply(T(ff), plan, cand, theta, s_cap, cap, True, soff)
        assert torch.equal(ii, idx)
        return o

    def L_of(ff):
        return float(torch.real(torch.sum(torch.conj(wv) * coefs(ff))).item())
    h = 1e-6
    node_off = np.concatenate([[0], np.cumsum([q.M.sum() for q in probs])])
    terms = (torch.abs(wv) * torch.abs(out.detach())).cpu().numpy()
    for fi in range(F):
        # a sample of function fi moves every output of fi: rounding noise of the central
        # difference ~ u ||w o out_fi||_2 / h (independent roundings), 8 times that allowed
        noise = 8 * np.finfo(np.float64).eps * float(np.linalg.norm(terms[fi])) / h
        for j in rng.integers(node_off[fi], node_off[fi + 1], 16):
            for unit in (1.0, 1j):
                e = np.zeros_like(f0)
                e[j] = unit
                fd = (L_of(f0 + h * e) - L_of(f0 - h * e)) / (2 * h)
                an = g[j].real if unit == 1.0 else g[j].imag
                assert fd == pytest.approx(an, rel=1e-5, abs=max(1e-8, noise)), (fi, int(j), unit, noise)
    # dot-product identity over every sample of the batch
    x = rng.standard_normal(f0.shape[0]) + 1j * rng.standard_normal(f0.shape[0])
    eps = 1e-4
    lin = (coefs(f0 + eps * x) - coefs(f0 - eps * x)) / (2 * eps)
    lhs = float(torch.real(torch.sum(torch.conj(wv) * lin)).item())
    rhs = float(np.real(np.vdot(g, x)))
    assert abs(lhs - rhs) <= 1e-7 * max(1.0, abs(rhs))


def test_graph_replay_matches_eager(m):
    say("graph replay")
    p = synth.small_config(3)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan = m.Plan(p.d, p.M, p.z, stream=s)
        freq = T(p.cand)
        f = m.mr1l_sample(plan, T(p.supp), T(p.coef))
        g, bm = m.mr1l_fft(plan, f, p.theta)
        ex = m.mr1l_extract(plan, freq, g, bm, p.theta, s_cap=40, cap=2000)
        s.synchronize()
        ref = ex["out_coef"].clone(), ex["out_idx"].clone(), ex["n_out"].clone()
        graph = m.Graph(plan)
        with graph:
            m.mr1l_fft(plan, f, p.theta, ghat=g, bitmap=bm)
            m.mr1l_extract(plan, freq, g, bm, p.theta, s_cap=40, cap=2000, out=ex)
        for rep in range(4):
            ex["out_coef"].zero_()
            ex["n_out"].zero_()
            s.synchronize()
            graph.launch(s)
            s.synchronize()
            assert torch.equal(ex["n_out"], ref[2])
            assert torch.equal(ex["out_idx"], ref[1])
            assert torch.equal(ex["out_coef"], ref[0])


def test_sample_graph_replay_keeps_its_scratch(m):
    """A graph that recorded mr1l_sample on plan A replays the same samples after a
    larger sample call on plan B on the same host thread and stream (each plan owns its
    term scratch, so B's growth cannot free or overwrite what A's graph uses)."""
    say("sample graph vs another plan's scratch")
    pa, pb = synth.small_config(4), synth.mid_config(1)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        A = m.Plan(pa.d, pa.M, pa.z, stream=s)
        B = m.Plan(pb.d, pb.M, pb.z, stream=s)
        supp, coef = T(pa.supp), T(pa.coef)
        fa = m.mr1l_sample(A, supp, coef, mode=1)          # sizes A's scratch
        s.synchronize()
        ref = fa.clone()
        graph = m.Graph(A)
        with graph:
            m.mr1l_sample(A, supp, coef, f=fa, mode=1)
        rng = np.random.default_rng(9)
        big = T(pb.cand)                                    # 10^5 terms: 50x A's
        bc = T(rng.standard_normal(pb.n) + 1j * rng.standard_normal(pb.n))
        for mode in (1, 2):
            fb = m.mr1l_sample(B, big, bc, mode=mode)
            for rep in range(3):
                fa.zero_()
                s.synchronize()
                graph.launch(s)
                s.synchronize()
                assert torch.equal(fa, ref), (mode, rep)
        s.synchronize()
    close(ref.cpu().numpy(), oracle.sample(pa.supp, pa.coef, pa.M, pa.z), 1e-11, "samples of A")
    fo = oracle.sample_nodes(pb.cand, bc.cpu().numpy(), pb.z[0], int(pb.M[0]), np.arange(0, int(pb.M[0]), 97))
    close(fb.cpu().numpy()[:int(pb.M[0])][::97], fo, 1e-11, "samples of B (bucket mode)")


def test_calls_on_a_plan_stream_other_than_the_current_one(m):
    """A plan bound to its own stream, called from torch's default stream: inputs made on
    the current stream are ready before the library reads them, and the results equal
    those of a plan on the current stream (the adjoint's temporary included)."""
    say("plan stream vs current stream")
    p = synth.mid_config(2)
    s = torch.cuda.Stream()
    P1 = m.Plan(p.d, p.M, p.z)
    P2 = m.Plan(p.d, p.M, p.z, stream=s)
    outs = []
    for plan in (P1, P2):
        f = m.mr1l_sample(plan, T(p.supp) * 1, T(p.coef) * 1)     # inputs made just now on the current stream
        g, bm = m.mr1l_fft(plan, f, p.theta)
        ex = m.mr1l_extract(plan, T(p.cand) + 0, g, bm, p.theta, s_cap=200, cap=4096)
        gf = m.mr1l_adjoint(plan, ex, torch.ones((1, 200), dtype=torch.complex64, device=dev()) * 0.5)
        outs.append((ex["out_idx"].cpu(), ex["out_coef"].cpu(), gf.cpu()))
    assert torch.equal(outs[0][0], outs[1][0])
    close(outs[1][1].numpy(), outs[0][1].numpy(), 1e-11, "coefficients")
    close(outs[1][2].numpy(), outs[0][2].numpy(), 1e-11, "adjoint")


def test_non_contiguous_arguments_are_refused(m):
    """The library reads row-major arrays through raw pointers: a transposed view (numpy
    fancy indexing along the second axis returns one) is refused, not read in the wrong
    order."""
    say("non-contiguous arguments")
    p = synth.small_config(0)
    plan = m.Plan(p.d, p.M, p.z)
    supp_f = torch.from_numpy(np.asfortranarray(p.supp)).to(dev())
    assert not supp_f.is_contiguous()
    with pytest.raises(m.Mr1lError):
        m.mr1l_sample(plan, supp_f, T(p.coef))
    f = m.mr1l_sample(plan, supp_f.contiguous(), T(p.coef))
    torch.cuda.synchronize()
    close(f.cpu().numpy(), oracle.sample(p.supp, p.coef, p.M, p.z), 1e-11, "samples")


# ------------------------------------------------------------------ driver
@pytest.mark.parametrize("seed", [0, 1])
def test_dimincr_matches_oracle_driver(m, seed):
    say("dimincr seed", seed)
    d, s = 6, 12
    freq, coef = synth.sparse_poly_box(seed, d=d, s=s, box=6)
    Mlat = synth.next_prime_above(10.33 * 2 * s)
    of, oc, ns = oracle.dimincr(freq, coef, N=6, s=s, s_local=2 * s, r=3, theta=1e-12, c=10.33, delta=0.9,
                                Mlat=Mlat, seed=100 + seed)
    gf, gc, gs = m.mr1l_dimincr(d, 6, s, 2 * s, 3, 1e-12, Mlat, 100 + seed, poly_freq=T(freq), poly_coef=T(coef))
    assert ns == gs
    assert np.array_equal(gf, of)
    close(gc, oc, 1e-11, "driver coefficients")
    truth = sorted(zip(map(tuple, freq.T.tolist()), coef))
    assert [tuple(r) for r in gf.tolist()] == [t[0] for t in truth]


def test_dimincr_sampling_callback_matches_builtin_sampler(m):
    """The driver with a sampling callback (here: the library sampler on a plan of the
    lattices and anchors the callback receives, written to the driver's buffer) gives the
    same support, coefficients and sample count as the built-in sampler, and the callback
    sees every repetition's lattices: r per step t < d, one at t = d."""
    import ctypes as C
    say("dimincr callback")
    d, s, N, r = 5, 10, 5, 3
    freq, coef = synth.sparse_poly_box(3, d=d, s=s, box=N)
    Mlat = synth.next_prime_above(10.33 * 2 * s)
    pf, pc = T(freq), T(coef)
    keep, calls = [], []

    def cb(user, t, L, Mp, zp, ancp, fptr, stream):
        Ms = np.ctypeslib.as_array(Mp, (L,)).copy()
        z = np.ctypeslib.as_array(zp, (L * t,)).copy().reshape(L, t)
        anc = None
        if t < d:
            anc = T(np.ctypeslib.as_array(ancp, (d - t,)).astype(np.int64).astype(np.uint32).view(np.int32))
        plan = m.Plan(t, Ms, z)
        rc = m.lib().mr1l_sample(plan.handle, d, None, s, pf.data_ptr(), pc.data_ptr(),
                                 None if anc is None else anc.data_ptr(), fptr, 1)
        keep.append((plan, anc))
        calls.append(t)
        return rc

    g0, c0, n0 = m.mr1l_dimincr(d, N, s, 2 * s, r, 1e-12, Mlat, 17, poly_freq=pf, poly_coef=pc)
    g1, c1, n1 = m.mr1l_dimincr(d, N, s, 2 * s, r, 1e-12, Mlat, 17, sample_fn=cb)
    torch.cuda.synchronize()
    assert calls == [t for t in range(2, d) for _ in range(r)] + [d]
    assert n0 == n1
    assert np.array_equal(g0, g1)
    assert np.array_equal(c0, c1)
    truth = sorted(zip(map(tuple, freq.T.tolist()), coef))
    assert [tuple(x) for x in g1.tolist()] == [t[0] for t in truth]


@pytest.mark.parametrize("d,s,N", [(4, 8, 60), (6, 12, 6)])
def test_dimincr_step1_matches_oracle_driver(m, d, s, N):
    """Algorithm 3 with Step 1: same single-coordinate sets, lattices and output as the
    oracle driver, and the true support."""
    say("dimincr step1", d, s, N)
    freq, coef = synth.sparse_poly_box(5, d=d, s=s, box=N)
    Mlat = synth.next_prime_above(10.33 * 2 * s)
    of, oc, ns = oracle.dimincr(freq, coef, N=N, s=s, s_local=2 * s, r=2, theta=1e-12, c=10.33, delta=0.9,
                                Mlat=Mlat, seed=91, step1=True)
    gf, gc, gs = m.mr1l_dimincr(d, N, s, 2 * s, 2, 1e-12, Mlat, 91, poly_freq=T(freq), poly_coef=T(coef),
                                step1=True)
    assert ns == gs
    assert np.array_equal(gf, of)
    close(gc, oc, 1e-11, "driver coefficients")
    truth = sorted(zip(map(tuple, freq.T.tolist()), coef))
    assert [tuple(r) for r in gf.tolist()] == [t[0] for t in truth]


def test_dimincr_least_squares_final_step_exact(m):
    """The least-squares final step (Remark 2.9) on a noise-free sparse polynomial: the
    same support as without it and coefficients exact to 1e-12 (relative)."""
    say("dimincr least squares")
    d, s, N = 6, 12, 6
    freq, coef = synth.sparse_poly_box(7, d=d, s=s, box=N)
    Mlat = synth.next_prime_above(10.33 * 2 * s)
    g0, c0, n0 = m.mr1l_dimincr(d, N, s, 2 * s, 2, 1e-12, Mlat, 5, poly_freq=T(freq), poly_coef=T(coef))
    g1, c1, n1 = m.mr1l_dimincr(d, N, s, 2 * s, 2, 1e-12, Mlat, 5, poly_freq=T(freq), poly_coef=T(coef),
                                lsq_iters=100)
    assert np.array_equal(g0, g1) and n0 == n1
    truth = sorted(zip(map(tuple, freq.T.tolist()), coef))
    assert [tuple(r) for r in g1.tolist()] == [t[0] for t in truth]
    close(c1, np.array([t[1] for t in truth]), 1e-12, "least-squares coefficients")


@pytest.mark.parametrize("step1", [False, True])
def test_dimincr_full_size_matches_oracle_and_truth(m, step1):
    """The dimension-incremental workload at full size: d = 25, s = 200 frequencies
    uniform in [-32, 32]^25, r = 5, s_local = 400, M = 4133, theta = 1e-12, with the
    full single-coordinate range or with Step 1.  The driver's result equals the oracle
    driver's (same lattices from the same SplitMix64 streams), recovers the support
    exactly, and its coefficients are exact to 1e-11 (relative l2)."""
    d, s, N, r, Mlat, seed = 25, 200, 32, 5, 4133, 1000
    freq, coef = synth.sparse_poly_box(0, d=d, s=s, box=N)
    say("dimincr full size: oracle", step1)
    of, oc, ns = oracle.dimincr(freq, coef, N=N, s=s, s_local=2 * s, r=r, theta=1e-12, c=10.33, delta=0.9,
                                Mlat=Mlat, seed=seed, step1=step1)
    say("dimincr full size: gpu", step1)
    gf, gc, gs = m.mr1l_dimincr(d, N, s, 2 * s, r, 1e-12, Mlat, seed, poly_freq=T(freq), poly_coef=T(coef),
                                step1=step1)
    assert gs == ns
    assert np.array_equal(gf, of)
    close(gc, oc, 1e-11, "driver coefficients")
    truth = sorted(zip(map(tuple, freq.T.tolist()), coef))
    assert [tuple(x) for x in gf.tolist()] == [t[0] for t in truth]
    c_truth = np.array([t[1] for t in truth])
    assert np.linalg.norm(gc - c_truth) / np.linalg.norm(c_truth) < 1e-11


@pytest.mark.parametrize("d,F,L", [(0, 1, 1), (65, 1, 1), (1, (1 << 20) + 1, 1), (1, 1, 65)])
def test_plan_create_rejects_out_of_range_shapes(m, d, F, L):
    """d, F and L beyond the documented ranges are argument errors (no plan, no launch)."""
    say("plan shape bounds", d, F, L)
    M = np.full(F * L, 7, np.int64)
    z = np.zeros((F * L, max(d, 1)), np.int64)
    with pytest.raises(m.Mr1lError):
        m.Plan(d, M, z[:, :d] if d else np.zeros((F * L, 0), np.int64), F=F)
