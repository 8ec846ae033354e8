#!/usr/bin/env python3
"""Throughput of the multiple-rank-1-lattice step on one MI355X.

Default workload ("large"): a batch of 64 functions, each with |Gamma| = 10^7
candidate frequencies uniform in [-512, 512]^10 (structure-of-arrays int64, 51 GB for
the batch), coefficients (1 + ||k||_1)^-2 with random unit phase on all of Gamma plus
1000 dominant entries of modulus 10, L = 20 lattices of prime size 16001 per function
with random generating vectors, complex128, theta = 1.  The samples are generated
once (untimed, bucket sampler) and stay resident in HBM.

One step = one pass of the method over the whole batch: the normalised lattice DFTs
with the non-zero bitmap (Algorithm 2, first loop) and the hash / vote / detected set
/ singleton masks / median and singleton coefficients / Algorithm 4 limit, as one
batched launch per stage.  value = candidates x lattices per second over the batch.

Also reported: per-stage times from HIP events recorded by the library on its stream,
the roofline of the dominant kernel (the vote pass), functions/s of the batched call
vs the per-function loop, a sampled parity check against the CPU oracle, and the
oracle's own throughput on a bounded sample (cpu_baseline).

Workload "batch": 512 functions with s log-uniform in [10, 1000], |Gamma| log-uniform
in [10^3, 10^6] from [-128, 128]^10, L = 8, M distinct primes in [8s, 16s],
noise-free, theta = 1e-12 (complex128, or complex64 with --c64).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PMC_FILE = os.path.join(ROOT, "profiles", "vote_large_pmc.json")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def vote_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("k_hash.hip", "mr1l_device.h"):
        with open(os.path.join(ROOT, "paper_2006_13053_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# ----------------------------------------------------------------------------- large
def setup_large(m, torch, F, n, seed=2026, distinct_m=False):
    import synth
    import synth.counter as sc
    d, L, M, box = 10, 20, 16001, 512
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(seed)
    if distinct_m:   # 20 distinct primes uniform in [15500, 16500] per function
        pr = synth.primes_in(15500, 16500)
        Ms = np.concatenate([rng.choice(pr, size=L, replace=False) for _ in range(F)]).astype(np.int64)
        zs = np.stack([np.stack([rng.integers(0, Ms[f * L + l], size=d, dtype=np.int64) for l in range(L)])
                       for f in range(F)])
    else:            # one size for every lattice: the smallest prime above 16000
        Ms = np.full(F * L, M, np.int64)
        zs = rng.integers(0, M, size=(F, L, d), dtype=np.int64)
    node_off = np.concatenate([[0], np.cumsum(Ms.reshape(F, L).sum(axis=1))]).astype(np.int64)
    nodes_f = int(node_off[1])
    t0 = time.time()
    gam = torch.empty((d, F * n), dtype=torch.int64, device=dev)      # batched SoA
    per = []                                                           # per-function SoA
    f_all = torch.empty(int(node_off[-1]), dtype=torch.complex128, device=dev)
    table = sc.phase_table(dev)
    plans = []
    for f in range(F):
        g = sc.candidates(seed, f, d, n, box, device=dev)
        gam[:, f * n:(f + 1) * n] = g
        per.append(g)
        c = sc.compressible_coefs(seed, f, g, table)
        dom = torch.from_numpy(sc.dominant_indices(seed, f, n, 1000)).to(dev)
        c[dom] = 10.0 * torch.from_numpy(sc.dominant_phases(seed, f, 1000)).to(dev)
        # sampled through a plan of its own, closed at once: its term scratch (10^7
        # terms x 96 B) is not kept by the per-function plans of the plain loop
        ps = m.Plan(d, Ms[f * L:(f + 1) * L], zs[f])
        m.mr1l_sample(ps, g, c, f=f_all[node_off[f]:node_off[f + 1]], mode=2)
        ps.close()
        plans.append(m.Plan(d, Ms[f * L:(f + 1) * L], zs[f]))
        del c
        if f % 8 == 7:
            torch.cuda.synchronize()
            log(f"  {f + 1}/{F} functions generated and sampled ({time.time() - t0:.1f}s)")
    torch.cuda.synchronize()
    log(f"generated {F} functions x {n} candidates and their samples in {time.time() - t0:.1f}s")
    plan = m.Plan(d, Ms, zs.reshape(-1), F=F)
    set_off = torch.arange(0, (F + 1) * n, n, dtype=torch.int64, device=dev)
    return dict(d=d, L=L, M=M, Ms=Ms.reshape(F, L), F=F, n=n, gam=gam, per=per, f=f_all, plan=plan, plans=plans,
                set_off=set_off, theta=1.0, zs=zs, seed=seed, box=box, nodes_f=nodes_f,
                cap=4096, s_cap=2048)


# ----------------------------------------------------------------------------- batch
def setup_batch(m, torch, F, seed=2027, c64=False, wl=None):
    import synth
    dev = torch.device("cuda", 0)
    dtype = torch.complex64 if c64 else torch.complex128
    wl = wl or synth.batch_workload(seed, F)
    d, L = wl.d, wl.L
    off, toff = wl.set_off, wl.term_off
    gam = torch.empty((d, int(off[-1])), dtype=torch.int64, device=dev)
    per, supp = [], []
    for f in range(F):
        g = wl.candidates(f, device=dev)
        gam[:, off[f]:off[f + 1]] = g
        per.append(g)
        supp.append(g[:, torch.from_numpy(wl.supp_idx[f]).to(dev)])
    supp = torch.cat(supp, dim=1).contiguous()
    coef = torch.from_numpy(np.concatenate(wl.coef)).to(dev).to(dtype)
    plan = m.Plan(d, wl.M, wl.z, F=F, dtype=dtype)
    f_all = m.mr1l_sample(plan, supp, coef, term_off=torch.from_numpy(toff).to(dev), mode=1)
    plans = [m.Plan(d, wl.M[f * L:(f + 1) * L], wl.z[f * L:(f + 1) * L], dtype=dtype) for f in range(F)]
    node_off = np.concatenate([[0], np.cumsum([int(wl.M[f * L:(f + 1) * L].sum()) for f in range(F)])])
    torch.cuda.synchronize()
    return dict(d=d, L=L, F=F, n=wl.n, gam=gam, per=per, f=f_all, plan=plan, plans=plans,
                set_off=torch.from_numpy(off).to(dev), theta=1e-3 if c64 else 1e-12, cap=4096,
                s_cap=2048, node_off=node_off, s=wl.s, dtype=dtype, wl=wl)


# ----------------------------------------------------------------------------- steps
def make_step(m, w):
    plan, f, gam, so = w["plan"], w["f"], w["gam"], w["set_off"]
    ghat, bm = m.mr1l_fft(plan, f, w["theta"])
    ex = m.mr1l_extract(plan, gam, ghat, bm, w["theta"], s_cap=w["s_cap"], cap=w["cap"], set_off=so,
                        want_w=False)

    def step():
        m.mr1l_fft(plan, f, w["theta"], ghat=ghat, bitmap=bm)
        m.mr1l_extract(plan, gam, ghat, bm, w["theta"], s_cap=w["s_cap"], cap=w["cap"], set_off=so, out=ex)
    return step, ex, ghat, bm


def timed_steps(torch, runner, steps, stream=None):
    """Run `steps` steps between two synchronisations -> (seconds, per-step ms from events
    recorded on `stream` (torch's current stream when None))."""
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for i in range(steps):
        runner()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return elapsed, [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]


def graph_runner(m, torch, plan, step):
    """Capture one step of `plan` into a HIP graph on a stream of its own -> (replay
    function, stream)."""
    s = torch.cuda.Stream()
    plan.set_stream(s)
    with torch.cuda.stream(s):
        step()
        s.synchronize()
        graph = m.Graph(plan)
        with graph:
            step()
        s.synchronize()

    def run():
        graph.launch(s)
    run.graph = graph
    return run, s


def stage_rooflines(w, plan, stages, ex, n_total, dtype):
    """Per-launch rooflines of the vote pass (8 d bytes per candidate + 8 per detection)
    and of the DFT stage (2 w bytes per node, nominal 5 M log2 M flops per lattice) from
    the stage times the library recorded on its stream."""
    st = {k: (v[0] / v[1] if v[1] else None) for k, v in stages.items()}
    vote_ms, fft_ms = st["vote"], st["fft"]
    nd = ex["n_det"].cpu().numpy()
    vbytes = 8.0 * w["d"] * n_total + 8.0 * float(np.minimum(nd, w["cap"]).sum())
    wb = 16 if dtype == "c128" else 8
    fbytes = 2.0 * wb * plan.nodes
    flops = float(sum(5.0 * int(mm) * np.log2(int(mm)) for mm in plan.M))
    fpeak = 78.6 if dtype == "c128" else 157.3
    vote = {"bound": "hbm", "kernel": "k_vote (hash + vote + compaction)", "achieved": vbytes / (vote_ms * 1e-3) / 1e9,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": vbytes / (vote_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "algorithmic_bytes_per_launch": vbytes, "vote_ms_per_launch": vote_ms}
    ffrac = fbytes / (fft_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
    fft = {"achieved": fbytes / (fft_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": ffrac, "target_frac": 0.6, "gap_to_target": 0.6 - ffrac,
           "bound": "in-register transforms and LDS exchanges (VALU busy 21-42% of the time); with "
                    "distinct sizes also one kernel-spectrum read per lattice, so the HBM traffic exceeds "
                    "the algorithmic bytes 2-5x",
           "ms_per_launch": fft_ms,
           "algorithmic_bytes_per_launch": fbytes, "nominal_flops_per_launch": flops,
           "achieved_TFLOPs": flops / (fft_ms * 1e-3) / 1e12, "peak_TFLOPs": fpeak}
    return st, vote, fft


def plain_pass(m, torch, w, reps=2):
    """Per-function loop: F separate plans, one fft + extract call pair each."""
    bufs = []
    nodes = [p.nodes for p in w["plans"]]
    off = np.concatenate([[0], np.cumsum(nodes)])
    for fi, pf in enumerate(w["plans"]):
        fv = w["f"][off[fi]:off[fi + 1]]
        g, b = m.mr1l_fft(pf, fv, w["theta"])
        e = m.mr1l_extract(pf, w["per"][fi], g, b, w["theta"], s_cap=w["s_cap"], cap=w["cap"], want_w=False)
        bufs.append((fv, g, b, e))
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        for fi, pf in enumerate(w["plans"]):
            fv, g, b, e = bufs[fi]
            m.mr1l_fft(pf, fv, w["theta"], ghat=g, bitmap=b)
            m.mr1l_extract(pf, w["per"][fi], g, b, w["theta"], s_cap=w["s_cap"], cap=w["cap"], out=e)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best, bufs


# ----------------------------------------------------------------------------- autograd
def autograd_timing(m, torch, w, reps=10):
    """Coefficients of Algorithm 4 as a differentiable function of the samples
    (LatticeCoefficients): forward alone (which also records the adjoint weights) vs
    forward + backward (the adjoint scatter and the inverse lattice DFTs) over the batch."""
    plan, f0, gam, so = w["plan"], w["f"], w["gam"], w["set_off"]
    f = f0.clone().requires_grad_(True)
    gen = torch.Generator(device=f.device).manual_seed(5)
    wv = torch.randn((w["F"], w["s_cap"]), dtype=f.dtype, device=f.device, generator=gen)

    def fwd():
        return m.LatticeCoefficients.apply(f, plan, gam, w["theta"], w["s_cap"], w["cap"], True, so)[0]

    def fwd_bwd():
        out = fwd()
        torch.real(torch.sum(torch.conj(wv) * out)).backward()
        f.grad = None
    res = {}
    for name, fn in (("forward_ms", lambda: fwd()), ("forward_backward_ms", fwd_bwd)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        res[name] = 1000.0 * (time.perf_counter() - t0) / reps
    res["backward_over_forward"] = res["forward_backward_ms"] / res["forward_ms"] - 1.0
    log(f"autograd: forward {res['forward_ms']:.3f} ms, forward+backward {res['forward_backward_ms']:.3f} ms")
    return res


# ----------------------------------------------------------------------------- dimincr
def bench_dimincr(m, torch, args):
    """Algorithm 3 Step 2 driver on the dimension-incremental workload: d = 25, s = 200
    frequencies uniform in [-32, 32]^25 with complex N(0,1) coefficients, r = 5,
    s_local = 400, one lattice size M = 4133, L by eq. (4.2), theta = 1e-12.  Each
    step is one full driver run on a new polynomial (seeds 0, 1, ...); the samples are
    taken inside the driver by the library's sampler."""
    import synth
    d, s, N, r, Mlat = 25, 200, 32, 5, 4133
    dev = torch.device("cuda", 0)
    runs = []
    for i in range(args.warmup + args.steps):
        seed = i % 5
        freq, coef = synth.sparse_poly_box(seed, d=d, s=s, box=N)
        pf = torch.from_numpy(freq).to(dev)
        pc = torch.from_numpy(coef).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gf, gc, ns = m.mr1l_dimincr(d, N, s, 2 * s, r, 1e-12, Mlat, 1000 + seed, poly_freq=pf, poly_coef=pc,
                                    step1=args.step1)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        truth = sorted(zip(map(tuple, freq.T.tolist()), coef))
        ok = [tuple(x) for x in gf.tolist()] == [t[0] for t in truth]
        err = (float(np.linalg.norm(gc - np.array([t[1] for t in truth])) / np.linalg.norm(coef))
               if ok else None)
        log(f"driver run {i} (seed {seed}): {dt:.3f} s, {ns} samples, support exact {ok}, rel err {err}")
        if i >= args.warmup:
            runs.append(dict(seed=seed, s=dt, samples=ns, support_exact=ok, rel_err=err))
    wall = float(np.median([x["s"] for x in runs]))
    out = {"metric": "dimension-incremental driver wall time", "value": wall, "unit": "s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1000.0 * wall,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c128",
           "data": "synthetic",
           "config": {"workload": "dimension-incremental: d=25, s=200 in [-32,32]^25, r=5, s_local=400, "
                                  "M=4133, L by eq. (4.2), theta=1e-12, Algorithm 3 "
                                  + ("Steps 1 and 2" if args.step1 else "Step 2 (full single-coordinate range)")},
           "runs": runs}
    if not args.no_cpu:
        import oracle
        freq, coef = synth.sparse_poly_box(0, d=d, s=s, box=N)
        t0 = time.perf_counter()
        of, oc, ns = oracle.dimincr(freq, coef, N=N, s=s, s_local=2 * s, r=r, theta=1e-12, c=10.33,
                                    delta=0.9, Mlat=Mlat, seed=1000, step1=args.step1)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": dt, "unit": "s", "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": "one full driver run (seed 0) of the oracle: direct DFTs, "
                                         "long-double arithmetic"}
    print(json.dumps(out), flush=True)


# ----------------------------------------------------------------------------- small / mid
def bench_plain(m, torch, args):
    """The small (d = 5, 2000 candidates, s = 20, L = 5, 100 seeds) and mid (d = 10, 10^5
    candidates, s = 100, L = 10, 40 dB, 20 seeds) configurations: one DFT + extract pass
    per function on resident samples, per-function calls (plain) and, for the small
    configuration, all 100 functions in one batched plan.  Launch-latency bound."""
    import synth
    dev = torch.device("cuda", 0)
    res = {}
    for name, mk, seeds in (("small", lambda sd: synth.small_config(sd), 100),
                            ("mid", lambda sd: synth.mid_config(sd), 20)):
        items = []
        for sd in range(seeds):
            p = mk(sd)
            plan = m.Plan(p.d, p.M, p.z)
            f = m.mr1l_sample(plan, torch.from_numpy(p.supp).to(dev), torch.from_numpy(p.coef).to(dev))
            if name == "mid":   # 40 dB complex Gaussian noise per lattice
                fn = f.cpu().numpy()
                f = torch.from_numpy(fn + synth.noise_for(fn, p.M, 40.0, sd)).to(dev)
            cand = torch.from_numpy(p.cand).to(dev)
            g, bm = m.mr1l_fft(plan, f, p.theta)
            ex = m.extract_buffers(plan, 4096, 2 * len(p.coef), 0, want_w=False)
            items.append((p, plan, f, cand, g, bm, ex))
        def one_pass():
            for p, plan, f, cand, g, bm, ex in items:
                m.mr1l_fft(plan, f, p.theta, ghat=g, bitmap=bm)
                m.mr1l_extract(plan, cand, g, bm, p.theta, s_cap=ex.s_cap, cap=4096, want_w=False, out=ex)
        for _ in range(args.warmup):
            one_pass()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            one_pass()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        cl = sum(p.cand.shape[1] * len(p.M) for p, *_ in items)
        res[name] = {"functions": seeds, "functions_per_s_plain": seeds / dt, "cand_lattices_per_s_plain": cl / dt,
                     "ms_per_function": 1000.0 * dt / seeds}
        log(name, f"plain: {seeds / dt:.0f} functions/s, {cl / dt:.3e} cand*lattices/s")
        for it in items:
            it[1].close()
    # small configuration batched: the 100 functions in one plan
    ps = [synth.small_config(sd) for sd in range(100)]
    plan = m.Plan(5, np.concatenate([p.M for p in ps]), np.concatenate([p.z for p in ps]), F=100)
    off = np.concatenate([[0], np.cumsum([p.cand.shape[1] for p in ps])]).astype(np.int64)
    toff = np.concatenate([[0], np.cumsum([len(p.coef) for p in ps])]).astype(np.int64)
    f = m.mr1l_sample(plan, torch.from_numpy(np.concatenate([p.supp for p in ps], axis=1)).to(dev),
                      torch.from_numpy(np.concatenate([p.coef for p in ps])).to(dev),
                      term_off=torch.from_numpy(toff).to(dev))
    cand = torch.from_numpy(np.concatenate([p.cand for p in ps], axis=1)).to(dev)
    so = torch.from_numpy(off).to(dev)
    g, bm = m.mr1l_fft(plan, f, 1e-12)
    ex = m.extract_buffers(plan, 4096, 40, 0, want_w=False)
    def batched():
        m.mr1l_fft(plan, f, 1e-12, ghat=g, bitmap=bm)
        m.mr1l_extract(plan, cand, g, bm, 1e-12, s_cap=40, cap=4096, set_off=so, want_w=False, out=ex)
    for _ in range(args.warmup):
        batched()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batched()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    res["small"]["functions_per_s_batched"] = 100 / dt
    log("small", f"batched: {100 / dt:.0f} functions/s")
    out = {"metric": "functions per second, small configuration, per-function calls", "value":
           res["small"]["functions_per_s_plain"], "unit": "functions/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": res["small"]["ms_per_function"] * 100, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
           "config": {"workload": "small: d=5, 2000 candidates in [-32,32]^5, s=20, L=5, 100 seeds; "
                                  "mid: d=10, 1e5 candidates in [-64,64]^10, s=100, L=10, 40 dB, 20 seeds; "
                                  "one step = one DFT + extract pass over every function"},
           "results": res}
    print(json.dumps(out), flush=True)


# ----------------------------------------------------------------------------- worst case (Section 4.1)
RANDOM_3D = dict(d=3, box=1000, n_gamma=10_000_000, n_active=1000, M=10331)
CROSS_8D = dict(d=8, bound=32, weight_exp=1.08, M=11047)
L_RANGE = tuple(range(9, 38, 2))


def _event_timer(torch):
    class T:
        def __init__(self):
            self.ms = 0.0

        def __enter__(self):
            self.a = torch.cuda.Event(enable_timing=True)
            self.b = torch.cuda.Event(enable_timing=True)
            self.a.record()
            return self

        def __exit__(self, *e):
            self.b.record()
            self.b.synchronize()
            self.ms += self.a.elapsed_time(self.b)
    return T()


def _add_stages(acc, plan):
    for k, (ms, cnt) in plan.profile_read().items():
        a = acc.setdefault(k, [0.0, 0])
        a[0] += ms
        a[1] += cnt


def worst_case_random_3d(m, torch, Ls=L_RANGE, reps=1000, batch=16, seed=41, n_gamma=None, cfg=RANDOM_3D,
                         stages=None):
    """Section 4.1.2: Gamma of n_gamma distinct points uniform in [-1000, 1000]^3 and I
    of 1000 points uniform in Gamma, new for each repetition (the same draw serves all
    L); for each L one random lattice configuration of size M = 10331, fixed over the
    repetitions.  Returns ({L: counts int64 [reps, 4]}, generation ms, method ms)."""
    import synth.counter as sc
    from paper_2006_13053_amd import worst_case as wc
    dev = torch.device("cuda", 0)
    d, box, na, M = cfg["d"], cfg["box"], cfg["n_active"], cfg["M"]
    n = n_gamma or cfg["n_gamma"]
    rng = np.random.default_rng(seed)
    runs = {L: wc.CountingRun(d, batch, L, M, np.tile(rng.integers(0, M, size=(L, d)), (batch, 1)),
                              profile=stages is not None) for L in Ls}
    set_off = torch.arange(batch + 1, dtype=torch.int64, device=dev) * n
    term_off = torch.arange(batch + 1, dtype=torch.int64, device=dev) * na
    n_act = torch.full((batch,), na, dtype=torch.int64, device=dev)
    cand = torch.empty((d, batch * n), dtype=torch.int64, device=dev)
    out = {L: [] for L in Ls}
    t_gen, t_run = _event_timer(torch), _event_timer(torch)
    nb = (reps + batch - 1) // batch
    for b in range(nb):
        with t_gen:
            for f in range(batch):
                rep = b * batch + f
                cand[:, f * n:(f + 1) * n] = sc.distinct_grid_points(seed * 1_000_003 + rep, n, d, box, device=dev)
            terms = cand.view(d, batch, n)[:, :, :na].reshape(d, batch * na).contiguous()
        with t_run:
            for L in Ls:
                out[L].append(runs[L].run(cand, set_off, n_act, terms, term_off).clone())
        if b % 8 == 7 or b == nb - 1:
            log(f"random 3d: {min(reps, (b + 1) * batch)}/{reps} repetitions")
    for r in runs.values():
        if stages is not None:
            _add_stages(stages, r.plan)
        r.close()
    res = {L: torch.cat(v).cpu().numpy()[:reps] for L, v in out.items()}
    return res, t_gen.ms, t_run.ms


def cross_8d_set(cfg=CROSS_8D):
    """Section 4.1.3: the unweighted hyperbolic cross Gamma (d = 8, bound 32) with the
    weighted cross I (weights t^1.08) listed first -> (Gamma [8, n] int64, |I|)."""
    import synth
    g = synth.hyperbolic_cross(cfg["d"], cfg["bound"])
    return synth.support_first(g, synth.weighted_cross_member(g, cfg["bound"], cfg["weight_exp"]))


def worst_case_cross_8d(m, torch, Ls=L_RANGE, reps=1000, batch=8, seed=43, cfg=CROSS_8D, gamma=None,
                        stages=None):
    """Section 4.1.3: Gamma and I fixed, a new random lattice configuration of size
    M = 11047 for every repetition.  Returns ({L: counts [reps, 4]}, setup ms, method ms)."""
    from paper_2006_13053_amd import worst_case as wc
    dev = torch.device("cuda", 0)
    d, M = cfg["d"], cfg["M"]
    t_gen, t_run = _event_timer(torch), _event_timer(torch)
    with t_gen:
        g, na = gamma if gamma is not None else cross_8d_set(cfg)
        n = g.shape[1]
        g = torch.from_numpy(g).to(dev)
        cand = g.repeat(1, batch)
        terms = g[:, :na].repeat(1, batch)
        del g
    set_off = torch.arange(batch + 1, dtype=torch.int64, device=dev) * n
    term_off = torch.arange(batch + 1, dtype=torch.int64, device=dev) * na
    n_act = torch.full((batch,), na, dtype=torch.int64, device=dev)
    rng = np.random.default_rng(seed)
    out = {L: [] for L in Ls}
    nb = (reps + batch - 1) // batch
    for L in Ls:
        run = wc.CountingRun(d, batch, L, M, rng.integers(0, M, size=(batch * L, d)), profile=stages is not None)
        with t_run:
            for b in range(nb):
                if b:
                    run.set_z(rng.integers(0, M, size=(batch * L, d)))
                out[L].append(run.run(cand, set_off, n_act, terms, term_off).clone())
        if stages is not None:
            _add_stages(stages, run.plan)
        run.close()
        log(f"cross 8d: L = {L} done")
    del cand, terms
    res = {L: torch.cat(v).cpu().numpy()[:reps] for L, v in out.items()}
    return res, t_gen.ms, t_run.ms


def bench_worst_case(m, torch, args):
    """Both experiments of Section 4.1 over L = 9, 11, ..., 37 with args.reps repetitions;
    success rates next to the printed ones, and the classification throughput."""
    from paper_2006_13053_amd import worst_case as wc
    gold = {}
    gpath = os.path.join(ROOT, "tests", "golden", "worst_case_success_rates.json")
    if os.path.exists(gpath):
        with open(gpath) as fh:
            gold = json.load(fh)
    exps, cl, run_ms, gen_ms, stages, vote_bytes = {}, 0.0, 0.0, 0.0, {}, 0.0
    todo = ("random_3d", "hyperbolic_cross_8d") if args.experiment == "both" else (args.experiment,)
    for name in todo:
        st = {}
        if name == "random_3d":
            res, g_ms, r_ms = worst_case_random_3d(m, torch, reps=args.reps, batch=16, stages=st)
            n_gamma, na, M, c, d, batch = RANDOM_3D["n_gamma"], RANDOM_3D["n_active"], RANDOM_3D["M"], 10.33, 3, 16
        else:
            res, g_ms, r_ms = worst_case_cross_8d(m, torch, reps=args.reps, batch=8, stages=st)
            n_gamma, na, M, c, d, batch = 10_665_297, 1069, CROSS_8D["M"], 10.33, 8, 8
        table = {}
        for L in sorted(res):
            sm = wc.summarize(res[L])
            sm["cor27_failure_bound"] = round(wc.cor27_failure_bound(n_gamma, c, L), 6)
            g = gold.get(name, {})
            sm["paper"] = {k: g[k][str(L)] for k in ("median", "median_r1l", "pfp_le10", "pfp_le100",
                                                      "max_pfn", "max_pfp") if str(L) in g.get(k, {})}
            table[str(L)] = sm
            cl += float(args.reps) * n_gamma * L
        exps[name] = {"reps": args.reps, "n_gamma": n_gamma, "n_active": na, "M": M, "method_ms": r_ms,
                      "input_ms": g_ms, "by_L": table}
        run_ms += r_ms
        gen_ms += g_ms
        vb = batch * n_gamma * d * 8.0
        for k, (ms, cnt) in st.items():
            a = stages.setdefault(k, [0.0, 0])
            a[0] += ms
            a[1] += cnt
        vote_bytes += vb * st.get("vote", (0.0, 0))[1]
        log(name, f"method {r_ms:.0f} ms, inputs {g_ms:.0f} ms")
    vote_ms, vote_n = stages.get("vote", (0.0, 0))
    roof = None
    if vote_n:
        ach = vote_bytes / (vote_ms / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": None, "kernel": "k_vote", "launches": vote_n,
                "bytes_per_launch_note": "candidates x d x 8 bytes of one batched launch (average over both "
                                         "experiments' launches)"}
    out = {"metric": "worst-case classifications (candidates x lattices) per second", "value": cl / (run_ms / 1e3),
           "unit": "candidate-lattices/s", "n_gpus": 1, "steps": args.reps, "warmup": 0,
           "ms_per_step": run_ms / (args.reps * len(todo)), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "c128", "data": "synthetic",
           "config": {"workload": "worst-case aliasing of Section 4.1 (Table 4.1): random Gamma of 1e7 points "
                                  "in [-1000,1000]^3 with |I| = 1000, M = 10331; 8-d hyperbolic cross "
                                  "(10,665,297) with the weighted cross I (1069), M = 11047; L = 9..37 odd; "
                                  "one step = one repetition over all L", "experiments": list(todo)},
           "stage_ms": {k: v[0] for k, v in stages.items()}, "input_generation_ms": gen_ms,
           "experiments": exps, "roofline": roof}
    if not args.no_cpu:
        import oracle
        import synth.counter as sc
        L = 21
        g = sc.distinct_grid_points(12345, RANDOM_3D["n_gamma"], 3, RANDOM_3D["box"]).numpy()
        z = np.random.default_rng(1).integers(0, RANDOM_3D["M"], size=(L, 3))
        t0 = time.perf_counter()
        oracle.pfpn(g, RANDOM_3D["n_active"], np.full(L, RANDOM_3D["M"]), z)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": RANDOM_3D["n_gamma"] * L / dt, "unit": "candidate-lattices/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"one repetition of the random 3-d experiment at L = {L} "
                                         f"(1e7 candidates), classification by direct alias counting: {dt:.2f} s"}
    print(json.dumps(out), flush=True)


# ----------------------------------------------------------------------------- Table 4.4
def bench_bspline(m, torch, args):
    """Algorithm 3 (Steps 1 and 2, Algorithm 4 as the detection method) on the test
    function eq. (4.3) in d = 10 over the (N, s) grid of Table 4.4: r = 5, s_local = 2s,
    delta = 0.999, theta = 1e-12, every lattice of size nextprime(10.33 s_local);
    args.reps runs per row (seeds 0, 1, ...).  Reports the largest relative L2 error
    and sample count per row next to the printed ones, and the wall time per run."""
    import synth
    gpath = os.path.join(ROOT, "tests", "golden", "table_4_4_bspline.json")
    with open(gpath) as fh:
        rows = json.load(fh)["rows"]
    if args.rows:
        rows = [r for r in rows if f"{r['N']}:{r['s']}" in args.rows.split(",")]
    orders, masks = synth.eq43_function()
    out_rows, times = [], []
    for row in rows:
        N, s = row["N"], row["s"]
        Mlat = synth.next_prime_above(10.33 * (s if args.m_of == "s" else 2 * s))
        errs, errs_ls, samp, ts = [], [], [], []
        for seed in range(args.reps):
            for lsq in (0, args.lsq_iters):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fr, co, ns = m.mr1l_dimincr(10, N, s, 2 * s, 5, 1e-12, Mlat, 1000 + seed, delta=0.999,
                                            cap=1 << 20, step1=True, bspline=(orders, masks), lsq_iters=lsq)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                e = synth.bspline_rel_l2_error(fr, co, orders, masks)
                if lsq:
                    errs_ls.append(e)
                else:
                    errs.append(e)
                    ts.append(dt)
                    samp.append(ns)
        log(f"N {N} s {s}: max rel L2 error {max(errs):.3e}, with least squares {max(errs_ls):.3e} "
            f"(printed {row['max_rel_l2_error']:.1e}), max samples {max(samp)} (printed {row['max_samples']}), "
            f"{np.mean(ts):.2f} s per run")
        out_rows.append(dict(N=N, s=s, M=Mlat, runs=args.reps, max_rel_l2_error=max(errs),
                             max_rel_l2_error_least_squares=max(errs_ls),
                             printed_max_rel_l2_error=row["max_rel_l2_error"], max_samples=max(samp),
                             printed_max_samples=row["max_samples"], s_per_run=float(np.mean(ts)),
                             s_runs=[round(float(x), 4) for x in ts]))
        times += ts
    out = {"metric": "dimension-incremental run time on the eq. (4.3) function (mean over the Table 4.4 grid)",
           "value": float(np.mean(times)), "unit": "s", "n_gpus": 1, "steps": len(times), "warmup": 0,
           "ms_per_step": 1000.0 * float(np.mean(times)), "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "c128", "data": "synthetic",
           "config": {"workload": "Table 4.4: f of eq. (4.3), d = 10, r = 5, s_local = 2s, delta = 0.999, "
                                  f"theta = 1e-12, Steps 1 and 2, M = nextprime(10.33 {args.m_of}); each run "
                                  "also with the least-squares final step",
                      "rows": [f"{r['N']}:{r['s']}" for r in out_rows]},
           "rows": out_rows}
    print(json.dumps(out), flush=True)


# ----------------------------------------------------------------------------- oracle legs
def copy_bandwidth(torch, nbytes=1 << 31):
    """Measured HBM rate of a plain device copy (torch's copy kernel): bytes read plus
    written over the best of three copies of nbytes, in GB/s (next to the 8 TB/s peak)."""
    a = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda")
    b = torch.empty_like(a)
    best = None
    for _ in range(4):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1)
        best = t if best is None else min(best, t)
    del a, b
    return 2.0 * nbytes / (best * 1e-3) / 1e9


def read_bandwidth(torch, nbytes=1 << 31):
    """Measured HBM rate of a plain device read (torch's int64 sum reduction over nbytes):
    bytes read over the best of four reductions, in GB/s (a read-only stream to set the
    vote pass, which only reads, against)."""
    a = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda")
    best = None
    for _ in range(4):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s = a.sum()
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1)
        best = t if best is None else min(best, t)
    assert int(s.item()) == nbytes // 8
    del a
    return nbytes / (best * 1e-3) / 1e9


def cpu_baseline_large(w, budget_s=10.0):
    """Oracle on one function of the batch, repeated until ~budget_s of CPU time: direct
    O(M^2) DFTs of its 20 lattices (on synthetic samples of the same size) and Algorithm 2
    + Remark 2.9 + Algorithm 4 over all of its candidates; value = candidates x lattices
    per second of one function."""
    import oracle
    import synth.counter as sc
    import torch
    d, L, n, seed = w["d"], w["L"], w["n"], w["seed"]
    Ms = np.ascontiguousarray(w["Ms"][0])
    z = w["zs"][0]
    rng = np.random.default_rng(7)
    nf = int(Ms.sum())
    fs = rng.standard_normal(nf) + 1j * rng.standard_normal(nf)
    # the oracle's own coefficients of function 0 (eq. (2.4): bucket sums of the polynomial)
    cand = sc.candidates(seed, 0, d, n, w["box"], device="cpu")
    coef = sc.compressible_coefs(seed, 0, cand, sc.phase_table("cpu"))
    dom = torch.from_numpy(sc.dominant_indices(seed, 0, n, 1000))
    coef[dom] = 10.0 * torch.from_numpy(sc.dominant_phases(seed, 0, 1000))
    cand_np = np.ascontiguousarray(cand.numpy())
    g_exact = oracle.bucket_sums(cand_np, coef.numpy(), Ms, z)
    reps, t_dft, t_ex = 0, 0.0, 0.0
    while reps == 0 or (t_dft + t_ex) < budget_s:
        t0 = time.perf_counter()
        oracle.dft(fs, Ms)
        t1 = time.perf_counter()
        ro = oracle.extract(cand_np, Ms, z, g_exact, w["theta"], s_cap=w["s_cap"], cap=w["cap"])
        t2 = time.perf_counter()
        t_dft += t1 - t0
        t_ex += t2 - t1
        reps += 1
    value = reps * n * L / (t_dft + t_ex)
    return dict(value=value, unit="candidates\u00b7lattices/s", cores=oracle.num_threads(), kind="oracle",
                cpu_model=cpu_model(),
                dft_s_per_rep=t_dft / reps, extract_s_per_rep=t_ex / reps,
                sample=(f"function 0 of the batch, {reps} repetitions: direct O(M^2) DFTs of its {L} lattices "
                        f"({t_dft / reps:.2f}s each) + Algorithm 2/Remark 2.9/Algorithm 4 over all {n} "
                        f"candidates ({t_ex / reps:.2f}s each)")), ro, g_exact


def unpack_bitmap(words, nodes):
    w = np.asarray(words).view(np.uint32)
    bits = ((w[:, None] >> np.arange(32, dtype=np.uint32)[None, :]) & 1).reshape(-1)
    return bits[:nodes].astype(bool)


def masks_u64(dm):
    w = np.asarray(dm).view(np.uint32).astype(np.uint64)
    return w if w.ndim == 1 else w[:, 0] | (w[:, 1] << np.uint64(32))


def compare_function(r, ro, go, theta, eps, tol):
    """One function's GPU pass (host arrays r) against the oracle's (ro) on the oracle's
    lattice values go: lattice values within tol of the largest modulus, the non-zero
    bitmap, detected count and indices and singleton masks bit-exact, median and
    post-processed coefficients within tol, Algorithm 4's entries and order equal up to
    moduli that tie within rounding.  Threshold decisions whose oracle modulus lies
    within the rounding band of theta are counted and left out (expected: none)."""
    res = {}
    gs = max(1e-300, float(np.abs(go).max()))
    res["ghat_rel_err"] = float(np.abs(r["ghat"] - go).max() / gs)
    band = np.abs(np.abs(go) - theta) <= 256 * eps * gs
    res["threshold_band"] = int(band.sum())
    res["bitmap_equal"] = bool(np.array_equal(r["bitmap"][~band], ((go.real ** 2 + go.imag ** 2)
                                                                   >= theta * theta)[~band]))
    res["n_det"] = int(r["n_det"])
    res["n_det_equal"] = res["n_det"] == int(ro["n_det"])
    res["det_idx_equal"] = bool(np.array_equal(r["det_idx"], ro["det_idx"]))
    res["det_mask_equal"] = bool(np.array_equal(r["det_mask"], ro["det_mask"]))
    same = res["det_idx_equal"]
    cs = max(1e-300, float(np.abs(ro["det_coef"]).max())) if ro["det_coef"].size else 1.0
    ms = max(1e-300, float(np.abs(ro["det_med"]).max())) if ro["det_med"].size else 1.0
    res["median_rel_err"] = float(np.abs(r["det_med"] - ro["det_med"]).max() / ms) if same and r["det_med"].size else 0.0
    res["coef_rel_err"] = float(np.abs(r["det_coef"] - ro["det_coef"]).max() / cs) if same and r["det_coef"].size else 0.0
    # Algorithm 4: same entries except ties at the smallest kept modulus, order by modulus
    oi, oc, gi, gc = ro["out_idx"], ro["out_coef"], r["out_idx"], r["out_coef"]
    lim_ok = gi.shape == oi.shape
    out_err = 0.0
    if lim_ok and oi.size:
        sc = max(1e-300, float(np.abs(oc).max()))
        delta = 256 * eps * sc
        omag = dict(zip(oi.tolist(), np.abs(oc).tolist()))
        mmin = float(np.abs(oc).min())
        boundary = {i for i, mg in omag.items() if abs(mg - mmin) <= delta}
        lim_ok = (set(oi.tolist()) - set(gi.tolist())) <= boundary
        seq = [omag.get(i, mmin) for i in gi.tolist()]
        lim_ok = lim_ok and all(seq[o] >= seq[o + 1] - delta for o in range(len(seq) - 1))
        ocd = dict(zip(oi.tolist(), oc.tolist()))
        out_err = max([abs(c - ocd[i]) / sc for i, c in zip(gi.tolist(), gc.tolist()) if i in ocd] or [0.0])
    res["limit_equal_up_to_ties"] = bool(lim_ok)
    res["out_coef_rel_err"] = float(out_err)
    res["ok"] = bool(res["threshold_band"] == 0 and res["bitmap_equal"] and res["n_det_equal"] and same
                     and res["det_mask_equal"] and res["ghat_rel_err"] <= tol and res["median_rel_err"] <= tol
                     and res["coef_rel_err"] <= tol and lim_ok and out_err <= tol)
    return res


def gpu_function(ex, ghat, bits, nodes_off, fi, cap):
    """Host copies of function fi's outputs of a batched pass (ghat and the unpacked
    bitmap of its nodes [nodes_off[fi], nodes_off[fi + 1]))."""
    a, b = int(nodes_off[fi]), int(nodes_off[fi + 1])
    nd = int(ex["n_det"][fi])
    k = min(nd, cap)
    no = int(ex["n_out"][fi])
    bits = bits[a:b]
    return dict(n_det=nd, ghat=ghat[a:b], bitmap=bits, det_idx=ex["det_idx"][fi, :k],
                det_mask=masks_u64(ex["det_mask"][fi, :k]), det_med=ex["det_med"][fi, :k],
                det_coef=ex["det_coef"][fi, :k], out_idx=ex["out_idx"][fi, :no], out_coef=ex["out_coef"][fi, :no])


def host_outputs(ex):
    return {k: (v.cpu().numpy() if v is not None and hasattr(v, "cpu") else v) for k, v in ex.items()}


def parity_large(m, torch, w, ex, ghat, bm, ro, g_exact):
    """Function 0 of the batched pass against the oracle over all of its candidates."""
    h = host_outputs(ex)
    gh = ghat[: w["nodes_f"]].cpu().numpy()
    bits = unpack_bitmap(bm[: (w["nodes_f"] + 31) // 32].cpu().numpy(), w["nodes_f"])
    r = gpu_function(h, gh, bits, [0, w["nodes_f"]], 0, w["cap"])
    res = compare_function(r, ro, g_exact, w["theta"], 2.0 ** -53, 1e-11)
    res["function"] = 0
    res["candidates"] = int(w["n"])
    return res


# ----------------------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=("large", "batch", "dimincr", "worst-case", "bspline", "plain"),
                    default="large")
    ap.add_argument("--lsq-iters", type=int, default=200,
                    help="bspline workload: CG iterations of the least-squares final step (second run per seed)")
    ap.add_argument("--m-of", choices=("s", "s_local"), default="s",
                    help="bspline workload: lattice size nextprime(10.33 s) or nextprime(10.33 s_local)")
    ap.add_argument("--rows", default="", help="bspline workload: comma-separated N:s rows of Table 4.4 (default all)")
    ap.add_argument("--reps", type=int, default=None,
                    help="worst-case workload: repetitions per L (1000); bspline workload: runs per row (3)")
    ap.add_argument("--experiment", choices=("both", "random_3d", "hyperbolic_cross_8d"), default="both",
                    help="worst-case workload: which experiment of Section 4.1")
    ap.add_argument("--functions", type=int, default=None)
    ap.add_argument("--candidates", type=int, default=10_000_000)
    ap.add_argument("--c64", action="store_true")
    ap.add_argument("--step1", action="store_true",
                    help="dimincr workload: single-coordinate sets from Algorithm 3 Step 1 instead of the full range")
    ap.add_argument("--distinct-m", action="store_true",
                    help="large workload with 20 distinct primes in [15500, 16500] per function instead of M = 16001")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle legs")
    ap.add_argument("--no-plain", action="store_true", help="skip the per-function loop")
    ap.add_argument("--no-batch", action="store_true",
                    help="large workload: skip the batched-workload leg (512 functions, graph vs per-function loop, "
                         "autograd)")
    ap.add_argument("--no-distinct-m", action="store_true",
                    help="large workload: skip the leg with 20 distinct lattice sizes per function")
    ap.add_argument("--graph", action="store_true", help="time a captured HIP graph of the step")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default DFT schedules instead of autotuning them before the timed steps")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the steps, copy 2 GiB once (a plain copy kernel of known size, used to scale "
                         "the FETCH_SIZE / WRITE_SIZE counters of profiled runs)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (--gpus 1): the library "
                          "has no multi-GPU path (sharding by candidates or by functions is not built)"}))
        sys.exit(2)

    import torch

    import paper_2006_13053_amd as m
    torch.cuda.set_device(0)
    m.lib()
    if args.workload == "dimincr":
        return bench_dimincr(m, torch, args)
    if args.workload == "worst-case":
        args.reps = args.reps or 1000
        return bench_worst_case(m, torch, args)
    if args.workload == "bspline":
        args.reps = args.reps or 3
        return bench_bspline(m, torch, args)
    if args.workload == "plain":
        return bench_plain(m, torch, args)

    if args.workload == "large":
        F = args.functions or 64
        w = setup_large(m, torch, F, args.candidates, distinct_m=args.distinct_m)
        msz = "20 distinct primes in [15500,16500] per function" if args.distinct_m else "M=16001"
        cfg = dict(workload="large compressible: d=10, |I|=1e7 per function in [-512,512]^10, "
                            "c_k=(1+|k|_1)^-2 x unit phase + 1000 dominants of modulus 10, L=20, "
                            f"{msz}, complex128, theta=1", functions=F, candidates_per_function=args.candidates,
                   lattices=20, M="15500..16500" if args.distinct_m else 16001, d=10)
        dtype = "c128"
    else:
        F = args.functions or 512
        w = setup_batch(m, torch, F, c64=args.c64)
        cfg = dict(workload="batched: 512 functions, d=10, s log-uniform [10,1000], |I| log-uniform "
                            "[1e3,1e6] from [-128,128]^10, L=8, M primes in [8s,16s], noise-free",
                   functions=F, candidates_total=int(w["gam"].shape[1]), lattices=8, d=10)
        dtype = "c64" if args.c64 else "c128"

    out = headline(m, torch, args, w, cfg, dtype, F)
    if args.workload == "large":
        if not args.no_cpu:
            log("oracle leg (CPU) ...")
            cpu, ro, g_exact = cpu_baseline_large(w)
            out["cpu_baseline"] = cpu
            out["parity"] = parity_large(m, torch, w, out.pop("_ex"), out.pop("_ghat"), out.pop("_bm"), ro, g_exact)
            log(f"parity of function 0 (all {w['n']} candidates): {out['parity']['ok']}")
        if not args.no_distinct_m and not args.distinct_m:
            out["distinct_m"] = distinct_m_leg(m, torch, args, w)
        for k in ("_ex", "_ghat", "_bm"):
            out.pop(k, None)
        w["plans"].clear()
        w["per"].clear()
        del w
        torch.cuda.empty_cache()
        if not args.no_batch:
            out["batch"] = batch_leg(m, torch, args)
    for k in ("_ex", "_ghat", "_bm"):
        out.pop(k, None)
    if args.copy_probe:
        a = torch.ones(1 << 28, dtype=torch.int64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = int(a.numel() * 8)
    print(json.dumps(out), flush=True)


def tune_schedules(w):
    """Autotune the batched plan's DFT schedules; the per-function plans take the same."""
    plan = w["plan"]
    tune = plan.fft_tune(reps=3)
    for pf in w["plans"]:
        for M in np.unique(pf.M):
            pf.fft_schedule(int(M), plan.fft_schedule(int(M)))
    return tune


def headline(m, torch, args, w, cfg, dtype, F):
    """The timed steps of the chosen workload -> the JSON line's fields."""
    plan = w["plan"]
    tune = None
    if not args.no_tune:
        tune = tune_schedules(w)
        log("DFT schedules (ms per batched DFT of each size's group): "
            + json.dumps({k: tune[k] for k in list(tune)[:4]}))
    log("setup done; warming up")
    step, ex, ghat, bm = make_step(m, w)
    n_total = int(w["gam"].shape[1])
    L = w["L"]
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = None
    if args.graph:
        runner, stream = graph_runner(m, torch, plan, step)
    else:
        runner = step
    plan.profile(not args.graph)
    elapsed, step_ms = timed_steps(torch, runner, args.steps, stream)
    stages = plan.profile_read() if not args.graph else {}
    plan.profile(False)
    ms_step = 1000.0 * elapsed / args.steps
    value = n_total * L / (elapsed / args.steps)

    out = {"metric": "candidates\u00b7lattices hashed+extracted/s and functions/s, batched vs plain, "
                     "at rel err \u22641e-11",
           "value": value, "unit": "candidates\u00b7lattices/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": cfg}
    out["functions_per_s_batched"] = F / (elapsed / args.steps)
    out["step_ms_median"] = float(np.median(step_ms))
    names = m.fft_schedule_names()
    out["fft_schedules"] = {str(int(M)): names[plan.fft_schedule(int(M))] for M in np.unique(plan.M)[:8]}
    if tune is not None:
        out["fft_tune_ms"] = {str(k): v for k, v in list(tune.items())[:8]}
    if stages:
        st, vote, fft = stage_rooflines(w, plan, stages, ex, n_total, dtype)
        out["stages_ms"] = st
        traffic = None
        if os.path.exists(PMC_FILE):
            with open(PMC_FILE) as fh:
                pmc = json.load(fh)
            wl = args.workload + ("-distinct-m" if args.distinct_m else "")
            if pmc.get("source_hash") == vote_source_hash() and pmc.get("workload") == wl:
                traffic = pmc.get("bytes_per_launch")
        vote["traffic"] = traffic
        vote["copy_GBps"] = copy_bandwidth(torch)
        vote["read_GBps"] = read_bandwidth(torch)
        out["roofline"] = {k: vote[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")}
        out["roofline"].update({k: v for k, v in vote.items() if k not in out["roofline"]})
        out["fft_roofline"] = fft
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step")
    if not args.no_plain:
        t_plain, _ = plain_pass(m, torch, w)
        log(f"plain per-function loop: {1000 * t_plain:.3f} ms")
        out["functions_per_s_plain"] = F / t_plain
        out["plain_ms_per_pass"] = 1000.0 * t_plain
    if args.workload == "batch":
        out["autograd"] = autograd_timing(m, torch, w)
    out["_ex"], out["_ghat"], out["_bm"] = ex, ghat, bm
    return out


def oracle_function(w, fi):
    """The oracle's lattice values (eq. (2.4) bucket sums of the polynomial) and its
    Algorithm 2 + Remark 2.9 + Algorithm 4 over every candidate of function fi of the
    large workload."""
    import oracle
    import synth.counter as sc
    import torch
    d, n, seed = w["d"], w["n"], w["seed"]
    Ms = np.ascontiguousarray(w["Ms"][fi])
    z = w["zs"][fi]
    cand = sc.candidates(seed, fi, d, n, w["box"], device="cpu")
    coef = sc.compressible_coefs(seed, fi, cand, sc.phase_table("cpu"))
    dom = torch.from_numpy(sc.dominant_indices(seed, fi, n, 1000))
    coef[dom] = 10.0 * torch.from_numpy(sc.dominant_phases(seed, fi, 1000))
    cand_np = np.ascontiguousarray(cand.numpy())
    g_exact = oracle.bucket_sums(cand_np, coef.numpy(), Ms, z)
    ro = oracle.extract(cand_np, Ms, z, g_exact, w["theta"], s_cap=w["s_cap"], cap=w["cap"])
    return ro, g_exact


def distinct_m_leg(m, torch, args, w):
    """The large workload (same candidates and coefficients) with 20 distinct primes
    uniform among the primes in [15500, 16500] per function: the DFT stage (every size
    has its own tables), the whole step, and function 0 against the oracle."""
    import synth
    import synth.counter as sc
    F, d, L, n, seed = w["F"], w["d"], w["L"], w["n"], w["seed"]
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(seed + 1)
    pr = synth.primes_in(15500, 16500)
    Ms = np.concatenate([rng.choice(pr, size=L, replace=False) for _ in range(F)]).astype(np.int64)
    zs = np.stack([np.stack([rng.integers(0, Ms[f * L + l], size=d, dtype=np.int64) for l in range(L)])
                   for f in range(F)])
    node_off = np.concatenate([[0], np.cumsum(Ms.reshape(F, L).sum(axis=1))]).astype(np.int64)
    f_all = torch.empty(int(node_off[-1]), dtype=torch.complex128, device=dev)
    table = sc.phase_table(dev)
    t0 = time.time()
    for f in range(F):
        c = sc.compressible_coefs(seed, f, w["per"][f], table)
        dom = torch.from_numpy(sc.dominant_indices(seed, f, n, 1000)).to(dev)
        c[dom] = 10.0 * torch.from_numpy(sc.dominant_phases(seed, f, 1000)).to(dev)
        ps = m.Plan(d, Ms[f * L:(f + 1) * L], zs[f])
        m.mr1l_sample(ps, w["per"][f], c, f=f_all[node_off[f]:node_off[f + 1]], mode=2)
        ps.close()
        del c
    torch.cuda.synchronize()
    log(f"distinct sizes: samples of {F} functions in {time.time() - t0:.1f}s")
    plan = m.Plan(d, Ms, zs.reshape(-1), F=F)
    w2 = dict(w, plan=plan, plans=[], f=f_all, Ms=Ms.reshape(F, L), zs=zs, nodes_f=int(node_off[1]))
    res = {"workload": "the large workload with 20 distinct primes uniform in [15500, 16500] per function",
           "distinct_sizes": int(np.unique(Ms).shape[0])}
    if not args.no_tune:
        tune_schedules(w2)
    names = m.fft_schedule_names()
    scheds = {}
    for M in np.unique(Ms):
        k = names[plan.fft_schedule(int(M))]
        scheds[k] = scheds.get(k, 0) + 1
    res["fft_schedules"] = scheds
    step, ex, ghat, bm = make_step(m, w2)
    for _ in range(args.warmup):
        step()
    plan.profile(True)
    elapsed, step_ms = timed_steps(torch, step, args.steps)
    stages = plan.profile_read()
    plan.profile(False)
    st, vote, fft = stage_rooflines(w2, plan, stages, ex, int(w["gam"].shape[1]), "c128")
    res.update(ms_per_step=1000.0 * elapsed / args.steps, step_ms_median=float(np.median(step_ms)),
               stages_ms=st, fft_roofline=fft, vote_roofline=vote)
    log(f"distinct sizes: {res['ms_per_step']:.3f} ms/step, DFT {st['fft']:.3f} ms")
    if not args.no_cpu:
        ro, g_exact = oracle_function(w2, 0)
        res["parity"] = parity_large(m, torch, w2, ex, ghat, bm, ro, g_exact)
        log(f"distinct sizes: parity of function 0: {res['parity']['ok']}")
    plan.close()
    return res


def batch_leg(m, torch, args):
    """The batched workload (512 functions, complex128) as extra keys of the line:
    functions/s of one pass replayed from a captured HIP graph, eagerly, and as the
    per-function loop; autograd forward vs forward + backward; the vote and DFT
    rooflines; every function against the oracle."""
    F = 512
    t0 = time.time()
    w = setup_batch(m, torch, F)
    log(f"batched workload: {F} functions, {int(w['gam'].shape[1])} candidates, set up in {time.time() - t0:.1f}s")
    plan = w["plan"]
    if not args.no_tune:
        tune_schedules(w)
    step, ex, ghat, bm = make_step(m, w)
    n_total = int(w["gam"].shape[1])
    steps = max(args.steps, 10)
    for _ in range(args.warmup):
        step()
    plan.profile(True)
    timed_steps(torch, step, steps)
    stages = plan.profile_read()
    plan.profile(False)
    st, vote, fft = stage_rooflines(w, plan, stages, ex, n_total, "c128")
    el_e, ms_e = timed_steps(torch, step, steps)
    run, s = graph_runner(m, torch, plan, step)
    for _ in range(args.warmup):
        run()
    el_g, ms_g = timed_steps(torch, run, steps, stream=s)
    plan.set_stream(torch.cuda.current_stream())
    t_plain, _ = plain_pass(m, torch, w)
    res = {"workload": "batched: 512 functions, d=10, s log-uniform [10,1000], |I| log-uniform [1e3,1e6] from "
                       "[-128,128]^10, L=8, M distinct primes in [8s,16s], noise-free, complex128, theta=1e-12",
           "functions": F, "candidates": n_total, "nodes": int(plan.nodes),
           "ms_per_pass_graph": 1000.0 * el_g / steps, "ms_per_pass_eager": 1000.0 * el_e / steps,
           "ms_per_pass_plain": 1000.0 * t_plain,
           "functions_per_s_graph": F * steps / el_g, "functions_per_s_eager": F * steps / el_e,
           "functions_per_s_plain": F / t_plain,
           "graph_over_plain": (F * steps / el_g) / (F / t_plain),
           "stages_ms": st, "vote_roofline": vote, "fft_roofline": fft}
    log(f"batched: graph {res['ms_per_pass_graph']:.3f} ms, eager {res['ms_per_pass_eager']:.3f} ms, "
        f"per-function loop {res['ms_per_pass_plain']:.3f} ms per pass")
    ag = autograd_timing(m, torch, w)
    ag["functions_per_s_forward"] = F / (ag["forward_ms"] * 1e-3)
    ag["functions_per_s_forward_backward"] = F / (ag["forward_backward_ms"] * 1e-3)
    res["autograd"] = ag
    if not args.no_cpu:
        res["parity"] = parity_batch(w, ex, ghat, bm)
        log(f"batched: parity over all {F} functions: {res['parity']['ok']}")
    return res


def parity_batch(w, ex, ghat, bm):
    """Every function of the batched pass (here: the buffers the graph replays wrote)
    against the oracle over all of its candidates, with the oracle's lattice values the
    eq. (2.4) bucket sums of the function's support."""
    import oracle
    wl = w["wl"]
    F, L = wl.F, wl.L
    t0 = time.perf_counter()
    cand = w["gam"].cpu().numpy()
    h = host_outputs(ex)
    gh = ghat.cpu().numpy()
    bits = unpack_bitmap(bm.cpu().numpy(), int(gh.shape[0]))
    node_off = np.concatenate([[0], np.cumsum(wl.M)]).astype(np.int64)[::L]
    soff = wl.set_off
    worst = {"ghat_rel_err": 0.0, "median_rel_err": 0.0, "coef_rel_err": 0.0, "out_coef_rel_err": 0.0}
    bad, band, ndet = [], 0, 0
    for fi in range(F):
        Mf, zf = wl.M[fi * L:(fi + 1) * L], wl.z[fi * L:(fi + 1) * L]
        cf = np.ascontiguousarray(cand[:, soff[fi]:soff[fi + 1]])
        go = oracle.bucket_sums(np.ascontiguousarray(cf[:, wl.supp_idx[fi]]), wl.coef[fi], Mf, zf)
        ro = oracle.extract(cf, Mf, zf, go, w["theta"], s_cap=w["s_cap"], cap=w["cap"])
        r = gpu_function(h, gh, bits, node_off, fi, w["cap"])
        c = compare_function(r, ro, go, w["theta"], 2.0 ** -53, 1e-11)
        for k in worst:
            worst[k] = max(worst[k], c[k])
        band += c["threshold_band"]
        ndet += c["n_det"]
        if not c["ok"]:
            bad.append(fi)
    return dict(functions=F, candidates=int(cand.shape[1]), functions_equal=F - len(bad), failed=bad[:20],
                detected=ndet, threshold_band=band, worst=worst, oracle_s=time.perf_counter() - t0,
                ok=not bad and band == 0)


if __name__ == "__main__":
    main()
