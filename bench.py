#!/usr/bin/env python3
"""Benchmark: encrypted semi-parallel GWAS on one MI355X.

A step is one call of the hot path, ``gwas_semiparallel``, on the paper-scale
workload: n = 245 samples, k = 4 covariates (intercept + 3 N(0,1)), m = 10643
SNPs packed two per complex slot (42 SNP batches of 256), RNS-CKKS with
N = 2^16, scale 2^40, q_0 of 60 bits, 26 rescale primes of 40 bits, 3 special
primes of 41 bits (key-switching digit groups of 3), kappa = 3 Newton passes.
Keys and encrypted inputs are resident in HBM before the timed region; the
encrypted numerators and denominators are ready in HBM at its end.  Data: seeded
synthetic genotypes and phenotypes with the shapes and distributions of the
paper's workload.

Two regions are timed.  The headline region runs the steps as a user would (the
logistic-regression part on a second stream, overlapping the per-batch work that
does not need it), with no kernel timing.  The roofline region runs the same
steps on one stream, where each kernel has the GPU to itself: one step with every
kernel timed picks the dominant kernel, then that kernel's launches are timed
over the region's steps.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_SAMPLES, K_COV, M_SNPS, KAPPA, LOG_N, LOG_SCALE = 245, 4, 10643, 3, 16, 40
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X, FP64 on the vector ALUs (an FMA counts 2)
CPU_SAMPLE_S = 12.0              # cpu_baseline: SNP batches run until this much oracle time has passed,
CPU_SAMPLE_MAX_BATCHES = 8       # or this many batches
WORKLOAD = ("encrypted semi-parallel GWAS n=245 k=4 m=10643, RNS-CKKS N=2^16, q_0 of 60 bits + L=26 primes of "
            "40 bits, scale=2^40, kappa=3; key switching with 3 special primes of 41 bits and digit groups of 3 "
            "(hybrid) in place of one 60-bit special prime")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def region_marker(tag: int):
    """A one-element torch fill kernel on the device: the GPU path itself launches no torch kernels, so in
    a profiler's kernel trace the dispatches between the two markers are exactly the timed steps."""
    import torch
    torch.full((1,), tag, dtype=torch.int64, device="cuda")


def galois_set(R):
    import paper_1902_04303_amd as P
    return P.gwas_galois_elements(LOG_N, R)


def gpu_leg(args):
    import torch

    import paper_1902_04303_amd as P
    from synth import config_seed, make_gwas_data

    torch.cuda.init()
    L = 7 * KAPPA + 5
    ctx = P.Context(LOG_N, L, LOG_SCALE, alpha=args.ks_alpha)
    lay = ctx.gwas_layout(N_SAMPLES, K_COV, M_SNPS, KAPPA)
    gal = galois_set(lay["R"])
    t0 = time.time()
    ctx.keygen(7, gal)
    torch.cuda.synchronize()
    log("[bench] keygen %.2fs (%d switching keys)" % (time.time() - t0, len(gal) + 1))
    d = make_gwas_data(N_SAMPLES, K_COV, M_SNPS, seed=config_seed(2))
    t0 = time.time()
    gin = ctx.gwas_pack_encrypt(d.X, d.y, d.S, KAPPA, 11)
    torch.cuda.synchronize()
    log("[bench] client encode+encrypt %.2fs, %d SNP batches" % (time.time() - t0, lay["n_batches"]))
    out = None
    for w in range(max(1, args.warmup)):
        out = ctx.gwas_semiparallel(gin)
        torch.cuda.synchronize()
        log("[bench] warmup %d done" % w)
    # headline region (markers 1, 2)
    c0 = ctx.counters()
    region_marker(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = ctx.gwas_semiparallel(gin)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    region_marker(2)
    c1 = ctx.counters()
    ms = (t1 - t0) * 1e3 / args.steps
    log("[bench] %d steps, %.1f ms/step" % (args.steps, ms))
    # roofline region (markers 3, 4): one stream, the dominant kernel's launches timed
    ctx.set_streams(1)
    ctx.kernel_timing(True)
    ctx.gwas_semiparallel(gin)
    torch.cuda.synchronize()
    ctx.kernel_timing(False)
    warm = ctx.kernel_report()
    dominant = max(warm.items(), key=lambda kv: kv[1][1])[0]
    ctx.kernel_timing_only(dominant)
    ctx.kernel_timing(True)
    region_marker(3)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        ctx.gwas_semiparallel(gin)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    region_marker(4)
    ctx.kernel_timing(False)
    kt = ctx.kernel_report()
    ms_one = (t3 - t2) * 1e3 / args.steps
    log("[bench] one stream: %.1f ms/step (dominant kernel %s timed)" % (ms_one, dominant))
    # key-switch region (markers 5, 6): every key switch of the steps timed as a whole on one stream
    ctx.kernel_timing_only("keyswitch")
    ctx.kernel_timing(True)
    region_marker(5)
    for _ in range(args.steps):
        ctx.gwas_semiparallel(gin)
    torch.cuda.synchronize()
    region_marker(6)
    ctx.kernel_timing(False)
    ks = ctx.kernel_report().get("keyswitch")
    ctx.kernel_timing_only(None)
    ctx.set_streams(2)
    # end-to-end with the host boundary (outside the timed region): finalize = D2H + decrypt + divide
    t4 = time.perf_counter()
    res = ctx.gwas_finalize(out)
    t5 = time.perf_counter()
    per_step = {k: (c1[k] - c0[k]) // args.steps for k in c0}
    return dict(ms=ms, ms_one_stream=ms_one, kernels=kt, warm_kernels=warm, counters=per_step, keyswitch=ks,
                finalize_ms=(t5 - t4) * 1e3,
                b_finite=int(np.isfinite(res["b"]).sum()), pool=ctx.pool_stats(), alpha=ctx.alpha)


def forms_leg(args):
    """Batched multi-job form vs the plain one-job-at-a-time path, and the serving loop under Poisson
    arrivals vs FIFO one job at a time, on a seeded mix of jobs with the batched configuration's size
    distribution (n ~ U{100..2000}, k = 4, m ~ logU[1e3, 5e4] scaled by args.forms_m_scale)."""
    import torch

    import paper_1902_04303_amd as P
    from synth import job_mix, make_gwas_data, poisson_arrivals

    L = 7 * KAPPA + 5
    ctx = P.Context(LOG_N, L, LOG_SCALE, alpha=args.ks_alpha)
    ctx.keygen(7, galois_set(2048))
    jobs = job_mix(args.forms_jobs, 301, args.forms_m_scale)
    snps = sum(m for _, _, m, _ in jobs)

    def pack_all():
        ins = []
        for n, k, m, ds in jobs:
            d = make_gwas_data(n, k, m, seed=ds)
            ins.append(ctx.gwas_pack_encrypt(d.X, d.y, d.S, KAPPA, ds))
        torch.cuda.synchronize()
        return ins

    ins = pack_all()
    # warm the pool with one job of the largest shape
    ctx.gwas_semiparallel(ins[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in ins:
        ctx.gwas_semiparallel(i)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    ctx.gwas_semiparallel_multi(ins, chunk=64)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    log("[bench] %d jobs (%d SNPs): plain %.2fs, batched %.2fs" % (len(jobs), snps, t_plain, t_batched))
    batched = {"jobs": len(jobs), "snps": snps, "plain_jobs_per_s": round(len(jobs) / t_plain, 3),
               "batched_jobs_per_s": round(len(jobs) / t_batched, 3),
               "ratio": round(t_plain / t_batched, 3), "m_scale": args.forms_m_scale}
    del ins

    def serve(max_jobs, burst=False):
        ins = pack_all()
        arrivals = [0.0] * len(ins) if burst else poisson_arrivals(len(ins), args.forms_rate, 302)
        srv = ctx.gwas_server(hbm_budget=0, max_jobs=max_jobs, chunk=64)
        t0 = time.perf_counter()
        ids = []
        for a, i in zip(arrivals, ins):
            while time.perf_counter() - t0 < a:
                time.sleep(0.001)
            ids.append(srv.submit(i))
        for jid, (_, _, m, _) in zip(ids, jobs):
            srv.poll(jid, m, wait=True)
        st = srv.stats()
        srv.close()
        return st

    cb = serve(64)
    fifo = serve(1)
    log("[bench] serving: continuous p50 %.0f ms p99 %.0f ms; FIFO p50 %.0f ms p99 %.0f ms" %
        (cb["p50_ms"], cb["p99_ms"], fifo["p50_ms"], fifo["p99_ms"]))
    # the same jobs all at once: requests that wait while others run, where continuous batching matters
    cb_b = serve(64, burst=True)
    fifo_b = serve(1, burst=True)
    log("[bench] serving, all jobs at once: continuous %.1f jobs/s p99 %.0f ms; FIFO %.1f jobs/s p99 %.0f ms" %
        (cb_b["jobs_per_s"], cb_b["p99_ms"], fifo_b["jobs_per_s"], fifo_b["p99_ms"]))
    rnd = lambda st: {k: (round(v, 2) if isinstance(v, float) else v) for k, v in st.items()}  # noqa: E731
    serving = {"jobs": len(jobs), "arrival_rate_per_s": args.forms_rate,
               "continuous": rnd(cb), "fifo_one_at_a_time": rnd(fifo),
               "burst": {"continuous": rnd(cb_b), "fifo_one_at_a_time": rnd(fifo_b)}}
    ctx.close()
    return batched, serving


def config5_leg(args):
    """The serving configuration: seeded Poisson arrivals (4 jobs/s) of jobs drawn from the batched
    configuration's size distribution, the continuous-batching server (admission by HBM footprint, keys
    resident, jobs that arrive while others run share launches) against the one-job-at-a-time FIFO
    server on the same trace.  Two regimes: (a) 256 jobs with m scaled by 0.25, so that every job can be
    encrypted before the run (inputs resident) and the server is not saturated; (b) 64 jobs at full m,
    whose encrypted inputs stay resident for the whole trace."""
    import torch

    import paper_1902_04303_amd as P
    from synth import job_mix, make_gwas_data, poisson_arrivals

    torch.cuda.empty_cache()
    L = 7 * KAPPA + 5
    ctx = P.Context(LOG_N, L, LOG_SCALE, alpha=args.ks_alpha)
    ctx.keygen(7, galois_set(2048))
    ctx.keep_projected(False)
    out = {}
    for label, count, m_scale in (("m_scale_0.25", args.config5_jobs, 0.25), ("full_m", 64, 1.0)):
        jobs = job_mix(count, 501, m_scale)
        arrivals = poisson_arrivals(count, 4.0, 502)
        data = [make_gwas_data(n, k, m, seed=ds) for n, k, m, ds in jobs]
        leg = {"jobs": count, "m_scale": m_scale, "arrival_rate_per_s": 4.0,
               "snps": int(sum(m for _, _, m, _ in jobs)), "arrivals_end_s": round(float(arrivals[-1]), 2)}
        for name, max_jobs in (("continuous", 64), ("fifo_one_at_a_time", 1)):
            ins = [ctx.gwas_pack_encrypt(dd.X, dd.y, dd.S, KAPPA, ds) for dd, (_, _, _, ds) in zip(data, jobs)]
            torch.cuda.synchronize()
            srv = ctx.gwas_server(hbm_budget=0, max_jobs=max_jobs, chunk=64)
            t0 = time.perf_counter()
            ids = []
            for a, i in zip(arrivals, ins):
                while time.perf_counter() - t0 < a:
                    time.sleep(0.0005)
                ids.append(srv.submit(i))
            del ins
            for q, (jid, (_, _, m, _)) in enumerate(zip(ids, jobs)):
                srv.poll(jid, m, wait=True)
                if q % 32 == 31:
                    log("[bench] config 5 %s %s: %d jobs done, %.1f s" % (label, name, q + 1, time.perf_counter() - t0))
            st = srv.stats()
            srv.close()
            ctx.pool_trim()
            torch.cuda.empty_cache()
            leg[name] = {k: (round(v, 2) if isinstance(v, float) else v) for k, v in st.items()}
            log("[bench] config 5 %s %s: %.2f jobs/s, p50 %.0f ms, p99 %.0f ms, peak %d in flight" %
                (label, name, st["jobs_per_s"], st["p50_ms"], st["p99_ms"], st.get("peak_jobs_in_flight", -1)))
        out[label] = leg
    ctx.close()
    return out


def m_layout_leg(args):
    """The M-materialised layout at the same workload (Alg. CP-REP-MatMult: M as n duplicated columns, each
    SNP batch in REP form, S' = sum_i Dup(M_i) S_rep(i) by one lazy tensor sum per batch instead of the
    factorised projection's rotations): ms per step with the REP inputs resident, their client encoding
    and encryption time and their HBM size, and b' against the FP64 GWAS."""
    import torch

    import paper_1902_04303_amd as P
    from oracle import gwas_fp64 as F
    from synth import config_seed, make_gwas_data

    L = 7 * KAPPA + 5
    ctx = P.Context(LOG_N, L, LOG_SCALE, alpha=args.ks_alpha)
    lay = ctx.gwas_layout(N_SAMPLES, K_COV, M_SNPS, KAPPA)
    ctx.keygen(7, galois_set(lay["R"]))
    d = make_gwas_data(N_SAMPLES, K_COV, M_SNPS, seed=config_seed(2))
    gin = ctx.gwas_pack_encrypt(d.X, d.y, d.S, KAPPA, 11)
    torch.cuda.synchronize()
    t0 = time.time()
    ctx.gwas_pack_encrypt_m(gin, d.X, d.S, 11)
    torch.cuda.synchronize()
    enc_s = time.time() - t0
    rep_bytes = gin.footprint()
    out = ctx.gwas_semiparallel(gin)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = ctx.gwas_semiparallel(gin)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    res = ctx.gwas_finalize(out)
    ref = F.modified_gwas(d.X, d.y, d.S, KAPPA)
    ok = ref.den > 1e-9 * np.max(ref.den)
    err = float(np.max(np.abs(res["b"] - ref.b)[ok] / np.maximum(np.abs(ref.b), ref.se)[ok]))
    log("[bench] M-materialised layout: %.1f ms/step (%.0f SNPs/s), REP inputs encrypted in %.1f s, input "
        "footprint %.1f GB, max error %.2g" % (ms, M_SNPS / (ms * 1e-3), enc_s, rep_bytes / 1e9, err))
    ctx.close()
    return {"ms_per_step": round(ms, 2), "snps_per_s": round(M_SNPS / (ms * 1e-3), 1),
            "client_rep_encrypt_s": round(enc_s, 2), "input_footprint_bytes": int(rep_bytes),
            "rep_ciphertexts": N_SAMPLES * lay["n_batches"] + N_SAMPLES * K_COV,
            "max_error_vs_fp64": err}


def config3_leg(args):
    """The batched configuration at full size: 64 seeded jobs, n ~ U{100..2000}, k = 4,
    m ~ logU[1e3, 5e4] (R from 128 to 2048), one key set; all inputs resident.  Plain = one job at a time
    (gwas_semiparallel, each job's outputs freed after it); batched = gwas_semiparallel_multi over all
    jobs (jobs of one (R, k, kappa) share every launch).  S' is not kept (gwas_keep_projected 0) so that the
    64 jobs' outputs fit beside their inputs.  A sample of jobs is checked bit for bit between the two."""
    import torch

    import paper_1902_04303_amd as P
    from synth import job_mix, make_gwas_data

    L = 7 * KAPPA + 5
    ctx = P.Context(LOG_N, L, LOG_SCALE, alpha=args.ks_alpha)
    ctx.keygen(7, galois_set(2048))
    ctx.keep_projected(False)
    jobs = job_mix(args.config3_jobs, 301, 1.0)
    t0 = time.time()
    ins = []
    for i, (n, k, m, seed) in enumerate(jobs):
        d = make_gwas_data(n, k, m, seed=seed)
        ins.append(ctx.gwas_pack_encrypt(d.X, d.y, d.S, KAPPA, 11))
        if i % 8 == 7:
            log("[bench] config 3: %d jobs encrypted" % (i + 1))
    torch.cuda.synchronize()
    enc_s = time.time() - t0
    snps = sum(m for _, _, m, _ in jobs)
    batches = sum(ctx.gwas_layout(n, k, m, KAPPA)["n_batches"] for n, k, m, _ in jobs)
    log("[bench] config 3: %d jobs, %d SNPs, %d SNP batches encrypted in %.1f s" % (len(jobs), snps, batches, enc_s))
    sample = [0, len(jobs) // 2, len(jobs) - 1]
    keep = {}

    def plain(tag):
        t0 = time.perf_counter()
        for i, gin in enumerate(ins):
            o = ctx.gwas_semiparallel(gin)
            if i in sample:
                keep[i] = ctx.export(o.ct(P.GwasOutput.NUM, 0), 0)
            del o
            if i % 16 == 15:
                torch.cuda.synchronize()
                log("[bench] config 3 plain (%s): %d jobs done, %.1f s" % (tag, i + 1, time.perf_counter() - t0))
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def batched(tag):
        t0 = time.perf_counter()
        outs = ctx.gwas_semiparallel_multi(ins, 64)
        torch.cuda.synchronize()
        s = time.perf_counter() - t0
        log("[bench] config 3 batched (%s): %.1f s" % (tag, s))
        return s, outs

    # each form once untimed first, so that the pool holds the blocks its shapes take (a cold pool pays
    # one allocator call per new block size); the pool is trimmed between the two forms
    plain("warm")
    plain_s = plain("timed")
    log("[bench] config 3 plain: %.1f s (%.2f jobs/s)" % (plain_s, len(jobs) / plain_s))
    ctx.pool_trim()   # the plain path's cached blocks (every job shape its own sizes) back to the allocator
    torch.cuda.empty_cache()
    _, outs = batched("warm")
    del outs
    batched_s, outs = batched("timed")
    same = all(np.array_equal(ctx.export(outs[i].ct(P.GwasOutput.NUM, 0), 0), keep[i]) for i in sample)
    log("[bench] config 3 batched: %.1f s (%.2f jobs/s), ratio %.3f, sample bit-identical: %s" %
        (batched_s, len(jobs) / batched_s, plain_s / batched_s, same))
    st = ctx.pool_stats()
    del outs
    del ins
    ctx.close()
    torch.cuda.empty_cache()
    return {"jobs": len(jobs), "snps": snps, "snp_batches": batches, "m_scale": 1.0,
            "client_encrypt_s": round(enc_s, 1), "plain_s": round(plain_s, 2), "batched_s": round(batched_s, 2),
            "plain_jobs_per_s": round(len(jobs) / plain_s, 3), "batched_jobs_per_s": round(len(jobs) / batched_s, 3),
            "batched_snps_per_s": round(snps / batched_s, 1), "ratio": round(plain_s / batched_s, 3),
            "target_ratio": 3.0, "sample_bit_identical": bool(same), "pool_peak_bytes": int(st["peak"])}


def config4_leg(args):
    """The large single job: n = 2000, k = 6, m = 100000 (R = 2048, 32 SNPs per ciphertext, 3125 SNP
    batches), kappa = 3, resident; then the same job in a context whose pool budget is below its working
    set, its SNP batches spilled to pinned host memory and prefetched chunk by chunk on a copy stream."""
    import torch

    import paper_1902_04303_amd as P
    from synth import config_seed, make_gwas_data

    n, k, m = 2000, 6, 100000
    L = 7 * KAPPA + 5
    d = make_gwas_data(n, k, m, seed=config_seed(4))
    out = {}
    for leg, budget in (("resident", 0), ("spilled", args.config4_budget_gb * (1 << 30))):
        ctx = P.Context(LOG_N, L, LOG_SCALE, alpha=args.ks_alpha, pool_budget=budget)
        ctx.keep_projected(False)
        lay = ctx.gwas_layout(n, k, m, KAPPA)
        ctx.keygen(7, galois_set(lay["R"]))
        gin = ctx.gwas_pack_encrypt(d.X, d.y, d.S, KAPPA, 11)
        fp = gin.footprint()
        if budget:
            gin.spill()
        torch.cuda.synchronize()
        o = ctx.gwas_semiparallel(gin)
        torch.cuda.synchronize()
        del o
        steps = max(1, min(args.steps, 2))
        t0 = time.perf_counter()
        for _ in range(steps):
            o = ctx.gwas_semiparallel(gin)
            del o
        torch.cuda.synchronize()
        s = (time.perf_counter() - t0) / steps
        st = ctx.pool_stats()
        out[leg] = {"seconds_per_job": round(s, 3), "snps_per_s": round(m / s, 1), "snp_batches": lay["n_batches"],
                    "input_footprint_bytes": int(fp), "pool_budget_bytes": int(budget),
                    "pool_peak_bytes": int(st["peak"])}
        log("[bench] config 4 %s: %.2f s per job (%.0f SNPs/s), pool peak %.1f GB" %
            (leg, s, m / s, st["peak"] / 1e9))
        ctx.close()
    return out


def kappa_sweep_leg(args):
    """kappa = 1, 2, 3 Newton passes on the same workload (Discussion: the SEAL run reduces kappa to 1 to fit
    its memory; depth table of the circuit): levels and limbs, ms per step, and the accuracy of the decrypted
    b' against the exact semi-parallel GWAS (Sikorska et al., IRLS with the exact sigmoid) by the paper's two
    methods (entries differing by more than e = 0.1, 0.01, 0.005, and the least-squares line of b' against
    b), plus the largest error against the FP64 modified GWAS of the same kappa.  kappa = 1 also runs with
    the homomorphic division (b' and err' as ciphertexts) on a chain longer by its levels."""
    import torch

    import paper_1902_04303_amd as P
    from oracle import gwas_circuit as G
    from oracle import gwas_fp64 as F
    from synth import config_seed, make_gwas_data

    d = make_gwas_data(N_SAMPLES, K_COV, M_SNPS, seed=config_seed(2))
    b_exact, _ = F.sikorska_gwas(d.X, d.y, d.S)
    rows = []
    for kappa, divide in ((1, False), (2, False), (3, False), (1, True)):
        L = G.circuit_depth(kappa) + (P.gwas_div_levels() if divide else 0)
        ctx = P.Context(LOG_N, L, LOG_SCALE, alpha=args.ks_alpha)
        lay = ctx.gwas_layout(N_SAMPLES, K_COV, M_SNPS, kappa)
        ctx.keygen(7, galois_set(lay["R"]))
        gin = ctx.gwas_pack_encrypt(d.X, d.y, d.S, kappa, 11)
        v = ctx.gwas_pack_normalisers(d.S, kappa, 11) if divide else None
        steps = max(1, min(args.steps, 3))
        out = ctx.gwas_semiparallel(gin)
        if divide:
            ctx.gwas_divide(out, v)
        torch.cuda.synchronize()
        c0 = ctx.counters()
        t0 = time.perf_counter()
        for _ in range(steps):
            out = ctx.gwas_semiparallel(gin)
            if divide:
                ctx.gwas_divide(out, v)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        c1 = ctx.counters()
        res = ctx.gwas_finalize_divided(out) if divide else ctx.gwas_finalize(out)
        ref = F.modified_gwas(d.X, d.y, d.S, kappa)
        ok = ref.den > 1e-9 * np.max(ref.den)
        g26 = float(np.max(np.abs(res["b"] - ref.b)[ok] / np.maximum(np.abs(ref.b), ref.se)[ok]))
        counts = F.accuracy_counts(b_exact[ok], res["b"][ok])
        slope, icpt = F.fit_line(b_exact[ok], res["b"][ok])
        row = {"kappa": kappa, "division": divide, "levels": L, "limbs_top": L + 1,
               "limbs_snp_batches": L + 1 - G.snp_depth(kappa), "ms_per_step": round(ms, 2),
               "snps_per_s": round(M_SNPS / (ms * 1e-3), 1),
               "keyswitches_per_step": (c1["keyswitches"] - c0["keyswitches"]) // steps,
               "max_error_vs_fp64_same_kappa": g26,
               "vs_exact_semi_parallel": {"different_entries": {str(e): c for e, (c, _) in counts.items()},
                                          "accuracy_pct": {str(e): round(pct, 2) for e, (_, pct) in counts.items()},
                                          "fit_line": [round(slope, 5), round(icpt, 6)], "snps": int(ok.sum())}}
        log("[bench] kappa %d%s: L = %d, %.1f ms/step, within 0.01 of exact: %.2f %%, fit %.4f x + %.5f" %
            (kappa, " with division" if divide else "", L, ms, counts[0.01][1], slope, icpt))
        rows.append(row)
        ctx.close()
    return rows


DEVICE_SOURCES = ["paper_1902_04303_amd/csrc/" + f
                  for f in ("ntt.hip", "kernels.hip", "modarith.h", "fmod64.h", "ckks_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def device_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in DEVICE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _counter_record():
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != device_source_digest():
        return None
    return rec


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter runs (FETCH_SIZE and WRITE_SIZE, each
    scaled by the same counter's reading for a device copy of known size), or None when there is no
    record for this kernel or the device sources changed since the counters were taken.  The figure is
    replayed from that file, not measured in this run."""
    rec = _counter_record()
    k = (rec or {}).get("kernels", {}).get(kernel)
    if k is None:
        return None
    return {"hbm_bytes_per_launch": int(k["hbm_bytes_per_launch"]),
            "source": "replayed from profiles/hbm_traffic.json (rocprofv3 FETCH_SIZE, WRITE_SIZE)"}


def measured_valu(kernel: str):
    """VALU issue of `kernel` from the committed SQ counter run (SQ_INSTS_VALU per launch over 256 CUs times
    the launch's cycles at 2.4 GHz in the kernel trace: wave64 VALU instructions per CU per cycle, the limit
    being 1), or None (no record, or the device sources changed since)."""
    rec = _counter_record()
    k = (rec or {}).get("valu", {}).get(kernel)
    if k is None:
        return None
    return {"valu_insts_per_cu_cycle": k["valu_insts_per_cu_cycle"], "frac": k["valu_insts_per_cu_cycle"],
            "source": "replayed from profiles/hbm_traffic.json (rocprofv3 SQ_INSTS_VALU over 256 CUs x the launch's "
                      "cycles at 2.4 GHz in the kernel trace)"}


def roofline(kernels, warm, steps):
    """The dominant kernel (largest share of kernel time in the one-stream step where every kernel is timed),
    measured with HIP events at the start and end of its own launches over the roofline region's steps.
    A kernel that declares algorithmic FP64 operations (the key-switch inner product, bound by its modular
    products) is placed against the FP64 vector peak, the others against HBM bandwidth.  Algorithmic bytes
    count an NTT as 16 N per limb transform (8 N per pass: the first pass's reads, the second pass's
    writes) plus a fused epilogue's operands; pass_bytes add the two-pass NTT's intermediate round trip."""
    name, (cnt, tot_ms, by, fl, pb) = max(kernels.items(), key=lambda kv: kv[1][1])
    avg_ms = tot_ms / cnt
    gbs = (by / cnt) / (avg_ms * 1e-3) / 1e9
    pass_gbs = (pb / cnt) / (avg_ms * 1e-3) / 1e9
    out = {"kernel": name}
    if fl > 0:
        tf = (fl / cnt) / (avg_ms * 1e-3) / 1e12
        out.update({"bound": "alu", "achieved": round(tf, 2), "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(tf / FP64_VECTOR_PEAK_TFLOPS, 4)})
    else:
        out.update({"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4)})
    tr = measured_traffic(name)
    out.update({"traffic": tr["hbm_bytes_per_launch"] if tr else None,
                "traffic_source": tr["source"] if tr else None,
                "launches_per_step": cnt // steps,
                "avg_launch_us": round(avg_ms * 1e3, 2), "algorithmic_bytes_per_launch": int(by / cnt),
                "algorithmic_hbm_gbs": round(gbs, 1), "pass_bytes_per_launch": int(pb / cnt),
                "pass_hbm_gbs": round(pass_gbs, 1), "pass_frac": round(pass_gbs / HBM_PEAK_GBS, 4),
                "algorithmic_fp64_ops_per_launch": int(fl / cnt),
                "share_of_kernel_time": round(warm[name][1] / sum(v[1] for v in warm.values()), 3)})
    v = measured_valu(name)
    if v:
        out["valu"] = v
    return out


def keyswitch_roofline(ks, steps):
    """Whole key switches (ModUp, inner product, ModDown: every kernel between the events around a key
    switch) against HBM: algorithmic bytes 8 N [count l + keys 2 G (l + alpha) + count 4 l] per call."""
    if not ks:
        return None
    cnt, ms, by, _, _ = ks
    gbs = by / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "calls_per_step": cnt // steps,
            "ms_per_step": round(ms / steps, 3), "algorithmic_bytes_per_step": int(by / steps)}


def ntt_aggregate(warm, limb_ntts):
    """Every NTT pass of one step (one stream, every kernel timed) against the transforms' own bytes:
    limb transforms x 16 N over the summed pass time."""
    ms = sum(v[1] for k, v in warm.items() if k.startswith("ntt_pass<"))
    by = limb_ntts * 16.0 * (1 << LOG_N)
    gbs = by / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "limb_transforms_per_step": int(limb_ntts),
            "ms_per_step": round(ms, 3)}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_op_times(C, G, p, o, rng):
    """Per-operation times of the oracle at the workload's ring (N = 2^16): one limb NTT, a key switch
    (relinearisation key) at 6, 15 and 27 limbs, a tensor product and a rescale at 27 limbs (ms)."""
    def rand_ct(depth):
        l = p.limbs_at_depth(depth)
        return C.Ct(np.stack([np.stack([rng.integers(0, q, size=p.N, dtype=np.uint64) for q in p.q[:l]])
                              for _ in range(2)]), depth, p.scales[depth])

    def timed(f, reps=1):
        t0 = time.perf_counter()
        for _ in range(reps):
            f()
        return round((time.perf_counter() - t0) * 1e3 / reps, 3)

    out = {}
    a = rand_ct(0)
    limb = np.ascontiguousarray(a.data[0, 1])
    ev = np.empty_like(limb)
    out["limb_ntt_ms"] = timed(lambda: C.lib().ref_to_eval(o._ctx, 1, C._p(limb), C._p(ev)), 5)
    for l in (6, 15, 27):
        d = np.ascontiguousarray(rand_ct(p.L + 1 - l).data[1])
        out["keyswitch_l%d_ms" % l] = timed(lambda: o.keyswitch(d, 0))
    b = rand_ct(0)
    out["tensor_l27_ms"] = timed(lambda: o.tensor([(a, b)]))
    out["rescale_l27_ms"] = timed(lambda: o.rescale(a))
    return out


def cpu_baseline_leg(alpha: int):
    """The CPU oracle on a bounded sample of the same workload: the per-batch part of whole 256-SNP batches
    (the fixed logistic-regression part is excluded, which favours the CPU), on every host thread; plus
    per-operation times on one thread and on every thread, and the FP64 plaintext GWAS."""
    from oracle import ckks as C
    from oracle import gwas_circuit as G
    from oracle import gwas_fp64 as F
    from synth import config_seed, make_gwas_data

    L = G.circuit_depth(KAPPA)
    p = C.make_params(LOG_N, L, LOG_SCALE, alpha)
    d = make_gwas_data(N_SAMPLES, K_COV, M_SNPS, seed=config_seed(2))
    lay = G.make_layout(p.N, N_SAMPLES, K_COV, M_SNPS)
    ds = G.snp_depth(KAPPA)
    o = C.Oracle(p)
    t0 = time.time()
    # the per-batch keys at the batch levels; relinearisation at full height for the per-operation times
    o.keygen(7, G.required_galois(p.N, lay.R), max_limbs=p.limbs_at_depth(ds), key_limbs={0: p.L + 1})
    log("[bench] cpu oracle keygen %.1fs" % (time.time() - t0))
    t0 = time.perf_counter()
    ref = F.modified_gwas(d.X, d.y, d.S, KAPPA)
    fp64_ms = (time.perf_counter() - t0) * 1e3
    A = F.xtx_inverse(d.X)
    enc = lambda v, depth, i: o.encrypt(C.encode(G.periodic_slots(v, lay), p.N, p.scales[depth]), depth,  # noqa
                                        p.scales[depth], 1000 + i)
    XA = d.X @ A
    fx = G.FixedPart(x=[enc(d.X[:, j], ds + 2, j) for j in range(K_COV)],
                     rr=[enc(XA[:, j], ds, 10 + j) for j in range(K_COV)],
                     w=enc(ref.w, ds + 3, 20), u=enc(ref.w * ref.z_proj, ds + 3, 21))
    K = G.diag_width(lay)
    if K:
        # the packed projection's diagonals, encrypted directly: Z_t (rotated right by t) at the SNP depth
        # and X_t at the SNP depth + 2, block row r holding column (r + t) mod K (0 beyond k or n)
        rows = np.arange(p.N // 2) % lay.R

        def diag(M, t):
            j = (rows + t) % K
            keep = (rows < N_SAMPLES) & (j < K_COV)
            v = np.zeros(p.N // 2)
            v[keep] = M[rows[keep], j[keep]]
            return v
        fx.zt = [o.encrypt(C.encode(np.roll(diag(XA, t), t), p.N, p.scales[ds]), ds, p.scales[ds], 40 + t)
                 for t in range(K)]
        fx.xt = [o.encrypt(C.encode(diag(d.X, t), p.N, p.scales[ds + 2]), ds + 2, p.scales[ds + 2], 50 + t)
                 for t in range(K)]
    # SNP batches in order until the timed oracle work reaches CPU_SAMPLE_S seconds (at most
    # CPU_SAMPLE_MAX_BATCHES); each batch's encryption is outside the timed part
    circ = G.Circuit(o, lay)
    ks0 = o.n_keyswitch
    t = 0.0
    nb = 0
    while nb < CPU_SAMPLE_MAX_BATCHES and (nb == 0 or t < CPU_SAMPLE_S):
        S = o.encrypt(C.encode(G.snp_batch_slots(d.S, lay, nb), p.N, p.scales[ds]), ds, p.scales[ds], 30 + nb)
        t0 = time.perf_counter()
        circ.run_batch(S, fx)
        t += time.perf_counter() - t0
        nb += 1
    cores = int(C.lib().ref_num_threads())
    log("[bench] cpu oracle: %d SNP batches (%d SNPs) in %.1fs on %d threads" % (nb, nb * lay.tau, t, cores))
    rng = np.random.default_rng(5)
    ops_all = oracle_op_times(C, G, p, o, rng)
    C.lib().ref_set_threads(1)
    try:
        ops_one = oracle_op_times(C, G, p, o, rng)
    finally:
        C.lib().ref_set_threads(0)
    log("[bench] cpu oracle per-op ms, %d threads: %s; 1 thread: %s" % (cores, ops_all, ops_one))
    whole = None
    try:
        with open(os.path.join(ROOT, "tests", "golden", "circuit_digests.json")) as fh:
            rec = json.load(fh)["gwas_n245_k4_m10643"]
        whole = {"seconds": rec["oracle_circuit_seconds"], "threads": rec["oracle_threads"],
                 "source": "whole circuit (fixed part and 42 SNP batches) timed offline by "
                           "tests/golden/make_circuit_digests.py on another host"}
    except (OSError, KeyError, ValueError):
        pass
    return {"value": round(nb * lay.tau / t, 3), "unit": "SNPs/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "per-batch part of the first %d 256-SNP batches of the same workload (S' = M S, numerator, "
                      "both denominators; %d key switches at <= 6 limbs), %.1f s of oracle time on %d threads; "
                      "the fixed logistic-regression part is excluded" % (nb, o.n_keyswitch - ks0, t, cores),
            "per_op_ms_all_threads": ops_all, "per_op_ms_one_thread": ops_one,
            "fp64_plaintext_gwas_ms": round(fp64_ms, 2), "whole_job_oracle": whole}


def copy_calibration(nbytes: int) -> int:
    """A device-to-device copy of nbytes (a fill kernel writes the source first): the known-size
    reference that scales HBM byte counters (FETCH_SIZE, WRITE_SIZE) to bytes."""
    import torch
    n = nbytes // 8
    src = torch.arange(n, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8}), flush=True)
    return 0


def run(args) -> int:
    g = gpu_leg(args)
    value = M_SNPS / (g["ms"] * 1e-3)
    rl = roofline(g["kernels"], g["warm_kernels"], args.steps)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_leg(g["alpha"])
    batched = serving = None
    if args.forms_jobs > 0:
        batched, serving = forms_leg(args)
    sweep = kappa_sweep_leg(args) if args.kappa_sweep else None
    mlay = m_layout_leg(args) if args.m_layout else None
    c3 = config3_leg(args) if args.config3_jobs > 0 else None
    c4 = config4_leg(args) if args.config4 else None
    c5 = config5_leg(args) if args.config5_jobs > 0 else None
    ks = keyswitch_roofline(g["keyswitch"], args.steps)
    ntt = ntt_aggregate(g["warm_kernels"], g["counters"]["limb_ntts"])
    line = {
        "metric": "encrypted SNPs/s at 245x4x10643",
        "value": round(value, 1),
        "unit": "SNPs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(g["ms"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n": N_SAMPLES, "k": K_COV, "m": M_SNPS, "kappa": KAPPA,
                   "log_n": LOG_N, "levels": 7 * KAPPA + 5, "log2_scale": LOG_SCALE, "ks_alpha": g["alpha"],
                   "snp_batches": 42,
                   "parallelism": "1 GPU"},
        "roofline": rl,
        "keyswitch": ks,
        "ntt_all_passes": ntt,
        "cpu_baseline": cpu,
        "batched": batched,
        "serving": serving,
        "kappa_sweep": sweep,
        "m_layout": mlay,
        "config3_batched_full": c3,
        "config4_large_job": c4,
        "config5_serving": c5,
        "per_step": g["counters"],
        "ms_per_step_one_stream": round(g["ms_one_stream"], 3),
        "finalize_ms": round(g["finalize_ms"], 1),
    }
    print(json.dumps(line), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ks-alpha", type=int, default=0, help="digit-group size of key switching (0: library default)")
    ap.add_argument("--forms-jobs", type=int, default=12, help="jobs in the batched / serving legs (0: skip)")
    ap.add_argument("--forms-m-scale", type=float, default=0.1, help="scale of the job SNP counts")
    ap.add_argument("--forms-rate", type=float, default=4.0, help="Poisson arrival rate (jobs/s)")
    ap.add_argument("--no-m-layout", dest="m_layout", action="store_false",
                    help="skip the M-materialised layout at the same workload")
    ap.add_argument("--config3-jobs", type=int, default=0,
                    help="run the batched configuration at full size with this many jobs (64: the configuration)")
    ap.add_argument("--config4", action="store_true", help="run the large single job (n=2000, k=6, m=100000)")
    ap.add_argument("--config5-jobs", type=int, default=0,
                    help="run the serving configuration with this many jobs at m x 0.25 (256: the configuration), "
                         "then 64 jobs at full m")
    ap.add_argument("--config4-budget-gb", type=int, default=48, help="pool budget of the spilled config-4 leg")
    ap.add_argument("--no-kappa-sweep", dest="kappa_sweep", action="store_false",
                    help="skip the kappa = 1, 2, 3 sweep (and the division run)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run one device copy of BYTES (byte-counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    if args.gpus != 1:
        print("bench.py runs on one GPU: this build measures the single-GPU path (the multi-GPU sharding is a "
              "design only); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        return 2
    return run(args)


if __name__ == "__main__":
    sys.exit(main())
