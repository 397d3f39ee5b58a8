"""GPU tests of the batched, serving and spill forms and of resource limits.

The arithmetic of a job is the same in every form.  Every job's inputs are the CPU oracle's own
ciphertexts (imported into the library), and every output ciphertext of every form is compared bit for
bit with the oracle's circuit on the same job (Alg. Semi Parallel GWAS): multi-job launches, one and two
streams, spilled SNP batches and jobs served in a mix.
"""
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import paper_1902_04303_amd as P  # noqa: E402
from oracle import ckks as C  # noqa: E402
from oracle import gwas_circuit as G  # noqa: E402
from synth import make_gwas_data  # noqa: E402

KAPPA = 3
LOG_N, SCALE_BITS = 10, 30
R_MAX = 64   # the keys cover every job's block size (R = 32 and 64 here)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = P.Context(LOG_N, G.circuit_depth(KAPPA), SCALE_BITS)
    c.keygen(7, G.required_galois(1 << LOG_N, R_MAX))
    return c


# (n, k, m, data seed): block sizes 32 and 64, ragged last batches, k = 3 and 4
JOBS = [(30, 4, 50, 101), (20, 4, 70, 102), (60, 4, 40, 103), (28, 4, 10, 104), (50, 3, 20, 105)]

KINDS = (P.GwasOutput.NUM, P.GwasOutput.DEN_EVEN, P.GwasOutput.DEN_ODD, P.GwasOutput.S_PROJ)
SINGLE = (P.GwasOutput.W, P.GwasOutput.W_INV, P.GwasOutput.Z_PROJ, P.GwasOutput.U)


@pytest.fixture(scope="module")
def oracle_jobs():
    """Each job encrypted and evaluated by the oracle (same keys as the library: seed 7)."""
    p = C.make_params(LOG_N, G.circuit_depth(KAPPA), SCALE_BITS)
    o = C.Oracle(p)
    o.keygen(7, G.required_galois(p.N, R_MAX))
    jobs = []
    for n, k, m, seed in JOBS:
        say("[oracle] job n=%d k=%d m=%d" % (n, k, m))
        d = make_gwas_data(n, k, m, seed=seed)
        inp = G.encrypt_inputs(o, G.encode_inputs(p, d.X, d.y, d.S, KAPPA), n, k, m, KAPPA, 11 + seed)
        lay = G.make_layout(p.N, n, k, m)
        out = G.Circuit(o, lay).run(inp)
        ref = {P.GwasOutput.NUM: [c.data for c in out.num], P.GwasOutput.DEN_EVEN: [c.data for c in out.den_even],
               P.GwasOutput.DEN_ODD: [c.data for c in out.den_odd], P.GwasOutput.S_PROJ: [c.data for c in out.S_proj],
               P.GwasOutput.W: [out.w.data], P.GwasOutput.W_INV: [out.w_inv.data],
               P.GwasOutput.Z_PROJ: [out.z_proj.data], P.GwasOutput.U: [out.u.data]}
        jobs.append((inp, lay, ref))
    return jobs


def pack(ctx, oracle_jobs, q):
    """Job q's oracle ciphertexts imported into the library."""
    inp, lay, _ = oracle_jobs[q]
    n, k, m, _ = JOBS[q]
    imp = lambda c: ctx.import_ct(c.data, c.depth, c.scale)  # noqa: E731
    return ctx.gwas_input_from_cts(n, k, m, KAPPA, [imp(c) for c in inp.x], imp(inp.y),
                                   [imp(inp.A[pr]) for pr in G.a_pairs(k)], [imp(c) for c in inp.S])


def outputs(ctx, out, n_batches):
    res = {}
    for which in KINDS:
        cts = []
        ch = 0
        got = 0
        while got < n_batches:
            ct = out.ct(which, ch)
            cnt = ct.count
            cts += [ctx.export(ct, i) for i in range(cnt)]
            got += cnt
            ch += 1
        res[which] = cts[:n_batches]
    for which in SINGLE:
        res[which] = [ctx.export(out.ct(which))]
    return res


def same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        assert len(a[k]) == len(b[k]), k
        for i, (x, y) in enumerate(zip(a[k], b[k])):
            assert np.array_equal(x, y), (k, i)


@pytest.fixture(scope="module")
def singles(oracle_jobs):
    return [ref for _, _, ref in oracle_jobs]


def nb(q):
    return G.make_layout(1 << LOG_N, *JOBS[q][:3]).n_batches


def test_single_jobs_match_oracle(ctx, oracle_jobs, singles):
    say("[gpu] single jobs")
    for q in range(len(JOBS)):
        same(outputs(ctx, ctx.gwas_semiparallel(pack(ctx, oracle_jobs, q)), nb(q)), singles[q])


def test_multi_job_matches_oracle(ctx, oracle_jobs, singles):
    say("[gpu] multi-job batched form")
    ins = [pack(ctx, oracle_jobs, q) for q in range(len(JOBS))]
    for chunk in (3, 64):
        outs = ctx.gwas_semiparallel_multi(ins, chunk=chunk)
        for q, o in enumerate(outs):
            same(outputs(ctx, o, nb(q)), singles[q])


def test_back_to_back_calls_match_oracle(ctx, oracle_jobs, singles):
    """Calls issued back to back without synchronisation: outputs dropped as soon as the next call returns
    (their blocks go back to both streams' pools while earlier calls may still run), an input imported
    between two calls, and every kept output compared with the oracle after one final synchronisation."""
    import torch
    say("[gpu] back-to-back calls")
    order = [0, 2, 4, 1, 3, 0, 4, 2]
    ins = {q: pack(ctx, oracle_jobs, q) for q in (0, 2, 4)}
    kept = []
    out = None
    for i, q in enumerate(order):
        if q not in ins:
            ins[q] = pack(ctx, oracle_jobs, q)   # imported between calls, no synchronisation
        out = ctx.gwas_semiparallel(ins[q])     # the previous output (unless kept) is freed here
        if i % 3 == 2:
            kept.append((q, out))
    kept.append((order[-1], out))
    torch.cuda.synchronize()
    for q, o in kept:
        same(outputs(ctx, o, nb(q)), singles[q])


def test_one_and_two_streams_agree(ctx, oracle_jobs, singles):
    """The circuit with the logistic-regression part on a second stream (the default) and in order on one
    stream give the oracle's ciphertexts."""
    say("[gpu] one stream vs two streams")
    for q in (0, 2, 4):
        ctx.set_streams(1)
        try:
            one = outputs(ctx, ctx.gwas_semiparallel(pack(ctx, oracle_jobs, q)), nb(q))
        finally:
            ctx.set_streams(2)
        same(one, singles[q])
        for chunk in (1, 2):   # several chunks: every chunk's S' is computed before the join
            two = outputs(ctx, ctx.gwas_semiparallel(pack(ctx, oracle_jobs, q), chunk), nb(q))
            same(two, singles[q])


def test_spilled_snp_batches_match_oracle(ctx, oracle_jobs, singles):
    say("[gpu] spill")
    inp = pack(ctx, oracle_jobs, 1)
    before = inp.footprint()
    inp.spill()
    assert inp.footprint() < before
    for chunk in (1, 2, 64):
        out = ctx.gwas_semiparallel(inp, chunk)
        same(outputs(ctx, out, nb(1)), singles[1])


def test_server_results_same_alone_and_in_mix(ctx, oracle_jobs, singles):
    say("[gpu] server")
    ins = [pack(ctx, oracle_jobs, q) for q in range(len(JOBS))]
    srv = ctx.gwas_server(hbm_budget=0, max_jobs=8, chunk=2)
    ids = []
    for inp in ins:
        ids.append(srv.submit(inp))
        time.sleep(0.002)         # arrivals while earlier jobs are on the GPU
    for q, jid in enumerate(ids):
        out = srv.poll(jid, JOBS[q][2], wait=True)
        same(outputs(ctx, out, nb(q)), singles[q])
    st = srv.stats()
    assert st["completed"] == len(JOBS)
    assert 0 < st["p50_ms"] <= st["p99_ms"]
    assert st["peak_jobs_in_flight"] >= 2        # work of several jobs overlapped
    srv.close()


def test_server_admission_budget_and_spill(ctx, oracle_jobs, singles):
    say("[gpu] server budget")
    ins = [pack(ctx, oracle_jobs, q) for q in (0, 1)]
    fp = max(i.footprint() for i in ins)
    srv = ctx.gwas_server(hbm_budget=int(fp * 1.2), max_jobs=8, chunk=4)
    ids = [srv.submit(i) for i in ins]
    for jid, q in zip(ids, (0, 1)):
        out = srv.poll(jid, JOBS[q][2], wait=True)
        same(outputs(ctx, out, nb(q)), singles[q])
    assert srv.stats()["peak_jobs_in_flight"] == 1   # only one fits the budget at a time
    srv.close()
    # a job larger than the whole budget runs with its SNP batches spilled to the host
    srv = ctx.gwas_server(hbm_budget=1024, max_jobs=8, chunk=4)
    jid = srv.submit(pack(ctx, oracle_jobs, 1))
    out = srv.poll(jid, JOBS[1][2], wait=True)
    same(outputs(ctx, out, nb(1)), singles[1])
    srv.close()


def test_server_cancel_queued(ctx, oracle_jobs):
    srv = ctx.gwas_server(hbm_budget=1, max_jobs=1, chunk=1)
    a = srv.submit(pack(ctx, oracle_jobs, 0))
    b = srv.submit(pack(ctx, oracle_jobs, 1))
    srv.cancel(b)
    with pytest.raises(P.CkksError) as e:
        srv.poll(b, JOBS[1][2], wait=True)
    assert e.value.code == -7
    assert srv.poll(a, JOBS[0][2], wait=True) is not None
    srv.close()


@pytest.mark.parametrize("delay_s", [0.0, 0.005, 0.05])
def test_server_cancel_admitted_or_running(ctx, oracle_jobs, singles, delay_s):
    """A long job cancelled after admission (during its fixed part or between its SNP-batch chunks,
    depending on the delay) returns its budget exactly once: the next two jobs, which fit the budget only
    one at a time, still run one at a time and give the oracle's ciphertexts."""
    say("[gpu] server cancel after %.3fs" % delay_s)
    d = make_gwas_data(30, 4, 1280, seed=777)   # 40 SNP batches, one per iteration at chunk 1
    long_job = ctx.gwas_pack_encrypt(d.X, d.y, d.S, KAPPA, 5)
    ins = [pack(ctx, oracle_jobs, q) for q in (0, 3)]
    fa, fb, fc = long_job.footprint(), ins[0].footprint(), ins[1].footprint()
    budget = int(max(fa, fb, fc) * 1.05)
    assert budget < fb + fc   # B and C fit only one at a time
    srv = ctx.gwas_server(hbm_budget=budget, max_jobs=8, chunk=1)
    a = srv.submit(long_job)
    time.sleep(delay_s)
    srv.cancel(a)
    b = srv.submit(ins[0])
    c = srv.submit(ins[1])
    with pytest.raises(P.CkksError) as e:
        srv.poll(a, 1280, wait=True)
    assert e.value.code == -7
    same(outputs(ctx, srv.poll(b, JOBS[0][2], wait=True), nb(0)), singles[0])
    same(outputs(ctx, srv.poll(c, JOBS[3][2], wait=True), nb(3)), singles[3])
    st = srv.stats()
    assert st["completed"] == 2
    assert st["peak_jobs_in_flight"] == 1
    srv.close()


def test_pool_budget_error_is_reported_and_context_survives():
    c = P.Context(LOG_N, 4, SCALE_BITS, pool_budget=1 << 20)
    with pytest.raises(P.CkksError) as e:
        c.keygen(1, [c.galois_rotate(1)] * 1 + [c.galois_rotate(2), c.galois_rotate(4)])
    assert e.value.code == -5
    st = c.pool_stats()
    assert st["in_use"] <= 1 << 20
    c.close()


def test_inputs_must_match_chain(ctx):
    c2 = P.Context(LOG_N, 12, SCALE_BITS)
    d = make_gwas_data(30, 4, 10, seed=1)
    with pytest.raises(P.CkksError) as e:
        c2.gwas_pack_encrypt(d.X, d.y, d.S, KAPPA, 1)
    assert e.value.code == -3
    c2.close()


def test_server_outputs_freed_while_worker_runs(ctx, oracle_jobs, singles):
    """Outputs polled and freed on the caller's thread while the server's worker runs the next jobs:
    freeing returns device buffers to the context's pool under the context's lock (the worker uses the
    same pool), and every result still matches the oracle."""
    say("[gpu] server: outputs freed during work")
    srv = ctx.gwas_server(hbm_budget=0, max_jobs=1, chunk=2)
    for rnd in range(3):
        ids = [(q, srv.submit(pack(ctx, oracle_jobs, q))) for q in range(len(JOBS))]
        for q, jid in ids:
            out = srv.poll(jid, JOBS[q][2], wait=True)
            same(outputs(ctx, out, nb(q)), singles[q])
            del out
    srv.close()
