"""GPU tests of the batched, serving and spill forms and of resource limits.

The arithmetic of a job is the same in every form, so outputs are compared bit
for bit with the plain single-job path (itself checked against the oracle in
test_gpu_parity.py).
"""
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import paper_1902_04303_amd as P  # noqa: E402
from oracle import gwas_circuit as G  # noqa: E402
from synth import make_gwas_data  # noqa: E402

KAPPA = 3
LOG_N, SCALE_BITS = 10, 30


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = P.Context(LOG_N, G.circuit_depth(KAPPA), SCALE_BITS)
    c.keygen(7, G.required_galois(1 << LOG_N, 64))
    return c


JOBS = [(30, 4, 50, 101), (20, 4, 70, 102), (60, 4, 40, 103), (28, 4, 10, 104), (50, 3, 20, 105)]


def pack(ctx, n, k, m, seed, enc=11):
    d = make_gwas_data(n, k, m, seed=seed)
    return ctx.gwas_pack_encrypt(d.X, d.y, d.S, KAPPA, enc + seed)


def outputs(ctx, out, n_batches):
    res = {}
    for which in (P.GwasOutput.NUM, P.GwasOutput.DEN_EVEN, P.GwasOutput.DEN_ODD, P.GwasOutput.S_PROJ):
        cts = []
        ch = 0
        got = 0
        while got < n_batches:
            ct = out.ct(which, ch)
            cnt = ct.count
            cts += [ctx.export(ct, i) for i in range(cnt)]
            got += cnt
            ch += 1
        res[which] = cts
    for which in (P.GwasOutput.W, P.GwasOutput.W_INV, P.GwasOutput.Z_PROJ, P.GwasOutput.U):
        res[which] = [ctx.export(out.ct(which))]
    return res


def same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        assert len(a[k]) == len(b[k]), k
        for x, y in zip(a[k], b[k]):
            assert np.array_equal(x, y), k


@pytest.fixture(scope="module")
def singles(ctx):
    ref = []
    for n, k, m, seed in JOBS:
        lay = ctx.gwas_layout(n, k, m, KAPPA)
        out = ctx.gwas_semiparallel(pack(ctx, n, k, m, seed))
        ref.append(outputs(ctx, out, lay["n_batches"]))
    return ref


def test_multi_job_matches_single_jobs(ctx, singles):
    say("[gpu] multi-job batched form")
    ins = [pack(ctx, n, k, m, seed) for n, k, m, seed in JOBS]
    for chunk in (3, 64):
        outs = ctx.gwas_semiparallel_multi(ins, chunk=chunk)
        for (n, k, m, seed), o, r in zip(JOBS, outs, singles):
            same(outputs(ctx, o, ctx.gwas_layout(n, k, m, KAPPA)["n_batches"]), r)


def test_one_and_two_streams_agree(ctx, singles):
    """The circuit with the logistic-regression part on a second stream (the default) and in order on one
    stream give the same ciphertexts."""
    say("[gpu] one stream vs two streams")
    for q in (0, 2, 4):
        n, k, m, seed = JOBS[q]
        lay = ctx.gwas_layout(n, k, m, KAPPA)
        ctx.set_streams(1)
        try:
            one = outputs(ctx, ctx.gwas_semiparallel(pack(ctx, n, k, m, seed)), lay["n_batches"])
        finally:
            ctx.set_streams(2)
        same(one, singles[q])
        for chunk in (1, 2):   # several chunks: every chunk's S' is computed before the join
            two = outputs(ctx, ctx.gwas_semiparallel(pack(ctx, n, k, m, seed), chunk), lay["n_batches"])
            same(two, singles[q])


def test_spilled_snp_batches_match_resident(ctx, singles):
    say("[gpu] spill")
    n, k, m, seed = JOBS[1]
    inp = pack(ctx, n, k, m, seed)
    before = inp.footprint()
    inp.spill()
    assert inp.footprint() < before
    for chunk in (1, 2, 64):
        out = ctx.gwas_semiparallel(inp, chunk)
        same(outputs(ctx, out, ctx.gwas_layout(n, k, m, KAPPA)["n_batches"]), singles[1])


def test_server_results_same_alone_and_in_mix(ctx, singles):
    say("[gpu] server")
    ins = [pack(ctx, n, k, m, seed) for n, k, m, seed in JOBS]
    srv = ctx.gwas_server(hbm_budget=0, max_jobs=8, chunk=2)
    ids = []
    for i, inp in enumerate(ins):
        ids.append(srv.submit(inp))
        time.sleep(0.002)         # arrivals while earlier jobs are on the GPU
    for jid, (n, k, m, seed), r in zip(ids, JOBS, singles):
        out = srv.poll(jid, m, wait=True)
        same(outputs(ctx, out, ctx.gwas_layout(n, k, m, KAPPA)["n_batches"]), r)
    st = srv.stats()
    assert st["completed"] == len(JOBS)
    assert 0 < st["p50_ms"] <= st["p99_ms"]
    assert st["peak_jobs_in_flight"] >= 2        # work of several jobs overlapped
    srv.close()


def test_server_admission_budget_and_spill(ctx, singles):
    say("[gpu] server budget")
    ins = [pack(ctx, *JOBS[i]) for i in (0, 1)]
    fp = max(i.footprint() for i in ins)
    srv = ctx.gwas_server(hbm_budget=int(fp * 1.2), max_jobs=8, chunk=4)
    ids = [srv.submit(i) for i in ins]
    for jid, i in zip(ids, (0, 1)):
        out = srv.poll(jid, JOBS[i][2], wait=True)
        same(outputs(ctx, out, ctx.gwas_layout(*JOBS[i][:3], KAPPA)["n_batches"]), singles[i])
    assert srv.stats()["peak_jobs_in_flight"] == 1   # only one fits the budget at a time
    srv.close()
    # a job larger than the whole budget runs with its SNP batches spilled to the host
    srv = ctx.gwas_server(hbm_budget=1024, max_jobs=8, chunk=4)
    jid = srv.submit(pack(ctx, *JOBS[1]))
    out = srv.poll(jid, JOBS[1][2], wait=True)
    same(outputs(ctx, out, ctx.gwas_layout(*JOBS[1][:3], KAPPA)["n_batches"]), singles[1])
    srv.close()


def test_server_cancel(ctx):
    srv = ctx.gwas_server(hbm_budget=1, max_jobs=1, chunk=1)
    a = srv.submit(pack(ctx, *JOBS[0]))
    b = srv.submit(pack(ctx, *JOBS[1]))
    srv.cancel(b)
    with pytest.raises(P.CkksError) as e:
        srv.poll(b, JOBS[1][2], wait=True)
    assert e.value.code == -7
    assert srv.poll(a, JOBS[0][2], wait=True) is not None
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
