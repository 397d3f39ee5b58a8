"""GPU tests of the circuit captured as a HIP graph (gwas_graph_*): every replay's output ciphertexts are
bit-identical to the eager call's and to the oracle's, with the context's own eager work and
synchronisations between replays; a second job of the same shape copied into the graph's input replays to
its own eager result; at the paper's dataset shape the replay is bit-identical too.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import paper_1902_04303_amd as P  # noqa: E402
from oracle import ckks as C  # noqa: E402
from oracle import gwas_circuit as G  # noqa: E402
from synth import config_seed, make_gwas_data  # noqa: E402

OUTS = (P.GwasOutput.NUM, P.GwasOutput.DEN_EVEN, P.GwasOutput.DEN_ODD, P.GwasOutput.S_PROJ)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    return torch


def exports(ctx, out, nb, k):
    r = [ctx.export(out.ct(P.GwasOutput.BETA, j)) for j in range(k)]
    for which in OUTS:
        ct = out.ct(which, 0)
        r += [ctx.export(ct, b) for b in range(nb)]
    return r


def same(a, b):
    return len(a) == len(b) and all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("n", [30, 24])   # one colSum and broadcast per covariate; packed projection
def test_graph_replays_match_oracle_and_eager(torch_dev, n):
    torch = torch_dev
    k, m, kappa, log_n, b = 4, 70, 3, 10, 30
    say("[gpu] graph n=%d m=%d" % (n, m))
    p = C.make_params(log_n, G.circuit_depth(kappa), b)
    d = make_gwas_data(n, k, m, seed=config_seed(1, 5))
    lay = G.make_layout(p.N, n, k, m)
    o = C.Oracle(p)
    o.keygen(7, G.required_galois(p.N, lay.R))
    inp = G.encrypt_inputs(o, G.encode_inputs(p, d.X, d.y, d.S, kappa), n, k, m, kappa, 11)
    ref = G.Circuit(o, lay).run(inp)
    want = [c.data for c in ref.beta]
    for lst in (ref.num, ref.den_even, ref.den_odd, ref.S_proj):
        want += [c.data for c in lst]
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        ctx = P.Context(log_n, p.L, b)
        ctx.keygen(7, G.required_galois(p.N, lay.R))
        imp = lambda c: ctx.import_ct(c.data, c.depth, c.scale)  # noqa: E731
        g1 = ctx.gwas_input_from_cts(n, k, m, kappa, [imp(c) for c in inp.x], imp(inp.y),
                                     [imp(inp.A[pr]) for pr in G.a_pairs(k)], [imp(c) for c in inp.S])
        d2 = make_gwas_data(n, k, m, seed=config_seed(1, 6))
        g2 = ctx.gwas_pack_encrypt(d2.X, d2.y, d2.S, kappa, 12)
        e1 = exports(ctx, ctx.gwas_semiparallel(g1), lay.n_batches, k)
        e2 = exports(ctx, ctx.gwas_semiparallel(g2), lay.n_batches, k)
        assert same(e1, want)
        graph = ctx.gwas_graph(g1)
        for rep in range(3):
            out = graph.launch()
            st.synchronize()
            assert same(exports(ctx, out, lay.n_batches, k), want), ("replay", rep)
            # the context's own eager work between replays
            assert same(exports(ctx, ctx.gwas_semiparallel(g2), lay.n_batches, k), e2)
            torch.cuda.synchronize()
        graph.set_input(g2)
        assert same(exports(ctx, graph.launch(), lay.n_batches, k), e2)
        graph.set_input(g1)
        assert same(exports(ctx, graph.launch(), lay.n_batches, k), want)
        res = ctx.gwas_finalize(graph.out)
        assert np.isfinite(res["b"]).sum() > 0
        graph.close()
        # the context is still usable after the graph is gone
        assert same(exports(ctx, ctx.gwas_semiparallel(g1), lay.n_batches, k), want)
        ctx.close()


def test_graph_at_dataset_shape(torch_dev):
    import time
    torch = torch_dev
    n, k, m, kappa, log_n, b = 245, 4, 10643, 3, 16, 40
    say("[gpu] graph at n=%d m=%d" % (n, m))
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        ctx = P.Context(log_n, G.circuit_depth(kappa), b)
        lay = ctx.gwas_layout(n, k, m, kappa)
        ctx.keygen(7, G.required_galois(1 << log_n, lay["R"]))
        d = make_gwas_data(n, k, m, seed=config_seed(2))
        gin = ctx.gwas_pack_encrypt(d.X, d.y, d.S, kappa, 11)
        eager = exports(ctx, ctx.gwas_semiparallel(gin), lay["n_batches"], k)
        graph = ctx.gwas_graph(gin)
        for rep in range(2):
            out = graph.launch()
            st.synchronize()
            assert same(exports(ctx, out, lay["n_batches"], k), eager), ("replay", rep)
        t0 = time.perf_counter()
        for _ in range(3):
            graph.launch()
        st.synchronize()
        tg = (time.perf_counter() - t0) / 3
        t0 = time.perf_counter()
        for _ in range(3):
            ctx.gwas_semiparallel(gin)
        st.synchronize()
        te = (time.perf_counter() - t0) / 3
        say("[gpu] dataset shape: graph replay %.1f ms, eager %.1f ms per call" % (tg * 1e3, te * 1e3))
        graph.close()
        ctx.close()


def test_tuner_schedules_are_bit_identical(torch_dev):
    """The autotuner's candidates (chunks of all, 32, 16, 8 SNP batches; one or two streams; the covariates'
    products stacked or not) all give the oracle's ciphertexts, and so does the schedule it records."""
    n, k, m, kappa, log_n, b = 30, 4, 700, 3, 10, 30
    say("[gpu] tuner n=%d m=%d" % (n, m))
    p = C.make_params(log_n, G.circuit_depth(kappa), b)
    d = make_gwas_data(n, k, m, seed=config_seed(1, 8))
    lay = G.make_layout(p.N, n, k, m)
    assert lay.n_batches == 22
    o = C.Oracle(p)
    o.keygen(7, G.required_galois(p.N, lay.R))
    inp = G.encrypt_inputs(o, G.encode_inputs(p, d.X, d.y, d.S, kappa), n, k, m, kappa, 11)
    ref = G.Circuit(o, lay).run(inp)
    ctx = P.Context(log_n, p.L, b)
    ctx.keygen(7, G.required_galois(p.N, lay.R))
    imp = lambda c: ctx.import_ct(c.data, c.depth, c.scale)  # noqa: E731
    gin = ctx.gwas_input_from_cts(n, k, m, kappa, [imp(c) for c in inp.x], imp(inp.y),
                                  [imp(inp.A[pr]) for pr in G.a_pairs(k)], [imp(c) for c in inp.S])

    def check(out, ch):
        for bi in range(lay.n_batches):
            for which, r in [(P.GwasOutput.NUM, ref.num), (P.GwasOutput.DEN_EVEN, ref.den_even),
                             (P.GwasOutput.DEN_ODD, ref.den_odd)]:
                assert np.array_equal(ctx.export(out.ct(which, bi // ch), bi % ch), r[bi].data), (which, bi, ch)

    t = ctx.gwas_tune(gin, 1)
    say("[gpu] tuner: %s" % t)
    assert t["candidates"] == 12 and t["chunk"] in (22, 16, 8) and t["streams"] in (1, 2) and t["stack"] in (0, 256)
    for streams in (2, 1):
        ctx.set_streams(streams)
        for stack in (0, 256, 40):
            ctx.set_stack(stack)
            for ch in (22, 16, 8):
                check(ctx.gwas_semiparallel(gin, ch), ch)
    ctx.set_streams(2)
    ctx.set_stack(0)
    ctx.use_tuned(True)
    check(ctx.gwas_semiparallel(gin), t["chunk"])
    ctx.close()
