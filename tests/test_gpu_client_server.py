"""GPU test of the client / server split (paper: Introduction and Methods: the data owner encrypts X, y,
(X^T X)^-1 and S and decrypts the result; the server computes on ciphertexts only).

The client context runs keygen and the packing, and exports the switching keys and the input
ciphertexts.  An evaluating context that never held the secret imports them and runs the circuit; it
cannot decrypt, finalise or export a secret.  The client imports the numerators and denominators back
and finalises.  Every ciphertext and every result equals the single-context run bit for bit.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import paper_1902_04303_amd as P  # noqa: E402
from synth import config_seed, make_gwas_data  # noqa: E402

LOG_N, SCALE_BITS, KAPPA = 13, 30, 3
N_, K_, M_ = 245, 4, 70   # R = 256, 32 SNPs per ciphertext: 3 batches, the last ragged


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


def _export_batch(ctx, ct):
    cnt, depth, _, scale = ct.info()
    return [ctx.export(ct, i) for i in range(cnt)], depth, scale


def test_client_server_split_is_bit_identical(torch_dev):
    L = 7 * KAPPA + 5
    client = P.Context(LOG_N, L, SCALE_BITS)
    lay = client.gwas_layout(N_, K_, M_, KAPPA)
    galois = P.gwas_galois_elements(LOG_N, lay["R"])
    say("[gpu] client keygen, %d Galois keys" % len(galois))
    client.keygen(7, galois)
    assert client.has_secret()
    d = make_gwas_data(N_, K_, M_, seed=config_seed(1, 3))
    gin = client.gwas_pack_encrypt(d.X, d.y, d.S, KAPPA, 11)
    # the single-context run (client and server in one context) as the reference
    ref_out = client.gwas_semiparallel(gin)
    ref = client.gwas_finalize(ref_out)
    kinds = (P.GwasOutput.NUM, P.GwasOutput.DEN_EVEN, P.GwasOutput.DEN_ODD)
    ref_cts = {w: _export_batch(client, ref_out.ct(w, 0))[0] for w in kinds}

    # client -> server: switching keys and input ciphertexts in canonical form
    keys = {0: client.export_switching_key(0)}
    keys.update({g: client.export_switching_key(g) for g in galois})
    pk = client.export_public_key()
    x = [_export_batch(client, gin.ct(P.GwasInput.X, j)) for j in range(K_)]
    y = _export_batch(client, gin.ct(P.GwasInput.Y))
    A = [_export_batch(client, gin.ct(P.GwasInput.A, a)) for a in range(K_ * (K_ + 1) // 2)]
    S, s_depth, s_scale = _export_batch(client, gin.ct(P.GwasInput.S))
    assert len(S) == lay["n_batches"] == 3

    say("[gpu] server: imports keys and ciphertexts")
    server = P.Context(LOG_N, L, SCALE_BITS)
    assert not server.has_secret()
    for kid, kk in keys.items():
        server.import_switching_key(kid, kk)
    server.import_public_key(pk)
    for kid in (0, galois[0], galois[-1]):
        assert np.array_equal(server.export_switching_key(kid), keys[kid])
    assert np.array_equal(server.export_public_key(), pk)

    def imp(rec):
        cts, depth, scale = rec
        return server.import_ct(cts[0], depth, scale)

    sin = server.gwas_input_from_cts(N_, K_, M_, KAPPA, [imp(r) for r in x], imp(y), [imp(r) for r in A],
                                     [server.import_ct(c, s_depth, s_scale) for c in S])
    sout = server.gwas_semiparallel(sin)
    # the server holds no secret: no decryption, no finalisation, no secret to export
    for call in (lambda: server.gwas_finalize(sout), lambda: server.decrypt(sout.ct(P.GwasOutput.NUM, 0)),
                 lambda: server.export_secret()):
        with pytest.raises(P.CkksError) as e:
            call()
        assert e.value.code == -4

    say("[gpu] server -> client: numerators and denominators")
    back = {}
    for w in kinds:
        cts, depth, scale = _export_batch(server, sout.ct(w, 0))
        for i, c in enumerate(cts):
            assert np.array_equal(c, ref_cts[w][i]), (w, i)   # bit-identical to the single-context run
        back[w] = [client.import_ct(c, depth, scale) for c in cts]
    cout = client.gwas_output_from_cts(N_, K_, M_, back[kinds[0]], back[kinds[1]], back[kinds[2]])
    res = client.gwas_finalize(cout)
    for key in ("b", "se", "err", "num", "den"):
        assert np.array_equal(res[key], ref[key]), key
    server.close()
    client.close()


def test_key_import_checks_size_and_range(torch_dev):
    ctx = P.Context(10, 3, 30)
    src = P.Context(10, 3, 30)
    src.keygen(5, [src.galois_rotate(1)])
    key = src.export_switching_key(0)
    with pytest.raises(P.CkksError) as e:
        ctx.import_switching_key(0, key[:, :, :, :-1])          # wrong size
    assert e.value.code == -1
    bad = key.copy()
    bad[0, 0, 0, 0] = np.uint64(2 ** 63)                      # residue out of range
    with pytest.raises(P.CkksError) as e:
        ctx.import_switching_key(0, bad)
    assert e.value.code == -1
    with pytest.raises(P.CkksError) as e:
        ctx.import_switching_key(4, key)                        # not a Galois element (even)
    assert e.value.code == -1
    with pytest.raises(P.CkksError) as e:                      # no public key yet: cannot encrypt
        ctx.encrypt(np.zeros(ctx.N, dtype=np.int64), 0, 2.0 ** 30, 1)
    assert e.value.code == -4
    ctx.import_switching_key(0, key)
    assert np.array_equal(ctx.export_switching_key(0), key)
    ctx.close()
    src.close()
