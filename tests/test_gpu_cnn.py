"""GPU encrypted CNN layers (slot packing, Eq. (enc_conv)) against the oracle
and the FP64 plaintext network."""
import numpy as np
import pytest

import workloads
from oracle import OracleCtx, cnn

pytestmark = pytest.mark.gpu

S_CONV, S_FC1, S_FC2 = 100000, 200000, 300000   # seed offsets of the weight ciphertexts


def _P():
    import paper_2102_00319_amd as P
    return P


def encrypt_images_gpu(g, pk, imgs, scale):
    """imgs [B][H][W] -> H*W ciphertexts, slot b of ciphertext (y, x) = imgs[b, y, x]."""
    B, H, W = imgs.shape
    return [g.encrypt(pk, g.encode(imgs[:, y, x], scale=scale), workloads.SEED_ENC + y * W + x)
            for y in range(H) for x in range(W)]


def test_small_cnn_bit_exact_and_logits():
    P = _P()
    g, o = P.Context.from_set("t_n12"), OracleCtx.from_set("t_n12")
    D = o.scale
    B, H, W, K, Cout, n1, n2 = o.N // 2, 6, 6, 3, 2, 3, 2
    Ho = Wo = 3
    imgs = workloads.images(workloads.SEED_DATA, B, H, W)
    cw = workloads.weights(workloads.SEED_DATA + 1, (Cout, 1, K, K))
    f1 = workloads.weights(workloads.SEED_DATA + 2, (n1, Cout * Ho * Wo))
    f2 = workloads.weights(workloads.SEED_DATA + 3, (n2, n1))
    s = g.keygen_secret(workloads.SEED_SECRET)
    so = s.astype(np.int64)
    pk, pko = g.keygen_pk(s, workloads.SEED_PK), o.keygen_pk(so, workloads.SEED_PK)
    rlk, rlko = g.keygen_relin(s, workloads.SEED_EVK), o.keygen_relin(so, workloads.SEED_EVK)
    L = o.L
    # client: images; model owner: weights (replicated constants) at the level each layer consumes
    X = encrypt_images_gpu(g, pk, imgs, D)
    Xo = [o.encrypt(pko, o.encode_rns(imgs[:, y, x], D, L), workloads.SEED_ENC + y * W + x, D)
          for y in range(H) for x in range(W)]
    for a, b in zip(X, Xo):
        assert np.array_equal(g.export_ct(a), b.data)
    Wc = g.encrypt_const_batch(pk, cw.ravel(), D, [workloads.SEED_ENC + S_CONV + t for t in range(cw.size)], L)
    W1 = g.encrypt_const_batch(pk, f1.ravel(), D, [workloads.SEED_ENC + S_FC1 + t for t in range(f1.size)], L - 2)
    W2 = g.encrypt_const_batch(pk, f2.ravel(), D, [workloads.SEED_ENC + S_FC2 + t for t in range(f2.size)], L - 4)
    Wco = [cnn.encrypt_const(o, pko, v, D, L, workloads.SEED_ENC + S_CONV + t) for t, v in enumerate(cw.ravel())]
    W1o = [cnn.encrypt_const(o, pko, v, D, L - 2, workloads.SEED_ENC + S_FC1 + t) for t, v in enumerate(f1.ravel())]
    W2o = [cnn.encrypt_const(o, pko, v, D, L - 4, workloads.SEED_ENC + S_FC2 + t) for t, v in enumerate(f2.ravel())]
    for a, b in zip(Wc + W1 + W2, Wco + W1o + W2o):
        assert np.array_equal(g.export_ct(a), b.data)
    g.op_counts()
    # cloud: conv -> x^2 -> fc1 -> x^2 -> fc2
    Y = g.conv2d_slot(rlk, X, H, W, 1, Wc, Cout, K, K, 2, 1, 1, Ho, Wo)
    A = g.square_act(rlk, Y)
    Z = g.fc_slot(rlk, A, W1, n1)
    A2 = g.square_act(rlk, Z)
    out = g.fc_slot(rlk, A2, W2, n2)
    ops = g.op_counts()
    cnt = cnn.Counter()
    Yo = cnn.enc_conv2d_slot(o, rlko, Xo, H, W, 1, Wco, Cout, K, K, 2, 1, 1, Ho, Wo, cnt)
    Ao = cnn.enc_square(o, rlko, Yo, cnt)
    Zo = cnn.enc_fc_slot(o, rlko, Ao, W1o, n1, cnt)
    A2o = cnn.enc_square(o, rlko, Zo, cnt)
    outo = cnn.enc_fc_slot(o, rlko, A2o, W2o, n2, cnt)
    for stage, (gg, oo) in enumerate([(Y, Yo), (A, Ao), (Z, Zo), (A2, A2o), (out, outo)]):
        for a, b in zip(gg, oo):
            assert np.array_equal(g.export_ct(a), b.data), "stage %d differs" % stage
            assert a.scale == b.scale
    assert (ops["ct_mult"], ops["ct_add"], ops["relin"], ops["rescale"]) == \
        (cnt.ct_mult, cnt.ct_add, cnt.relin, cnt.rescale)
    assert ops["ct_mult"] == cnn.conv_op_count(H, W, K, K, 2, 1, 1, Ho, Wo, 1, Cout) + 18 + 18 * 3 + 3 + 3 * 2
    # user: decrypt the scores and compare with the FP64 network
    ref = cnn.slot_cnn_fp64(imgs, cw, f1, f2, 2, 1, 1, Ho, Wo)
    for r in range(n2):
        got, _ = g.decode(g.decrypt(s, out[r]), n=B)
        assert np.abs(got - ref[:, r]).max() < 1e-3


def test_config2_cnn_logits_reduced_fc1():
    """Config 2 at full ring size and batch (N = 2^14, 8 limbs, 8192 images per
    ciphertext, conv 5x5 stride 2 x 5 channels = 845 outputs) with FC1 reduced to
    845 -> 10 so that the weight set stays small; one conv output is checked
    bit-exact against the oracle."""
    P = _P()
    g = P.Context.from_set("c2_n14")
    D = g.scale
    B, H, W, K, Cout = g.N // 2, 28, 28, 5, 5
    Ho = Wo = 13
    n1, n2 = 10, 10
    imgs = workloads.images(workloads.SEED_DATA, B, H, W)
    cw = workloads.weights(workloads.SEED_DATA + 1, (Cout, 1, K, K))
    f1 = workloads.weights(workloads.SEED_DATA + 2, (n1, Cout * Ho * Wo))
    f2 = workloads.weights(workloads.SEED_DATA + 3, (n2, n1))
    s = g.keygen_secret(workloads.SEED_SECRET)
    pk = g.keygen_pk(s, workloads.SEED_PK)
    rlk = g.keygen_relin(s, workloads.SEED_EVK)
    L = g.L
    X = encrypt_images_gpu(g, pk, imgs, D)
    Wc = g.encrypt_const_batch(pk, cw.ravel(), D, [workloads.SEED_ENC + S_CONV + t for t in range(cw.size)], L)
    W1 = g.encrypt_const_batch(pk, f1.ravel(), D, [workloads.SEED_ENC + S_FC1 + t for t in range(f1.size)], L - 2)
    W2 = g.encrypt_const_batch(pk, f2.ravel(), D, [workloads.SEED_ENC + S_FC2 + t for t in range(f2.size)], L - 4)
    g.op_counts()
    Y = g.conv2d_slot(rlk, X, H, W, 1, Wc, Cout, K, K, 2, 1, 1, Ho, Wo)
    out = g.fc_slot(rlk, g.square_act(rlk, g.fc_slot(rlk, g.square_act(rlk, Y), W1, n1)), W2, n2)
    ops = g.op_counts()
    assert ops["ct_mult"] == 20480 + 845 + 845 * n1 + n1 + n1 * n2
    assert ops["relin"] == ops["rescale"] == 845 + 845 + n1 + n1 + n2
    ref = cnn.slot_cnn_fp64(imgs, cw, f1, f2, 2, 1, 1, Ho, Wo)
    worst = 0.0
    for r in range(n2):
        got, _ = g.decode(g.decrypt(s, out[r]), n=B)
        worst = max(worst, float(np.abs(got - ref[:, r]).max()))
    print("config-2 logits: max |encrypted - FP64| = %.3e" % worst)
    assert worst < 1e-3
    # sampled output: Y[0] (channel 0, position (0, 0)) recomputed by the oracle from the same ciphertexts
    o = OracleCtx.from_set("c2_n14")
    so = s.astype(np.int64)
    rlko = o.keygen_relin(so, workloads.SEED_EVK)
    from oracle.ckks import Ct
    cnt = cnn.Counter()
    pairs = []
    for p in range(K):
        for q in range(K):
            y, x = p - 1, q - 1
            if 0 <= y < H and 0 <= x < W:
                pairs.append((Ct(g.export_ct(X[y * W + x]), D), Ct(g.export_ct(Wc[p * K + q]), D)))
    y0 = cnn._mac_relin_rescale(o, rlko, pairs, cnt)
    assert np.array_equal(g.export_ct(Y[0]), y0.data)


def test_config2_cnn_full_fc1_100(capsys):
    """Config 2 as configured: N = 2^14, 8 limbs, 8192 images per ciphertext, conv 5x5
    stride 2 x 5 channels, x^2, FC 845 -> 100 (84,500 weight ciphertexts, 124 GiB), x^2,
    FC 100 -> 10: the scores within 1e-3 of FP64; and the FC1 layer on the network's
    own activations bit-exact against the oracle for one output over its first 8
    inputs (the whole 845-input sum is out of the oracle's reach in test time)."""
    P = _P()
    g = P.Context.from_set("c2_n14")
    D = g.scale
    B, H, W, K, Cout = g.N // 2, 28, 28, 5, 5
    Ho = Wo = 13
    n1, n2 = 100, 10
    imgs = workloads.images(workloads.SEED_DATA, B, H, W)
    cw = workloads.weights(workloads.SEED_DATA + 1, (Cout, 1, K, K))
    f1 = workloads.weights(workloads.SEED_DATA + 2, (n1, Cout * Ho * Wo))
    f2 = workloads.weights(workloads.SEED_DATA + 3, (n2, n1))
    s = g.keygen_secret(workloads.SEED_SECRET)
    pk = g.keygen_pk(s, workloads.SEED_PK)
    rlk = g.keygen_relin(s, workloads.SEED_EVK)
    L = g.L
    X = P.CtArray(encrypt_images_gpu(g, pk, imgs, D))
    Wc = P.CtArray(g.encrypt_const_batch(pk, cw.ravel(), D, [workloads.SEED_ENC + S_CONV + t for t in range(cw.size)], L))
    W1 = P.CtArray(g.encrypt_const_batch(pk, f1.ravel(), D, [workloads.SEED_ENC + S_FC1 + t for t in range(f1.size)],
                                         L - 2))
    W2 = P.CtArray(g.encrypt_const_batch(pk, f2.ravel(), D, [workloads.SEED_ENC + S_FC2 + t for t in range(f2.size)],
                                         L - 4))
    Y = g.conv2d_slot(rlk, X, H, W, 1, Wc, Cout, K, K, 2, 1, 1, Ho, Wo)
    A = g.square_act(rlk, Y)
    Z = g.fc_slot(rlk, A, W1, n1)
    out = g.fc_slot(rlk, g.square_act(rlk, Z), W2, n2)
    ref = cnn.slot_cnn_fp64(imgs, cw, f1, f2, 2, 1, 1, Ho, Wo)
    worst = 0.0
    for r in range(n2):
        got, _ = g.decode(g.decrypt(s, out[r]), n=B)
        worst = max(worst, float(np.abs(got - ref[:, r]).max()))
    with capsys.disabled():
        print("config-2 (FC1 = 100) logits: max |encrypted - FP64| = %.3e" % worst, flush=True)
    assert worst < 1e-3
    # FC1 output 0 over the first 8 activations, on the GPU and on the oracle
    z8 = g.fc_slot(rlk, A[:8], [W1[i] for i in range(8)], 1)[0]
    o = OracleCtx.from_set("c2_n14")
    so = s.astype(np.int64)
    rlko = o.keygen_relin(so, workloads.SEED_EVK)
    from oracle.ckks import Ct
    pairs = [(Ct(g.export_ct(A[i]), A[i].scale), Ct(g.export_ct(W1[i]), D)) for i in range(8)]
    zo = cnn._mac_relin_rescale(o, rlko, pairs, cnn.Counter())
    assert np.array_equal(g.export_ct(z8), zo.data)
    assert z8.scale == zo.scale


@pytest.mark.parametrize("H,W,Cin,Cout,K,stride,pad", [(3, 4, 2, 9, 2, 1, 0), (6, 6, 1, 3, 3, 2, 1)])
def test_conv_tiles_bit_exact(H, W, Cin, Cout, K, stride, pad):
    """Conv shapes whose outputs fill the multiply-accumulate tiles in every way:
    runs of 8 channels and of 1, two neighbouring windows per tile, windows cut by
    padding (single-group tiles), several input channels per window."""
    P = _P()
    g, o = P.Context.from_set("t_n12"), OracleCtx.from_set("t_n12")
    D, L, B = o.scale, o.L, o.N // 2
    Ho, Wo = (H + pad - K) // stride + 1, (W + pad - K) // stride + 1
    imgs = workloads.images(workloads.SEED_DATA + 7, B, Cin * H, W)
    cw = workloads.weights(workloads.SEED_DATA + 8, (Cout, Cin, K, K))
    s = g.keygen_secret(workloads.SEED_SECRET)
    so = s.astype(np.int64)
    pk, pko = g.keygen_pk(s, workloads.SEED_PK), o.keygen_pk(so, workloads.SEED_PK)
    rlk, rlko = g.keygen_relin(s, workloads.SEED_EVK), o.keygen_relin(so, workloads.SEED_EVK)
    X = encrypt_images_gpu(g, pk, imgs, D)
    Xo = [o.encrypt(pko, o.encode_rns(imgs[:, y, x], D, L), workloads.SEED_ENC + y * W + x, D)
          for y in range(Cin * H) for x in range(W)]
    Wc = g.encrypt_const_batch(pk, cw.ravel(), D, [workloads.SEED_ENC + S_CONV + t for t in range(cw.size)], L)
    Wco = [cnn.encrypt_const(o, pko, v, D, L, workloads.SEED_ENC + S_CONV + t) for t, v in enumerate(cw.ravel())]
    Y = g.conv2d_slot(rlk, X, H, W, Cin, Wc, Cout, K, K, stride, pad, pad, Ho, Wo)
    Yo = cnn.enc_conv2d_slot(o, rlko, Xo, H, W, Cin, Wco, Cout, K, K, stride, pad, pad, Ho, Wo, cnn.Counter())
    assert len(Y) == len(Yo) == Cout * Ho * Wo
    for i, (a, b) in enumerate(zip(Y, Yo)):
        assert np.array_equal(g.export_ct(a), b.data), "output %d differs" % i
        assert a.scale == b.scale
