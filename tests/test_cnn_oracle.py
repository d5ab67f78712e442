"""CPU checks of the CNN layer definitions used by the encrypted recipes:
the op-count formula of the paper and the FP64 network shape arithmetic."""
import math

import numpy as np

import workloads
from oracle import OracleCtx, cnn


def test_conv_count_matches_paper_formula_without_padding():
    # Sec. 3: (M-P+1)(N-Q+1)PQ CT-CT mults for an M x N image and P x Q kernel, stride 1, no padding
    for (M, N, P, Q) in [(28, 28, 3, 3), (8, 6, 2, 3), (5, 5, 5, 5)]:
        Ho, Wo = M - P + 1, N - Q + 1
        assert cnn.conv_op_count(M, N, P, Q, 1, 0, 0, Ho, Wo, 1, 1) == (M - P + 1) * (N - Q + 1) * P * Q


def test_paper_network_shapes():
    # Sec. 4.3: 28x28 input, 3x3 conv without padding -> 26x26, 2x2 mean pool -> 13x13, 28 filters
    assert 28 - 3 + 1 == 26 and 26 // 2 == 13 and 13 * 13 * 28 == 4732
    # Table 1 / Sec. 4.3: one filter's conv is 26*26*9 = 6084 CT-CT mults
    assert cnn.conv_op_count(28, 28, 3, 3, 1, 0, 0, 26, 26, 1, 1) == 6084


def test_config2_conv_counts():
    # 28x28, 5x5 stride 2, pad top/left 1 -> 13x13 x 5 channels = 845 outputs
    H = W = 28
    Ho = Wo = (H + 1 - 5) // 2 + 1
    assert Ho == 13 and 13 * 13 * 5 == 845
    n = cnn.conv_op_count(H, W, 5, 5, 2, 1, 1, Ho, Wo, 1, 5)
    assert n == 20480   # in-bounds taps only


def test_fp64_forward_matches_direct_sum():
    rs = np.random.default_rng(0)
    x = rs.uniform(0, 1, (3, 6, 6))
    w = rs.normal(0, 0.1, (2, 1, 3, 3))
    f1 = rs.normal(0, 0.1, (3, 18))
    f2 = rs.normal(0, 0.1, (2, 3))
    out = cnn.slot_cnn_fp64(x, w, f1, f2, 2, 1, 1, 3, 3)
    # independent evaluation by explicit zero padding and slicing
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)))
    conv = np.zeros((3, 2, 3, 3))
    for co in range(2):
        for i in range(3):
            for j in range(3):
                conv[:, co, i, j] = (xp[:, 2 * i:2 * i + 3, 2 * j:2 * j + 3] * w[co, 0]).sum(axis=(1, 2))
    h = (conv ** 2).reshape(3, -1)
    ref = ((h @ f1.T) ** 2) @ f2.T
    assert np.allclose(out, ref, rtol=1e-12, atol=1e-14)


def test_paper_network_on_oracle():
    """The paper's network (Sec. 4.3) shrunk to N = 2^12: 6x6 images, conv 3x3 x 2
    filters without padding, ActPool with g/4 folded, FC 8 -> 2; scores within 1e-3
    of the FP64 network with the exact 2x2 mean of g."""
    o = OracleCtx.from_set("t_n12")
    D, B = o.scale, o.N // 2
    imgs = workloads.images(workloads.SEED_DATA, B, 6, 6)
    wc = workloads.weights(workloads.SEED_DATA + 1, (2, 1, 3, 3))
    wfc = workloads.weights(workloads.SEED_DATA + 2, (2, 8))
    s = o.keygen_secret(workloads.SEED_SECRET)
    pk = o.keygen_pk(s, workloads.SEED_PK)
    rlk = o.keygen_relin(s, workloads.SEED_EVK)
    X = [o.encrypt(pk, o.encode_rns(imgs[:, y, x], D, o.L), workloads.SEED_ENC + y * 6 + x, D)
         for y in range(6) for x in range(6)]
    # conv weights at D sqrt(c2 / 4): the depth-1 activation's output scale (S^2 / c2 per
    # rescale) then returns to about D, leaving the scores room below q0
    swc = D * math.sqrt(0.09 / 4.0)
    Wc = [cnn.encrypt_const(o, pk, v, swc, o.L, workloads.SEED_ENC + 100000 + t) for t, v in enumerate(wc.ravel())]
    Wf = [cnn.encrypt_const(o, pk, v, D, 2, workloads.SEED_ENC + 200000 + t) for t, v in enumerate(wfc.ravel())]
    cnt = cnn.Counter()
    _, Z = cnn.enc_paper_cnn(o, rlk, X, Wc, Wf, 2, 3, 6, 6, 2, cnt)
    assert abs(math.log2(Z[0].scale) - math.log2(D)) < 1.0
    ref = cnn.paper_cnn_fp64(imgs, wc, wfc)
    for r in range(2):
        re, _ = o.decode(o.decrypt(Z[r], s), Z[r].scale, n=B)
        assert np.abs(re - ref[:, r]).max() < 1e-3
    assert cnt.ct_mult == 2 * 4 * 4 * 9 + 2 * 4 * 4 + 8 * 2
    assert cnt.relin == 2 * 16 + 2 * 16 + 2   # conv outputs, one product each in g, FC outputs


def test_slot_cnn_on_oracle():
    """The slot CNN's recipe (conv with stride 2 and padding 1 on top and left,
    padded taps skipped; x^2; FC; x^2; FC) shrunk to N = 2^12 with 6x6 images, two
    filters, FC 18 -> 3 -> 2: scores within 1e-3 of the FP64 network, and the
    operation counts of the recipe (one product per in-bounds tap and input,
    one relinearisation and one rescale per output)."""
    o = OracleCtx.from_set("t_n12")
    D, B = o.scale, o.N // 2
    H = W = 6
    C, K, S = 2, 3, 2
    Ho = Wo = (H + 1 - K) // S + 1
    imgs = workloads.images(workloads.SEED_DATA, B, H, W)
    wc = workloads.weights(workloads.SEED_DATA + 1, (C, 1, K, K))
    f1 = workloads.weights(workloads.SEED_DATA + 2, (3, C * Ho * Wo))
    f2 = workloads.weights(workloads.SEED_DATA + 3, (2, 3))
    s = o.keygen_secret(workloads.SEED_SECRET)
    pk = o.keygen_pk(s, workloads.SEED_PK)
    rlk = o.keygen_relin(s, workloads.SEED_EVK)
    L = o.L
    X = [o.encrypt(pk, o.encode_rns(imgs[:, y, x], D, L), workloads.SEED_ENC + y * W + x, D)
         for y in range(H) for x in range(W)]
    Wc = [cnn.encrypt_const(o, pk, v, D, L, workloads.SEED_ENC + 100 + t) for t, v in enumerate(wc.ravel())]
    W1 = [cnn.encrypt_const(o, pk, v, D, L - 2, workloads.SEED_ENC + 200 + t) for t, v in enumerate(f1.ravel())]
    W2 = [cnn.encrypt_const(o, pk, v, D, L - 4, workloads.SEED_ENC + 300 + t) for t, v in enumerate(f2.ravel())]
    cnt = cnn.Counter()
    Y = cnn.enc_conv2d_slot(o, rlk, X, H, W, 1, Wc, C, K, K, S, 1, 1, Ho, Wo, cnt)
    A = cnn.enc_square(o, rlk, Y, cnt)
    Z = cnn.enc_fc_slot(o, rlk, A, W1, 3, cnt)
    A2 = cnn.enc_square(o, rlk, Z, cnt)
    out = cnn.enc_fc_slot(o, rlk, A2, W2, 2, cnt)
    ref = cnn.slot_cnn_fp64(imgs, wc, f1, f2, S, 1, 1, Ho, Wo)
    for r in range(2):
        assert out[r].level == L - 5
        re, _ = o.decode(o.decrypt(out[r], s), out[r].scale, n=B)
        assert np.abs(re - ref[:, r]).max() < 1e-3
    taps = cnn.conv_op_count(H, W, K, K, S, 1, 1, Ho, Wo, 1, C)
    assert cnt.ct_mult == taps + C * Ho * Wo + 3 * C * Ho * Wo + 3 + 2 * 3
    assert cnt.relin == cnt.rescale == C * Ho * Wo * 2 + 3 * 2 + 2
