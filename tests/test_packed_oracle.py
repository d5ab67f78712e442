"""Within-image packed CNN on the CPU oracle: the FP64 network's building blocks
against library routines, the encrypted recipes against the FP64 network, the
activation polynomial's special cases, and the slot layouts of the two
codebases against each other."""
import numpy as np
import pytest
import scipy.signal

import workloads
from oracle import OracleCtx, cnn

FH = FW = 16
H = W = 12
K = 3
COEF = (0.47, 0.5, 0.09, -0.005)
G_PAPER = (0.47, 0.50, 0.09)   # g of Eq. (approxReLU)


def test_fp64_blocks_against_library_routines():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((3, 2, 8, 8))
    w = rng.standard_normal((4, 2, 3, 3))
    got = cnn.conv2d_same_fp64(x, w)
    for b in range(3):
        for co in range(4):
            ref = sum(scipy.signal.correlate2d(x[b, ci], w[co, ci], mode="same") for ci in range(2))
            assert np.allclose(got[b, co], ref, atol=1e-12)
    p = cnn.avgpool2_fp64(x)
    for i in range(4):
        for j in range(4):
            assert np.allclose(p[:, :, i, j], x[:, :, 2 * i:2 * i + 2, 2 * j:2 * j + 2].mean(axis=(2, 3)))
    assert np.allclose(cnn.poly_fp64(x, COEF), np.polyval(COEF[::-1], x))


def test_frame_layout():
    imgs = np.arange(2 * 3 * 3, dtype=np.float64).reshape(2, 3, 3) + 1
    v = cnn.frame_pack(imgs, 4, 4)
    assert v.shape == (32,)
    assert v[16 + 1 * 4 + 2] == imgs[1, 1, 2]
    assert np.count_nonzero(v) == 18
    # a left rotation by dy*frame_w + dx brings pixel (y+dy, x+dx) to (y, x); the guard gives zeros
    r = np.roll(v, -(1 * 4 + 1))
    assert r[0] == imgs[0, 1, 1] and r[2] == 0.0 and r[16 + 1 * 4 + 1] == imgs[1, 2, 2]


def _setup(o, c1, c2, ncls):
    B = (o.N // 2) // (FH * FW)
    imgs = workloads.images(workloads.SEED_DATA, B, H, W)
    w1 = workloads.weights(workloads.SEED_DATA + 1, (c1, 1, K, K))
    w2 = workloads.weights(workloads.SEED_DATA + 2, (c2, c1, K, K))
    wfc = workloads.weights(workloads.SEED_DATA + 3, (ncls, c2 * (H // 4) * (W // 4)))
    s = o.keygen_secret(workloads.SEED_SECRET)
    pk = o.keygen_pk(s, workloads.SEED_PK)
    return B, imgs, w1, w2, wfc, s, pk


def run_packed_oracle(o, imgs, w1, w2, wfc, s, pk, coef, deg, cnt):
    """The whole packed network on the oracle; returns the logits ciphertexts and every stage."""
    D = o.scale
    B = imgs.shape[0]
    c1, c2, ncls = w1.shape[0], w2.shape[0], wfc.shape[0]
    rlk = o.keygen_relin(s, workloads.SEED_EVK)
    steps = cnn.packed_rotation_steps(K, FW, FH * FW)
    gks = {r: o.keygen_rot(s, r, workloads.SEED_EVK + 1 + i) for i, r in enumerate(steps)}
    L = o.L
    d = (2 if deg == 3 else 1) + 2   # levels of one conv, activation and pool
    X = [o.encrypt(pk, o.encode_rns(cnn.frame_pack(imgs, FH, FW), D, L), workloads.SEED_ENC, D)]
    W1 = [cnn.encrypt_const(o, pk, v, D, L, workloads.SEED_ENC + 100000 + t) for t, v in enumerate(w1.ravel())]
    W2 = [cnn.encrypt_const(o, pk, v, D, L - d, workloads.SEED_ENC + 200000 + t) for t, v in enumerate(w2.ravel())]
    hp = H // 4
    Wf = []
    for r in range(ncls):
        rows = wfc[r].reshape(c2, hp * hp)
        for c in range(c2):
            v = cnn.fc_weight_slots(rows[c], hp, hp, FH, FW, B, 4)
            Wf.append(o.encrypt(pk, o.encode_rns(v, D, L - 2 * d), workloads.SEED_ENC + 300000 + r * c2 + c, D))
    stages = {}
    Y = cnn.enc_conv2d_packed(o, rlk, gks, X, 1, W1, c1, K, 1, FW, cnt)
    A = cnn.enc_poly_act(o, rlk, Y, coef, deg, cnt)
    l = A[0].level
    P = cnn.enc_avgpool2x2(o, gks, A, 1, FW, cnn.pool_mask(o, H, W, FH, FW, 1, float(o.q[l - 1]), l),
                           float(o.q[l - 1]), cnt)
    stages.update(conv1=Y, act1=A, pool1=P)
    Y = cnn.enc_conv2d_packed(o, rlk, gks, P, c1, W2, c2, K, 2, FW, cnt)
    A = cnn.enc_poly_act(o, rlk, Y, coef, deg, cnt)
    l = A[0].level
    P = cnn.enc_avgpool2x2(o, gks, A, 2, FW, cnn.pool_mask(o, H, W, FH, FW, 2, float(o.q[l - 1]), l),
                           float(o.q[l - 1]), cnt)
    stages.update(conv2=Y, act2=A, pool2=P)
    Z = cnn.enc_fc_packed(o, rlk, gks, P, Wf, ncls, FH * FW, cnt)
    stages["fc"] = Z
    return Z, stages, (X, W1, W2, Wf)


@pytest.mark.parametrize("coef,deg", [(COEF, 3), (G_PAPER, 2)])
def test_packed_network_logits_and_counts(coef, deg):
    """Small within-image network (N = 2^12, 8 images of 12 x 12 in 16 x 16 frames,
    2 and 3 channels, 2 classes, 11 limbs at scale 2^49): decrypted scores equal the
    FP64 network to 1e-3, and the operation counts follow the recipe; with the
    paper's quadratic g each activation takes one level instead of two."""
    o = OracleCtx.from_set("t4_n12")
    c1, c2, ncls = 2, 3, 2
    B, imgs, w1, w2, wfc, s, pk = _setup(o, c1, c2, ncls)
    cnt = cnn.Counter()
    Z, _, _ = run_packed_oracle(o, imgs, w1, w2, wfc, s, pk, coef, deg, cnt)
    assert Z[0].level == o.L - (9 if deg == 3 else 7)
    ref = cnn.packed_cnn_fp64(imgs, w1, w2, wfc, coef)
    F = FH * FW
    for r in range(ncls):
        re, _ = o.decode(o.decrypt(Z[r], s), Z[r].scale)
        assert np.abs(re[np.arange(B) * F] - ref[:, r]).max() < 1e-3
    kk = K * K
    act = 2 if deg == 3 else 1
    assert cnt.ct_mult == c1 * kk + c2 * c1 * kk + act * (c1 + c2) + ncls * c2
    assert cnt.relin == c1 + c2 + act * (c1 + c2) + ncls
    assert cnt.rotate == (kk - 1) * (1 + c1) + 2 * (c1 + c2) + ncls * 8


@pytest.mark.parametrize("coef,deg", [((0.0, 1.0, 0.0, 0.0), 3), ((0.3, -0.2, 0.7, 0.0), 3), ((0.3, -0.2, 0.7), 2),
                                      ((-0.3, 0.2, 0.05), 2)])
def test_poly_act_special_cases(coef, deg):
    """(0, 1, 0, 0) is the identity up to noise; a zero cubic term reduces to the
    quadratic, and the degree-2 form agrees with it (its constant term is an integer
    near 2^79, or a negative one near 2^82 for the last case)."""
    o = OracleCtx.from_set("t4_n12")
    n = o.N // 2
    s = o.keygen_secret(workloads.SEED_SECRET)
    pk = o.keygen_pk(s, workloads.SEED_PK)
    rlk = o.keygen_relin(s, workloads.SEED_EVK)
    m = workloads.slot_messages(11, n)
    x = o.encrypt(pk, o.encode_rns(m, o.scale, 5), workloads.SEED_ENC, o.scale)
    cnt = cnn.Counter()
    (y,) = cnn.enc_poly_act(o, rlk, [x], coef, deg, cnt)
    assert y.level == (4 if deg == 2 else 3)
    re, _ = o.decode(o.decrypt(y, s), y.scale)
    assert np.abs(re - cnn.poly_fp64(m, coef)).max() < 1e-6
    assert cnt.relin == (2 if deg == 3 else 1)


def test_layouts_of_both_codebases_agree():
    """The library's client-side layouts (frame packing, pool masks, FC weight
    slots) against the oracle's, written separately."""
    from paper_2102_00319_amd import networks
    o = OracleCtx.from_set("t4_n12")
    net = networks.PackedCNN(H=H, W=W, frame_h=FH, frame_w=FW, c1=2, c2=3, n_classes=2)

    class _N:
        N = o.N
    B = (o.N // 2) // (FH * FW)
    imgs = workloads.images(workloads.SEED_DATA, B, H, W)
    assert np.array_equal(networks.frame_pack(imgs, FH, FW), cnn.frame_pack(imgs, FH, FW))
    wrow = np.arange(9, dtype=np.float64) + 1
    assert np.array_equal(net.fc_slots(_N, wrow), cnn.fc_weight_slots(wrow, 3, 3, FH, FW, B, 4))
    for dil in (1, 2):
        a = np.sort(networks.grid_slots(H, W, FH, FW, B, 2 * dil))
        b = np.sort(cnn.frame_positions(H, W, FH, FW, B, 2 * dil))
        assert np.array_equal(a, b)
    assert net.rotation_steps() == cnn.packed_rotation_steps(K, FW, FH * FW)


def run_packed_oracle_plain(o, imgs, w1, w2, wfc, s, coef, cnt):
    """The within-image network with the model in the clear (constants and
    plaintext FC weights); returns the scores ciphertexts and every stage."""
    D = o.scale
    B = imgs.shape[0]
    c1, c2, ncls = w1.shape[0], w2.shape[0], wfc.shape[0]
    pk = o.keygen_pk(s, workloads.SEED_PK)
    rlk = o.keygen_relin(s, workloads.SEED_EVK)
    steps = cnn.packed_rotation_steps(K, FW, FH * FW)
    gks = {r: o.keygen_rot(s, r, workloads.SEED_EVK + 1 + i) for i, r in enumerate(steps)}
    L = o.L
    X = [o.encrypt(pk, o.encode_rns(cnn.frame_pack(imgs, FH, FW), D, L), workloads.SEED_ENC, D)]
    st = {}
    Y = cnn.enc_conv2d_packed_pw(o, gks, X, 1, w1, c1, K, 1, FW, float(o.q[L - 1]), cnt)
    A = cnn.enc_poly_act(o, rlk, Y, coef, 3, cnt)
    l = A[0].level
    P = cnn.enc_avgpool2x2(o, gks, A, 1, FW, cnn.pool_mask(o, H, W, FH, FW, 1, float(o.q[l - 1]), l),
                           float(o.q[l - 1]), cnt)
    st.update(conv1=Y, act1=A, pool1=P)
    l = P[0].level
    Y = cnn.enc_conv2d_packed_pw(o, gks, P, c1, w2, c2, K, 2, FW, float(o.q[l - 1]), cnt)
    A = cnn.enc_poly_act(o, rlk, Y, coef, 3, cnt)
    l = A[0].level
    P = cnn.enc_avgpool2x2(o, gks, A, 2, FW, cnn.pool_mask(o, H, W, FH, FW, 2, float(o.q[l - 1]), l),
                           float(o.q[l - 1]), cnt)
    st.update(conv2=Y, act2=A, pool2=P)
    l = P[0].level
    hp = H // 4
    sc = float(o.q[l - 1])
    Wpt = []
    for r in range(ncls):
        rows = wfc[r].reshape(c2, hp * hp)
        for c in range(c2):
            Wpt.append(o.encode_rns(cnn.fc_weight_slots(rows[c], hp, hp, FH, FW, B, 4), sc, l))
    Z = cnn.enc_fc_packed_pw(o, gks, P, Wpt, sc, ncls, FH * FW, cnt)
    st["fc"] = Z
    return Z, st


def test_packed_network_plain_model():
    """The same network with an unencrypted model (constant conv taps, plaintext
    FC weights): scores within 1e-3 of FP64, relinearisations only in the activations."""
    o = OracleCtx.from_set("t4_n12")
    c1, c2, ncls = 2, 3, 2
    B, imgs, w1, w2, wfc, s, _ = _setup(o, c1, c2, ncls)
    cnt = cnn.Counter()
    Z, _ = run_packed_oracle_plain(o, imgs, w1, w2, wfc, s, COEF, cnt)
    ref = cnn.packed_cnn_fp64(imgs, w1, w2, wfc, COEF)
    for r in range(ncls):
        re, _ = o.decode(o.decrypt(Z[r], s), Z[r].scale)
        assert np.abs(re[np.arange(B) * FH * FW] - ref[:, r]).max() < 1e-3
    assert cnt.relin == 2 * (c1 + c2) and cnt.ct_mult == 2 * (c1 + c2)
    assert cnt.rotate == (K * K - 1) * (1 + c1) + 2 * (c1 + c2) + ncls * 8


def test_strided_padded_conv_against_scipy():
    """The FP64 convolution with stride and one-sided padding against scipy's
    correlate2d of the zero-padded image, sampled at the strided positions."""
    rng = np.random.default_rng(6)
    x = rng.standard_normal((2, 2, 9, 7))
    w = rng.standard_normal((3, 2, 3, 3))
    for stride, pt, pl in [(1, 0, 0), (2, 1, 1), (2, 0, 1), (3, 2, 0)]:
        Ho = (9 + pt - 3) // stride + 1
        Wo = (7 + pl - 3) // stride + 1
        got = cnn.conv2d_fp64(x, w, stride, pt, pl, Ho, Wo)
        for b in range(2):
            for co in range(3):
                ref = 0.0
                for ci in range(2):
                    xp = np.pad(x[b, ci], ((pt, 3), (pl, 3)))
                    full = scipy.signal.correlate2d(xp, w[co, ci], mode="valid")
                    ref = ref + full[::stride, ::stride][:Ho, :Wo]
                assert np.allclose(got[b, co], ref, atol=1e-12)
