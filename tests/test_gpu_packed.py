"""GPU within-image packed CNN (rotation-sum convolutions, polynomial activation,
2x2 average pooling, rotate-and-sum FC) against the oracle and the FP64 network."""
import sys

import numpy as np
import pytest

import workloads
from oracle import OracleCtx, cnn
from oracle.ckks import Ct
from test_packed_oracle import COEF, FH, FW, G_PAPER, H, K, W, _setup, run_packed_oracle

pytestmark = pytest.mark.gpu

SEEDS = (workloads.SEED_ENC + 100000, workloads.SEED_ENC + 200000, workloads.SEED_ENC + 300000)


def _P():
    import paper_2102_00319_amd as P
    from paper_2102_00319_amd import networks
    return P, networks


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("coef,deg", [(COEF, 3), (G_PAPER, 2)])
def test_small_packed_network_bit_exact(coef, deg):
    """N = 2^12, 8 images of 12 x 12 in 16 x 16 frames: every stage's ciphertexts
    equal the oracle's, operation counts match, scores within 1e-3 of FP64; with the
    cubic activation and with the paper's quadratic g (depth 1, weights two levels higher)."""
    P, networks = _P()
    g, o = P.Context.from_set("t4_n12"), OracleCtx.from_set("t4_n12")
    c1, c2, ncls = 2, 3, 2
    B, imgs, w1, w2, wfc, s, pk_o = _setup(o, c1, c2, ncls)
    cnt = cnn.Counter()
    Zo, st, (Xo, W1o, W2o, Wfo) = run_packed_oracle(o, imgs, w1, w2, wfc, s, pk_o, coef, deg, cnt)
    _say("oracle network done (deg %d)" % deg)
    net = networks.PackedCNN(H=H, W=W, frame_h=FH, frame_w=FW, k=K, c1=c1, c2=c2, n_classes=ncls, coef=coef,
                             deg=deg)
    sg = g.keygen_secret(workloads.SEED_SECRET)
    assert np.array_equal(sg.astype(np.int64), s)
    pk = g.keygen_pk(sg, workloads.SEED_PK)
    rlk, gks = net.keygen(g, sg, workloads.SEED_EVK)
    X = net.encrypt_images(g, pk, imgs, workloads.SEED_ENC)
    W1, W2, Wf = net.encrypt_weights(g, pk, w1, w2, wfc, SEEDS)
    for a, b in zip(X + W1 + W2 + Wf, Xo + W1o + W2o + Wfo):
        assert np.array_equal(g.export_ct(a), b.data)
    g.op_counts()
    Y = g.conv2d_packed(rlk, gks, X, W1, c1, K, 1, FW)
    A = g.poly_act(rlk, Y, coef, deg)
    Pl = g.avgpool2x2(gks, A, 1, FW, net.pool_mask(g, 1, A[0].limbs))
    Y2 = g.conv2d_packed(rlk, gks, Pl, W2, c2, K, 2, FW)
    A2 = g.poly_act(rlk, Y2, coef, deg)
    P2 = g.avgpool2x2(gks, A2, 2, FW, net.pool_mask(g, 2, A2[0].limbs))
    Z = g.fc_packed(rlk, gks, P2, Wf, ncls, FH * FW)
    ops = g.op_counts()
    for name, got in [("conv1", Y), ("act1", A), ("pool1", Pl), ("conv2", Y2), ("act2", A2), ("pool2", P2),
                      ("fc", Z)]:
        for a, b in zip(got, st[name]):
            assert np.array_equal(g.export_ct(a), b.data), "stage %s differs" % name
            assert a.scale == b.scale, name
    assert (ops["ct_mult"], ops["relin"], ops["rotate"], ops["rescale"], ops["pt_mult"], ops["pt_add"],
            ops["ct_add"]) == (cnt.ct_mult, cnt.relin, cnt.rotate, cnt.rescale, cnt.pt_mult, cnt.pt_add, cnt.ct_add)
    assert (ops["ct_mult"], ops["relin"], ops["rotate"]) == net.op_counts()
    ref = cnn.packed_cnn_fp64(imgs, w1, w2, wfc, coef)
    got = net.decrypt_scores(g, sg, Z, B)
    assert np.abs(got - ref).max() < 1e-3
    # the composed forward pass, and the one-ciphertext-per-call form, give the same ciphertexts
    Z2 = net.forward(g, rlk, gks, X, (W1, W2, Wf))
    Z3 = net.forward_per_op(g, rlk, gks, X, (W1, W2, Wf))
    for a, b, c in zip(Z2, Z, Z3):
        assert np.array_equal(g.export_ct(a), g.export_ct(b))
        assert np.array_equal(g.export_ct(c), g.export_ct(b))
        assert c.scale == b.scale


@pytest.mark.parametrize("coef,deg", [((0.3, -0.2, 0.7), 2), ((-0.3, 0.2, 0.05), 2), ((0.0, 1.0, 0.0, 0.0), 3)])
def test_poly_act_forms_bit_exact(coef, deg):
    P, _ = _P()
    g, o = P.Context.from_set("t4_n12"), OracleCtx.from_set("t4_n12")
    n = o.N // 2
    sg = g.keygen_secret(workloads.SEED_SECRET)
    s = sg.astype(np.int64)
    pk, pko = g.keygen_pk(sg, workloads.SEED_PK), o.keygen_pk(s, workloads.SEED_PK)
    rlk, rlko = g.keygen_relin(sg, workloads.SEED_EVK), o.keygen_relin(s, workloads.SEED_EVK)
    xs, xo = [], []
    for i in range(3):
        m = workloads.slot_messages(20 + i, n)
        xs.append(g.encrypt(pk, g.encode(m, scale=g.scale, limbs=6), workloads.SEED_ENC + i))
        xo.append(o.encrypt(pko, o.encode_rns(m, o.scale, 6), workloads.SEED_ENC + i, o.scale))
    ys = g.poly_act(rlk, xs, coef, deg)
    yo = cnn.enc_poly_act(o, rlko, xo, coef, deg, cnn.Counter())
    for a, b in zip(ys, yo):
        assert a.limbs == (5 if deg == 2 else 4)
        assert np.array_equal(g.export_ct(a), b.data)
        assert a.scale == b.scale


def test_packed_layer_errors():
    P, networks = _P()
    g = P.Context.from_set("t4_n12")
    sg = g.keygen_secret(workloads.SEED_SECRET)
    pk = g.keygen_pk(sg, workloads.SEED_PK)
    rlk = g.keygen_relin(sg, workloads.SEED_EVK)
    x = g.encrypt(pk, g.encode(np.zeros(4), scale=g.scale), workloads.SEED_ENC)
    w = g.encrypt_const_batch(pk, np.ones(9), g.scale, list(range(9)), g.L)
    with pytest.raises(P.FheError):   # no Galois keys
        g.conv2d_packed(rlk, {}, [x], w, 1, 3, 1, FW)
    with pytest.raises(P.FheError):   # even kernel size
        g.conv2d_packed(rlk, {}, [x], w[:4], 1, 2, 1, FW)
    with pytest.raises(P.FheError):   # frame not a power of two
        g.fc_packed(rlk, {}, [x], [x], 1, 24)
    with pytest.raises(P.FheError):   # degree 4
        g.poly_act(rlk, [x], (0, 1, 0, 0, 1), 4)
    with pytest.raises(P.FheError):   # degree 2 with a quadratic coefficient that is not positive
        g.poly_act(rlk, [x], (0.1, 1.0, -0.5), 2)
    net = networks.PackedCNN(H=H, W=W, frame_h=FH, frame_w=FW, c1=1, c2=1, n_classes=1)
    with pytest.raises(P.FheError):   # mask at another level
        g.avgpool2x2({}, [x], 1, FW, net.pool_mask(g, 1, g.L - 1))


def test_config4_network_full_size():
    """The deep CNN at full size: N = 2^16, 24 limbs at scale 2^49, dnum 3; 32
    images of 28 x 28 in 32 x 32 frames; conv 3x3 x 8, cubic, pool, conv 3x3 x 16,
    cubic, pool, FC 784 -> 10.  Scores within 1e-3 of FP64, operation counts of the
    recipe, and sampled stages recomputed by the oracle from the GPU's ciphertexts."""
    P, networks = _P()
    g = P.Context.from_set("c4_n16")
    net = networks.PackedCNN()
    B = net.images_per_ct(g)
    assert B == 32
    imgs = workloads.images(workloads.SEED_DATA, B, 28, 28)
    w1 = workloads.weights(workloads.SEED_DATA + 1, (8, 1, 3, 3))
    w2 = workloads.weights(workloads.SEED_DATA + 2, (16, 8, 3, 3))
    wfc = workloads.weights(workloads.SEED_DATA + 3, (10, 784))
    sg = g.keygen_secret(workloads.SEED_SECRET)
    pk = g.keygen_pk(sg, workloads.SEED_PK)
    rlk, gks = net.keygen(g, sg, workloads.SEED_EVK)
    assert len(gks) == 22
    X = net.encrypt_images(g, pk, imgs, workloads.SEED_ENC)
    W1, W2, Wf = net.encrypt_weights(g, pk, w1, w2, wfc, SEEDS)
    _say("keys and weights ready")
    g.op_counts()
    Y = g.conv2d_packed(rlk, gks, X, W1, 8, 3, 1, 32)
    A = g.poly_act(rlk, Y, COEF, 3)
    Pl = g.avgpool2x2(gks, A, 1, 32, net.pool_mask(g, 1, A[0].limbs))
    Y2 = g.conv2d_packed(rlk, gks, Pl, W2, 16, 3, 2, 32)
    A2 = g.poly_act(rlk, Y2, COEF, 3)
    P2 = g.avgpool2x2(gks, A2, 2, 32, net.pool_mask(g, 2, A2[0].limbs))
    Z = g.fc_packed(rlk, gks, P2, Wf, 10, 1024)
    ops = g.op_counts()
    assert (ops["ct_mult"], ops["relin"], ops["rotate"]) == (1432, 82, 220) == net.op_counts()
    assert Z[0].limbs == 15
    ref = cnn.packed_cnn_fp64(imgs, w1, w2, wfc, COEF)
    got = net.decrypt_scores(g, sg, Z, B)
    err = float(np.abs(got - ref).max())
    _say("config-4 scores: max |encrypted - FP64| = %.3e" % err)
    assert err < 1e-3
    # sampled: pool of channel 0 (two rotations, mask product, rescale) from the GPU's input
    o = OracleCtx.from_set("c4_n16")
    s = sg.astype(np.int64)
    steps = net.rotation_steps()
    gko = {r: o.keygen_rot(s, r, workloads.SEED_EVK + 1 + steps.index(r)) for r in (1, 32)}
    l = A[0].limbs
    mask = cnn.pool_mask(o, 28, 28, 32, 32, 1, float(o.q[l - 1]), l)
    a0 = Ct(g.export_ct(A[0]), A[0].scale)
    (p0,) = cnn.enc_avgpool2x2(o, gko, [a0], 1, 32, mask, float(o.q[l - 1]), cnn.Counter())
    assert np.array_equal(g.export_ct(Pl[0]), p0.data)
    assert Pl[0].scale == p0.scale
    _say("sampled pool stage bit-exact")


def test_small_plain_model_bit_exact():
    """The within-image network with the model in the clear: the scores ciphertexts
    equal the oracle's and decrypt to the FP64 network within 1e-3."""
    from test_packed_oracle import run_packed_oracle_plain
    P, networks = _P()
    g, o = P.Context.from_set("t4_n12"), OracleCtx.from_set("t4_n12")
    c1, c2, ncls = 2, 3, 2
    B, imgs, w1, w2, wfc, s, _ = _setup(o, c1, c2, ncls)
    cnt = cnn.Counter()
    Zo, st = run_packed_oracle_plain(o, imgs, w1, w2, wfc, s, COEF, cnt)
    _say("oracle plain-model network done")
    net = networks.PackedCNN(H=H, W=W, frame_h=FH, frame_w=FW, k=K, c1=c1, c2=c2, n_classes=ncls, coef=COEF)
    sg = g.keygen_secret(workloads.SEED_SECRET)
    pk = g.keygen_pk(sg, workloads.SEED_PK)
    rlk, gks = net.keygen(g, sg, workloads.SEED_EVK)
    X = net.encrypt_images(g, pk, imgs, workloads.SEED_ENC)
    Wpt = net.plain_fc_weights(g, wfc, g.L - 8)
    g.op_counts()
    Y = g.conv2d_packed_pw(gks, X, w1, c1, K, 1, FW, float(g.q[g.L - 1]))
    A = g.poly_act(rlk, Y, COEF, 3)
    Pl = g.avgpool2x2(gks, A, 1, FW, net.pool_mask(g, 1, A[0].limbs))
    Y2 = g.conv2d_packed_pw(gks, Pl, w2, c2, K, 2, FW, float(g.q[Pl[0].limbs - 1]))
    A2 = g.poly_act(rlk, Y2, COEF, 3)
    P2 = g.avgpool2x2(gks, A2, 2, FW, net.pool_mask(g, 2, A2[0].limbs))
    Z = g.fc_packed_pw(gks, P2, Wpt, ncls, FH * FW)
    ops = g.op_counts()
    for name, got in [("conv1", Y), ("act1", A), ("pool1", Pl), ("conv2", Y2), ("act2", A2), ("pool2", P2),
                      ("fc", Z)]:
        for a, b in zip(got, st[name]):
            assert np.array_equal(g.export_ct(a), b.data), "stage %s differs" % name
            assert a.scale == b.scale, name
    assert (ops["relin"], ops["rotate"]) == (cnt.relin, cnt.rotate)
    # the composed forward pass gives the same ciphertexts
    for a, b in zip(net.forward_plain(g, rlk, gks, X, w1, w2, Wpt), Z):
        assert np.array_equal(g.export_ct(a), g.export_ct(b))
    ref = cnn.packed_cnn_fp64(imgs, w1, w2, wfc, COEF)
    assert np.abs(net.decrypt_scores(g, sg, Z, B) - ref).max() < 1e-3
