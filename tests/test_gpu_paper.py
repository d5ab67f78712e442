"""The paper's network (Sec. 4.3: conv 3x3 x 28 without padding, ActPool with
g(u) = 0.47 + 0.50u + 0.09u^2, FC 4732 -> 10) on the GPU: bit-exact against the
oracle at N = 2^12, and at the paper's ring (N = 2^15, 16384 images) within 1e-3
of the FP64 network.  The full-size case reports every stage as it ends (past
pytest's output capture), so a long run is never silent."""
import math
import time

import numpy as np
import pytest

import workloads
from oracle import OracleCtx, cnn

pytestmark = pytest.mark.gpu


def test_paper_network_small_bit_exact():
    import paper_2102_00319_amd as P
    from paper_2102_00319_amd import networks
    g, o = P.Context.from_set("t_n12"), OracleCtx.from_set("t_n12")
    D, B = o.scale, o.N // 2
    imgs = workloads.images(workloads.SEED_DATA, B, 6, 6)
    wc = workloads.weights(workloads.SEED_DATA + 1, (2, 1, 3, 3))
    wfc = workloads.weights(workloads.SEED_DATA + 2, (2, 8))
    net = networks.PaperCNN(H=6, W=6, K=3, C=2, n_classes=2, band=1)
    sg = g.keygen_secret(workloads.SEED_SECRET)
    s = sg.astype(np.int64)
    pk, pko = g.keygen_pk(sg, workloads.SEED_PK), o.keygen_pk(s, workloads.SEED_PK)
    rlk, rlko = g.keygen_relin(sg, workloads.SEED_EVK), o.keygen_relin(s, workloads.SEED_EVK)
    X = net.encrypt_images(g, pk, imgs, workloads.SEED_ENC)
    Wc, Wf = net.encrypt_weights(g, pk, wc, wfc, (workloads.SEED_ENC + 100000, workloads.SEED_ENC + 200000))
    swc = D * math.sqrt(0.09 / 4.0)      # the conv weights' scale, computed here on its own
    Xo = [o.encrypt(pko, o.encode_rns(imgs[:, y, x], D, o.L), workloads.SEED_ENC + y * 6 + x, D)
          for y in range(6) for x in range(6)]
    Wco = [cnn.encrypt_const(o, pko, v, swc, o.L, workloads.SEED_ENC + 100000 + t) for t, v in enumerate(wc.ravel())]
    Wfo = [cnn.encrypt_const(o, pko, v, D, 2, workloads.SEED_ENC + 200000 + t) for t, v in enumerate(wfc.ravel())]
    for a, b in zip(list(X) + list(Wc) + list(Wf), Xo + Wco + Wfo):
        assert np.array_equal(g.export_ct(a), b.data)
        assert a.scale == b.scale
    stages, Zo = cnn.enc_paper_cnn(o, rlko, Xo, Wco, Wfo, 2, 3, 6, 6, 2, cnn.Counter())
    # stage by stage through the layer entry points
    Y = g.conv2d_slot(rlk, X, 6, 6, 1, Wc, 2, 3, 3, 1, 0, 0, 4, 4)
    A = g.poly_act(rlk, Y, net.coef4, 2)
    Pp = g.pool2x2_sum_slot(A, 2, 4, 4)
    for name, got in [("conv", Y), ("act", A), ("pool", Pp)]:
        for a, b in zip(got, stages[name]):
            assert np.array_equal(g.export_ct(a), b.data), name
            assert a.scale == b.scale, name
    # the banded forward pass gives the oracle's scores bit for bit
    g.op_counts()
    Z = net.forward(g, rlk, {}, X, (Wc, Wf))
    ops = g.op_counts()
    for a, b in zip(Z, Zo):
        assert np.array_equal(g.export_ct(a), b.data)
        assert a.scale == b.scale
    assert ops["ct_mult"] == net.op_counts()["ct_mult"] and ops["relin"] == net.op_counts()["relin"]
    ref = cnn.paper_cnn_fp64(imgs, wc, wfc)
    assert np.abs(net.decrypt_scores(g, sg, Z, B) - ref).max() < 1e-3


def test_paper_network_full_size(capsys):
    import torch
    import paper_2102_00319_amd as P
    from paper_2102_00319_amd import networks
    t0 = time.time()

    def say(msg):
        with capsys.disabled():
            print("[paper N=2^15 %6.1f s] %s" % (time.time() - t0, msg), flush=True)

    g = P.Context.from_set("p_n15")
    B = g.N // 2
    assert B == 16384
    imgs = workloads.images(workloads.SEED_DATA, B, 28, 28)
    wc = workloads.weights(workloads.SEED_DATA + 1, (28, 1, 3, 3))
    wfc = workloads.weights(workloads.SEED_DATA + 2, (10, 4732))
    net = networks.PaperCNN(band=2)
    sg = g.keygen_secret(workloads.SEED_SECRET)
    pk = g.keygen_pk(sg, workloads.SEED_PK)
    rlk, _ = net.keygen(g, sg, workloads.SEED_EVK)
    say("keys ready")
    X = net.encrypt_images(g, pk, imgs, workloads.SEED_ENC, progress=say)
    W = net.encrypt_weights(g, pk, wc, wfc, (workloads.SEED_ENC + 100000, workloads.SEED_ENC + 200000))
    torch.cuda.synchronize()
    say("weights encrypted: %d conv at %d limbs, %d FC at 2 limbs" % (len(W[0]), g.L, len(W[1])))
    torch.cuda.reset_peak_memory_stats()
    g.op_counts()
    t1 = time.time()
    Z = net.forward(g, rlk, {}, X, W, progress=say)
    torch.cuda.synchronize()
    t_fwd = time.time() - t1
    ops = g.op_counts()
    say("forward pass %.2f s; torch peak %.1f GiB, library scratch %.2f GiB" %
        (t_fwd, torch.cuda.max_memory_allocated() / 2 ** 30, g.scratch_bytes() / 2 ** 30))
    assert ops["ct_mult"] == net.op_counts()["ct_mult"] == 18928 * 9 + 18928 + 47320
    assert ops["relin"] == net.op_counts()["relin"]
    got = net.decrypt_scores(g, sg, Z, B)
    say("scores decrypted")
    ref = cnn.paper_cnn_fp64(imgs, wc, wfc)
    err = float(np.abs(got - ref).max())
    say("max |encrypted - FP64| = %.3e over %d images x 10 classes" % (err, B))
    assert err < 1e-3
