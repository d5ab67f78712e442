"""The paper's printed values (tests/golden/paper_printed_values.json, each with
its passage) against the code's parameter sets, network definition, operation
counts and level use."""
import json
import os

import workloads
from oracle import cnn

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_printed_values.json")))


def test_ring_of_the_paper_network():
    r = GOLD["ring"]
    s = workloads.load_params("p_n15")
    N = 1 << s["log_n"]
    assert r["phi_m"] == r["m"] // 2 == N          # power-of-two m: phi(m) = m/2 = ring degree
    assert r["slots"] == N // 2


def test_network_definition():
    from paper_2102_00319_amd.networks import PaperCNN
    n, g = PaperCNN(), GOLD["network"]
    assert (n.H, n.W) == tuple(g["image"]) and n.C == g["filters"] and (n.K, n.K) == tuple(g["kernel"])
    assert (n.Ho, n.Wo) == (g["image"][0] - g["kernel"][0] + 1, g["image"][1] - g["kernel"][1] + 1)  # no padding
    assert n.n_in_fc == g["flatten"] == g["fc"][0] and n.n_classes == g["fc"][1]
    assert tuple(n.coef) == tuple(GOLD["activation"]["coefficients"])


def test_conv_count_formula():
    f = GOLD["conv_count"]["formula_inputs"]
    M, N, P, Q = f["M"], f["N"], f["P"], f["Q"]
    assert cnn.conv_op_count(M, N, P, Q, 1, 0, 0, M - P + 1, N - Q + 1, 1, 1) == (M - P + 1) * (N - Q + 1) * P * Q


def test_depth_of_conv_and_activation():
    """Levels the oracle's recipe consumes: one for the conv and one for the quadratic
    activation, as the paper states: one 3x3 window and one filter at N = 2^12."""
    import numpy as np
    from oracle import OracleCtx
    o = OracleCtx.from_set("t_n12")
    D, L = o.scale, o.L
    s = o.keygen_secret(workloads.SEED_SECRET)
    pk, rlk = o.keygen_pk(s, workloads.SEED_PK), o.keygen_relin(s, workloads.SEED_EVK)
    img = workloads.images(workloads.SEED_DATA, 4, 3, 3)
    X = [o.encrypt(pk, o.encode_rns(img[:, y, x], D, L), workloads.SEED_ENC + 3 * y + x, D)
         for y in range(3) for x in range(3)]
    Wc = [cnn.encrypt_const(o, pk, v, D, L, workloads.SEED_ENC + 100 + t)
          for t, v in enumerate(np.full(9, 0.1))]
    Y = cnn.enc_conv2d_slot(o, rlk, X, 3, 3, 1, Wc, 1, 3, 3, 1, 0, 0, 1, 1, cnn.Counter())
    A = cnn.enc_poly_act(o, rlk, Y, GOLD["activation"]["coefficients"], 2, cnn.Counter())
    d = GOLD["depth"]
    assert Y[0].data.shape[1] == L - d["conv"]
    assert A[0].data.shape[1] == L - d["conv"] - d["activation"]
