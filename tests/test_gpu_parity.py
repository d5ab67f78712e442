"""GPU parity: every library operation, called through the C ABI, against the
CPU oracle on the same seeded inputs.  Integer results must be bit-exact
(canonical coefficient-domain residues); decoded slots are compared in FP64.

Sizes: N = 2^12 (one NTT pass), 2^14 (one pass, 1024-thread groups), 2^15 and
2^16 (column + row passes); levels include ragged last key-switching digits
and the one-limb floor of rescale."""
import numpy as np
import pytest

import workloads
from oracle import OracleCtx, ckks

pytestmark = pytest.mark.gpu


def _fhe():
    import paper_2102_00319_amd as P
    return P


@pytest.fixture(scope="module")
def sets():
    cache = {}

    def get(name):
        if name not in cache:
            P = _fhe()
            cache[name] = (P.Context.from_set(name), OracleCtx.from_set(name))
        return cache[name]
    return get


def rand_ct(o, l, polys, seed):
    return workloads.uniform_residues(seed, o.q[:l] * polys, o.N).reshape(polys, l, o.N)


def eq(a, b):
    a, b = np.asarray(a, dtype=np.uint64), np.asarray(b, dtype=np.uint64)
    assert a.shape == b.shape
    bad = np.argwhere(a != b)
    assert bad.size == 0, "mismatch at %s (of %d)" % (bad[:5].tolist(), len(bad))


# ------------------------------------------------------------------ NTT
@pytest.mark.parametrize("name", ["c1_n12", "c2_n14", "c3_n15", "c4_n16"])
def test_ntt_roundtrip_and_ring_product(sets, name):
    g, o = sets(name)
    l = min(o.L, 4)
    x = rand_ct(o, l, 2, 1)
    p = workloads.uniform_residues(2, o.q[:l], o.N)
    cx = g.import_ct(x, 1.0)
    eq(g.export_ct(cx), x)                          # iNTT(NTT(x)) == x
    cp = g.import_limbs(p, list(range(l)))
    prod = g.mul_pt(cx, _fhe().Plaintext(cp, 1.0))
    want = o.mul_pt(ckks.Ct(x, 1.0), p, 1.0).data
    eq(g.export_ct(prod), want)


def test_ntt_special_primes_batch(sets):
    g, o = sets("c4_n16")
    mods = list(range(o.L, o.L + o.K)) * 3
    x = workloads.uniform_residues(3, [o.moduli[m] for m in mods], o.N)
    t = g.import_limbs(x, mods)
    eq(g.export_limbs(t, mods), x)


# -------------------------------------------------------------- samplers / keys
def test_secret_and_public_key_parity(sets):
    g, o = sets("c1_n12")
    s = g.keygen_secret(workloads.SEED_SECRET)
    so = o.keygen_secret(workloads.SEED_SECRET)
    assert np.array_equal(s.astype(np.int64), so)
    pk = g.keygen_pk(s, workloads.SEED_PK)
    eq(g.export_ct(pk), o.keygen_pk(so, workloads.SEED_PK))


@pytest.mark.parametrize("name", ["c1_n12", "c3_n13"])
def test_relin_and_rotation_key_parity(sets, name):
    g, o = sets(name)
    s = g.keygen_secret(7)
    so = s.astype(np.int64)
    rlk = g.keygen_relin(s, 11)
    eq(g.export_evk(rlk), o.keygen_relin(so, 11))
    for step in [1, -3]:
        gk = g.keygen_rot(s, step, 12)
        assert gk.galois == o.galois_elt(step)
        eq(g.export_evk(gk), o.keygen_rot(so, step, 12))


# ------------------------------------------------------- encode / encrypt
@pytest.mark.parametrize("name", ["c1_n12", "c2_n14"])
def test_encode_parity(sets, name):
    g, o = sets(name)
    n = o.N // 2
    re, im = workloads.complex_messages(3, n)
    pt = g.encode(re, im, scale=o.scale, limbs=2)
    got = g.export_limbs(pt.data, [0, 1])
    want = o.encode_rns(re, o.scale, 2, im)
    eq(got, want)
    # fewer values than slots, real only
    pt = g.encode(re[:100], None, scale=o.scale, limbs=1)
    eq(g.export_limbs(pt.data, [0]), o.encode_rns(re[:100], o.scale, 1))


def test_encrypt_decrypt_decode_parity(sets):
    g, o = sets("c1_n12")
    s = g.keygen_secret(1)
    so = s.astype(np.int64)
    pk = g.keygen_pk(s, 2)
    pko = o.keygen_pk(so, 2)
    n = o.N // 2
    z = workloads.slot_messages(4, n)
    coeff = o.encode(z, None, o.scale)
    for l in [3, 1]:
        pt = g.encode_coeffs(coeff, o.scale, limbs=l)
        ct = g.encrypt(pk, pt, 99)
        cto = o.encrypt(pko, o.small_to_rns(coeff, l), 99, o.scale)
        eq(g.export_ct(ct), cto.data)
        dec = g.decrypt(s, ct)
        eq(g.export_limbs(dec.data, list(range(l))), o.decrypt(cto, so))
        re, im = g.decode(dec)
        mo = o.decrypt(cto, so)
        ro, io = o.decode(mo, o.scale)
        dmax = max(np.abs(re - ro).max(), np.abs(im - io).max())
        nd = int(np.sum(re != ro) + np.sum(im != io))
        # Both sides sum the same N products in FP64 in different orders; any order is
        # within (N + 1) u sum_k |m_k| of the exact sum (u = 2^-53), so they differ by
        # at most twice that, over the scale.
        mk = _centered_lift(mo, o.q)
        bound = 2 * (o.N + 1) * 2.0 ** -53 * float(sum(abs(v) for v in mk)) / o.scale
        print("decode l=%d: %d of %d values differ, max |diff| %.3e (bound %.3e)" % (l, nd, 2 * n, dmax, bound))
        assert dmax <= bound
        assert np.abs(re - z).max() < 1e-3
        # selected slots equal the full decode
        sel = [0, 1, 7, n - 1, n // 2]
        rs, is_ = g.decode_slots(dec, sel)
        assert np.array_equal(rs, re[sel]) and np.array_equal(is_, im[sel])


def _centered_lift(m, q):
    """Plaintext coefficients from limb 0 (one limb) or limbs 0 and 1 by CRT, centered."""
    if m.shape[0] == 1:
        return [int(x) - q[0] if int(x) > q[0] // 2 else int(x) for x in m[0]]
    Q = q[0] * q[1]
    inv = pow(q[0], -1, q[1])
    out = []
    for x0, x1 in zip(m[0], m[1]):
        x = int(x0) + q[0] * (((int(x1) - int(x0)) * inv) % q[1])
        out.append(x - Q if x > Q // 2 else x)
    return out


# ------------------------------------------------------------ arithmetic
def test_add_sub_mulconst_parity(sets):
    g, o = sets("c1_n12")
    a, b = rand_ct(o, 3, 2, 5), rand_ct(o, 3, 2, 6)
    ga, gb = g.import_ct(a, 1.0), g.import_ct(b, 1.0)
    eq(g.export_ct(g.add(ga, gb)), o.add(ckks.Ct(a, 1.0), ckks.Ct(b, 1.0)).data)
    eq(g.export_ct(g.sub(ga, gb)), o.sub(ckks.Ct(a, 1.0), ckks.Ct(b, 1.0)).data)
    got = g.mul_const(ga, -0.37, 2.0 ** 20)
    eq(g.export_ct(got), o.mul_const(ckks.Ct(a, 1.0), round(-0.37 * 2 ** 20)).data)
    p = workloads.uniform_residues(7, o.q, o.N)
    gp = _fhe().Plaintext(g.import_limbs(p, [0, 1, 2]), 1.0)
    eq(g.export_ct(g.add_pt(ga, gp)), o.add_pt(ckks.Ct(a, 1.0), p).data)


def test_sum_pool_and_drop_level_parity(sets):
    """The 2x2 sum pooling over slot-packed maps (three additions per output, the
    paper network's pool with 1/4 folded into the activation) and the level drop,
    against the oracle's additions and limb slicing: 2 channels of 4 x 6 maps."""
    from oracle import cnn
    g, o = sets("c1_n12")
    C_, H, W = 2, 4, 6
    xs = [rand_ct(o, 3, 2, 900 + i) for i in range(C_ * H * W)]
    gx = [g.import_ct(x, 1.0) for x in xs]
    got = g.pool2x2_sum_slot(gx, C_, H, W)
    ref = cnn.enc_sum_pool2x2_slot(o, [ckks.Ct(x, 1.0) for x in xs], C_, H, W, cnn.Counter())
    assert len(got) == len(ref) == C_ * (H // 2) * (W // 2)
    for a, b in zip(got, ref):
        eq(g.export_ct(a), b.data)
    for lim in (1, 2):
        d = g.drop_level(gx[5], lim)
        assert d.limbs == lim and d.scale == gx[5].scale
        eq(g.export_ct(d), xs[5][:, :lim])


@pytest.mark.parametrize("n", [1, 5, 25])
def test_tensor_mac_parity(sets, n):
    g, o = sets("c2_n14")
    l = 5
    As = [rand_ct(o, l, 2, 100 + i) for i in range(n)]
    Bs = [rand_ct(o, l, 2, 200 + i) for i in range(n)]
    got = g.mul_acc([g.import_ct(x, 1.0) for x in As], [g.import_ct(x, 1.0) for x in Bs])
    want = o.mul_acc([ckks.Ct(x, 1.0) for x in As], [ckks.Ct(x, 1.0) for x in Bs])
    eq(g.export_ct(got), want.data)


@pytest.mark.parametrize("name,levels", [("c1_n12", [3, 2]), ("c2_n14", [8, 2]), ("c4_n16", [3])])
def test_rescale_parity(sets, name, levels):
    g, o = sets(name)
    for l in levels:
        for polys in [2, 3]:
            x = rand_ct(o, l, polys, 10 + l)
            got = g.rescale(g.import_ct(x, 2.0 ** 60))
            want = o.rescale(ckks.Ct(x, 2.0 ** 60))
            eq(g.export_ct(got), want.data)
            assert got.scale == want.scale
    # in place (output aliases the input buffer)
    x = rand_ct(o, levels[0], 2, 3)
    gx = g.import_ct(x, 1.0)
    out = _fhe().Ciphertext(gx.data.view(-1)[: 2 * (levels[0] - 1) * o.N].view(2, levels[0] - 1, o.N), 1.0)
    g.rescale(gx, out)
    eq(g.export_ct(out), o.rescale(ckks.Ct(x, 1.0)).data)


def test_rescale_floor_raises(sets):
    g, o = sets("c1_n12")
    P = _fhe()
    x = g.import_ct(rand_ct(o, 1, 2, 1), 1.0)
    with pytest.raises(P.FheError) as e:
        g.rescale(x, g.new_ct(1))
    assert e.value.code == P.fhe.FHE_ELEVEL


# ----------------------------------------------------------- key switching
@pytest.mark.parametrize("name,levels", [("c1_n12", [3, 2, 1]), ("c2_n14", [8, 5]), ("c3_n15", [16, 7, 1])])
def test_keyswitch_parity_random_key(sets, name, levels):
    g, o = sets(name)
    M = o.L + o.K
    evk = workloads.uniform_residues(50, o.moduli * (2 * o.dnum), o.N).reshape(o.dnum, 2, M, o.N)
    gk = g.import_evk(evk)
    for l in levels:
        d = workloads.uniform_residues(60 + l, o.q[:l], o.N)
        gd = g.import_limbs(d, list(range(l)))
        got = g.keyswitch(gk, gd)
        eq(g.export_ct(got), o.keyswitch(d, evk))


def test_keyswitch_batch_matches_single(sets):
    g, o = sets("c3_n15")
    M = o.L + o.K
    keys, ds = [], []
    for b in range(3):
        evk = workloads.uniform_residues(70 + b, o.moduli * (2 * o.dnum), o.N)
        keys.append(g.import_evk(evk))
        ds.append(g.import_limbs(workloads.uniform_residues(80 + b, o.q[:9], o.N), list(range(9))))
    outs = g.keyswitch_batch(keys, ds)
    for b in range(3):
        single = g.keyswitch(keys[b], ds[b])
        assert np.array_equal(g.export_ct(outs[b]), g.export_ct(single))


@pytest.mark.parametrize("name,l", [("c1_n12", 3), ("c3_n15", 16), ("c4_n16", 24), ("c4_n16", 7)])
def test_keyswitch_fused_row_inner_matches_split(sets, name, l):
    """The row pass of the converted digits fused into the key inner product gives
    the same key switch as the two separate kernels, and as the oracle."""
    g, o = sets(name)
    evk_np = workloads.uniform_residues(300 + l, o.moduli * (2 * o.dnum), o.N).reshape(o.dnum, 2, o.L + o.K, o.N)
    d_np = [workloads.uniform_residues(310 + l + i, o.q[:l], o.N) for i in range(2)]
    evk = g.import_evk(evk_np)
    ds = [g.import_limbs(d, list(range(l))) for d in d_np]
    evk2 = workloads.uniform_residues(320 + l, o.moduli * (2 * o.dnum), o.N).reshape(o.dnum, 2, o.L + o.K, o.N)
    keys = [evk, g.import_evk(evk2)]
    outs = {}
    for fuse in (1, 0):
        g.set_tuning("ks_fuse_row_inner", fuse)
        outs[fuse] = [g.export_ct(x) for x in g.keyswitch_batch(keys, ds)]
    g.set_tuning("ks_fuse_row_inner", 1)
    for a, b in zip(outs[1], outs[0]):
        assert np.array_equal(a, b)
    if o.N <= 1 << 15 or l < 10:
        eq(outs[1][0], o.keyswitch(d_np[0], evk_np))


@pytest.mark.parametrize("name,l", [("c3_n15", 16), ("c4_n16", 24), ("c4_n16", 9)])
def test_tuning_knobs_same_results(sets, name, l):
    """The row passes of the key switch and the rescale in 128- or 256-thread
    workgroups give the same rotations and rescales."""
    g, o = sets(name)
    s = g.keygen_secret(9)
    keys = [g.keygen_rot(s, r, 70 + r) for r in (1, 3)]
    xs = [g.import_ct(rand_ct(o, l, 2, 400 + i), 1.0) for i in range(2)]
    res = {}
    for wg in (128, 256):
        g.set_tuning("row_wg", wg)
        rot = g.rotate_batch(keys, xs, [1, 3])
        res[wg] = [g.export_ct(x) for x in rot] + [g.export_ct(x) for x in g.rescale_batch(rot)]
    g.set_tuning("row_wg", 128)
    for a, b in zip(res[128], res[256]):
        assert np.array_equal(a, b)
    P = _fhe()
    with pytest.raises(P.FheError):
        g.set_tuning("row_wg", 64)


def test_keyswitch_batch_shared_keys(sets):
    """Items that share a key at one level share the key reads of the inner
    product (groups of at most 8): batches with interleaved keys and a group split
    in two equal single calls and the oracle."""
    g, o = sets("c3_n15")
    keys_np = [workloads.uniform_residues(90 + b, o.moduli * (2 * o.dnum), o.N).reshape(o.dnum, 2, o.L + o.K, o.N)
               for b in range(2)]
    keys = [g.import_evk(k) for k in keys_np]
    for l, plan in [(9, [0] * 6 + [1] * 2 + [0] * 5 + [1] * 3), (4, [1, 0, 1])]:
        ds_np = [workloads.uniform_residues(100 + i, o.q[:l], o.N) for i in range(len(plan))]
        ds = [g.import_limbs(d, list(range(l))) for d in ds_np]
        outs = g.keyswitch_batch([keys[k] for k in plan], ds)
        for i, k in enumerate(plan):
            assert np.array_equal(g.export_ct(outs[i]), g.export_ct(g.keyswitch(keys[k], ds[i]))), (l, i)
        # members of every group, both halves of the split one
        for i in ((0, 6, 9, 12, 15) if l == 9 else (0, 1)):
            eq(g.export_ct(outs[i]), o.keyswitch(ds_np[i], keys_np[plan[i]]))


def test_rotate_batch_gathered(sets):
    """Batched rotations read c1 and c0 through the Galois permutation inside the key
    switch (no permuted copy): equal to single rotations (which stage a permuted
    copy) and to the oracle, at N = 2^15 (two-pass transforms), shared and distinct
    keys."""
    g, o = sets("c3_n15")
    s = g.keygen_secret(5)
    steps = [1, -1, 28, 1, 5]
    keys = {r: g.keygen_rot(s, r, 60 + r % 64) for r in set(steps)}
    for l in (9, 2):
        xs_np = [rand_ct(o, l, 2, 200 + 10 * l + i) for i in range(len(steps))]
        xs = [g.import_ct(x, 1.0) for x in xs_np]
        outs = g.rotate_batch([keys[r] for r in steps], xs, steps)
        for i, r in enumerate(steps):
            assert np.array_equal(g.export_ct(outs[i]), g.export_ct(g.rotate(keys[r], xs[i], r))), (l, i)
    gko = o.keygen_rot(s.astype(np.int64), 28, 60 + 28)
    eq(g.export_ct(outs[2]), o.rotate(ckks.Ct(xs_np[2], 1.0), 28, gko).data)


def test_relin_rotate_parity(sets):
    g, o = sets("c1_n12")
    s = g.keygen_secret(3)
    so = s.astype(np.int64)
    rlk = g.keygen_relin(s, 4)
    rlko = o.keygen_relin(so, 4)
    x3 = rand_ct(o, 3, 3, 21)
    got = g.relin(rlk, g.import_ct(x3, 1.0))
    eq(g.export_ct(got), o.relin(ckks.Ct(x3, 1.0), rlko).data)
    for step in [1, -1, 5]:
        gk = g.keygen_rot(s, step, 30 + step)
        gko = o.keygen_rot(so, step, 30 + step)
        for l in [3, 2]:
            x = rand_ct(o, l, 2, 40 + l)
            got = g.rotate(gk, g.import_ct(x, 1.0), step)
            eq(g.export_ct(got), o.rotate(ckks.Ct(x, 1.0), step, gko).data)
    P = _fhe()
    with pytest.raises(P.FheError) as e:
        g.rotate(gk, g.import_ct(rand_ct(o, 3, 2, 1), 1.0), 2)
    assert e.value.code == P.fhe.FHE_ENOKEY


def test_end_to_end_mult_rotate_c1(sets):
    """Config 1: encode, encrypt, HMult + relin + rescale, rotate by 1, decrypt, decode."""
    g, o = sets("c1_n12")
    n = o.N // 2
    s = g.keygen_secret(workloads.SEED_SECRET)
    pk = g.keygen_pk(s, workloads.SEED_PK)
    rlk = g.keygen_relin(s, workloads.SEED_EVK)
    gk = g.keygen_rot(s, 1, workloads.SEED_EVK + 1)
    a, b = workloads.slot_messages(1, n), workloads.slot_messages(2, n)
    ca = g.encrypt(pk, g.encode(a, scale=o.scale), workloads.SEED_ENC)
    cb = g.encrypt(pk, g.encode(b, scale=o.scale), workloads.SEED_ENC + 1)
    m = g.mul_relin_rescale(rlk, ca, cb)
    r = g.rotate(gk, m, 1)
    # bit-exact against the oracle pipeline from the same seeds
    so = s.astype(np.int64)
    pko = o.keygen_pk(so, workloads.SEED_PK)
    rlko = o.keygen_relin(so, workloads.SEED_EVK)
    gko = o.keygen_rot(so, 1, workloads.SEED_EVK + 1)
    cao = o.encrypt(pko, o.encode_rns(a, o.scale, o.L), workloads.SEED_ENC, o.scale)
    cbo = o.encrypt(pko, o.encode_rns(b, o.scale, o.L), workloads.SEED_ENC + 1, o.scale)
    ro = o.rotate(o.mul_relin_rescale(cao, cbo, rlko), 1, gko)
    eq(g.export_ct(r), ro.data)
    got, _ = g.decode(g.decrypt(s, r))
    assert np.abs(got - np.roll(a * b, -1)).max() < 1e-2   # scale 2^20 after the rescale


# ------------------------------------------- the key switch at N=2^16, l=24
def test_keyswitch_parity_n16_full_level(sets):
    g, o = sets("c4_n16")
    M = o.L + o.K
    evk = workloads.uniform_residues(90, o.moduli * (2 * o.dnum), o.N).reshape(o.dnum, 2, M, o.N)
    gk = g.import_evk(evk)
    for l in [24, 17]:
        d = workloads.uniform_residues(91 + l, o.q[:l], o.N)
        got = g.keyswitch(gk, g.import_limbs(d, list(range(l))))
        eq(g.export_ct(got), o.keyswitch(d, evk))


def test_rotation_batch_as_benchmarked(sets):
    """The benchmark's configuration: 8 fresh ciphertexts at N = 2^16, l = 24 rotated by
    1..8 with 8 distinct Galois keys in one fhe_rotate_batch, with the default tuning.
    Two sampled outputs are recomputed by the oracle from the same keys and inputs."""
    g, o = sets("c4_n16")
    s = g.keygen_secret(workloads.SEED_SECRET)
    so = s.astype(np.int64)
    pk = g.keygen_pk(s, workloads.SEED_PK)
    steps = list(range(1, 9))
    gks = [g.keygen_rot(s, r, workloads.SEED_EVK + r) for r in steps]
    cts = [g.encrypt(pk, g.encode(workloads.slot_messages(workloads.SEED_DATA + b, 64), scale=g.scale, limbs=g.L),
                     workloads.SEED_ENC + b) for b in range(8)]
    outs = g.rotate_batch(gks, cts, steps)
    for b in (0, 5):
        gko = o.keygen_rot(so, steps[b], workloads.SEED_EVK + steps[b])
        assert np.array_equal(g.export_evk(gks[b]), gko)
        ref = o.rotate(ckks.Ct(g.export_ct(cts[b]), cts[b].scale), steps[b], gko)
        eq(g.export_ct(outs[b]), ref.data)


def test_keyswitch_knobs_give_the_same_bits(sets):
    """The key switch's kernel knobs (the five-kernel fused form or the seven-kernel
    one; data used once loaded and stored non-temporally or not) give the
    same bits every way, for rotations with distinct keys and for relinearisations
    that share one key."""
    import torch
    g, _ = sets("c3_n15")
    s = g.keygen_secret(workloads.SEED_SECRET)
    pk = g.keygen_pk(s, workloads.SEED_PK)
    rlk = g.keygen_relin(s, workloads.SEED_EVK)
    steps = [1, -1, 28, 5, 7]
    gks = [g.keygen_rot(s, r, workloads.SEED_EVK + 1 + i) for i, r in enumerate(steps)]
    cts = [g.encrypt(pk, g.encode(workloads.slot_messages(workloads.SEED_DATA + b, 64), scale=g.scale,
                                  limbs=9 + b), workloads.SEED_ENC + b) for b in range(len(steps))]
    c3 = [g.mul(c, c) for c in cts]

    def run():
        rot = g.rotate_batch(gks, [cts[0]] * len(steps), steps)
        rel = [g.relin(rlk, c) for c in c3]
        rel += g.relin_batch(rlk, c3[:1] * 3)
        torch.cuda.synchronize()
        return [x.data.clone() for x in rot + rel]
    ref = run()
    for fuse, nt in ((0, 0), (0, 1), (1, 0), (1, 1)):
        g.set_tuning("ks_fuse_row_inner", fuse)
        g.set_tuning("ks_nt", nt)
        got = run()
        for i, (a, b) in enumerate(zip(got, ref)):
            assert torch.equal(a, b), (fuse, nt, i)
    g.set_tuning("ks_fuse_row_inner", 1)
    g.set_tuning("ks_nt", 1)
