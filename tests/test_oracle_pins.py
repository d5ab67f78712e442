"""Pins for the CPU oracle: each test checks it against something other than
itself -- Python big integers, sympy, numpy's Philox, mpmath, closed forms and
invariants of the scheme -- so that a dropped term, a wrong sign or index or a
transposed operand in the oracle fails at least one of them."""
import math

import mpmath
import numpy as np
import pytest
import sympy

import workloads
from oracle import OracleCtx, ckks

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def small_primes(log_n, count, bits=30):
    two_n = 2 << log_n
    out, c = [], ((1 << bits) - 2) // two_n
    while len(out) < count:
        q = c * two_n + 1
        if sympy.isprime(q):
            out.append(q)
        c -= 1
    return out


def crt(res, mods):
    return int(sympy.ntheory.modular.crt(mods, [int(r) for r in res])[0])


def centered(x, m):
    x %= m
    return x - m if x > m // 2 else x


def schoolbook(a, b, q):
    n = len(a)
    out = [0] * n
    for i in range(n):
        for j in range(n):
            if i + j < n:
                out[i + j] += int(a[i]) * int(b[j])
            else:
                out[i + j - n] -= int(a[i]) * int(b[j])
    return [x % q for x in out]


@pytest.fixture(scope="module")
def tiny():
    q = small_primes(4, 3, 30)
    p = small_primes(4, 2, 31)
    return OracleCtx(4, q, p, dnum=2, cdt=workloads.load_params("c1_n12")["cdt"])


@pytest.fixture(scope="module")
def c1():
    return OracleCtx.from_set("c1_n12")


# ------------------------------------------------------------ parameters
def test_param_primes_are_ntt_friendly_primes():
    data = workloads.load_params()
    for name, s in data["sets"].items():
        n2 = 2 << s["log_n"]
        allp = [int(x) for x in s["q"]] + [int(x) for x in s["p"]]
        assert len(set(allp)) == len(allp), name
        for q in allp:
            assert sympy.isprime(q), (name, q)
            assert (q - 1) % n2 == 0, (name, q)
            assert q < 2 ** 50, (name, q)


def test_param_q0_is_largest_below_bound():
    # "below(b)" rule: no NTT-friendly prime lies between q0 and 2^b
    s = workloads.load_params("c4_n16")
    q0, n2 = s["q"][0], 2 << s["log_n"]
    for c in range(q0 // n2 + 1, (2 ** 50 - 1) // n2 + 1):
        assert not sympy.isprime(c * n2 + 1)


def test_is_prime_matches_sympy():
    rs = np.random.default_rng(5)
    L = ckks.lib()
    for x in list(rs.integers(2, 2 ** 62, size=300, dtype=np.uint64)) + [2, 3, 4, 561, 1105, 2 ** 61 - 1]:
        assert bool(L.or_is_prime(int(x))) == sympy.isprime(int(x))


def test_min_psi_is_minimal_primitive_root():
    L = ckks.lib()
    for (q, n) in [(97, 16), (257, 64), (7681, 256), (12289, 512)]:
        psi = L.or_min_psi(q, n)
        assert pow(psi, n, q) == q - 1
        roots = [x for x in range(1, q) if pow(x, n, q) == q - 1]
        assert psi == min(roots)


# ------------------------------------------------------------------- NTT
def test_ntt_is_evaluation_at_odd_powers(tiny):
    rs = np.random.default_rng(1)
    for m in range(3):
        q, psi = tiny.moduli[m], tiny.psi(m)
        a = rs.integers(0, q, size=tiny.N, dtype=np.uint64)
        got = tiny.ntt(m, a)
        for k in range(tiny.N):
            x = pow(psi, 2 * k + 1, q)
            assert int(got[k]) == sum(int(a[i]) * pow(x, i, q) for i in range(tiny.N)) % q
        assert np.array_equal(tiny.intt(m, got), a)


@pytest.mark.parametrize("log_n", [3, 5, 6])
def test_polymul_matches_schoolbook(log_n):
    q = small_primes(log_n, 1, 40)
    o = OracleCtx(log_n, q, [], dnum=1)
    rs = np.random.default_rng(log_n)
    a = rs.integers(0, q[0], size=o.N, dtype=np.uint64)
    b = rs.integers(0, q[0], size=o.N, dtype=np.uint64)
    assert [int(x) for x in o.polymul(0, a, b)] == schoolbook(a, b, q[0])


def test_polymul_spot_coefficients_n4096(c1):
    rs = np.random.default_rng(2)
    q = c1.q[0]
    a = rs.integers(0, q, size=c1.N, dtype=np.uint64)
    b = rs.integers(0, q, size=c1.N, dtype=np.uint64)
    c = c1.polymul(0, a, b)
    A, B = [int(x) for x in a], [int(x) for x in b]
    for k in [0, 1, 2047, 4095]:
        s = sum(A[i] * B[k - i] for i in range(k + 1)) - sum(A[i] * B[c1.N + k - i] for i in range(k + 1, c1.N))
        assert int(c[k]) == s % q
    assert np.array_equal(c1.intt(0, c1.ntt(0, a)), a)


# ---------------------------------------------------------------- Philox
def test_philox_matches_numpy():
    L = ckks.lib()
    rs = np.random.default_rng(3)
    for _ in range(20):
        key = rs.integers(0, 2 ** 64, size=2, dtype=np.uint64)
        ctr = rs.integers(0, 2 ** 63, size=4, dtype=np.uint64)
        ref = np.random.Philox(key=key, counter=ctr).random_raw(4)   # numpy uses counter+1
        out = (ckks.C.c_uint64 * 4)()
        c2 = ctr.copy()
        c2[0] += np.uint64(1)
        L.or_philox4x64_10((ckks.C.c_uint64 * 2)(*[int(x) for x in key]),
                           (ckks.C.c_uint64 * 4)(*[int(x) for x in c2]), out)
        assert [int(x) for x in out] == [int(x) for x in ref]


# -------------------------------------------------------------- samplers
def test_uniform_sampler_statistics(c1):
    u = c1.sample_uniform(11, ckks.TAG_UNIFORM, 0, [0, 3])
    for row, q in zip(u, [c1.q[0], c1.p[0]]):
        assert row.max() < q
        hist = np.bincount((row.astype(np.float64) / q * 16).astype(int), minlength=16)
        chi2 = ((hist - len(row) / 16) ** 2 / (len(row) / 16)).sum()
        assert chi2 < 60   # 15 dof; p ~ 1e-7
    assert not np.array_equal(u[0], c1.sample_uniform(12, ckks.TAG_UNIFORM, 0, [0])[0])
    assert np.array_equal(u, c1.sample_uniform(11, ckks.TAG_UNIFORM, 0, [0, 3]))


def test_ternary_sampler_statistics(c1):
    s = np.concatenate([c1.sample_ternary(20 + i, ckks.TAG_SECRET, 0) for i in range(8)])
    vals, counts = np.unique(s, return_counts=True)
    assert list(vals) == [-1, 0, 1]
    assert np.all(np.abs(counts / len(s) - 1 / 3) < 0.01)


def test_gauss_table_and_sampler(c1):
    cdt = workloads.load_params("c1_n12")["cdt"]
    assert all(a < b for a, b in zip(cdt, cdt[1:])) and cdt[-1] < 2 ** 64
    # P(e = 0) from the table vs the Jacobi theta normalisation (independent closed form)
    sig = mpmath.mpf(3.2)
    z = mpmath.jtheta(3, 0, mpmath.exp(-1 / (2 * sig ** 2)))
    assert abs(cdt[0] / 2 ** 64 - float(1 / z)) < 1e-6   # tail beyond 19 is < 1e-8
    e = np.concatenate([c1.sample_gauss(30 + i, ckks.TAG_ERROR, 0) for i in range(16)])
    assert np.abs(e).max() <= 19
    assert abs(e.mean()) < 0.05
    assert abs(e.var() - 3.2 ** 2) < 0.25
    assert abs(np.mean(e == 0) - cdt[0] / 2 ** 64) < 0.005


# ------------------------------------------------------------------ keys
def _centered_crt(rows, mods):
    N = rows.shape[1]
    M = math.prod(mods)
    return [centered(crt(rows[:, k], mods), M) for k in range(N)]


def test_public_key_is_rlwe_sample(c1):
    s = c1.keygen_secret(7)
    pk = c1.keygen_pk(s, 8)
    for i, q in enumerate(c1.q):
        sr = c1.small_to_rns(s, modidx=[i])[0]
        e = (pk[0, i] + c1.polymul(i, pk[1, i], sr)) % np.uint64(q)   # b + a s = e (small)
        ec = np.array([centered(int(x), q) for x in e])
        assert np.abs(ec).max() <= 19
        if i == 0:
            e0 = ec
        assert np.array_equal(ec, e0)
    assert np.abs(e0).max() > 0


def test_evk_gadget_structure(tiny):
    s = tiny.sample_ternary(1, ckks.TAG_SECRET, 0)
    s2 = tiny.square_small(s)
    # s^2 by big-integer schoolbook
    assert [int(x) for x in s2] == [centered(v, 2 ** 62) for v in schoolbook(s % 2 ** 62, s % 2 ** 62, 2 ** 62)]
    evk = tiny.keygen_evk(s, s2, 5)
    P = math.prod(tiny.p)
    n = tiny.L + tiny.K
    for j in range(tiny.dnum):
        lo, hi = j * tiny.alpha, min((j + 1) * tiny.alpha, tiny.L)
        rows = []
        for i in range(n):
            q = tiny.moduli[i]
            sr = tiny.small_to_rns(s, modidx=[i])[0]
            v = (evk[j, 0, i] + tiny.polymul(i, evk[j, 1, i], sr)) % np.uint64(q)
            g = (P % q) if lo <= i < hi else 0
            v = np.array([(int(x) - g * int(y)) % q for x, y in zip(v, s2)], dtype=object)
            rows.append([centered(int(x), q) for x in v])
        rows = np.array(rows)
        assert np.abs(rows).max() <= 19
        assert (rows == rows[0]).all()
    # gadget identity: sum_j [d]_{Q_j} * Q^_j * [Q^_j^-1]_{Q_j} == d (mod Q)
    Q = math.prod(tiny.q)
    d = 123456789123456789 % Q
    acc = 0
    for j in range(tiny.dnum):
        Qj = math.prod(tiny.q[j * tiny.alpha:(j + 1) * tiny.alpha])
        Qh = Q // Qj
        acc += (d % Qj) * Qh * pow(Qh, -1, Qj)
    assert acc % Q == d


# ---------------------------------------------------- encrypt / decrypt
def test_encrypt_decrypt_noise_bound(c1):
    s = c1.keygen_secret(1)
    pk = c1.keygen_pk(s, 2)
    rs = np.random.default_rng(4)
    m = np.array([rs.integers(0, q, size=c1.N, dtype=np.uint64) for q in c1.q])
    ct = c1.encrypt(pk, m, 3, 1.0)
    d = c1.decrypt(ct, s)
    diff = np.array([(d[i].astype(object) - m[i].astype(object)) % q for i, q in enumerate(c1.q)])
    noise = _centered_crt(diff, c1.q)
    assert max(abs(x) for x in noise) <= 19 * (2 * c1.N + 1)
    assert max(abs(x) for x in noise) > 0


# ------------------------------------------------------------- encoding
def test_encode_constant_closed_form(c1):
    for c in [0.25, -0.7, 1.0]:
        coeff = c1.encode(np.full(c1.N // 2, c), None, 2.0 ** 30)
        assert coeff[0] == round(c * 2 ** 30)
        assert np.all(coeff[1:] == 0)


def test_encode_matches_mpmath_and_slot_order():
    q = small_primes(4, 2, 40)
    o = OracleCtx(4, q, [], dnum=1)
    N, n, scale = o.N, o.N // 2, 2.0 ** 20
    rs = np.random.default_rng(9)
    re, im = rs.uniform(-1, 1, n), rs.uniform(-1, 1, n)
    coeff = o.encode(re, im, scale)
    mpmath.mp.dps = 40
    zeta = mpmath.exp(1j * mpmath.pi / N)
    for k in range(N):
        v = 0
        for j in range(n):
            r = zeta ** (pow(5, j, 2 * N))
            z = mpmath.mpc(re[j], im[j])
            v += z * r ** (-k) + mpmath.conj(z) * mpmath.conj(r) ** (-k)
        exact = v.real * scale / N
        assert abs(int(coeff[k]) - float(exact)) <= 0.5 + 1e-6
    # evaluation at zeta^(5^j) recovers slot j (pins the slot order)
    for j in range(n):
        r = zeta ** pow(5, j, 2 * N)
        val = sum(int(coeff[k]) * r ** k for k in range(N)) / scale
        assert abs(complex(val) - complex(re[j], im[j])) < N / scale


def test_decode_encode_roundtrip(c1):
    n = c1.N // 2
    re, im = workloads.complex_messages(5, n)
    m = c1.encode_rns(re, 2.0 ** 30, 2, im)
    r2, i2 = c1.decode(m, 2.0 ** 30)
    err = max(np.abs(r2 - re).max(), np.abs(i2 - im).max())
    assert err < (n / 2.0 ** 30) and err < 1e-6


# ------------------------------------------------------ basis conversion
def test_bconv_identity(tiny):
    rs = np.random.default_rng(6)
    src, dst = [0, 1, 2], [3, 4]
    B = math.prod(tiny.moduli[i] for i in src)
    x = np.array([rs.integers(0, tiny.moduli[i], size=tiny.N, dtype=np.uint64) for i in src])
    y = tiny.bconv(x, src, dst)
    for k in range(tiny.N):
        X = crt(x[:, k], [tiny.moduli[i] for i in src])
        us = set()
        for d_i, d in enumerate(dst):
            c = tiny.moduli[d]
            # y = X + u*B (mod c) for one integer 0 <= u < len(src)
            cands = [u for u in range(len(src)) if (X + u * B) % c == int(y[d_i, k])]
            assert cands, (k, d)
            us.add(cands[0])
        assert len(us) == 1


# ------------------------------------------------- key switch / relin
def _ks_error(o, ks, d, s_from, s):
    l = d.shape[0]
    rows = []
    for i in range(l):
        q = o.q[i]
        sr = o.small_to_rns(s, modidx=[i])[0]
        sf = o.small_to_rns(s_from, modidx=[i])[0]
        v = (ks[0, i].astype(object) + o.polymul(i, ks[1, i], sr).astype(object)
             - o.polymul(i, d[i], sf).astype(object)) % q
        rows.append(v)
    return _centered_crt(np.array(rows), o.q[:l])


def test_keyswitch_invariant(tiny):
    s = tiny.sample_ternary(2, ckks.TAG_SECRET, 0)
    s_from = tiny.square_small(s)
    evk = tiny.keygen_evk(s, s_from, 9)
    rs = np.random.default_rng(7)
    for l in [3, 2]:
        d = np.array([rs.integers(0, q, size=tiny.N, dtype=np.uint64) for q in tiny.q[:l]])
        ks = tiny.keyswitch(d, evk)
        err = _ks_error(tiny, ks, d, s_from, s)
        maxQj = max(math.prod(tiny.q[j * tiny.alpha:(j + 1) * tiny.alpha]) for j in range(tiny.dnum))
        bound = tiny.dnum * tiny.alpha * tiny.N * 19 * maxQj / math.prod(tiny.p) + (tiny.K + 1) * (tiny.N + 1)
        assert max(abs(x) for x in err) <= bound


def test_keyswitch_galois_identity_and_invariant(tiny):
    """The rotation form of the key switch: with g = 1 it is the plain key switch;
    with a Galois element it is a key switch of sigma_g(d) (same invariant and error
    bound as the plain one, with sigma_g(d) for d); and it is another valid result
    than the plain key switch of sigma_g(d), since the fast conversion of a negated
    coefficient differs from the negated conversion by a multiple of the digit modulus."""
    s = tiny.sample_ternary(2, ckks.TAG_SECRET, 0)
    rs = np.random.default_rng(17)
    for l in [3, 2]:
        d = np.array([rs.integers(0, q, size=tiny.N, dtype=np.uint64) for q in tiny.q[:l]])
        s_from = tiny.square_small(s)
        evk = tiny.keygen_evk(s, s_from, 9)
        assert np.array_equal(tiny.keyswitch_galois(d, evk, 1), tiny.keyswitch(d, evk))
        for r in (1, -3):
            g = tiny.galois_elt(r)
            sg = tiny.automorph_small(s, g)
            gk = tiny.keygen_evk(s, sg, 30 + r)
            dg = tiny.automorph(d, g)
            ks = tiny.keyswitch_galois(d, gk, g)
            err = _ks_error(tiny, ks, dg, sg, s)
            maxQj = max(math.prod(tiny.q[j * tiny.alpha:(j + 1) * tiny.alpha]) for j in range(tiny.dnum))
            bound = tiny.dnum * tiny.alpha * tiny.N * 19 * maxQj / math.prod(tiny.p) + (tiny.K + 1) * (tiny.N + 1)
            assert max(abs(x) for x in err) <= bound
            assert not np.array_equal(ks, tiny.keyswitch(dg, gk))


def test_relin_preserves_decryption(c1):
    s = c1.keygen_secret(1)
    rlk = c1.keygen_relin(s, 4)
    rs = np.random.default_rng(8)
    x = ckks.Ct(np.array([[rs.integers(0, q, size=c1.N, dtype=np.uint64) for q in c1.q] for _ in range(3)]), 1.0)
    r = c1.relin(x, rlk)
    d3, d2 = c1.decrypt(x, s), c1.decrypt(r, s)
    diff = np.array([(d2[i].astype(object) - d3[i].astype(object)) % q for i, q in enumerate(c1.q)])
    err = _centered_crt(diff, c1.q)
    assert max(abs(x) for x in err) < 2 ** 30


# ---------------------------------------------------------------- rescale
def test_rescale_is_exact_rounding(c1):
    rs = np.random.default_rng(10)
    ct = ckks.Ct(np.array([[rs.integers(0, q, size=c1.N, dtype=np.uint64) for q in c1.q] for _ in range(2)]), 2.0 ** 60)
    out = c1.rescale(ct)
    Q, Q1, ql = math.prod(c1.q), math.prod(c1.q[:2]), c1.q[2]
    for p in range(2):
        for k in range(0, c1.N, 97):
            x = centered(crt(ct.data[p, :, k], c1.q), Q)
            want = (2 * x + ql) // (2 * ql)      # round(x / ql), no ties (ql odd)
            got = centered(crt(out.data[p, :, k], c1.q[:2]), Q1)
            assert got == want
    assert out.scale == 2.0 ** 60 / ql


# ----------------------------------------------------- automorphism / rotate
def test_automorphism_permutes_evaluations(tiny):
    rs = np.random.default_rng(11)
    q, N = tiny.q[0], tiny.N
    a = rs.integers(0, q, size=N, dtype=np.uint64)
    for r in [1, 3, -1]:
        g = tiny.galois_elt(r)
        assert g == pow(5, r % (N // 2), 2 * N)
        A, S = tiny.ntt(0, a), tiny.ntt(0, tiny.automorph(a[None], g)[0])
        for k in range(N):
            kk = (((2 * k + 1) * g) % (2 * N) - 1) // 2
            assert S[k] == A[kk]
    g, h = tiny.galois_elt(1), tiny.galois_elt(2)
    assert np.array_equal(tiny.automorph(tiny.automorph(a[None], g), h), tiny.automorph(a[None], (g * h) % (2 * N)))


def test_end_to_end_mult_and_rotate(c1):
    n = c1.N // 2
    s = c1.keygen_secret(workloads.SEED_SECRET)
    pk = c1.keygen_pk(s, workloads.SEED_PK)
    rlk = c1.keygen_relin(s, workloads.SEED_EVK)
    gk = c1.keygen_rot(s, 1, workloads.SEED_EVK + 1)
    a, b = workloads.slot_messages(1, n), workloads.slot_messages(2, n)
    D = c1.scale
    ca = c1.encrypt(pk, c1.encode_rns(a, D, c1.L), workloads.SEED_ENC, D)
    cb = c1.encrypt(pk, c1.encode_rns(b, D, c1.L), workloads.SEED_ENC + 1, D)
    m = c1.mul_relin_rescale(ca, cb, rlk)
    # The rescale divides by a ~2^40 prime, leaving scale 2^20; its rounding
    # term (c0 + c1*s rounding, |c1*s| ~ sqrt(2N/3)/2 per coefficient) gives a
    # slot error of about sqrt(N) * 26 / 2^20 ~ 2e-3, so the bound is 1e-2.
    assert m.scale == D * D / c1.q[2]
    got, _ = c1.decode(c1.decrypt(m, s), m.scale)
    assert np.abs(got - a * b).max() < 1e-2
    rot = c1.rotate(m, 1, gk)
    got, _ = c1.decode(c1.decrypt(rot, s), rot.scale)
    assert np.abs(got - np.roll(a * b, -1)).max() < 1e-2
    # fresh noise v*e + e0 + e1*s: ~240 per coefficient, ~6e-5 per slot at 2^30
    got, _ = c1.decode(c1.decrypt(c1.add(ca, cb), s), D)
    assert np.abs(got - (a + b)).max() < 1e-3
