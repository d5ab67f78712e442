"""Pins for the oracle's element-wise and small-polynomial entry points against
Python big-integer arithmetic written from the definitions (per-limb modular
sum and difference, negacyclic schoolbook products, polynomial composition for
X -> X^g).  Each check is built so that a swapped operand, a dropped term or a
wrong limb index in the oracle changes the result."""
import math

import numpy as np
import pytest
import sympy

import workloads
from oracle import OracleCtx, ckks
from oracle.ckks import Ct

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def small_primes(log_n, count, bits):
    two_n = 2 << log_n
    out, c = [], ((1 << bits) - 2) // two_n
    while len(out) < count:
        q = c * two_n + 1
        if sympy.isprime(q):
            out.append(q)
        c -= 1
    return out


def negacyclic(a, b, q):
    """c_k = sum_{i+j=k} a_i b_j - sum_{i+j=k+N} a_i b_j mod q, in Python integers."""
    n = len(a)
    out = [0] * n
    for i in range(n):
        ai = int(a[i])
        for j in range(n):
            if i + j < n:
                out[i + j] += ai * int(b[j])
            else:
                out[i + j - n] -= ai * int(b[j])
    return [x % q for x in out]


@pytest.fixture(scope="module")
def tiny():
    # N = 16, three 30-bit primes and two 31-bit special primes
    return OracleCtx(4, small_primes(4, 3, 30), small_primes(4, 2, 31), dnum=2,
                     cdt=workloads.load_params("c1_n12")["cdt"])


def rand_ct(o, rs, polys, l):
    return Ct(np.array([[rs.integers(0, q, size=o.N, dtype=np.uint64) for q in o.q[:l]]
                        for _ in range(polys)]), 1.0)


def rows(o, x, l):
    """[polys][l][N] -> nested Python ints."""
    return [[[int(v) for v in x[p, i]] for i in range(l)] for p in range(x.shape[0])]


@pytest.mark.parametrize("l,polys", [(1, 2), (2, 3), (3, 2)])
def test_add_and_sub_are_limbwise_sum_and_difference(tiny, l, polys):
    rs = np.random.default_rng(100 + l)
    a, b = rand_ct(tiny, rs, polys, l), rand_ct(tiny, rs, polys, l)
    A, B = rows(tiny, a.data, l), rows(tiny, b.data, l)
    s, d = tiny.add(a, b).data, tiny.sub(a, b).data
    assert s.shape == d.shape == (polys, l, tiny.N)
    for p in range(polys):
        for i in range(l):
            q = tiny.q[i]
            assert [int(v) for v in s[p, i]] == [(x + y) % q for x, y in zip(A[p][i], B[p][i])]
            assert [int(v) for v in d[p, i]] == [(x - y) % q for x, y in zip(A[p][i], B[p][i])]
    # on the CRT integers: sub(a, b) + b == a (mod Q_l), and sub(a, b) != sub(b, a)
    back = tiny.add(tiny.sub(a, b), b).data
    assert np.array_equal(back, a.data)
    assert not np.array_equal(d, tiny.sub(b, a).data)


def test_add_pt_touches_c0_only(tiny):
    rs = np.random.default_rng(7)
    for l in (1, 3):
        ct = rand_ct(tiny, rs, 2, l)
        pt = np.array([rs.integers(0, q, size=tiny.N, dtype=np.uint64) for q in tiny.q[:l]])
        out = tiny.add_pt(ct, pt).data
        for i in range(l):
            q = tiny.q[i]
            assert [int(v) for v in out[0, i]] == [(int(x) + int(y)) % q for x, y in zip(ct.data[0, i], pt[i])]
        assert np.array_equal(out[1], ct.data[1])


def test_mul_pt_is_negacyclic_product_of_each_poly(tiny):
    rs = np.random.default_rng(8)
    for l in (1, 3):
        ct = rand_ct(tiny, rs, 2, l)
        pt = np.array([rs.integers(0, q, size=tiny.N, dtype=np.uint64) for q in tiny.q[:l]])
        out = tiny.mul_pt(ct, pt, 2.0)
        assert out.scale == 2.0
        for p in range(2):
            for i in range(l):
                assert [int(v) for v in out.data[p, i]] == negacyclic(ct.data[p, i], pt[i], tiny.q[i])


@pytest.mark.parametrize("const", [0, 1, 12345, -7, -(1 << 70) - 3, (1 << 65) + 11])
def test_mul_const_reduces_the_integer_per_limb(tiny, const):
    rs = np.random.default_rng(9)
    ct = rand_ct(tiny, rs, 2, 3)
    out = tiny.mul_const(ct, const, 4.0)
    assert out.scale == 4.0
    for p in range(2):
        for i in range(3):
            q = tiny.q[i]
            assert [int(v) for v in out.data[p, i]] == [(int(x) * const) % q for x in ct.data[p, i]]


def test_tensor_components_are_the_three_products(tiny):
    rs = np.random.default_rng(10)
    for l in (1, 2):
        a, b = rand_ct(tiny, rs, 2, l), rand_ct(tiny, rs, 2, l)
        a.scale, b.scale = 3.0, 5.0
        t = tiny.tensor(a, b)
        assert t.data.shape == (3, l, tiny.N) and t.scale == 15.0
        for i in range(l):
            q = tiny.q[i]
            a0, a1, b0, b1 = a.data[0, i], a.data[1, i], b.data[0, i], b.data[1, i]
            assert [int(v) for v in t.data[0, i]] == negacyclic(a0, b0, q)
            mid = [(x + y) % q for x, y in zip(negacyclic(a0, b1, q), negacyclic(a1, b0, q))]
            assert [int(v) for v in t.data[1, i]] == mid
            assert [int(v) for v in t.data[2, i]] == negacyclic(a1, b1, q)


def test_mul_acc_sums_the_pairs(tiny):
    rs = np.random.default_rng(11)
    l, n = 2, 4
    As = [rand_ct(tiny, rs, 2, l) for _ in range(n)]
    Bs = [rand_ct(tiny, rs, 2, l) for _ in range(n)]
    acc = tiny.mul_acc(As, Bs).data
    for i in range(l):
        q = tiny.q[i]
        want = [[0] * tiny.N for _ in range(3)]
        for a, b in zip(As, Bs):
            a0, a1, b0, b1 = a.data[0, i], a.data[1, i], b.data[0, i], b.data[1, i]
            parts = [negacyclic(a0, b0, q),
                     [(x + y) % q for x, y in zip(negacyclic(a0, b1, q), negacyclic(a1, b0, q))],
                     negacyclic(a1, b1, q)]
            for c in range(3):
                want[c] = [(x + y) % q for x, y in zip(want[c], parts[c])]
        for c in range(3):
            assert [int(v) for v in acc[c, i]] == want[c]


def test_decrypt_two_and_three_polys(tiny):
    rs = np.random.default_rng(12)
    s = tiny.sample_ternary(3, ckks.TAG_SECRET, 0)
    sq = [0] * tiny.N                                   # s^2 over the integers, negacyclic
    for i in range(tiny.N):
        for j in range(tiny.N):
            k = i + j
            if k < tiny.N:
                sq[k] += int(s[i]) * int(s[j])
            else:
                sq[k - tiny.N] -= int(s[i]) * int(s[j])
    for polys in (2, 3):
        ct = rand_ct(tiny, rs, polys, 3)
        m = tiny.decrypt(ct, s)
        for i in range(3):
            q = tiny.q[i]
            si = [int(v) % q for v in s]
            want = [int(v) for v in ct.data[0, i]]
            want = [(x + y) % q for x, y in zip(want, negacyclic(ct.data[1, i], si, q))]
            if polys == 3:
                want = [(x + y) % q for x, y in zip(want, negacyclic(ct.data[2, i], [v % q for v in sq], q))]
            assert [int(v) for v in m[i]] == want


def test_small_to_rns_and_automorph_small(tiny):
    s = np.array([-3, 5, 0, -1, 2, 7, -9, 1, 0, 0, 4, -2, 6, -5, 3, -8], dtype=np.int64)
    r = tiny.small_to_rns(s)
    for i, q in enumerate(tiny.q):
        assert [int(v) for v in r[i]] == [int(v) % q for v in s]
    N = tiny.N
    for step in (1, 3, -1):
        g = tiny.galois_elt(step)
        # s(X^g) written out as a polynomial of degree (N-1) g, then reduced by X^N = -1
        full = [0] * ((N - 1) * g + 1)
        for i in range(N):
            full[i * g] += int(s[i])
        red = [0] * N
        for e, v in enumerate(full):
            red[e % N] += v if (e // N) % 2 == 0 else -v
        assert [int(v) for v in tiny.automorph_small(s, g)] == red
        # the same map on residues (or_automorph) agrees with it limb by limb
        got = tiny.automorph(r, g)
        for i, q in enumerate(tiny.q):
            assert [int(v) for v in got[i]] == [v % q for v in red]


def test_drop_level_keeps_the_residues_of_the_smaller_modulus(tiny):
    rs = np.random.default_rng(13)
    ct = rand_ct(tiny, rs, 2, 3)
    d = tiny.drop_level(ct, 2)
    assert d.data.shape == (2, 2, tiny.N) and d.scale == ct.scale
    Q2 = math.prod(tiny.q[:2])
    for p in range(2):
        for k in range(tiny.N):
            X = int(sympy.ntheory.modular.crt(tiny.q, [int(v) for v in ct.data[p, :, k]])[0])
            Y = int(sympy.ntheory.modular.crt(tiny.q[:2], [int(v) for v in d.data[p, :, k]])[0])
            assert X % Q2 == Y


def test_keygen_secret_is_uniform_ternary():
    o = OracleCtx.from_set("c1_n12")
    s = np.concatenate([o.keygen_secret(40 + i) for i in range(8)])
    vals, counts = np.unique(s, return_counts=True)
    assert list(vals) == [-1, 0, 1]
    assert np.all(np.abs(counts / len(s) - 1 / 3) < 0.01)
    assert not np.array_equal(o.keygen_secret(40), o.keygen_secret(41))
