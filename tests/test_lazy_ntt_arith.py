"""The forward transform's lazy reduction (the upper butterfly input reduced on every
other stage only), emulated exactly on the CPU: integer-valued doubles with IEEE
round-to-nearest-even, the FMA's single rounding done on Python integers.  The
transform must equal the reduced one modulo q, and every intermediate must stay
below 4q (< 2^52 for q < 2^50), where the FP64 modular product stays exact."""
import json
import os
import random

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def fl(v):          # the double nearest to the integer v, as an integer
    return int(float(v))


def fma(a, b, c):   # one rounding of a*b + c
    return fl(a * b + c)


def mulmod(a, b, q, qinv):
    h = fl(a * b)
    lo = a * b - h                  # exact low part (an FMA)
    assert abs(lo) < 2 ** 53
    qt = int(round(float(h) * qinv))   # rint: round half to even
    r = fma(-qt, q, h)
    assert abs(r) < 2 ** 53
    return fl(r + lo)


def redc(x, q, qinv):
    return fma(-int(round(float(x) * qinv)), q, x)


def ntt_fwd(x, q, psi_brv, lazy):
    qinv = 1.0 / q
    n = len(x)
    x = list(x)
    worst, t, m, stage = 0, n, 1, 0
    while m < n:
        t //= 2
        for i in range(m):
            w = psi_brv[m + i]
            for j in range(2 * i * t, 2 * i * t + t):
                X = x[j] if (lazy and stage % 2 == 1) else redc(x[j], q, qinv)
                V = mulmod(x[j + t], w, q, qinv)
                x[j], x[j + t] = X + V, X - V
                worst = max(worst, abs(x[j]), abs(x[j + t]))
        m *= 2
        stage += 1
    return x, worst


def test_lazy_forward_transform_is_exact_and_bounded():
    sets = json.load(open(os.path.join(ROOT, "workloads", "params.json")))["sets"]
    q = max(int(v) for v in sets["c4_n16"]["q"] + sets["c4_n16"]["p"])   # the largest prime, just below 2^50
    assert q < 2 ** 50
    n = 256
    g = 3
    while True:
        psi = pow(g, (q - 1) // (2 * n), q)
        if pow(psi, n, q) == q - 1:
            break
        g += 1
    bits = n.bit_length() - 1
    psi_brv = [pow(psi, int(format(i, "0%db" % bits)[::-1], 2), q) for i in range(n)]
    rng = random.Random(5)
    for trial in range(4):
        # lazy inputs as a previous pass leaves them (|x| < 3.9q), and the extreme values
        a = [rng.randrange(-int(3.9 * q), int(3.9 * q)) for _ in range(n)]
        if trial == 3:
            a = [int(3.9 * q) - 1 if i % 2 else -(int(3.9 * q) - 1) for i in range(n)]
        ref, _ = ntt_fwd([v % q for v in a], q, psi_brv, False)
        got, worst = ntt_fwd(a, q, psi_brv, True)
        assert all((u - v) % q == 0 for u, v in zip(ref, got))
        assert worst < 4 * q
