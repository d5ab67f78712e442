"""Writes workloads/params.json: the parameter sets (explicit prime chains) and the
discrete-Gaussian cumulative table.  Test infrastructure: run by hand,
`python -m oracle.params`; the JSON it writes is committed and is the only
place either side gets its primes from.

Prime rule (the paper fixes none; it runs HElib with m = 2^16, r = 35 and a
modulus of L bits, Sec. 4.2 "Impact of FHE parameters"):
  * every prime q satisfies q = 1 (mod 2N) so that the negacyclic NTT exists;
  * every prime is below 2^50;
  * "below(b)": scan q = c*2N + 1 downward from 2^b;
  * "near(D)": nearest such primes to D, alternating below / above, so that the
    scale drifts as little as possible across rescales.
Gaussian table: sigma = 3.2, support |e| <= 19 (6 sigma);
  cdt[i] = floor(2^64 * P(|e| <= i)) for i = 0..18 with P proportional to
  exp(-x^2 / (2 sigma^2)) on the integers of [-19, 19] (computed at 80 digits).
"""
import json
import os

import mpmath

from .ckks import is_prime_py

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(os.path.dirname(HERE), "workloads", "params.json")


def primes_below(bits, two_n, count, exclude=()):
    out = []
    c = ((1 << bits) - 2) // two_n
    while len(out) < count:
        q = c * two_n + 1
        if q < (1 << bits) and q not in exclude and is_prime_py(q):
            out.append(q)
        c -= 1
    return out


def primes_near(target, two_n, count, exclude=()):
    below, above = [], []
    c_lo = (target - 1) // two_n
    c_hi = c_lo + 1
    out = []
    while len(out) < count:
        want_below = len(out) % 2 == 0
        if want_below:
            while True:
                q = c_lo * two_n + 1
                c_lo -= 1
                if q not in exclude and is_prime_py(q):
                    out.append(q)
                    break
        else:
            while True:
                q = c_hi * two_n + 1
                c_hi += 1
                if q not in exclude and is_prime_py(q):
                    out.append(q)
                    break
    del below, above
    return out


def make_set(name, log_n, q0_bits, n_rest, rest_target_bits, n_special, special_bits, scale_bits,
             dnum, note):
    two_n = 2 << log_n
    q0 = primes_below(q0_bits, two_n, 1)
    if rest_target_bits is None:
        rest = primes_below(q0_bits, two_n, n_rest, exclude=set(q0))
    else:
        rest = primes_near(1 << rest_target_bits, two_n, n_rest, exclude=set(q0))
    q = q0 + rest
    p = primes_below(special_bits, two_n, n_special, exclude=set(q))
    return {
        "name": name, "log_n": log_n, "q": [str(x) for x in q], "p": [str(x) for x in p],
        "dnum": dnum, "scale": float(2 ** scale_bits), "note": note,
    }


def gauss_cdt(sigma=3.2, tail=19):
    mpmath.mp.dps = 80
    w = [mpmath.exp(-mpmath.mpf(x) ** 2 / (2 * mpmath.mpf(sigma) ** 2)) for x in range(tail + 1)]
    z = w[0] + 2 * sum(w[1:])
    cdt, acc = [], w[0]
    for i in range(tail):
        if i > 0:
            acc += 2 * w[i]
        cdt.append(int(mpmath.floor(acc / z * mpmath.mpf(2) ** 64)))
    return cdt


def build_all():
    sets = [
        make_set("c1_n12", 12, 40, 2, None, 1, 50, 30, 3,
                 "primitives: 3 x ~40-bit primes, 1 special ~50-bit, scale 2^30"),
        make_set("c2_n14", 14, 40, 7, 40, 2, 41, 40, 4,
                 "slot-packed CNN: 8 primes of ~40 bits (q0 below 2^40, q1..q7 nearest 2^40), 2 special "
                 "~2^41, dnum 4 (digits of 2 limbs under P ~ 2^82; log QP ~ 402 bits), scale 2^40 (scale "
                 "2^30 misses the 1e-3 logit bound: fresh noise of inputs and weights)"),
        make_set("c3_n13", 13, 45, 3, 40, 1, 46, 40, 4,
                 "uneven batch N=2^13: q0 ~2^45, 3 primes nearest 2^40, 1 special"),
        make_set("c3_n15", 15, 45, 15, 40, 4, 46, 40, 4,
                 "uneven batch N=2^15: q0 ~2^45, 15 primes nearest 2^40, 4 special, dnum 4"),
        make_set("c4_n16", 16, 50, 23, 49, 8, 50, 49, 3,
                 "key switch / deep CNN: q0 ~2^50, 23 primes nearest 2^49, 8 special, dnum 3"),
        make_set("t_n12", 12, 40, 5, 30, 2, 41, 30, 3,
                 "small CNN tests: q0 ~2^40, 5 primes nearest 2^30, 2 special ~2^41, dnum 3"),
        make_set("t4_n12", 12, 50, 10, 49, 4, 50, 49, 3,
                 "small within-image CNN tests: q0 ~2^50, 10 primes nearest 2^49, 4 special, dnum 3, "
                 "scale 2^49 (the deep-CNN chain shortened to 11 limbs)"),
        make_set("p_n15", 15, 50, 15, 40, 4, 50, 40, 4,
                 "the paper's ring (m = 2^16): q0 ~2^50, 15 primes nearest 2^40, 4 special"),
    ]
    return {"sigma": 3.2, "gauss_tail": 19, "cdt": [str(x) for x in gauss_cdt()],
            "sets": {s["name"]: s for s in sets}}


if __name__ == "__main__":
    data = build_all()
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1)
    print("wrote", OUT)
