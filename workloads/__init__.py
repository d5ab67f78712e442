"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no homomorphic arithmetic: it only reads the parameter file
and draws plain random numbers (messages, images, weights, residues) from
numpy generators with fixed seeds.  Both the GPU path and the CPU oracle take
their inputs from here.

Input recipe (the paper evaluates on MNIST, Sec. 4.3 "Dataset and Inference
Results"; MNIST is not available here, so same-shaped synthetic data stands in):
  * images: 28x28 single channel, pixels uniform on [0, 1];
  * weights: normal, mean 0, standard deviation 0.1;
  * slot messages for the primitive tests: uniform on [-1, 1];
  * random ring elements (key-switch inputs): uniform residues below each prime.
"""
import json
import os

import numpy as np

MASTER_SEED = 210200319
SEED_DATA = MASTER_SEED + 1
SEED_SECRET = MASTER_SEED + 2
SEED_PK = MASTER_SEED + 3
SEED_EVK = MASTER_SEED + 4          # + key index
SEED_ENC = MASTER_SEED + 1000       # + ciphertext index
SEED_BATCH = MASTER_SEED + 3000

_HERE = os.path.dirname(os.path.abspath(__file__))
PARAMS_PATH = os.path.join(_HERE, "params.json")


def load_params(name=None):
    """Parameter set `name` with integer primes and the Gaussian table, or the raw file."""
    with open(PARAMS_PATH) as f:
        data = json.load(f)
    if name is None:
        return data
    s = dict(data["sets"][name])
    s["q"] = [int(x) for x in s["q"]]
    s["p"] = [int(x) for x in s["p"]]
    s["cdt"] = [int(x) for x in data["cdt"]]
    return s


def rng(seed):
    return np.random.default_rng(int(seed))


def slot_messages(seed, n, lo=-1.0, hi=1.0):
    return rng(seed).uniform(lo, hi, size=n)


def complex_messages(seed, n, amp=1.0):
    g = rng(seed)
    return g.uniform(-amp, amp, size=n), g.uniform(-amp, amp, size=n)


def images(seed, count, h=28, w=28):
    return rng(seed).uniform(0.0, 1.0, size=(count, h, w))


def weights(seed, shape, std=0.1):
    return rng(seed).normal(0.0, std, size=shape)


def uniform_residues(seed, moduli, n):
    """[len(moduli)][n] uint64, entry (i, k) uniform in [0, moduli[i])."""
    g = rng(seed)
    out = np.empty((len(moduli), n), dtype=np.uint64)
    for i, q in enumerate(moduli):
        out[i] = g.integers(0, int(q), size=n, dtype=np.uint64)
    return out


def small_ints(seed, n, bound):
    return rng(seed).integers(-bound, bound + 1, size=n, dtype=np.int64)


# Batched uneven workload: independent jobs over three ring degrees, each job
# multiplies two fresh ciphertexts at a random level, relinearises, rescales and
# rotates the product by +1, -1, +ROW, -ROW (ROW = 28, one image row).
UNEVEN_SETS = ("c3_n13", "c2_n14", "c3_n15")
UNEVEN_ROW = 28
UNEVEN_STEPS = (1, -1, UNEVEN_ROW, -UNEVEN_ROW)


def uneven_jobs(seed=SEED_BATCH, n_jobs=256, sets=UNEVEN_SETS):
    """List of (parameter set, level) per job: set uniform over `sets`, level
    uniform in 2 .. L of that set."""
    g = rng(seed)
    Ls = [len(load_params(s)["q"]) for s in sets]
    out = []
    for _ in range(n_jobs):
        i = int(g.integers(0, len(sets)))
        out.append((sets[i], int(g.integers(2, Ls[i] + 1))))
    return out
