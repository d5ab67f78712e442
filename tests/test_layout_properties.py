"""Index facts the key-switching kernels rely on, checked on the CPU over every ring
degree they run at (2^10 .. 2^16), written here from their definitions:

* the NTT-domain Galois map (position x holds the evaluation at psi^(2 brv(x) + 1); the
  automorphism X -> X^g moves it to the position whose exponent is (2 brv(x) + 1) g mod 2N)
  sends each row of N/8 consecutive positions onto one row, and each aligned pair
  (2p, 2p + 1) onto an aligned pair, possibly swapped;
* a radix-16 round's local index splits into a lane part and a register part with
  disjoint bits, so both parts can be added (and padded for LDS) separately;
* after a forward row pass whose last round covers one bit, registers 2m and 2m + 1 of a
  lane hold adjacent positions, and the lanes' pairs are consecutive."""
import random

import pytest

LOGR = 4


def brv(x, bits):
    return int(format(x, "0%db" % bits)[::-1], 2) if bits else 0


def galois_pos(x, g, logN):
    """The position the NTT-domain value at x comes from under X -> X^g."""
    N = 1 << logN
    e = (2 * brv(x, logN) + 1) * g % (2 * N)
    return brv((e - 1) // 2, logN)


def elem_local(LOGT, tau, k, blo, rho):
    fr = ((k >> rho) << LOGT) | tau
    return ((fr >> blo) << (blo + rho)) | ((k & ((1 << rho) - 1)) << blo) | (fr & ((1 << blo) - 1))


def lds_pad(g):
    return g + (g >> LOGR)


@pytest.mark.parametrize("logN", range(10, 17))
def test_galois_map_keeps_rows_and_pairs(logN):
    N, G = 1 << logN, 1 << (logN - 3)
    rng = random.Random(logN)
    for _ in range(12):
        g = rng.randrange(1, 2 * N, 2)
        perm = [galois_pos(x, g, logN) for x in range(N)]
        assert sorted(perm) == list(range(N))            # a permutation
        for r in range(8):
            assert len({perm[x] // G for x in range(r * G, (r + 1) * G)}) == 1
        for p in range(0, N, 2):
            assert perm[p] ^ 1 == perm[p + 1]
        # the inverse element gives the inverse permutation
        ginv = pow(g, -1, 2 * N)
        inv = [galois_pos(x, ginv, logN) for x in range(N)]
        assert all(inv[perm[x]] == x for x in range(0, N, 7))


@pytest.mark.parametrize("LOGG", range(7, 14))
def test_round_index_splits_into_lane_and_register_parts(LOGG):
    LOGT = LOGG - LOGR
    T = 1 << LOGT
    NR = (LOGG + LOGR - 1) // LOGR
    rounds = [(LOGG - r * LOGR - min(LOGR, LOGG - r * LOGR), min(LOGR, LOGG - r * LOGR)) for r in range(NR)]
    for blo, rho in rounds:
        seen = set()
        for tau in range(T):
            for k in range(1 << LOGR):
                a, b = elem_local(LOGT, tau, 0, blo, rho), elem_local(LOGT, 0, k, blo, rho)
                full = elem_local(LOGT, tau, k, blo, rho)
                assert a & b == 0 and full == a + b
                assert lds_pad(full) == lds_pad(a) + lds_pad(b)
                assert (full >> (blo + 1)) == (a >> (blo + 1)) + (b >> (blo + 1))
                seen.add(full)
        assert seen == set(range(1 << LOGG))             # every element once per round


@pytest.mark.parametrize("LOGG", range(7, 14))
def test_forward_output_pairs(LOGG):
    LOGT = LOGG - LOGR
    NR = (LOGG + LOGR - 1) // LOGR
    RL = LOGG - (NR - 1) * LOGR
    for tau in range(1 << LOGT):
        for m in range(8):
            a = elem_local(LOGT, tau, 2 * m, 0, RL)
            assert a % 2 == 0 and elem_local(LOGT, tau, 2 * m + 1, 0, RL) == a + 1
    if RL == 1:   # a group's lanes hold consecutive pairs: 16-byte accesses coalesce
        lanes = min(64, 1 << LOGT)
        for m in range(8):
            assert [elem_local(LOGT, tau, 2 * m, 0, RL) for tau in range(lanes)] == \
                [elem_local(LOGT, 0, 2 * m, 0, RL) + 2 * tau for tau in range(lanes)]
