"""Ragged work lists (operations at mixed levels in one launch sequence) against
the oracle's one-at-a-time operations."""
import numpy as np
import pytest

import workloads
from oracle import OracleCtx

pytestmark = pytest.mark.gpu


def _P():
    import paper_2102_00319_amd as P
    return P


def _keys(g, o, steps):
    sg = g.keygen_secret(workloads.SEED_SECRET)
    s = sg.astype(np.int64)
    pk, pko = g.keygen_pk(sg, workloads.SEED_PK), o.keygen_pk(s, workloads.SEED_PK)
    rlk, rlko = g.keygen_relin(sg, workloads.SEED_EVK), o.keygen_relin(s, workloads.SEED_EVK)
    gks = {r: g.keygen_rot(sg, r, workloads.SEED_EVK + 1 + i) for i, r in enumerate(steps)}
    gko = {r: o.keygen_rot(s, r, workloads.SEED_EVK + 1 + i) for i, r in enumerate(steps)}
    return sg, pk, pko, rlk, rlko, gks, gko


@pytest.mark.parametrize("name,levels", [("t4_n12", [2, 3, 5, 7, 9, 11, 4]), ("c1_n12", [3, 2, 3])])
def test_ragged_work_list_bit_exact(name, levels):
    P = _P()
    g, o = P.Context.from_set(name), OracleCtx.from_set(name)
    n, D = o.N // 2, o.scale
    steps = [1, -1, 5]
    sg, pk, pko, rlk, rlko, gks, gko = _keys(g, o, steps)
    ops, expect = [], []
    for j, l in enumerate(levels):
        ma, mb = workloads.slot_messages(100 + j, n), workloads.slot_messages(200 + j, n)
        a = g.encrypt(pk, g.encode(ma, scale=D, limbs=l), workloads.SEED_ENC + 2 * j)
        b = g.encrypt(pk, g.encode(mb, scale=D, limbs=l), workloads.SEED_ENC + 2 * j + 1)
        ao = o.encrypt(pko, o.encode_rns(ma, D, l), workloads.SEED_ENC + 2 * j, D)
        bo = o.encrypt(pko, o.encode_rns(mb, D, l), workloads.SEED_ENC + 2 * j + 1, D)
        m = P.BatchOp(P.fhe.OP_MUL_RELIN_RESCALE, a, rlk, b=b, out=g.new_ct(l - 1, 2))
        ops.append(m)
        mo = o.mul_relin_rescale(ao, bo, rlko)
        expect.append(mo)
        for r in steps[: 1 + j % 3]:
            ops.append(P.BatchOp(P.fhe.OP_ROTATE, m.out, gks[r], step=r))
            expect.append(o.rotate(mo, r, gko[r]))
    g.op_counts()
    outs = g.batch_run(ops)
    cnt = g.op_counts()
    assert cnt["relin"] == len(levels) and cnt["rotate"] == len(ops) - len(levels)
    for i, (x, y) in enumerate(zip(outs, expect)):
        assert np.array_equal(g.export_ct(x), y.data), "entry %d differs" % i
        assert x.scale == y.scale


def test_work_list_errors():
    P = _P()
    g = P.Context.from_set("t4_n12")
    sg = g.keygen_secret(workloads.SEED_SECRET)
    pk = g.keygen_pk(sg, workloads.SEED_PK)
    rlk = g.keygen_relin(sg, workloads.SEED_EVK)
    gk = g.keygen_rot(sg, 1, workloads.SEED_EVK + 1)
    a = g.encrypt(pk, g.encode(np.zeros(4), scale=g.scale, limbs=4), 1)
    b = g.encrypt(pk, g.encode(np.zeros(4), scale=g.scale, limbs=3), 2)
    with pytest.raises(P.FheError):   # operands at different levels
        g.batch_run([P.BatchOp(P.fhe.OP_MUL_RELIN_RESCALE, a, rlk, b=b)])
    with pytest.raises(P.FheError):   # key of another step
        g.batch_run([P.BatchOp(P.fhe.OP_ROTATE, a, gk, step=2)])
    with pytest.raises(P.FheError):   # output aliasing its own input
        g.batch_run([P.BatchOp(P.fhe.OP_ROTATE, a, gk, step=1, out=a)])
    o1 = g.new_ct(4, 2)
    with pytest.raises(P.FheError):   # two outputs overlap
        g.batch_run([P.BatchOp(P.fhe.OP_ROTATE, a, gk, step=1, out=o1), P.BatchOp(P.fhe.OP_ROTATE, a, gk, step=1, out=o1)])
