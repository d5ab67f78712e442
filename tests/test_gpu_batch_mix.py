"""The uneven batch as benchmarked (256 jobs over N = 2^13, 2^14, 2^15, levels
uniform in 2..L, each a product with relinearisation and rescale and its 4
rotations), run as one batch by the runtime in the autotuner's configurations;
jobs at every ring degree are compared bit for bit with the oracle's
one-at-a-time operations on the same inputs."""
import numpy as np
import pytest
import torch

import workloads
from oracle import OracleCtx

pytestmark = pytest.mark.gpu


def test_uneven_mix_jobs_bit_exact():
    import paper_2102_00319_amd as P
    from paper_2102_00319_amd import runtime
    torch.cuda.set_device(0)
    spec = workloads.uneven_jobs(workloads.SEED_BATCH, 256)
    steps = workloads.UNEVEN_STEPS
    ctxs, keys, pks = {}, {}, {}
    for name in workloads.UNEVEN_SETS:
        g = P.Context.from_set(name, stream=torch.cuda.Stream())
        s = g.keygen_secret(workloads.SEED_SECRET)
        pks[name] = (g.keygen_pk(s, workloads.SEED_PK), s)
        rlk = g.keygen_relin(s, workloads.SEED_EVK)
        keys[name] = (rlk, {r: g.keygen_rot(s, r, workloads.SEED_EVK + 1 + i) for i, r in enumerate(steps)})
        ctxs[name] = g
    msgs, jobs = [], []
    for j, (name, l) in enumerate(spec):
        g, (pk, _) = ctxs[name], pks[name]
        ma = workloads.slot_messages(workloads.SEED_DATA + 2 * j, 64)
        mb = workloads.slot_messages(workloads.SEED_DATA + 2 * j + 1, 64)
        a = g.encrypt(pk, g.encode(ma, scale=g.scale, limbs=l), workloads.SEED_ENC + 2 * j)
        b = g.encrypt(pk, g.encode(mb, scale=g.scale, limbs=l), workloads.SEED_ENC + 2 * j + 1)
        msgs.append((ma, mb))
        jobs.append((name, a, b))
    ub = runtime.UnevenBatch(ctxs, keys, jobs, steps)
    # the lowest-level job of every ring degree and the highest-level one of N = 2^13
    pick = {}
    for j, (name, l) in enumerate(spec):
        if name not in pick or l < spec[pick[name]][1]:
            pick[name] = j
    hi = max((j for j, (n, _) in enumerate(spec) if n == "c3_n13"), key=lambda j: spec[j][1])
    chosen = sorted(set(pick.values()) | {hi})
    for cfg in ({"graph": False, "concurrent": True, "chunk": 0}, {"graph": True, "concurrent": True, "chunk": 0}):
        ub.run(cfg)
        torch.cuda.synchronize()
        for j in chosen:
            name, l = spec[j]
            o = OracleCtx.from_set(name)
            s = pks[name][1].astype(np.int64)
            pko = o.keygen_pk(s, workloads.SEED_PK)
            rlko = o.keygen_relin(s, workloads.SEED_EVK)
            ma, mb = msgs[j]
            ao = o.encrypt(pko, o.encode_rns(ma, o.scale, l), workloads.SEED_ENC + 2 * j, o.scale)
            bo = o.encrypt(pko, o.encode_rns(mb, o.scale, l), workloads.SEED_ENC + 2 * j + 1, o.scale)
            mo = o.mul_relin_rescale(ao, bo, rlko)
            g = ctxs[name]
            assert np.array_equal(g.export_ct(ub.products[j]), mo.data), (cfg, j, name, l)
            for i, r in enumerate(steps):
                ro = o.rotate(mo, r, o.keygen_rot(s, r, workloads.SEED_EVK + 1 + i))
                assert np.array_equal(g.export_ct(ub.rotations[j][i]), ro.data), (cfg, j, name, l, r)
    ub.close()
