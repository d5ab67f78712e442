"""fhe_keyswitch_batch_static (scratch in the library's static device array, no
allocation) against fhe_keyswitch_batch on the same inputs, bit for bit: two calls
in a row, the second with a smaller batch at fewer limbs, and a batch beyond the
static array refused before anything runs."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


def _inputs(g, n, limbs, seed):
    ds = [g.import_limbs(workloads.uniform_residues(seed + b, g.q[:limbs], g.N), list(range(limbs)))
          for b in range(n)]
    return ds


@pytest.mark.parametrize("name,first,second", [("c3_n15", (6, 16), (2, 9)), ("c4_n16", (2, 24), (1, 13))])
def test_static_keyswitch_matches_the_allocating_one(name, first, second):
    import paper_2102_00319_amd as P
    torch.cuda.set_device(0)
    g = P.Context.from_set(name)
    s = g.keygen_secret(workloads.SEED_SECRET)
    keys = [g.keygen_relin(s, workloads.SEED_EVK + 7 * i) for i in range(first[0])]
    for call, (n, limbs) in enumerate([first, second]):
        ds = _inputs(g, n, limbs, 500 + 100 * call)
        ref = g.keyswitch_batch(keys[:n], ds)
        outs = [g.new_ct(limbs, 2) for _ in range(n)]
        g.keyswitch_batch_static(keys[:n], ds, outs)
        torch.cuda.synchronize()
        for a, b in zip(outs, ref):
            assert torch.equal(a.data, b.data), (name, call)
        print("%s call %d: %d key switches at %d limbs bit-exact" % (name, call, n, limbs), flush=True)


def test_static_keyswitch_refuses_a_batch_beyond_the_array():
    import paper_2102_00319_amd as P
    from paper_2102_00319_amd.fhe import FheError
    torch.cuda.set_device(0)
    g = P.Context.from_set("c4_n16")
    s = g.keygen_secret(workloads.SEED_SECRET)
    key = g.keygen_relin(s, workloads.SEED_EVK)
    ds = [g.empty(24, g.N) for _ in range(3)]     # 3 x 104 MiB of scratch > 256 MiB
    outs = [g.new_ct(24, 2) for _ in range(3)]
    with pytest.raises(FheError) as e:
        g.keyswitch_batch_static([key] * 3, ds, outs)
    assert e.value.code == -6 and "static array" in str(e.value)
