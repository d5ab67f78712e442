"""Host logic of bench.py: the algorithmic byte model of the key-switch kernels, the
one-GPU guard and the committed-counter lookup (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_inner_product_bytes_per_key_switch():
    # N = 2^16, l = 24, K = 8, dnum 3 (alpha 8): per key switch the three digits and
    # both key polynomials over 32 limbs (3 * 3 * 32) plus u over 32 limbs (2 * 32)
    limb = (1 << 16) * 8
    b, _ = bench.kernel_model("ks_inner", 1 << 16, 24, 8, 8, 8, 3, 24)
    assert b == 8 * (3 * 3 * 32 + 2 * 32) * limb == 1476395008


def test_fused_path_bytes_per_key_switch():
    """The fused path (row passes inside the inner products, uQ kept on chip, uP's inverse
    row pass inside the special-prime inner product) against the split path, in limbs
    per key switch at N = 2^16, l = 24, K = 8, dnum 3 (the rotation addend included)."""
    args = (1 << 16, 24, 8, 8, 8, 3, 24)
    limb = (1 << 16) * 8
    cats = ["ks_intt_first", "bconv_up", "ntt_fwd_row", "ks_inner", "ntt_inv_row", "bconv_down", "ks_moddown_final"]

    def limbs(fused):
        return {c: bench.kernel_model(c, *args, fused=fused)[0] // (8 * limb) for c in cats}
    f, s = limbs(True), limbs(False)
    assert f["ntt_fwd_row"] == f["ntt_inv_row"] == 0 and s["ntt_fwd_row"] == 2 * 72 and s["ntt_inv_row"] == 32
    # special primes: 3 digits of D_j, both key polynomials, uP out
    assert f["ks_inner"] == 3 * 8 + 3 * 2 * 8 + 2 * 8 == 88
    # Q limbs: 3 digits of D_j and both keys, z in, addend in, out
    assert f["ks_moddown_final"] == 3 * 3 * 24 + 2 * 24 + 24 + 2 * 24 == 336
    assert sum(f.values()) == 632 and sum(s.values()) == 48 + 96 + 144 + 352 + 32 + 64 + 168
    # the same flops for the transforms: every converted limb still gets its row pass
    fl = lambda fused, c: bench.kernel_model(c, *args, fused=fused)[1]
    assert sum(fl(True, c) for c in cats) == sum(fl(False, c) for c in cats)


def test_conversion_targets():
    # ModUp: each of the 3 digits (8 limbs) converts to the other 16 + 8 limbs
    limb = (1 << 16) * 8
    b, _ = bench.kernel_model("bconv_up", 1 << 16, 24, 8, 8, 1, 3, 24)
    assert b == (24 + 3 * 24) * limb


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_counter_lookup_needs_matching_source():
    assert bench.measured_traffic("no_such_kernel", "fused") is None
    # the committed counters are those of the fused form
    assert bench.measured_traffic("ks_moddown_final", "split") is None
    assert bench.measured_traffic("ks_moddown_final", "fused") is None   # taken with non-temporal streams


def test_source_digest_ignores_comments(tmp_path):
    a, b, c = tmp_path / "a.hip", tmp_path / "b.hip", tmp_path / "c.hip"
    a.write_text("int f(int x)\n{\n    return x + 1;\n}\n")
    b.write_text("// a comment\nint f(int x)   // trailing\n{\n\n    return x + 1;\n}\n")
    c.write_text("int f(int x)\n{\n    return x + 2;\n}\n")
    assert bench.source_digest(str(a)) == bench.source_digest(str(b)) != bench.source_digest(str(c))
