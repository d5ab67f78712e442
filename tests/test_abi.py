"""The C ABI library loads and exports every symbol declared in include/fhe.h, and
refuses invalid parameter sets on the host (no compute calls: this runs without a
GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "fhe.h")).read()
    return sorted(set(re.findall(r"^(?:fhe_status|void|const char \*|uint32_t|uint64_t|size_t)\s*\*?(fhe_\w+)\(",
                                 src, re.M)))


def test_header_declares_entry_points():
    names = declared()
    assert len(names) >= 30
    assert {"fhe_ctx_create", "fhe_keyswitch", "fhe_rotate", "fhe_relin", "fhe_rescale", "fhe_mul_acc"} <= set(names)


def test_library_exports_every_declared_symbol():
    path = os.path.join(ROOT, "paper_2102_00319_amd", "libfhe.so")
    if not os.path.exists(path):
        import paper_2102_00319_amd.build as b
        b.build()
    lib = ctypes.CDLL(path)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2102_00319_amd import fhe
    assert set(declared()) <= set(fhe.exported_symbols())


def _create(fhe, log_n, q, p, dnum):
    qa = (ctypes.c_uint64 * len(q))(*q)
    pa = (ctypes.c_uint64 * max(1, len(p)))(*(p or [0]))
    prm = fhe.fhe_params(log_n, len(q), len(p), dnum, qa, pa if p else None, None, 0)
    h = ctypes.c_void_p()
    rc = fhe.lib().fhe_ctx_create(ctypes.byref(prm), None, 0, ctypes.byref(h))
    return rc, fhe.lib().fhe_last_error().decode()


def test_invalid_parameters_refused_before_any_device_call():
    """Parameter validation (the error paths of context creation) runs on the host:
    every one of these is refused with FHE_EPARAM whether or not a GPU is present."""
    from paper_2102_00319_amd import fhe
    import workloads
    s = workloads.load_params("c1_n12")
    q, p = [int(x) for x in s["q"]], [int(x) for x in s["p"]]
    cases = [
        (9, q, p, 1, "log_n"),                                  # ring degree out of range
        (12, q, p, len(q) + 1, "dnum"),                         # more digits than limbs
        (12, [q[0] + 2] + q[1:], p, 1, "modulus 0"),           # not prime / not 1 mod 2N
        (12, q, [q[0]], 1, "modulus 3"),                        # special prime repeats a q
        (12, [(1 << 50) + 8193] + q[1:], p, 1, "modulus 0"),    # above 2^50
        (13, q, p, 1, "modulus"),                               # 1 mod 2^13 but not mod 2^14
    ]
    for log_n, qq, pp, dnum, what in cases:
        rc, msg = _create(fhe, log_n, qq, pp, dnum)
        assert rc == fhe.FHE_EPARAM, (log_n, dnum, msg)
        assert what in msg, msg


def test_size_helpers_without_a_context():
    """The sizing helpers are host-only and answer 0 for a null context."""
    from paper_2102_00319_amd import fhe
    assert fhe.lib().fhe_ct_bytes(None, 24, 2) == 0
    assert fhe.lib().fhe_evk_bytes(None) == 0
