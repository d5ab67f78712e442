"""Python binding of libfhe.so (include/fhe.h): argument marshalling only.

Every computation runs in the HIP library; torch provides device memory (int64
tensors used as raw 64-bit residue storage) and the current HIP stream.  If
the library is missing this module raises at import time: there is no CPU
fallback.
"""
import atexit
import ctypes as C
import os
import weakref

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfhe.so")

FHE_OK, FHE_EINVAL, FHE_ELEVEL, FHE_ESCALE, FHE_ENOKEY, FHE_EPARAM, FHE_ENOMEM, FHE_EDEVICE = 0, -1, -2, -3, -4, -5, -6, -7
_NAMES = {-1: "EINVAL", -2: "ELEVEL", -3: "ESCALE", -4: "ENOKEY", -5: "EPARAM", -6: "ENOMEM", -7: "EDEVICE"}


class FheError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("FHE_%s: %s" % (_NAMES.get(code, str(code)), msg))
        self.code = code


class fhe_params(C.Structure):
    _fields_ = [("log_n", C.c_uint32), ("n_q", C.c_uint32), ("n_p", C.c_uint32), ("dnum", C.c_uint32),
                ("q", C.POINTER(C.c_uint64)), ("p", C.POINTER(C.c_uint64)), ("cdt", C.POINTER(C.c_uint64)),
                ("n_cdt", C.c_uint32)]


class fhe_ct(C.Structure):
    _fields_ = [("d", C.c_void_p), ("limbs", C.c_uint32), ("polys", C.c_uint32), ("scale", C.c_double)]


class fhe_pt(C.Structure):
    _fields_ = [("d", C.c_void_p), ("limbs", C.c_uint32), ("scale", C.c_double)]


class fhe_evk(C.Structure):
    _fields_ = [("d", C.c_void_p), ("galois", C.c_uint64)]


class fhe_op(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("step", C.c_int32), ("a", C.POINTER(fhe_ct)), ("b", C.POINTER(fhe_ct)),
                ("key", C.POINTER(fhe_evk)), ("out", C.POINTER(fhe_ct))]


OP_MUL_RELIN_RESCALE, OP_ROTATE = 1, 2


class BatchOp:
    """One entry of a work list for Context.batch_run: kind OP_MUL_RELIN_RESCALE
    (a, b, key = relinearisation key) or OP_ROTATE (a, step, key = Galois key);
    out is allocated when None.  a (and b) may be the out of an earlier entry."""

    def __init__(self, kind, a, key, b=None, step=0, out=None):
        self.kind, self.a, self.b, self.key, self.step, self.out = kind, a, b, key, int(step), out


if not os.path.exists(LIB_PATH):
    raise ImportError("libfhe.so is not built (run paper_2102_00319_amd/build.py or __graft_entry__.build())")
_lib = C.CDLL(LIB_PATH)

_P = C.c_void_p
_sig = {
    "fhe_ctx_create": [C.POINTER(fhe_params), _P, C.c_uint64, C.POINTER(_P)],
    "fhe_set_stream": [_P, _P],
    "fhe_ntt": [_P, _P, C.c_uint32, _P], "fhe_intt": [_P, _P, C.c_uint32, _P],
    "fhe_export_limbs": [_P, _P, C.c_uint32, _P, _P], "fhe_import_limbs": [_P, _P, C.c_uint32, _P, _P],
    "fhe_keygen_secret": [_P, C.c_uint64, _P],
    "fhe_keygen_pk": [_P, _P, C.c_uint64, C.POINTER(fhe_ct)],
    "fhe_keygen_relin": [_P, _P, C.c_uint64, C.POINTER(fhe_evk)],
    "fhe_keygen_rot": [_P, _P, C.c_int32, C.c_uint64, C.POINTER(fhe_evk)],
    "fhe_encode": [_P, _P, _P, C.c_uint32, C.c_double, C.POINTER(fhe_pt)],
    "fhe_encode_coeffs": [_P, _P, C.POINTER(fhe_pt)],
    "fhe_encrypt": [_P, C.POINTER(fhe_ct), C.POINTER(fhe_pt), C.c_uint64, C.POINTER(fhe_ct)],
    "fhe_decrypt": [_P, _P, C.POINTER(fhe_ct), C.POINTER(fhe_pt)],
    "fhe_decode": [_P, C.POINTER(fhe_pt), _P, _P, C.c_uint32],
    "fhe_add": [_P, C.POINTER(fhe_ct), C.POINTER(fhe_ct), C.POINTER(fhe_ct)],
    "fhe_sub": [_P, C.POINTER(fhe_ct), C.POINTER(fhe_ct), C.POINTER(fhe_ct)],
    "fhe_add_pt": [_P, C.POINTER(fhe_ct), C.POINTER(fhe_pt), C.POINTER(fhe_ct)],
    "fhe_mul_pt": [_P, C.POINTER(fhe_ct), C.POINTER(fhe_pt), C.POINTER(fhe_ct)],
    "fhe_mul_const": [_P, C.POINTER(fhe_ct), C.c_double, C.c_double, C.POINTER(fhe_ct)],
    "fhe_mul": [_P, C.POINTER(fhe_ct), C.POINTER(fhe_ct), C.POINTER(fhe_ct)],
    "fhe_mul_acc": [_P, C.POINTER(fhe_ct), C.POINTER(fhe_ct), C.c_uint32, C.POINTER(fhe_ct)],
    "fhe_relin": [_P, C.POINTER(fhe_evk), C.POINTER(fhe_ct), C.POINTER(fhe_ct)],
    "fhe_rescale": [_P, C.POINTER(fhe_ct), C.POINTER(fhe_ct)],
    "fhe_drop_level": [_P, C.POINTER(fhe_ct), C.c_uint32, C.POINTER(fhe_ct)],
    "fhe_rotate": [_P, C.POINTER(fhe_evk), C.POINTER(fhe_ct), C.c_int32, C.POINTER(fhe_ct)],
    "fhe_keyswitch": [_P, C.POINTER(fhe_evk), _P, C.c_uint32, C.POINTER(fhe_ct)],
    "fhe_keyswitch_batch": [_P, C.POINTER(fhe_evk), _P, C.c_uint32, C.c_uint32, C.POINTER(fhe_ct)],
    "fhe_keyswitch_batch_static": [_P, C.POINTER(fhe_evk), _P, C.c_uint32, C.c_uint32, C.POINTER(fhe_ct)],
    "fhe_ctx_set_allocator": [_P, _P, _P, _P],
    "fhe_ctx_release_buffers": [_P],
    "fhe_rotate_batch": [_P, C.POINTER(fhe_evk), C.POINTER(fhe_ct), _P, C.c_uint32, C.POINTER(fhe_ct)],
    "fhe_profile_enable": [_P, C.c_char_p],
    "fhe_op_counts": [_P, _P],
    "fhe_relin_batch": [_P, C.POINTER(fhe_evk), C.POINTER(fhe_ct), C.c_uint32, C.POINTER(fhe_ct)],
    "fhe_rescale_batch": [_P, C.POINTER(fhe_ct), C.c_uint32, C.POINTER(fhe_ct)],
    "fhe_conv2d_slot": [_P, C.POINTER(fhe_evk), C.POINTER(fhe_ct), C.c_uint32, C.c_uint32, C.c_uint32,
                        C.POINTER(fhe_ct), C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                        C.c_uint32, C.c_uint32, C.POINTER(fhe_ct)],
    "fhe_fc_slot": [_P, C.POINTER(fhe_evk), C.POINTER(fhe_ct), C.c_uint32, C.POINTER(fhe_ct), C.c_uint32,
                    C.POINTER(fhe_ct)],
    "fhe_square_act": [_P, C.POINTER(fhe_evk), C.POINTER(fhe_ct), C.c_uint32, C.POINTER(fhe_ct)],
    "fhe_encrypt_const_batch": [_P, C.POINTER(fhe_ct), _P, C.c_uint32, C.c_double, _P, C.POINTER(fhe_ct)],
    "fhe_profile_read": [_P, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_uint64)],
    "fhe_add_const": [_P, C.POINTER(fhe_ct), C.c_double, C.POINTER(fhe_ct)],
    "fhe_decode_slots": [_P, C.POINTER(fhe_pt), _P, C.c_uint32, _P, _P],
    "fhe_pool2x2_sum_slot": [_P, C.POINTER(fhe_ct), C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(fhe_ct)],
    "fhe_conv2d_packed_pw": [_P, C.POINTER(fhe_evk), C.c_uint32, C.POINTER(fhe_ct), C.c_uint32, _P, C.c_uint32,
                             C.c_uint32, C.c_uint32, C.c_uint32, C.c_double, C.POINTER(fhe_ct)],
    "fhe_fc_packed_pw": [_P, C.POINTER(fhe_evk), C.c_uint32, C.POINTER(fhe_ct), C.c_uint32, C.POINTER(fhe_pt),
                         C.c_uint32, C.c_uint32, C.POINTER(fhe_ct)],
    "fhe_batch_run": [_P, C.POINTER(fhe_op), C.c_uint32],
    "fhe_graph_begin": [_P, C.c_uint32, C.c_uint64, C.POINTER(_P)],
    "fhe_graph_end": [_P, C.c_uint32, _P],
    "fhe_graph_launch": [_P, _P],
    "fhe_ctx_set_tuning": [_P, C.c_char_p, C.c_uint64],
    "fhe_conv2d_packed": [_P, C.POINTER(fhe_evk), C.POINTER(fhe_evk), C.c_uint32, C.POINTER(fhe_ct), C.c_uint32,
                          C.POINTER(fhe_ct), C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(fhe_ct)],
    "fhe_poly_act": [_P, C.POINTER(fhe_evk), C.POINTER(fhe_ct), C.c_uint32, C.POINTER(C.c_double), C.c_uint32,
                     C.POINTER(fhe_ct)],
    "fhe_avgpool2x2": [_P, C.POINTER(fhe_evk), C.c_uint32, C.POINTER(fhe_ct), C.c_uint32, C.c_uint32, C.c_uint32,
                       C.POINTER(fhe_pt), C.POINTER(fhe_ct)],
    "fhe_fc_packed": [_P, C.POINTER(fhe_evk), C.POINTER(fhe_evk), C.c_uint32, C.POINTER(fhe_ct), C.c_uint32,
                      C.POINTER(fhe_ct), C.c_uint32, C.c_uint32, C.POINTER(fhe_ct)],
}
for _n, _a in _sig.items():
    getattr(_lib, _n).argtypes = _a
    getattr(_lib, _n).restype = C.c_int32
_lib.fhe_ctx_destroy.argtypes = [_P]
_lib.fhe_ctx_destroy.restype = None
_lib.fhe_last_error.restype = C.c_char_p
_lib.fhe_graph_destroy.argtypes = [_P]
_lib.fhe_graph_destroy.restype = None
for _n, _r in [("fhe_ring_degree", C.c_uint32), ("fhe_modulus", C.c_uint64), ("fhe_evk_bytes", C.c_size_t),
               ("fhe_ct_bytes", C.c_size_t),
               ("fhe_galois_elt", C.c_uint64), ("fhe_scratch_bytes", C.c_uint64), ("fhe_workspace_bytes", C.c_uint64)]:
    getattr(_lib, _n).restype = _r
_lib.fhe_workspace_bytes.argtypes = [_P]
_lib.fhe_ring_degree.argtypes = [_P]
_lib.fhe_modulus.argtypes = [_P, C.c_uint32]
_lib.fhe_evk_bytes.argtypes = [_P]
_lib.fhe_ct_bytes.argtypes = [_P, C.c_uint32, C.c_uint32]
_lib.fhe_galois_elt.argtypes = [_P, C.c_int32]
_lib.fhe_scratch_bytes.argtypes = [_P]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
# contexts whose buffers come from torch: closed before the interpreter tears torch down
_TORCH_ALLOC_CTXS = weakref.WeakSet()


@atexit.register
def _close_torch_alloc_ctxs():
    for ctx in list(_TORCH_ALLOC_CTXS):
        ctx.close()


def lib():
    return _lib


def exported_symbols():
    return sorted(_sig) + ["fhe_ctx_destroy", "fhe_last_error", "fhe_ring_degree", "fhe_modulus", "fhe_evk_bytes",
                           "fhe_ct_bytes",
                           "fhe_galois_elt", "fhe_scratch_bytes", "fhe_workspace_bytes", "fhe_graph_destroy"]


def _check(rc):
    if rc != FHE_OK:
        raise FheError(rc, _lib.fhe_last_error().decode())


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Ciphertext:
    """Device ciphertext [polys][limbs][N] (int64 storage of 64-bit residues) and its scale."""

    def __init__(self, data, scale):
        self.data = data
        self.scale = float(scale)

    @property
    def polys(self):
        return self.data.shape[0]

    @property
    def limbs(self):
        return self.data.shape[1]

    def s(self):
        return fhe_ct(self.data.data_ptr(), self.limbs, self.polys, self.scale)


class CtArray:
    """Ciphertexts whose C descriptor array is built once (model weights, reused by every
    forward pass: building 10^5 descriptors in Python costs ~0.1 s per call).  Behaves
    like a read-only list.  The descriptors hold device addresses: after moving the
    ciphertexts' data (eviction to host and back), call refresh(); a layer call checks
    the first and last address and raises FheError when they are stale."""

    def __init__(self, cts):
        self.cts = list(cts)
        self.refresh()

    def refresh(self):
        self.arr = (fhe_ct * len(self.cts))(*[x.s() for x in self.cts])

    def check(self):
        if self.cts and (self.arr[0].d != self.cts[0].data.data_ptr() or
                         self.arr[len(self.cts) - 1].d != self.cts[-1].data.data_ptr()):
            raise FheError(-1, "packed ciphertext array is stale: refresh() it after moving its data")

    def __len__(self):
        return len(self.cts)

    def __getitem__(self, i):
        return self.cts[i]

    def __iter__(self):
        return iter(self.cts)

    def __add__(self, other):
        return self.cts + list(other)

    def __radd__(self, other):
        return list(other) + self.cts


class Plaintext:
    def __init__(self, data, scale):
        self.data = data
        self.scale = float(scale)

    @property
    def limbs(self):
        return self.data.shape[0]

    def s(self):
        return fhe_pt(self.data.data_ptr(), self.limbs, self.scale)


class EvalKey:
    def __init__(self, data, galois):
        self.data = data
        self.galois = int(galois)

    def s(self):
        return fhe_evk(self.data.data_ptr(), self.galois)


class Context:
    """A parameter set on the current GPU; wraps fhe_ctx."""

    def __init__(self, log_n, q, p, dnum, cdt, scale=None, device="cuda", hbm_budget=0, stream=None):
        self.device = torch.device(device)
        self.log_n, self.N = int(log_n), 1 << int(log_n)
        self.q, self.p = [int(x) for x in q], [int(x) for x in p]
        self.L, self.K, self.dnum = len(self.q), len(self.p), int(dnum)
        self.scale = scale
        self._qa = np.array(self.q, dtype=np.uint64)
        self._pa = np.array(self.p if self.p else [0], dtype=np.uint64)
        self._ca = np.array(cdt if len(cdt) else [0], dtype=np.uint64)
        prm = fhe_params(self.log_n, self.L, self.K, self.dnum, self._qa.ctypes.data_as(C.POINTER(C.c_uint64)),
                         self._pa.ctypes.data_as(C.POINTER(C.c_uint64)),
                         self._ca.ctypes.data_as(C.POINTER(C.c_uint64)), len(cdt))
        with torch.cuda.device(self.device):
            st = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.stream = st
            h = C.c_void_p()
            _check(_lib.fhe_ctx_create(C.byref(prm), C.c_void_p(st.cuda_stream), int(hbm_budget), C.byref(h)))
        self._h = h
        self.alpha = (self.L + self.dnum - 1) // self.dnum
        self._kept = None      # list receiving every buffer empty() allocates, when set

    @classmethod
    def from_set(cls, name, **kw):
        import workloads
        s = workloads.load_params(name)
        return cls(s["log_n"], s["q"], s["p"], s["dnum"], s["cdt"], scale=s["scale"], **kw)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.fhe_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------- allocation
    def empty(self, *shape):
        # allocate on the context's stream, so that the caching allocator orders
        # the reuse of freed blocks after this stream's kernels
        if self.stream == torch.cuda.current_stream(self.device):
            t = torch.empty(shape, dtype=torch.int64, device=self.device)
        else:
            with torch.cuda.stream(self.stream):
                t = torch.empty(shape, dtype=torch.int64, device=self.device)
        if self._kept is not None:
            self._kept.append(t)
        return t

    def keep_allocations(self, kept):
        """From now on every buffer this context allocates is also appended to `kept`
        (None stops): a captured launch sequence must find its intermediates where the
        capture put them, so none may return to torch's cache while the graph lives."""
        self._kept = kept

    def use_stream(self, stream):
        """Enqueue this context's work on another torch stream from now on."""
        torch.cuda.synchronize(self.device)
        _check(_lib.fhe_set_stream(self._h, C.c_void_p(stream.cuda_stream)))
        self.stream = stream

    def new_ct(self, limbs, polys=2, scale=1.0):
        return Ciphertext(self.empty(polys, limbs, self.N), scale)

    def new_pt(self, limbs, scale=1.0):
        return Plaintext(self.empty(limbs, self.N), scale)

    def new_evk(self):
        return EvalKey(self.empty(self.dnum, 2, self.L + self.K, self.N), 0)

    def set_tuning(self, key, value):
        _check(_lib.fhe_ctx_set_tuning(self._h, key.encode(), int(value)))

    def galois_elt(self, step):
        return int(_lib.fhe_galois_elt(self._h, int(step)))

    def scratch_bytes(self):
        return int(_lib.fhe_scratch_bytes(self._h))

    def library_bytes(self):
        """Device memory the context's growable buffers hold (scratch and layer workspace)."""
        return int(_lib.fhe_scratch_bytes(self._h)) + int(_lib.fhe_workspace_bytes(self._h))

    def release_buffers(self):
        """Give back the context's scratch and layer workspace (fhe_ctx_release_buffers)."""
        _check(_lib.fhe_ctx_release_buffers(self._h))

    def use_torch_allocator(self):
        """Take the context's scratch and layer workspace from torch's caching allocator
        (fhe_ctx_set_allocator), on the context's stream: the library's memory then shares
        torch's cache and its accounting.  A refused allocation fails the call that needed
        it (FHE_ENOMEM) before any work."""
        dev = self.device.index if self.device.index is not None else torch.cuda.current_device()
        me = weakref.ref(self)

        def alloc(nbytes, hip_stream, user):
            ctx = me()
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev, ctx.stream if ctx else None)
            except torch.OutOfMemoryError:
                return None

        def free(ptr, user):
            torch.cuda.caching_allocator_delete(ptr)

        self._alloc_cbs = (_ALLOC_FN(alloc), _FREE_FN(free))   # kept alive with the context
        _check(_lib.fhe_ctx_set_allocator(self._h, C.cast(self._alloc_cbs[0], C.c_void_p),
                                          C.cast(self._alloc_cbs[1], C.c_void_p), None))
        _TORCH_ALLOC_CTXS.add(self)

    # ---------------------------------------------------- limbs / IO
    @staticmethod
    def _mods(modidx):
        return np.ascontiguousarray(np.array(modidx, dtype=np.uint32))

    def ntt(self, t, modidx):
        m = self._mods(modidx)
        _check(_lib.fhe_ntt(self._h, _ptr(t), len(m), m.ctypes.data_as(C.c_void_p)))

    def intt(self, t, modidx):
        m = self._mods(modidx)
        _check(_lib.fhe_intt(self._h, _ptr(t), len(m), m.ctypes.data_as(C.c_void_p)))

    def export_limbs(self, t, modidx):
        m = self._mods(modidx)
        out = np.empty((len(m), self.N), dtype=np.uint64)
        flat = t.view(-1)
        for a in range(0, len(m), 128):          # the C call takes at most 128 limbs
            mm = np.ascontiguousarray(m[a:a + 128])
            _check(_lib.fhe_export_limbs(self._h, C.c_void_p(flat[a * self.N:].data_ptr()), len(mm),
                                         mm.ctypes.data_as(C.c_void_p), out[a:a + 128].ctypes.data_as(C.c_void_p)))
        return out

    def import_limbs(self, arr, modidx, out=None):
        m = self._mods(modidx)
        a = np.ascontiguousarray(np.asarray(arr, dtype=np.uint64).reshape(len(m), self.N))
        if out is None:
            out = self.empty(len(m), self.N)
        flat = out.view(-1)
        for s in range(0, len(m), 128):
            mm = np.ascontiguousarray(m[s:s + 128])
            part = np.ascontiguousarray(a[s:s + 128])
            _check(_lib.fhe_import_limbs(self._h, part.ctypes.data_as(C.c_void_p), len(mm),
                                         mm.ctypes.data_as(C.c_void_p), C.c_void_p(flat[s * self.N:].data_ptr())))
        return out

    def export_ct(self, ct):
        """Canonical coefficient-domain residues [polys][limbs][N] (numpy uint64)."""
        mods = list(range(ct.limbs)) * ct.polys
        return self.export_limbs(ct.data, mods).reshape(ct.polys, ct.limbs, self.N)

    def import_ct(self, arr, scale):
        arr = np.asarray(arr, dtype=np.uint64)
        polys, limbs = arr.shape[0], arr.shape[1]
        t = self.import_limbs(arr.reshape(-1, self.N), list(range(limbs)) * polys).view(polys, limbs, self.N)
        return Ciphertext(t, scale)

    def import_evk(self, arr, galois=0):
        M = self.L + self.K
        t = self.import_limbs(np.asarray(arr).reshape(-1, self.N), list(range(M)) * (2 * self.dnum))
        return EvalKey(t.view(self.dnum, 2, M, self.N), galois)

    def export_evk(self, evk):
        M = self.L + self.K
        return self.export_limbs(evk.data, list(range(M)) * (2 * self.dnum)).reshape(self.dnum, 2, M, self.N)

    # ---------------------------------------------------------- client
    def keygen_secret(self, seed):
        s = np.empty(self.N, dtype=np.int8)
        _check(_lib.fhe_keygen_secret(self._h, int(seed), s.ctypes.data_as(C.c_void_p)))
        return s

    def keygen_pk(self, s, seed):
        s = np.ascontiguousarray(s, dtype=np.int8)
        pk = self.new_ct(self.L, 2, 0.0)
        st = pk.s()
        _check(_lib.fhe_keygen_pk(self._h, s.ctypes.data_as(C.c_void_p), int(seed), C.byref(st)))
        return pk

    def keygen_relin(self, s, seed):
        s = np.ascontiguousarray(s, dtype=np.int8)
        k = self.new_evk()
        st = k.s()
        _check(_lib.fhe_keygen_relin(self._h, s.ctypes.data_as(C.c_void_p), int(seed), C.byref(st)))
        k.galois = st.galois
        return k

    def keygen_rot(self, s, step, seed):
        s = np.ascontiguousarray(s, dtype=np.int8)
        k = self.new_evk()
        st = k.s()
        _check(_lib.fhe_keygen_rot(self._h, s.ctypes.data_as(C.c_void_p), int(step), int(seed), C.byref(st)))
        k.galois = st.galois
        return k

    def encode(self, re, im=None, scale=None, limbs=None):
        re = np.ascontiguousarray(re, dtype=np.float64)
        imv = None if im is None else np.ascontiguousarray(im, dtype=np.float64)
        pt = self.new_pt(self.L if limbs is None else limbs, scale if scale is not None else self.scale)
        st = pt.s()
        _check(_lib.fhe_encode(self._h, re.ctypes.data_as(C.c_void_p),
                               None if imv is None else imv.ctypes.data_as(C.c_void_p), len(re), float(pt.scale),
                               C.byref(st)))
        return pt

    def encode_coeffs(self, coeff, scale, limbs=None):
        coeff = np.ascontiguousarray(coeff, dtype=np.int64)
        pt = self.new_pt(self.L if limbs is None else limbs, scale)
        st = pt.s()
        _check(_lib.fhe_encode_coeffs(self._h, coeff.ctypes.data_as(C.c_void_p), C.byref(st)))
        return pt

    def encrypt(self, pk, pt, seed):
        out = self.new_ct(pt.limbs, 2, pt.scale)
        a, b, o = pk.s(), pt.s(), out.s()
        _check(_lib.fhe_encrypt(self._h, C.byref(a), C.byref(b), int(seed), C.byref(o)))
        return out

    def decrypt(self, s, ct):
        s = np.ascontiguousarray(s, dtype=np.int8)
        pt = self.new_pt(ct.limbs, ct.scale)
        a, o = ct.s(), pt.s()
        _check(_lib.fhe_decrypt(self._h, s.ctypes.data_as(C.c_void_p), C.byref(a), C.byref(o)))
        return pt

    def decode(self, pt, n=None):
        n = self.N // 2 if n is None else n
        re = np.empty(n, dtype=np.float64)
        im = np.empty(n, dtype=np.float64)
        a = pt.s()
        _check(_lib.fhe_decode(self._h, C.byref(a), re.ctypes.data_as(C.c_void_p), im.ctypes.data_as(C.c_void_p), n))
        return re, im

    def decode_slots(self, pt, slots):
        """Values of the listed slots (re, im)."""
        idx = np.ascontiguousarray(slots, dtype=np.uint32)
        n = len(idx)
        re = np.empty(n, dtype=np.float64)
        im = np.empty(n, dtype=np.float64)
        a = pt.s()
        _check(_lib.fhe_decode_slots(self._h, C.byref(a), idx.ctypes.data_as(C.c_void_p), n,
                                     re.ctypes.data_as(C.c_void_p), im.ctypes.data_as(C.c_void_p)))
        return re, im

    # ---------------------------------------------------------- server
    def _bin(self, fn, a, b, out):
        x, y, o = a.s(), b.s(), out.s()
        _check(fn(self._h, C.byref(x), C.byref(y), C.byref(o)))
        out.scale = o.scale
        return out

    def add(self, a, b, out=None):
        return self._bin(_lib.fhe_add, a, b, out or self.new_ct(a.limbs, a.polys))

    def sub(self, a, b, out=None):
        return self._bin(_lib.fhe_sub, a, b, out or self.new_ct(a.limbs, a.polys))

    def add_pt(self, a, p, out=None):
        return self._bin(_lib.fhe_add_pt, a, p, out or self.new_ct(a.limbs, a.polys))

    def mul_pt(self, a, p, out=None):
        return self._bin(_lib.fhe_mul_pt, a, p, out or self.new_ct(a.limbs, a.polys))

    def mul(self, a, b, out=None):
        return self._bin(_lib.fhe_mul, a, b, out or self.new_ct(a.limbs, 3))

    def mul_const(self, a, value, const_scale, out=None):
        out = out or self.new_ct(a.limbs, a.polys)
        x, o = a.s(), out.s()
        _check(_lib.fhe_mul_const(self._h, C.byref(x), float(value), float(const_scale), C.byref(o)))
        out.scale = o.scale
        return out

    def mul_acc(self, alist, blist, out=None):
        n = len(alist)
        A = (fhe_ct * n)(*[a.s() for a in alist])
        B = (fhe_ct * n)(*[b.s() for b in blist])
        out = out or self.new_ct(alist[0].limbs, 3)
        o = out.s()
        _check(_lib.fhe_mul_acc(self._h, A, B, n, C.byref(o)))
        out.scale = o.scale
        return out

    def relin(self, rlk, ct3, out=None):
        out = out or self.new_ct(ct3.limbs, 2)
        k, x, o = rlk.s(), ct3.s(), out.s()
        _check(_lib.fhe_relin(self._h, C.byref(k), C.byref(x), C.byref(o)))
        out.scale = o.scale
        return out

    def rescale(self, ct, out=None):
        out = out or self.new_ct(ct.limbs - 1, ct.polys)
        x, o = ct.s(), out.s()
        _check(_lib.fhe_rescale(self._h, C.byref(x), C.byref(o)))
        out.scale = o.scale
        return out

    def drop_level(self, ct, limbs):
        out = self.new_ct(limbs, ct.polys)
        x, o = ct.s(), out.s()
        _check(_lib.fhe_drop_level(self._h, C.byref(x), int(limbs), C.byref(o)))
        out.scale = o.scale
        return out

    def rotate(self, gk, ct, step, out=None):
        out = out or self.new_ct(ct.limbs, 2)
        k, x, o = gk.s(), ct.s(), out.s()
        _check(_lib.fhe_rotate(self._h, C.byref(k), C.byref(x), int(step), C.byref(o)))
        out.scale = o.scale
        return out

    def keyswitch(self, evk, d, out=None):
        limbs = d.shape[0]
        out = out or self.new_ct(limbs, 2)
        k, o = evk.s(), out.s()
        _check(_lib.fhe_keyswitch(self._h, C.byref(k), _ptr(d), limbs, C.byref(o)))
        return out

    def keyswitch_batch(self, evks, ds, outs=None):
        n = len(ds)
        limbs = ds[0].shape[0]
        outs = outs or [self.new_ct(limbs, 2) for _ in range(n)]
        K = (fhe_evk * n)(*[e.s() for e in evks])
        D = (C.c_void_p * n)(*[d.data_ptr() for d in ds])
        O = (fhe_ct * n)(*[o.s() for o in outs])
        _check(_lib.fhe_keyswitch_batch(self._h, K, D, limbs, n, O))
        return outs

    def keyswitch_batch_static(self, evks, ds, outs):
        """fhe_keyswitch_batch_static: the outputs must be allocated by the caller."""
        n = len(ds)
        limbs = ds[0].shape[0]
        K = (fhe_evk * n)(*[e.s() for e in evks])
        D = (C.c_void_p * n)(*[d.data_ptr() for d in ds])
        O = (fhe_ct * n)(*[o.s() for o in outs])
        _check(_lib.fhe_keyswitch_batch_static(self._h, K, D, limbs, n, O))
        return outs

    def rotate_batch(self, gks, cts, steps, outs=None):
        n = len(cts)
        outs = outs or [self.new_ct(cts[0].limbs, 2) for _ in range(n)]
        K = (fhe_evk * n)(*[k.s() for k in gks])
        I = (fhe_ct * n)(*[x.s() for x in cts])
        S = (C.c_int32 * n)(*[int(x) for x in steps])
        O = (fhe_ct * n)(*[o.s() for o in outs])
        _check(_lib.fhe_rotate_batch(self._h, K, I, C.cast(S, C.c_void_p), n, O))
        for i, o in enumerate(outs):
            o.scale = O[i].scale
        return outs

    # ------------------------------------------------------- measurement
    def profile_enable(self, category):
        _check(_lib.fhe_profile_enable(self._h, None if category is None else category.encode()))

    def profile_read(self, category):
        ms, cnt = C.c_double(), C.c_uint64()
        _check(_lib.fhe_profile_read(self._h, category.encode(), C.byref(ms), C.byref(cnt)))
        return ms.value, cnt.value

    # ----------------------------------------------------------- batches
    @staticmethod
    def _arr(cts):
        if isinstance(cts, CtArray):
            cts.check()
            return cts.arr
        return (fhe_ct * len(cts))(*[x.s() for x in cts])

    @staticmethod
    def _back(arr, cts):
        for i, x in enumerate(cts):
            x.scale = arr[i].scale

    def relin_batch(self, rlk, cts3, outs=None):
        outs = outs or [self.new_ct(x.limbs, 2) for x in cts3]
        k, I, O = rlk.s(), self._arr(cts3), self._arr(outs)
        _check(_lib.fhe_relin_batch(self._h, C.byref(k), I, len(cts3), O))
        self._back(O, outs)
        return outs

    def rescale_batch(self, cts, outs=None):
        outs = outs or [self.new_ct(x.limbs - 1, x.polys) for x in cts]
        I, O = self._arr(cts), self._arr(outs)
        _check(_lib.fhe_rescale_batch(self._h, I, len(cts), O))
        self._back(O, outs)
        return outs

    def op_counts(self):
        """(ct_mult, ct_add, pt_mult, pt_add, relin, rescale, rotate) since the last call."""
        out = (C.c_uint64 * 8)()
        _check(_lib.fhe_op_counts(self._h, out))
        return dict(zip(["ct_mult", "ct_add", "pt_mult", "pt_add", "relin", "rescale", "rotate"], list(out)[:7]))

    # ------------------------------------------------------------ layers
    def encrypt_const_batch(self, pk, values, scale, seeds, limbs):
        values = np.ascontiguousarray(values, dtype=np.float64).ravel()
        seeds = np.ascontiguousarray(seeds, dtype=np.uint64).ravel()
        outs = [self.new_ct(limbs, 2, scale) for _ in range(len(values))]
        O = self._arr(outs)
        _check(_lib.fhe_encrypt_const_batch(self._h, C.byref(pk.s()), values.ctypes.data_as(C.c_void_p), len(values),
                                            float(scale), seeds.ctypes.data_as(C.c_void_p), O))
        self._back(O, outs)
        return outs

    def conv2d_slot(self, rlk, X, H, W, Cin, Wt, Cout, kh, kw, stride, pad_t, pad_l, Ho, Wo):
        l = X[0].limbs
        Y = [self.new_ct(l - 1, 2) for _ in range(Cout * Ho * Wo)]
        XA, WA, YA = self._arr(X), self._arr(Wt), self._arr(Y)
        _check(_lib.fhe_conv2d_slot(self._h, C.byref(rlk.s()), XA, H, W, Cin, WA, Cout, kh, kw, stride, pad_t, pad_l,
                                    Ho, Wo, YA))
        self._back(YA, Y)
        return Y

    def fc_slot(self, rlk, x, Wt, n_out):
        l = x[0].limbs
        y = [self.new_ct(l - 1, 2) for _ in range(n_out)]
        XA, WA, YA = self._arr(x), self._arr(Wt), self._arr(y)
        _check(_lib.fhe_fc_slot(self._h, C.byref(rlk.s()), XA, len(x), WA, n_out, YA))
        self._back(YA, y)
        return y

    def pool2x2_sum_slot(self, x, C_, H, W):
        y = [self.new_ct(x[0].limbs, 2) for _ in range(C_ * (H // 2) * (W // 2))]
        XA, YA = self._arr(x), self._arr(y)
        _check(_lib.fhe_pool2x2_sum_slot(self._h, XA, C_, H, W, YA))
        self._back(YA, y)
        return y

    def square_act(self, rlk, x):
        y = [self.new_ct(v.limbs - 1, 2) for v in x]
        XA, YA = self._arr(x), self._arr(y)
        _check(_lib.fhe_square_act(self._h, C.byref(rlk.s()), XA, len(x), YA))
        self._back(YA, y)
        return y

    # -------------------------------------------- within-image packed layers
    def _keys(self, gks):
        keys = list(gks.values()) if isinstance(gks, dict) else list(gks)
        return (fhe_evk * max(1, len(keys)))(*[k.s() for k in keys]), len(keys)

    def conv2d_packed(self, rlk, gks, X, Wt, Cout, k, dilation, frame_w):
        l = X[0].limbs
        Y = [self.new_ct(l - 1, 2) for _ in range(Cout)]
        K, nk = self._keys(gks)
        XA, WA, YA = self._arr(X), self._arr(Wt), self._arr(Y)
        _check(_lib.fhe_conv2d_packed(self._h, C.byref(rlk.s()), K, nk, XA, len(X), WA, Cout, k, dilation, frame_w,
                                      YA))
        self._back(YA, Y)
        return Y

    def poly_act(self, rlk, xs, coef, deg):
        y = [self.new_ct(v.limbs - (1 if deg == 2 else 2), 2) for v in xs]
        cf = (C.c_double * 4)(*[float(v) for v in (list(coef) + [0.0] * 4)[:4]])
        XA, YA = self._arr(xs), self._arr(y)
        _check(_lib.fhe_poly_act(self._h, C.byref(rlk.s()), XA, len(xs), cf, deg, YA))
        self._back(YA, y)
        return y

    def avgpool2x2(self, gks, xs, dilation, frame_w, mask):
        y = [self.new_ct(v.limbs - 1, 2) for v in xs]
        K, nk = self._keys(gks)
        XA, YA = self._arr(xs), self._arr(y)
        m = mask.s()
        _check(_lib.fhe_avgpool2x2(self._h, K, nk, XA, len(xs), dilation, frame_w, C.byref(m), YA))
        self._back(YA, y)
        return y

    def fc_packed(self, rlk, gks, xs, Wt, n_out, frame_slots):
        l = xs[0].limbs
        y = [self.new_ct(l - 1, 2) for _ in range(n_out)]
        K, nk = self._keys(gks)
        XA, WA, YA = self._arr(xs), self._arr(Wt), self._arr(y)
        _check(_lib.fhe_fc_packed(self._h, C.byref(rlk.s()), K, nk, XA, len(xs), WA, n_out, frame_slots, YA))
        self._back(YA, y)
        return y

    def conv2d_packed_pw(self, gks, X, w, Cout, k, dilation, frame_w, wscale):
        l = X[0].limbs
        Y = [self.new_ct(l - 1, 2) for _ in range(Cout)]
        K, nk = self._keys(gks)
        wv = np.ascontiguousarray(w, dtype=np.float64).ravel()
        XA, YA = self._arr(X), self._arr(Y)
        _check(_lib.fhe_conv2d_packed_pw(self._h, K, nk, XA, len(X), wv.ctypes.data_as(C.c_void_p), Cout, k, dilation,
                                         frame_w, float(wscale), YA))
        self._back(YA, Y)
        return Y

    def fc_packed_pw(self, gks, xs, Wpt, n_out, frame_slots):
        l = xs[0].limbs
        y = [self.new_ct(l - 1, 2) for _ in range(n_out)]
        K, nk = self._keys(gks)
        WA = (fhe_pt * len(Wpt))(*[w.s() for w in Wpt])
        XA, YA = self._arr(xs), self._arr(y)
        _check(_lib.fhe_fc_packed_pw(self._h, K, nk, XA, len(xs), WA, n_out, frame_slots, YA))
        self._back(YA, y)
        return y

    def add_const(self, a, value, out=None):
        out = out or self.new_ct(a.limbs, a.polys)
        x, o = a.s(), out.s()
        _check(_lib.fhe_add_const(self._h, C.byref(x), float(value), C.byref(o)))
        out.scale = o.scale
        return out

    def batch_run(self, ops):
        """Run a work list (BatchOp entries) through fhe_batch_run; returns the outputs."""
        for op in ops:
            if op.out is None:
                lv = op.a.limbs - 1 if op.kind == OP_MUL_RELIN_RESCALE else op.a.limbs
                op.out = self.new_ct(lv, 2)
        descs, keys = {}, {}

        def d(ct):
            if id(ct) not in descs:
                descs[id(ct)] = ct.s()
            return C.pointer(descs[id(ct)])

        def k(key):
            if id(key) not in keys:
                keys[id(key)] = key.s()
            return C.pointer(keys[id(key)])
        arr = (fhe_op * max(1, len(ops)))()
        for i, op in enumerate(ops):
            arr[i].kind = op.kind
            arr[i].step = op.step
            arr[i].a = d(op.a)
            arr[i].b = d(op.b) if op.b is not None else C.POINTER(fhe_ct)()
            arr[i].key = k(op.key)
            arr[i].out = d(op.out)
        _check(_lib.fhe_batch_run(self._h, arr, len(ops)))
        for op in ops:
            op.out.scale = descs[id(op.out)].scale
        return [op.out for op in ops]

    def mul_relin_rescale(self, rlk, a, b):
        return self.rescale(self.relin(rlk, self.mul(a, b)))


class Graph:
    """A captured HIP graph over one or more contexts (fhe_graph_*)."""

    def __init__(self, handle, ctxs):
        self._h = handle
        self._ctxs = ctxs   # keep the contexts (and their device tables) alive

    def launch(self, stream=None):
        _check(_lib.fhe_graph_launch(self._h, None if stream is None else C.c_void_p(stream.cuda_stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.fhe_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def capture_graph(ctxs, fn, table_bytes=0):
    """Capture the work fn() enqueues on the contexts' streams into one graph.
    fn must only enqueue work on those contexts: outputs preallocated, scratch
    already sized by the same calls run once eagerly."""
    ctxs = list(ctxs)
    arr = (C.c_void_p * len(ctxs))(*[c._h.value for c in ctxs])
    h = C.c_void_p()
    _check(_lib.fhe_graph_begin(arr, len(ctxs), int(table_bytes), C.byref(h)))
    err = None
    try:
        fn()
    except Exception as e:   # still end the capture, then report
        err = e
    rc = _lib.fhe_graph_end(arr, len(ctxs), h)
    if err is not None:
        raise err
    _check(rc)
    return Graph(h, ctxs)
