"""ctypes front end of the C oracle (test infrastructure only).

Ciphertexts here are coefficient-domain numpy uint64 arrays shaped
[polys][limbs][N] together with the scale they carry (the CKKS scale
bookkeeping of Cheon-Kim-Kim-Song 2017: a product multiplies scales, a rescale
divides by the dropped prime).
"""
import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_u64p = C.POINTER(C.c_uint64)
_i64p = C.POINTER(C.c_int64)
_u32p = C.POINTER(C.c_uint32)
_dblp = C.POINTER(C.c_double)

TAG_SECRET, TAG_UNIFORM, TAG_ERROR, TAG_EPHEMERAL = 1, 2, 3, 4

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        L.or_ctx_new.restype = C.c_void_p
        L.or_ctx_new.argtypes = [C.c_uint32, _u64p, C.c_uint32, _u64p, C.c_uint32, C.c_uint32]
        L.or_ctx_free.argtypes = [C.c_void_p]
        for fn in ("or_modulus", "or_psi"):
            getattr(L, fn).restype = C.c_uint64
            getattr(L, fn).argtypes = [C.c_void_p, C.c_uint32]
        L.or_alpha.restype = C.c_uint32
        L.or_alpha.argtypes = [C.c_void_p]
        L.or_is_prime.restype = C.c_int
        L.or_is_prime.argtypes = [C.c_uint64]
        L.or_min_psi.restype = C.c_uint64
        L.or_min_psi.argtypes = [C.c_uint64, C.c_uint32]
        L.or_galois_elt.restype = C.c_uint64
        L.or_galois_elt.argtypes = [C.c_void_p, C.c_int64]
        L.or_encode.restype = C.c_int
        L.or_rescale.restype = C.c_int
        _LIB = L
    return _LIB


def _p(a, t=_u64p):
    return a.ctypes.data_as(t)


def is_prime_py(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.3e24 (first 12 prime bases)."""
    if n < 2:
        return False
    bases = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37]
    for b in bases:
        if n % b == 0:
            return n == b
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in bases:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def load_params(name=None):
    """Parameter sets written by oracle/params.py (explicit primes)."""
    from workloads import load_params as _lp
    return _lp(name)


@dataclass
class Ct:
    """Coefficient-domain ciphertext [polys][limbs][N] plus its scale."""
    data: np.ndarray
    scale: float

    @property
    def level(self):
        return self.data.shape[1]

    @property
    def polys(self):
        return self.data.shape[0]


class OracleCtx:
    def __init__(self, log_n, q, p, dnum, cdt=None):
        self.log_n = int(log_n)
        self.N = 1 << self.log_n
        self.q = [int(x) for x in q]
        self.p = [int(x) for x in p]
        self.L, self.K, self.dnum = len(self.q), len(self.p), int(dnum)
        qa = np.array(self.q, dtype=np.uint64)
        pa = np.array(self.p if self.p else [0], dtype=np.uint64)
        h = lib().or_ctx_new(self.log_n, _p(qa), self.L, _p(pa), self.K, self.dnum)
        if not h:
            raise ValueError("invalid parameter set")
        self._h = C.c_void_p(h)
        self.alpha = lib().or_alpha(self._h)
        self.cdt = np.array(cdt if cdt is not None else [], dtype=np.uint64)
        self.moduli = self.q + self.p

    @classmethod
    def from_set(cls, name):
        s = load_params(name)
        o = cls(s["log_n"], s["q"], s["p"], s["dnum"], s["cdt"])
        o.scale = s["scale"]
        return o

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _LIB is not None:
            _LIB.or_ctx_free(h)
            self._h = None

    # ------------------------------------------------------------ basics
    def psi(self, m):
        return lib().or_psi(self._h, m)

    def ntt(self, m, a):
        a = np.ascontiguousarray(a, dtype=np.uint64)
        out = np.empty(self.N, dtype=np.uint64)
        lib().or_ntt(self._h, C.c_uint32(m), _p(a), _p(out))
        return out

    def intt(self, m, a):
        a = np.ascontiguousarray(a, dtype=np.uint64)
        out = np.empty(self.N, dtype=np.uint64)
        lib().or_intt(self._h, C.c_uint32(m), _p(a), _p(out))
        return out

    def polymul(self, m, a, b):
        a = np.ascontiguousarray(a, dtype=np.uint64)
        b = np.ascontiguousarray(b, dtype=np.uint64)
        out = np.empty(self.N, dtype=np.uint64)
        lib().or_polymul(self._h, C.c_uint32(m), _p(a), _p(b), _p(out))
        return out

    def galois_elt(self, r):
        return int(lib().or_galois_elt(self._h, C.c_int64(int(r))))

    # ---------------------------------------------------------- sampling
    def sample_uniform(self, seed, tag, poly_id, modidx):
        idx = np.array(modidx, dtype=np.uint32)
        out = np.empty((len(idx), self.N), dtype=np.uint64)
        lib().or_sample_uniform(self._h, C.c_uint64(seed), C.c_uint64(tag), C.c_uint64(poly_id),
                                C.c_uint32(len(idx)), _p(idx, _u32p), _p(out))
        return out

    def sample_ternary(self, seed, tag, poly_id):
        out = np.empty(self.N, dtype=np.int64)
        lib().or_sample_ternary(self._h, C.c_uint64(seed), C.c_uint64(tag), C.c_uint64(poly_id),
                                _p(out, _i64p))
        return out

    def sample_gauss(self, seed, tag, poly_id):
        out = np.empty(self.N, dtype=np.int64)
        lib().or_sample_gauss(self._h, C.c_uint64(seed), C.c_uint64(tag), C.c_uint64(poly_id),
                              _p(self.cdt), C.c_uint32(len(self.cdt)), _p(out, _i64p))
        return out

    def small_to_rns(self, a, nlimbs=None, modidx=None):
        if modidx is None:
            modidx = list(range(self.L if nlimbs is None else nlimbs))
        idx = np.array(modidx, dtype=np.uint32)
        a = np.ascontiguousarray(a, dtype=np.int64)
        out = np.empty((len(idx), self.N), dtype=np.uint64)
        lib().or_small_to_rns(self._h, _p(a, _i64p), C.c_uint32(len(idx)), _p(idx, _u32p), _p(out))
        return out

    # --------------------------------------------------------------- keys
    def keygen_secret(self, seed):
        s = np.empty(self.N, dtype=np.int64)
        lib().or_keygen_secret(self._h, C.c_uint64(seed), _p(s, _i64p))
        return s

    def keygen_pk(self, s, seed):
        pk = np.empty((2, self.L, self.N), dtype=np.uint64)
        lib().or_keygen_pk(self._h, _p(np.ascontiguousarray(s, dtype=np.int64), _i64p), C.c_uint64(seed),
                           _p(self.cdt), C.c_uint32(len(self.cdt)), _p(pk))
        return pk

    def square_small(self, s):
        out = np.empty(self.N, dtype=np.int64)
        lib().or_square_small(self._h, _p(np.ascontiguousarray(s, dtype=np.int64), _i64p), _p(out, _i64p))
        return out

    def automorph_small(self, s, g):
        out = np.empty(self.N, dtype=np.int64)
        lib().or_automorph_small(self._h, _p(np.ascontiguousarray(s, dtype=np.int64), _i64p),
                                 C.c_uint64(g), _p(out, _i64p))
        return out

    def keygen_evk(self, s, s_from, seed):
        evk = np.empty((self.dnum, 2, self.L + self.K, self.N), dtype=np.uint64)
        lib().or_keygen_evk(self._h, _p(np.ascontiguousarray(s, dtype=np.int64), _i64p),
                            _p(np.ascontiguousarray(s_from, dtype=np.int64), _i64p), C.c_uint64(seed),
                            _p(self.cdt), C.c_uint32(len(self.cdt)), _p(evk))
        return evk

    def keygen_relin(self, s, seed):
        return self.keygen_evk(s, self.square_small(s), seed)

    def keygen_rot(self, s, r, seed):
        return self.keygen_evk(s, self.automorph_small(s, self.galois_elt(r)), seed)

    # ------------------------------------------------- encrypt / decrypt
    def encrypt(self, pk, m, seed, scale):
        m = np.ascontiguousarray(m, dtype=np.uint64)
        l = m.shape[0]
        ct = np.empty((2, l, self.N), dtype=np.uint64)
        lib().or_encrypt(self._h, _p(np.ascontiguousarray(pk)), _p(m), C.c_uint32(l), C.c_uint64(seed),
                         _p(self.cdt), C.c_uint32(len(self.cdt)), _p(ct))
        return Ct(ct, float(scale))

    def decrypt(self, ct, s):
        d = np.ascontiguousarray(ct.data)
        m = np.empty((ct.level, self.N), dtype=np.uint64)
        lib().or_decrypt(self._h, _p(d), C.c_uint32(ct.polys), C.c_uint32(ct.level),
                         _p(np.ascontiguousarray(s, dtype=np.int64), _i64p), _p(m))
        return m

    def encode(self, re, im=None, scale=None):
        re = np.ascontiguousarray(re, dtype=np.float64)
        imp = None if im is None else np.ascontiguousarray(im, dtype=np.float64)
        out = np.empty(self.N, dtype=np.int64)
        rc = lib().or_encode(self._h, _p(re, _dblp), None if imp is None else _p(imp, _dblp),
                             C.c_uint32(len(re)), C.c_double(scale), _p(out, _i64p))
        if rc != 0:
            raise OverflowError("encode: slot count or coefficient out of range")
        return out

    def decode(self, m, scale, n=None):
        m = np.ascontiguousarray(m, dtype=np.uint64)
        n = self.N // 2 if n is None else n
        re = np.empty(n, dtype=np.float64)
        im = np.empty(n, dtype=np.float64)
        lib().or_decode(self._h, _p(m), C.c_uint32(m.shape[0]), C.c_double(scale), _p(re, _dblp),
                        _p(im, _dblp), C.c_uint32(n))
        return re, im

    def encode_rns(self, re, scale, l, im=None):
        return self.small_to_rns(self.encode(re, im, scale), l)

    # ------------------------------------------------------------ ops
    def _binop(self, fn, a, b, scale):
        out = np.empty_like(a.data)
        fn(self._h, _p(np.ascontiguousarray(a.data)), _p(np.ascontiguousarray(b.data)),
           C.c_uint32(a.polys), C.c_uint32(a.level), _p(out))
        return Ct(out, scale)

    def add(self, a, b):
        return self._binop(lib().or_add, a, b, a.scale)

    def sub(self, a, b):
        return self._binop(lib().or_sub, a, b, a.scale)

    def add_pt(self, ct, pt):
        out = np.empty_like(ct.data)
        lib().or_add_pt(self._h, _p(np.ascontiguousarray(ct.data)), _p(np.ascontiguousarray(pt, dtype=np.uint64)),
                        C.c_uint32(ct.level), _p(out))
        return Ct(out, ct.scale)

    def mul_pt(self, ct, pt, pt_scale):
        out = np.empty_like(ct.data)
        lib().or_mul_pt(self._h, _p(np.ascontiguousarray(ct.data)), _p(np.ascontiguousarray(pt, dtype=np.uint64)),
                        C.c_uint32(ct.level), _p(out))
        return Ct(out, ct.scale * pt_scale)

    def mul_const(self, ct, const_int, const_scale=1.0):
        """Multiply by an integer constant (reduced per limb)."""
        res = np.array([int(const_int) % q for q in self.q[:ct.level]], dtype=np.uint64)
        out = np.empty_like(ct.data)
        lib().or_mul_const(self._h, _p(np.ascontiguousarray(ct.data)), C.c_uint32(ct.polys),
                           C.c_uint32(ct.level), _p(res), _p(out))
        return Ct(out, ct.scale * const_scale)

    def tensor(self, a, b):
        out = np.empty((3, a.level, self.N), dtype=np.uint64)
        lib().or_tensor(self._h, _p(np.ascontiguousarray(a.data)), _p(np.ascontiguousarray(b.data)),
                        C.c_uint32(a.level), _p(out))
        return Ct(out, a.scale * b.scale)

    def mul_acc(self, alist, blist):
        n = len(alist)
        l = alist[0].level
        keep = [np.ascontiguousarray(x.data) for x in alist] + [np.ascontiguousarray(x.data) for x in blist]
        pa = (_u64p * n)(*[_p(x) for x in keep[:n]])
        pb = (_u64p * n)(*[_p(x) for x in keep[n:]])
        out = np.empty((3, l, self.N), dtype=np.uint64)
        lib().or_mul_acc(self._h, pa, pb, C.c_uint32(n), C.c_uint32(l), _p(out))
        return Ct(out, alist[0].scale * blist[0].scale)

    def bconv(self, x, src, dst):
        x = np.ascontiguousarray(x, dtype=np.uint64)
        s = np.array(src, dtype=np.uint32)
        d = np.array(dst, dtype=np.uint32)
        y = np.empty((len(d), self.N), dtype=np.uint64)
        lib().or_bconv(self._h, _p(x), _p(s, _u32p), C.c_uint32(len(s)), _p(d, _u32p), C.c_uint32(len(d)), _p(y))
        return y

    def keyswitch(self, d, evk):
        d = np.ascontiguousarray(d, dtype=np.uint64)
        l = d.shape[0]
        ks = np.empty((2, l, self.N), dtype=np.uint64)
        lib().or_keyswitch(self._h, _p(d), C.c_uint32(l), _p(np.ascontiguousarray(evk)), _p(ks))
        return ks

    def keyswitch_galois(self, d, evk, g):
        """Key switch of sigma_g(d) in the form rotations use: d's digits extended,
        then every extended limb mapped by X -> X^g (see or_keyswitch_galois)."""
        d = np.ascontiguousarray(d, dtype=np.uint64)
        l = d.shape[0]
        ks = np.empty((2, l, self.N), dtype=np.uint64)
        lib().or_keyswitch_galois(self._h, _p(d), C.c_uint32(l), _p(np.ascontiguousarray(evk)), C.c_uint64(int(g)),
                                  _p(ks))
        return ks

    def relin(self, ct3, rlk):
        out = np.empty((2, ct3.level, self.N), dtype=np.uint64)
        lib().or_relin(self._h, _p(np.ascontiguousarray(ct3.data)), C.c_uint32(ct3.level),
                       _p(np.ascontiguousarray(rlk)), _p(out))
        return Ct(out, ct3.scale)

    def rescale(self, ct):
        l = ct.level
        if l < 2:
            raise ValueError("rescale at level 1")
        out = np.empty((ct.polys, l - 1, self.N), dtype=np.uint64)
        lib().or_rescale(self._h, _p(np.ascontiguousarray(ct.data)), C.c_uint32(ct.polys), C.c_uint32(l), _p(out))
        return Ct(out, ct.scale / float(self.q[l - 1]))

    def drop_level(self, ct, l):
        return Ct(np.ascontiguousarray(ct.data[:, :l]), ct.scale)

    def automorph(self, a, g):
        a = np.ascontiguousarray(a, dtype=np.uint64)
        out = np.empty_like(a)
        lib().or_automorph(self._h, _p(a), C.c_uint32(a.shape[0]), C.c_uint64(g), _p(out))
        return out

    def rotate(self, ct, r, gk):
        out = np.empty_like(ct.data)
        lib().or_rotate(self._h, _p(np.ascontiguousarray(ct.data)), C.c_uint32(ct.level), C.c_int64(int(r)),
                        _p(np.ascontiguousarray(gk)), _p(out))
        return Ct(out, ct.scale)

    def mul_relin_rescale(self, a, b, rlk):
        return self.rescale(self.relin(self.tensor(a, b), rlk))
