"""Encrypted CNN layers on the CPU oracle, and the FP64 plaintext network they
approximate (test infrastructure only).

Slot packing (Sec. 3 "Convolution Operator", Fig. 2): ciphertext X[c][y][x]
holds pixel (y, x) of channel c of every image in the batch, one image per
slot; weight ciphertext W[...] holds one weight replicated in every slot, i.e.
the constant polynomial round(w * scale).  A convolution output is the inner
product of Eq. (enc_conv) over the in-bounds taps of its window (zero padding
skipped), followed by relinearisation and one rescale.  Activation x^2 and
fully connected layers (Sec. 2.3, Z = f(WX), no bias) follow the same pattern.
"""
import numpy as np

from . import ckks


# ------------------------------------------------------------ FP64 network
def conv2d_fp64(x, w, stride, pad_t, pad_l, Ho, Wo):
    """x: [B][Cin][H][W], w: [Cout][Cin][kh][kw] -> [B][Cout][Ho][Wo] (zero padding)."""
    B, Cin, H, W = x.shape
    Cout, _, kh, kw = w.shape
    out = np.zeros((B, Cout, Ho, Wo))
    for co in range(Cout):
        for i in range(Ho):
            for j in range(Wo):
                acc = np.zeros(B)
                for ci in range(Cin):
                    for p in range(kh):
                        for q in range(kw):
                            y, xx = i * stride + p - pad_t, j * stride + q - pad_l
                            if 0 <= y < H and 0 <= xx < W:
                                acc += x[:, ci, y, xx] * w[co, ci, p, q]
                out[:, co, i, j] = acc
    return out


def slot_cnn_fp64(images, conv_w, fc1_w, fc2_w, stride, pad_t, pad_l, Ho, Wo):
    """conv -> x^2 -> flatten (c, y, x) -> fc1 -> x^2 -> fc2, in FP64."""
    x = images[:, None] if images.ndim == 3 else images
    h = conv2d_fp64(x, conv_w, stride, pad_t, pad_l, Ho, Wo) ** 2
    h = h.reshape(h.shape[0], -1)
    h = (h @ fc1_w.T) ** 2
    return h @ fc2_w.T


# -------------------------------------------------------- encrypted layers
class Counter:
    def __init__(self):
        self.ct_mult = self.ct_add = self.relin = self.rescale = 0


def _mac_relin_rescale(o, rlk, pairs, cnt):
    acc = o.mul_acc([a for a, _ in pairs], [b for _, b in pairs])
    cnt.ct_mult += len(pairs)
    cnt.ct_add += len(pairs) - 1
    cnt.relin += 1
    cnt.rescale += 1
    return o.rescale(o.relin(acc, rlk))


def enc_conv2d_slot(o, rlk, X, H, W, Cin, Wt, Cout, kh, kw, stride, pad_t, pad_l, Ho, Wo, cnt):
    Y = []
    for co in range(Cout):
        for i in range(Ho):
            for j in range(Wo):
                pairs = []
                for ci in range(Cin):
                    for p in range(kh):
                        for q in range(kw):
                            y, x = i * stride + p - pad_t, j * stride + q - pad_l
                            if 0 <= y < H and 0 <= x < W:
                                pairs.append((X[(ci * H + y) * W + x], Wt[((co * Cin + ci) * kh + p) * kw + q]))
                Y.append(_mac_relin_rescale(o, rlk, pairs, cnt))
    return Y


def enc_square(o, rlk, xs, cnt):
    return [_mac_relin_rescale(o, rlk, [(x, x)], cnt) for x in xs]


def enc_fc_slot(o, rlk, xs, Wt, n_out, cnt):
    n_in = len(xs)
    return [_mac_relin_rescale(o, rlk, [(xs[i], Wt[r * n_in + i]) for i in range(n_in)], cnt) for r in range(n_out)]


def encrypt_const(o, pk, value, scale, limbs, seed):
    """Weight replicated in every slot: the constant polynomial round(value * scale)."""
    coeff = np.zeros(o.N, dtype=np.int64)
    coeff[0] = int(np.rint(value * scale))
    return o.encrypt(pk, o.small_to_rns(coeff, limbs), seed, scale)


def conv_op_count(H, W, kh, kw, stride, pad_t, pad_l, Ho, Wo, Cin, Cout):
    """CT-CT multiplications of the slot convolution: one per in-bounds tap.
    Without padding and with stride 1 this is (M-P+1)(N-Q+1)PQ per channel pair
    (Sec. 3, the count after Eq. (enc_conv))."""
    n = 0
    for i in range(Ho):
        for j in range(Wo):
            for p in range(kh):
                for q in range(kw):
                    y, x = i * stride + p - pad_t, j * stride + q - pad_l
                    n += 0 <= y < H and 0 <= x < W
    return n * Cin * Cout
