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
    """x: [B][Cin][H][W], w: [Cout][Cin][kh][kw] -> [B][Cout][Ho][Wo] (zero padding).
    out[b, co, i, j] = sum over (ci, p, q) of x[b, ci, i*stride + p - pad_t, j*stride + q - pad_l]
    * w[co, ci, p, q], taps outside the image counting as zero: the windows of a
    zero-padded copy of x, contracted with the weights by one matrix product."""
    B, Cin, H, W = x.shape
    Cout, _, kh, kw = w.shape
    pb = max(0, (Ho - 1) * stride + kh - pad_t - H)
    pr = max(0, (Wo - 1) * stride + kw - pad_l - W)
    xp = np.zeros((B, Cin, pad_t + H + pb, pad_l + W + pr))
    xp[:, :, pad_t:pad_t + H, pad_l:pad_l + W] = x
    win = np.lib.stride_tricks.sliding_window_view(xp, (kh, kw), axis=(2, 3))   # [B][Cin][y][x][p][q]
    win = win[:, :, :(Ho - 1) * stride + 1:stride, :(Wo - 1) * stride + 1:stride]
    out = np.tensordot(win, w, axes=([1, 4, 5], [1, 2, 3]))                     # [B][Ho][Wo][Cout]
    return np.ascontiguousarray(out.transpose(0, 3, 1, 2))


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
        self.rotate = self.pt_mult = self.pt_add = 0


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


# ------------------------------------------- within-image packing (deep CNN)
# A ciphertext holds one channel of a batch of images, each image in its own
# frame of frame_h x frame_w slots (row-major, zero guard to the right and
# below); image b, pixel (y, x) sits in slot b*frame_h*frame_w + y*frame_w + x.
# The slot rotation of Sec. 3 (Fig. 2 "rotation") then moves whole neighbour
# pixels: a left rotation by dy*frame_w + dx brings pixel (y+dy, x+dx) to (y, x).
def frame_pack(img, frame_h, frame_w):
    """img [B][H][W] -> slot vector of B * frame_h * frame_w values."""
    B, H, W = img.shape
    v = np.zeros((B, frame_h, frame_w))
    v[:, :H, :W] = img
    return v.ravel()


def frame_positions(H, W, frame_h, frame_w, n_frames, dil):
    """Slot indices of the valid positions (y, x) = (dil*i, dil*j), y < H, x < W, of every frame."""
    ys, xs = np.arange(0, H, dil), np.arange(0, W, dil)
    one = (ys[:, None] * frame_w + xs[None, :]).ravel()
    return (np.arange(n_frames)[:, None] * (frame_h * frame_w) + one[None, :]).ravel()


def conv2d_same_fp64(x, w):
    """Stride 1, zero padding k // 2 on every side."""
    k = w.shape[2]
    return conv2d_fp64(x, w, 1, k // 2, k // 2, x.shape[2], x.shape[3])


def poly_fp64(x, coef):
    c = list(coef) + [0.0] * (4 - len(coef))
    return c[0] + c[1] * x + c[2] * x * x + c[3] * x * x * x


def avgpool2_fp64(x):
    B, C, H, W = x.shape
    return x.reshape(B, C, H // 2, 2, W // 2, 2).mean(axis=(3, 5))


def packed_cnn_fp64(images, w1, w2, wfc, coef):
    """conv 3x3 same -> poly -> avg pool 2x2 -> conv 3x3 same -> poly -> avg pool
    -> flatten (c, y, x) -> fc, in FP64."""
    x = images[:, None] if images.ndim == 3 else images
    h = avgpool2_fp64(poly_fp64(conv2d_same_fp64(x, w1), coef))
    h = avgpool2_fp64(poly_fp64(conv2d_same_fp64(h, w2), coef))
    return h.reshape(h.shape[0], -1) @ wfc.T


def conv_steps(k, dil, frame_w):
    """Rotation step of each tap (p, q) of a k x k 'same' kernel, row-major."""
    return [dil * ((p - k // 2) * frame_w + (q - k // 2)) for p in range(k) for q in range(k)]


def add_const(o, ct, value):
    """ct + value: the constant polynomial round(value * ct.scale) added to c0.
    The integer is exact at any size (a Python int), reduced per limb."""
    m = int(np.rint(value * ct.scale))
    pt = np.zeros((ct.level, o.N), dtype=np.uint64)
    pt[:, 0] = [m % int(q) for q in o.q[:ct.level]]
    return o.add_pt(ct, pt)


def enc_conv2d_packed(o, rlk, gks, X, Cin, Wt, Cout, k, dil, frame_w, cnt):
    """Y[co] = Rescale(Relin( sum_ci sum_(p,q) rot(X[ci], step(p,q)) (x) W[co][ci][p][q] )),
    the weights replicated scalars; gks maps a step to its Galois key."""
    steps = conv_steps(k, dil, frame_w)
    R = []
    for ci in range(Cin):
        row = []
        for r in steps:
            if r == 0:
                row.append(X[ci])
            else:
                row.append(o.rotate(X[ci], r, gks[r]))
                cnt.rotate += 1
        R.append(row)
    Y = []
    for co in range(Cout):
        pairs = [(R[ci][t], Wt[(co * Cin + ci) * k * k + t]) for ci in range(Cin) for t in range(k * k)]
        Y.append(_mac_relin_rescale(o, rlk, pairs, cnt))
    return Y


def enc_poly_act(o, rlk, xs, coef, deg, cnt):
    """Polynomial activation; deg 3 at depth 2, deg 2 at depth 1 (Sec. 3).
    deg 3: (c3 u + c2) u^2 + (c1 u + c0).  A constant multiplier c at plaintext
    scale s is the integer round(c s); the branch c3 u uses s = q_(l-1) so that
    its rescale keeps u's scale, and the linear branch's scale is chosen so that
    it lands on the product's scale.
    deg 2: Relin(u (x) u), whose plain value is u^2 at scale S^2, is read as c2 u^2
    at scale S' = S^2 / c2, so the leading coefficient costs no multiplication;
    c1 u joins at that scale as round(c1 S / c2) u, c0 as round(c0 S'), and one
    rescale ends it."""
    out = []
    for x in xs:
        l = x.level
        ql, ql2 = o.q[l - 1], o.q[l - 2]
        if deg == 3:
            u2 = _mac_relin_rescale(o, rlk, [(x, x)], cnt)
            a = o.rescale(o.mul_const(x, int(np.rint(coef[3] * float(ql))), float(ql)))
            a = add_const(o, a, coef[2])
            p = _mac_relin_rescale(o, rlk, [(a, u2)], cnt)
            s1 = p.scale * float(ql2) / x.scale
            b = o.rescale(o.mul_const(o.drop_level(x, l - 1), int(np.rint(coef[1] * s1)), s1))
            b = add_const(o, b, coef[0])
            cnt.pt_mult += 2
            cnt.pt_add += 2
            cnt.rescale += 2
            cnt.ct_add += 1
            out.append(o.add(p, b))
        elif deg == 2:
            if not coef[2] > 0:
                raise ValueError("deg 2 needs a positive quadratic coefficient (a factor of the scale)")
            S = x.scale
            Sp = S * S / coef[2]
            t = o.relin(o.tensor(x, x), rlk)
            b = o.mul_const(x, int(np.rint(coef[1] * S / coef[2])))
            u = o.add(ckks.Ct(t.data, Sp), ckks.Ct(b.data, Sp))
            u = add_const(o, u, coef[0])
            out.append(o.rescale(u))
            cnt.ct_mult += 1
            cnt.relin += 1
            cnt.pt_mult += 1
            cnt.pt_add += 1
            cnt.ct_add += 1
            cnt.rescale += 1
        else:
            raise ValueError("deg must be 2 or 3")
    return out


def pool_mask(o, H, W, frame_h, frame_w, dil, scale, limbs):
    """Plaintext 0.25 at the positions that survive a 2x2 pool of inputs at
    dilation dil (y, x multiples of 2 dil inside the image), 0 elsewhere."""
    n = o.N // 2
    v = np.zeros(n)
    v[frame_positions(H, W, frame_h, frame_w, n // (frame_h * frame_w), 2 * dil)] = 0.25
    return o.encode_rns(v, scale, limbs)


def enc_avgpool2x2(o, gks, xs, dil, frame_w, mask, mask_scale, cnt):
    """s = x + rot(x, dil); s = s + rot(s, frame_w dil); y = Rescale(s * mask)
    (the 2x2 mean lands on the window's top-left position; the mask keeps those)."""
    out = []
    for x in xs:
        t = o.add(x, o.rotate(x, dil, gks[dil]))
        t = o.add(t, o.rotate(t, frame_w * dil, gks[frame_w * dil]))
        out.append(o.rescale(o.mul_pt(t, mask, mask_scale)))
        cnt.rotate += 2
        cnt.ct_add += 2
        cnt.pt_mult += 1
        cnt.rescale += 1
    return out


def enc_fc_packed(o, rlk, gks, xs, Wt, n_out, frame_slots, cnt):
    """z[r] = Rescale(Relin(sum_c x[c] (x) W[r][c])), then z += rot(z, i) for
    i = 1, 2, 4, ..., frame_slots/2: slot 0 of every frame holds the class score."""
    n_in = len(xs)
    out = []
    for r in range(n_out):
        z = _mac_relin_rescale(o, rlk, [(xs[c], Wt[r * n_in + c]) for c in range(n_in)], cnt)
        i = 1
        while i < frame_slots:
            z = o.add(z, o.rotate(z, i, gks[i]))
            cnt.rotate += 1
            cnt.ct_add += 1
            i *= 2
        out.append(z)
    return out


def fc_weight_slots(wrow, Hp, Wp, frame_h, frame_w, n_frames, dil):
    """Slot vector of one FC weight ciphertext: weight (i, j) of a channel at
    frame position (dil i, dil j) of every frame, zero elsewhere."""
    v = np.zeros(n_frames * frame_h * frame_w)
    pos = frame_positions(Hp * dil, Wp * dil, frame_h, frame_w, n_frames, dil)
    v[pos] = np.tile(np.asarray(wrow, dtype=np.float64).ravel(), n_frames)
    return v


def packed_rotation_steps(k, frame_w, frame_slots, n_pools=2):
    """Every rotation step the packed network uses (conv taps at dilation 1, 2, pools, fc sums)."""
    st = set()
    dil = 1
    for _ in range(n_pools):
        st.update(r for r in conv_steps(k, dil, frame_w) if r)
        st.update([dil, frame_w * dil])
        dil *= 2
    i = 1
    while i < frame_slots:
        st.add(i)
        i *= 2
    return sorted(st)


# ------------------------------------------------------ the paper's network
G_PAPER = (0.47, 0.50, 0.09)   # Eq. (approxReLU)


def paper_cnn_fp64(images, wc, wfc, coef=G_PAPER, chunk=512):
    """conv KxK stride 1 no padding -> g -> 2x2 mean (Eq. (ActPool)) -> flatten (c, y, x) -> FC.
    Images are independent; they go through in chunks so that the intermediates stay small."""
    x = images[:, None] if images.ndim == 3 else images
    K = wc.shape[2]
    H, W = x.shape[2], x.shape[3]
    out = np.empty((x.shape[0], wfc.shape[0]))
    for b0 in range(0, x.shape[0], chunk):
        y = conv2d_fp64(x[b0:b0 + chunk], wc, 1, 0, 0, H - K + 1, W - K + 1)
        p = avgpool2_fp64(poly_fp64(y, coef))
        out[b0:b0 + chunk] = p.reshape(p.shape[0], -1) @ wfc.T
    return out


def enc_sum_pool2x2_slot(o, xs, C, H, W, cnt):
    """y[c][i][j] = x[c][2i][2j] + x[c][2i][2j+1] + x[c][2i+1][2j] + x[c][2i+1][2j+1]."""
    out = []
    for c in range(C):
        for i in range(H // 2):
            for j in range(W // 2):
                def at(yy, xx):
                    return xs[(c * H + yy) * W + xx]
                t = o.add(at(2 * i, 2 * j), at(2 * i, 2 * j + 1))
                t = o.add(t, at(2 * i + 1, 2 * j))
                out.append(o.add(t, at(2 * i + 1, 2 * j + 1)))
                cnt.ct_add += 3
    return out


def enc_paper_cnn(o, rlk, X, Wc, Wf, C, K, H, W, n_classes, cnt, coef=G_PAPER):
    """The paper's network on the oracle: conv, g/4 on every output (depth 1), sum
    pooling (= the mean of g), drop to two limbs, FC; returns (stages, scores)."""
    Ho, Wo = H - K + 1, W - K + 1
    Y = enc_conv2d_slot(o, rlk, X, H, W, 1, Wc, C, K, K, 1, 0, 0, Ho, Wo, cnt)
    A = enc_poly_act(o, rlk, Y, tuple(c / 4.0 for c in coef), 2, cnt)
    Pp = enc_sum_pool2x2_slot(o, A, C, Ho, Wo, cnt)
    Pd = [o.drop_level(p, 2) for p in Pp]
    Z = enc_fc_slot(o, rlk, Pd, Wf, n_classes, cnt)
    return {"conv": Y, "act": A, "pool": Pp, "fc": Z}, Z


# -------------------------------------- within-image packing, plain model
def enc_conv2d_packed_pw(o, gks, X, Cin, w, Cout, k, dil, frame_w, wscale, cnt):
    """Y[co] = Rescale( sum_ci sum_t rot(X[ci], s_t) * round(w[co][ci][t] * wscale) )."""
    steps = conv_steps(k, dil, frame_w)
    R = []
    for ci in range(Cin):
        row = []
        for r in steps:
            if r == 0:
                row.append(X[ci])
            else:
                row.append(o.rotate(X[ci], r, gks[r]))
                cnt.rotate += 1
        R.append(row)
    w = np.asarray(w, dtype=np.float64).reshape(Cout, Cin, k * k)
    Y = []
    for co in range(Cout):
        acc = None
        for ci in range(Cin):
            for t in range(k * k):
                term = o.mul_const(R[ci][t], int(np.rint(w[co, ci, t] * wscale)), wscale)
                acc = term if acc is None else o.add(acc, term)
                cnt.pt_mult += 1
        cnt.ct_add += Cin * k * k - 1
        cnt.rescale += 1
        Y.append(o.rescale(acc))
    return Y


def enc_fc_packed_pw(o, gks, xs, Wpt, pt_scale, n_out, frame_slots, cnt):
    """z[r] = Rescale( sum_c x[c] * W[r][c] ) with plaintext weights, then rotate-and-sum."""
    n_in = len(xs)
    out = []
    for r in range(n_out):
        acc = None
        for c in range(n_in):
            term = o.mul_pt(xs[c], Wpt[r * n_in + c], pt_scale)
            acc = term if acc is None else o.add(acc, term)
            cnt.pt_mult += 1
        cnt.ct_add += n_in - 1
        cnt.rescale += 1
        z = o.rescale(acc)
        i = 1
        while i < frame_slots:
            z = o.add(z, o.rotate(z, i, gks[i]))
            cnt.rotate += 1
            cnt.ct_add += 1
            i *= 2
        out.append(z)
    return out
