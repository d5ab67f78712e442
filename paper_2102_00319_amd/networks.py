"""Encrypted CNNs composed from the layer entry points of libfhe.

Roles follow the paper's setting (Sec. 2.1): the user holds the secret key,
encrypts images and decrypts scores; the model owner encrypts the weights under
the user's public key (Sec. 3, "both image and model encrypted"); the cloud runs
`forward` on ciphertexts only.

PackedCNN -- within-image packing: one ciphertext per channel, a batch of images
each in a frame_h x frame_w frame of slots (zero guard right and below):
    conv k x k same (c1 channels) -> poly act -> 2x2 avg pool
    -> conv k x k same (c2 channels, dilation 2) -> poly act -> 2x2 avg pool
    -> fully connected (flatten order (c, y, x)) -> score in slot 0 of each frame.
Every CT x CT product is followed by relinearisation and one rescale, so a
forward pass takes 9 levels with the cubic activation: conv 1, act 2, pool 1,
conv 1, act 2, pool 1, fc 1 (7 with the quadratic one, whose depth is 1).
"""
import math

import numpy as np

from .fhe import CtArray

# ------------------------------------------------------------ slot layouts


def frame_pack(images, frame_h, frame_w):
    """images [B][H][W] -> slot vector, image b pixel (y, x) at b*frame_h*frame_w + y*frame_w + x."""
    B, H, W = images.shape
    if H > frame_h or W > frame_w:
        raise ValueError("image larger than its frame")
    out = np.zeros(B * frame_h * frame_w)
    for b in range(B):
        base = b * frame_h * frame_w
        for y in range(H):
            out[base + y * frame_w: base + y * frame_w + W] = images[b, y]
    return out


def grid_slots(H, W, frame_h, frame_w, n_frames, step):
    """Slots of the grid positions (step*i, step*j) inside an H x W image, every frame, row-major per frame."""
    rows = range(0, H, step)
    cols = range(0, W, step)
    return np.array([f * frame_h * frame_w + y * frame_w + x
                     for f in range(n_frames) for y in rows for x in cols], dtype=np.int64)


class PackedCNN:
    def __init__(self, H=28, W=28, frame_h=32, frame_w=32, k=3, c1=8, c2=16, n_classes=10,
                 coef=(0.47, 0.5, 0.09, -0.005), deg=3):
        if H % 4 or W % 4:
            raise ValueError("image sides must be multiples of 4 (two 2x2 pools)")
        if frame_h - H < 2 * (k // 2) or frame_w - W < 2 * (k // 2):
            raise ValueError("zero guard too small for the second convolution's dilation")
        self.H, self.W, self.fh, self.fw, self.k = H, W, frame_h, frame_w, k
        self.c1, self.c2, self.n_classes, self.coef, self.deg = c1, c2, n_classes, tuple(coef), deg
        self.frame = frame_h * frame_w
        if self.frame & (self.frame - 1):
            raise ValueError("frame size must be a power of two")
        self._masks = {}

    # -------------------------------------------------------------- plan
    def conv_steps(self, dil):
        h = self.k // 2
        return [dil * ((p - h) * self.fw + (q - h)) for p in range(self.k) for q in range(self.k)]

    def rotation_steps(self):
        st = set()
        for dil in (1, 2):
            st.update(r for r in self.conv_steps(dil) if r)
            st.update([dil, self.fw * dil])
        i = 1
        while i < self.frame:
            st.add(i)
            i *= 2
        return sorted(st)

    def images_per_ct(self, ctx):
        return (ctx.N // 2) // self.frame

    @property
    def act_depth(self):
        return 2 if self.deg == 3 else 1

    @property
    def depth(self):
        return 2 * (self.act_depth + 2) + 1

    # -------------------------------------------------------------- user
    def keygen(self, ctx, s, seed):
        """Relinearisation key (seed) and one Galois key per rotation step (seed + 1 + i)."""
        rlk = ctx.keygen_relin(s, seed)
        gks = {r: ctx.keygen_rot(s, r, seed + 1 + i) for i, r in enumerate(self.rotation_steps())}
        return rlk, gks

    def encrypt_images(self, ctx, pk, images, seed, scale=None):
        B = images.shape[0]
        if B > self.images_per_ct(ctx):
            raise ValueError("more images than frames in one ciphertext")
        v = frame_pack(images, self.fh, self.fw)
        return [ctx.encrypt(pk, ctx.encode(v, scale=scale or ctx.scale), seed)]

    def decrypt_scores(self, ctx, s, Z, B):
        out = np.empty((B, len(Z)))
        slots = np.arange(B) * self.frame   # the score of image b sits at its frame's first slot
        for r, z in enumerate(Z):
            out[:, r], _ = ctx.decode_slots(ctx.decrypt(s, z), slots)
        return out

    # ------------------------------------------------------- model owner
    def weight_levels(self, top):
        d = self.act_depth + 2
        return top, top - d, top - 2 * d

    def fc_slots(self, ctx, wrow):
        """One FC weight ciphertext's slots: weight (y, x) of a channel at frame position (4y, 4x)."""
        nf = self.images_per_ct(ctx)
        v = np.zeros(ctx.N // 2)
        v[grid_slots(self.H, self.W, self.fh, self.fw, nf, 4)] = np.tile(np.asarray(wrow, np.float64).ravel(), nf)
        return v

    def encrypt_weights(self, ctx, pk, w1, w2, wfc, seeds, top=None, scale=None):
        """w1 [c1][1][k][k], w2 [c2][c1][k][k] as slot-replicated constants, wfc [classes][c2*(H/4)*(W/4)]
        as masked slot vectors; seeds = (conv1, conv2, fc) base seeds, one per ciphertext from there."""
        top = ctx.L if top is None else top
        D = scale or ctx.scale
        l1, l2, l3 = self.weight_levels(top)
        W1 = ctx.encrypt_const_batch(pk, w1.ravel(), D, [seeds[0] + t for t in range(w1.size)], l1)
        W2 = ctx.encrypt_const_batch(pk, w2.ravel(), D, [seeds[1] + t for t in range(w2.size)], l2)
        hp, wp = self.H // 4, self.W // 4
        Wf = []
        for r in range(self.n_classes):
            rows = np.asarray(wfc[r]).reshape(self.c2, hp * wp)
            for c in range(self.c2):
                pt = ctx.encode(self.fc_slots(ctx, rows[c]), scale=D, limbs=l3)
                Wf.append(ctx.encrypt(pk, pt, seeds[2] + r * self.c2 + c))
        return CtArray(W1), CtArray(W2), CtArray(Wf)

    # -------------------------------------------------------------- cloud
    def pool_mask(self, ctx, dil, limbs):
        """0.25 at the grid of step 2*dil, at scale q_(limbs-1) so that the rescale keeps the scale."""
        key = (ctx.N, tuple(ctx.q), dil, limbs)   # a network object may serve several parameter sets
        if key not in self._masks:
            v = np.zeros(ctx.N // 2)
            v[grid_slots(self.H, self.W, self.fh, self.fw, self.images_per_ct(ctx), 2 * dil)] = 0.25
            m = ctx.encode(v, scale=float(ctx.q[limbs - 1]), limbs=limbs)
            ctx.stream.synchronize()   # other streams may read the cached mask next
            self._masks.setdefault(key, m)
        return self._masks[key]

    def forward(self, ctx, rlk, gks, X, weights):
        W1, W2, Wf = weights
        Y = ctx.conv2d_packed(rlk, gks, X, W1, self.c1, self.k, 1, self.fw)
        A = ctx.poly_act(rlk, Y, self.coef, self.deg)
        P = ctx.avgpool2x2(gks, A, 1, self.fw, self.pool_mask(ctx, 1, A[0].limbs))
        Y = ctx.conv2d_packed(rlk, gks, P, W2, self.c2, self.k, 2, self.fw)
        A = ctx.poly_act(rlk, Y, self.coef, self.deg)
        P = ctx.avgpool2x2(gks, A, 2, self.fw, self.pool_mask(ctx, 2, A[0].limbs))
        return ctx.fc_packed(rlk, gks, P, Wf, self.n_classes, self.frame)

    def forward_per_op(self, ctx, rlk, gks, X, weights):
        """The same network with one ciphertext per library call, the unbatched form that
        batching is measured against: every rotation, every output's products +
        relinearisation + rescale, every activation and pool, every rotate-and-sum step is
        its own call.  Gives the same ciphertexts as forward()."""
        W1, W2, Wf = weights

        def conv(xs, wt, cout, dil):
            steps = self.conv_steps(dil)
            kk, cin = len(steps), len(xs)
            rot = [[x if s == 0 else ctx.rotate(gks[s], x, s) for s in steps] for x in xs]
            out = []
            for co in range(cout):
                a = [rot[ci][t] for ci in range(cin) for t in range(kk)]
                b = [wt[(co * cin + ci) * kk + t] for ci in range(cin) for t in range(kk)]
                out.append(ctx.rescale(ctx.relin(rlk, ctx.mul_acc(a, b))))
            return out

        def act(ys):
            return [ctx.poly_act(rlk, [y], self.coef, self.deg)[0] for y in ys]

        def pool(xs, dil):
            return [ctx.avgpool2x2(gks, [x], dil, self.fw, self.pool_mask(ctx, dil, x.limbs))[0] for x in xs]

        P = pool(act(conv(X, W1, self.c1, 1)), 1)
        P = pool(act(conv(P, W2, self.c2, 2)), 2)
        out = []
        for r in range(self.n_classes):
            z = ctx.rescale(ctx.relin(rlk, ctx.mul_acc(P, [Wf[r * self.c2 + c] for c in range(self.c2)])))
            i = 1
            while i < self.frame:
                z = ctx.add(z, ctx.rotate(gks[i], z, i))
                i *= 2
            out.append(z)
        return out

    # ---------------------------------------------- plain (unencrypted) model
    def plain_fc_weights(self, ctx, wfc, limbs):
        """FC weights as plaintexts at `limbs` limbs, scale q_(limbs-1) (the rescale keeps the scale)."""
        hp, wp = self.H // 4, self.W // 4
        sc = float(ctx.q[limbs - 1])
        out = []
        for r in range(self.n_classes):
            rows = np.asarray(wfc[r]).reshape(self.c2, hp * wp)
            for c in range(self.c2):
                out.append(ctx.encode(self.fc_slots(ctx, rows[c]), scale=sc, limbs=limbs))
        return out

    def forward_plain(self, ctx, rlk, gks, X, w1, w2, Wfc_pt):
        """Forward pass with the model in the clear: conv taps multiply by integer
        constants (scale q_(l-1)), FC weights are plaintexts; activations and pools as
        in forward().  One relinearisation per activation product only."""
        l = X[0].limbs
        Y = ctx.conv2d_packed_pw(gks, X, w1, self.c1, self.k, 1, self.fw, float(ctx.q[l - 1]))
        A = ctx.poly_act(rlk, Y, self.coef, self.deg)
        P = ctx.avgpool2x2(gks, A, 1, self.fw, self.pool_mask(ctx, 1, A[0].limbs))
        l = P[0].limbs
        Y = ctx.conv2d_packed_pw(gks, P, w2, self.c2, self.k, 2, self.fw, float(ctx.q[l - 1]))
        A = ctx.poly_act(rlk, Y, self.coef, self.deg)
        P = ctx.avgpool2x2(gks, A, 2, self.fw, self.pool_mask(ctx, 2, A[0].limbs))
        return ctx.fc_packed_pw(gks, P, Wfc_pt, self.n_classes, self.frame)

    def op_counts(self):
        """Expected (ct_mult, relin, rotate) of one forward pass."""
        kk, nz = self.k * self.k, self.k * self.k - 1
        act = 2 if self.deg == 3 else 1
        ct_mult = self.c1 * kk + self.c2 * self.c1 * kk + act * (self.c1 + self.c2) + self.n_classes * self.c2
        relin = self.c1 + self.c2 + act * (self.c1 + self.c2) + self.n_classes
        rot = nz * (1 + self.c1) + 2 * (self.c1 + self.c2) + self.n_classes * int(np.log2(self.frame))
        return ct_mult, relin, rot


class SlotCNN:
    """Slot packing (Sec. 3, Fig. 2): one ciphertext per pixel holding that pixel of
    every image of the batch, one weight ciphertext per weight (replicated):
        conv K x K stride s, zero padding pad on top and left (Cout channels) -> x^2
        -> FC (Cout*Ho*Wo -> fc1) -> x^2 -> FC (fc1 -> n_classes).
    Images of one client may occupy any slot range [off, off + B): ciphertexts of
    requests with disjoint ranges add up to one batch (slot merging)."""

    def __init__(self, H=28, W=28, K=5, Cout=5, stride=2, pad=1, fc1=100, n_classes=10):
        self.H, self.W, self.K, self.Cout, self.stride, self.pad = H, W, K, Cout, stride, pad
        self.Ho = (H + pad - K) // stride + 1
        self.Wo = (W + pad - K) // stride + 1
        self.fc1, self.n_classes = fc1, n_classes

    @property
    def depth(self):
        return 4

    def slots(self, ctx):
        return ctx.N // 2

    def keygen(self, ctx, s, seed):
        return ctx.keygen_relin(s, seed), {}

    def encrypt_images(self, ctx, pk, images, seed, slot_offset=0, scale=None):
        B = images.shape[0]
        if slot_offset + B > self.slots(ctx):
            raise ValueError("images beyond the slot count")
        out = []
        for y in range(self.H):
            for x in range(self.W):
                v = np.zeros(slot_offset + B)
                v[slot_offset:] = images[:, y, x]
                out.append(ctx.encrypt(pk, ctx.encode(v, scale=scale or ctx.scale), seed + y * self.W + x))
        return out

    def encrypt_weights(self, ctx, pk, cw, f1, f2, seeds, top=None, scale=None):
        top = ctx.L if top is None else top
        D = scale or ctx.scale
        Wc = ctx.encrypt_const_batch(pk, cw.ravel(), D, [seeds[0] + t for t in range(cw.size)], top)
        W1 = ctx.encrypt_const_batch(pk, f1.ravel(), D, [seeds[1] + t for t in range(f1.size)], top - 2)
        W2 = ctx.encrypt_const_batch(pk, f2.ravel(), D, [seeds[2] + t for t in range(f2.size)], top - 4)
        return CtArray(Wc), CtArray(W1), CtArray(W2)

    def forward(self, ctx, rlk, gks, X, weights):
        Wc, W1, W2 = weights
        Y = ctx.conv2d_slot(rlk, X, self.H, self.W, 1, Wc, self.Cout, self.K, self.K, self.stride, self.pad,
                            self.pad, self.Ho, self.Wo)
        Z = ctx.fc_slot(rlk, ctx.square_act(rlk, Y), W1, self.fc1)
        return ctx.fc_slot(rlk, ctx.square_act(rlk, Z), W2, self.n_classes)

    def decrypt_scores(self, ctx, s, Z, B, slot_offset=0):
        out = np.empty((B, len(Z)))
        slots = np.arange(slot_offset, slot_offset + B)
        for r, z in enumerate(Z):
            out[:, r], _ = ctx.decode_slots(ctx.decrypt(s, z), slots)
        return out


class PaperCNN:
    """The paper's network (Sec. 4.3) with slot packing (one image per slot):
        conv K x K, stride 1, no padding, C filters -> ActPool (g on every output,
        then the mean of each 2x2 window, Eq. (ActPool)) -> FC (C*Hp*Wp -> classes).
    g(u) = 0.47 + 0.50 u + 0.09 u^2 (Eq. (approxReLU)); the 1/4 of the mean is folded
    into g's coefficients, so that pooling is three additions.  The conv and ActPool
    run in bands of pooled rows (the conv outputs of one band are freed before the
    next), and the pooled maps drop to two limbs before the FC, whose weights the
    model owner encrypts at that level.

    Scales: the depth-1 activation reads Relin(u (x) u) as c2 u^2 at scale S^2 / c2,
    so its output scale is 1/c2 times that of u^2 (44x for g/4).  The conv weights
    are therefore encrypted at scale D * sqrt(c2), which puts the conv output at
    about D sqrt(c2) and the activation output back at about D; the FC output then
    sits near D at one limb, with log2(q0 / D) bits of room for the scores."""

    def __init__(self, H=28, W=28, K=3, C=28, n_classes=10, coef=(0.47, 0.50, 0.09), band=1):
        self.H, self.W, self.K, self.C, self.n_classes = H, W, K, C, n_classes
        self.Ho, self.Wo = H - K + 1, W - K + 1
        if self.Ho % 2 or self.Wo % 2:
            raise ValueError("conv output sides must be even (2x2 pooling)")
        self.Hp, self.Wp = self.Ho // 2, self.Wo // 2
        self.coef = tuple(coef)
        self.coef4 = tuple(c / 4.0 for c in coef)
        self.band = band

    @property
    def n_in_fc(self):
        return self.C * self.Hp * self.Wp

    def conv_weight_scale(self, D):
        """Scale of the conv weight ciphertexts for input scale D (see the class note)."""
        return D * math.sqrt(self.coef4[2])

    def keygen(self, ctx, s, seed):
        return ctx.keygen_relin(s, seed), {}

    def encrypt_images(self, ctx, pk, images, seed, slot_offset=0, scale=None, progress=None):
        B = images.shape[0]
        out = []
        for y in range(self.H):
            for x in range(self.W):
                v = np.zeros(slot_offset + B)
                v[slot_offset:] = images[:, y, x]
                out.append(ctx.encrypt(pk, ctx.encode(v, scale=scale or ctx.scale), seed + y * self.W + x))
            if progress:
                progress("images: row %d of %d encrypted" % (y + 1, self.H))
        return out

    def encrypt_weights(self, ctx, pk, wc, wfc, seeds, top=None, scale=None):
        """wc [C][1][K][K] at the top level and scale conv_weight_scale(D); wfc
        [classes][C*Hp*Wp] at two limbs and scale D."""
        top = ctx.L if top is None else top
        D = scale or ctx.scale
        Wc = ctx.encrypt_const_batch(pk, wc.ravel(), self.conv_weight_scale(D),
                                     [seeds[0] + t for t in range(wc.size)], top)
        Wf = ctx.encrypt_const_batch(pk, wfc.ravel(), D, [seeds[1] + t for t in range(wfc.size)], 2)
        return CtArray(Wc), CtArray(Wf)

    def forward(self, ctx, rlk, gks, X, weights, progress=None):
        Wc, Wf = weights
        pooled = [None] * self.n_in_fc
        for i0 in range(0, self.Hp, self.band):
            i1 = min(self.Hp, i0 + self.band)
            rows = 2 * (i1 - i0)
            Xs = X[2 * i0 * self.W:(2 * i1 + self.K - 1) * self.W]
            Y = ctx.conv2d_slot(rlk, Xs, rows + self.K - 1, self.W, 1, Wc, self.C, self.K, self.K, 1, 0, 0,
                                rows, self.Wo)
            A = ctx.poly_act(rlk, Y, self.coef4, 2)
            del Y
            Pb = ctx.pool2x2_sum_slot(A, self.C, rows, self.Wo)
            del A
            for c in range(self.C):
                for i in range(i1 - i0):
                    for j in range(self.Wp):
                        p = Pb[(c * (i1 - i0) + i) * self.Wp + j]
                        pooled[(c * self.Hp + i0 + i) * self.Wp + j] = ctx.drop_level(p, 2)
            if progress:
                progress("forward: pooled rows %d..%d of %d enqueued" % (i0, i1 - 1, self.Hp))
        return ctx.fc_slot(rlk, pooled, Wf, self.n_classes)

    def decrypt_scores(self, ctx, s, Z, B, slot_offset=0):
        out = np.empty((B, len(Z)))
        slots = np.arange(slot_offset, slot_offset + B)
        for r, z in enumerate(Z):
            out[:, r], _ = ctx.decode_slots(ctx.decrypt(s, z), slots)
        return out

    def op_counts(self):
        n_conv = self.C * self.Ho * self.Wo
        return {"ct_mult": n_conv * self.K * self.K + n_conv + self.n_in_fc * self.n_classes,
                "relin": n_conv * 2 + self.n_classes}
