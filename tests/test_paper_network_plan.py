"""Host-side plan of the paper's network at full size (Sec. 4.3: N = 2^15, 16384
images, conv 3x3 x 28, ActPool, FC 4732 -> 10), checked on the CPU before any GPU
run: the scale bookkeeping leaves room for the scores of the synthetic workload,
and a dry run of the forward pass with stand-in ciphertexts bounds the device
memory it holds."""
import math
import weakref

import numpy as np

import workloads
from oracle import cnn
from paper_2102_00319_amd import fhe, networks

ROOM_BITS = 4            # the library's rule for layer outputs (FHE_SCALE_ROOM_BITS)
HBM_BYTES = 288e9


def test_scales_leave_room_for_the_scores():
    s = workloads.load_params("p_n15")
    q = [int(x) for x in s["q"]]
    D = float(s["scale"])
    net = networks.PaperCNN()
    c2 = net.coef4[2]
    swc = net.conv_weight_scale(D)
    assert swc == D * math.sqrt(0.09 / 4.0)
    L = len(q)
    s_conv = D * swc / q[L - 1]                       # 16 -> 15 limbs
    s_act = s_conv * s_conv / c2 / q[L - 2]           # depth 1: 15 -> 14 limbs
    s_fc = s_act * D / q[1]                           # dropped to 2 limbs, FC -> 1 limb
    logq = [math.log2(x) for x in q]
    for sc, limbs in [(s_conv, L - 1), (s_act, L - 2), (s_fc, 1)]:
        assert math.log2(sc) <= sum(logq[:limbs]) - 1 - ROOM_BITS
    # the workload's scores (FP64 network, same seeds as the GPU run)
    imgs = workloads.images(workloads.SEED_DATA, 16384, 28, 28)
    wc = workloads.weights(workloads.SEED_DATA + 1, (28, 1, 3, 3))
    wfc = workloads.weights(workloads.SEED_DATA + 2, (10, 4732))
    ref = cnn.paper_cnn_fp64(imgs, wc, wfc)
    top = float(np.abs(ref).max())
    assert 1.0 < top < 64.0
    assert math.log2(s_fc) + math.log2(top) < logq[0] - 1 - 2   # two bits more than a wrap needs


class _Buf:
    """Stand-in device buffer: counts its bytes while it is referenced."""

    def __init__(self, meter, shape):
        self.shape = shape
        self.nbytes = 8 * math.prod(shape)
        meter.alloc(self.nbytes)
        weakref.finalize(self, meter.free, self.nbytes)


class _Meter:
    def __init__(self):
        self.live = self.peak = 0

    def alloc(self, n):
        self.live += n
        self.peak = max(self.peak, self.live)

    def free(self, n):
        self.live -= n


class _Ct:
    def __init__(self, meter, polys, limbs, N, scale=1.0):
        self.data = _Buf(meter, (polys, limbs, N))
        self.scale = scale

    @property
    def limbs(self):
        return self.data.shape[1]

    def s(self):
        return fhe.fhe_ct(0, self.limbs, 2, self.scale)


class _StandInCtx:
    """The calls PaperCNN makes, with the shapes the library gives their outputs."""

    def __init__(self, name):
        s = workloads.load_params(name)
        self.N, self.L, self.K = 1 << s["log_n"], len(s["q"]), len(s["p"])
        self.scale = float(s["scale"])
        self.meter = _Meter()

    def new_ct(self, limbs, polys=2):
        return _Ct(self.meter, polys, limbs, self.N)

    def encode(self, v, scale=None):
        return _Ct(self.meter, 1, self.L, self.N)

    def encrypt(self, pk, pt, seed):
        return self.new_ct(pt.limbs)

    def keygen_relin(self, s, seed):
        return _Buf(self.meter, (4, 2, self.L + self.K, self.N))

    def encrypt_const_batch(self, pk, values, scale, seeds, limbs):
        return [self.new_ct(limbs) for _ in range(len(values))]

    def conv2d_slot(self, rlk, X, H, W, Cin, Wt, Cout, kh, kw, stride, pt, pl, Ho, Wo):
        return [self.new_ct(X[0].limbs - 1) for _ in range(Cout * Ho * Wo)]

    def poly_act(self, rlk, Y, coef, deg):
        return [self.new_ct(y.limbs - 1) for y in Y]

    def pool2x2_sum_slot(self, A, C, H, W):
        return [self.new_ct(A[0].limbs) for _ in range(C * (H // 2) * (W // 2))]

    def drop_level(self, ct, limbs):
        return self.new_ct(limbs)

    def fc_slot(self, rlk, x, Wt, n_out):
        return [self.new_ct(x[0].limbs - 1) for _ in range(n_out)]


def dry_run_peak(band):
    ctx = _StandInCtx("p_n15")
    net = networks.PaperCNN(band=band)
    rlk, _ = net.keygen(ctx, None, 0)
    imgs = np.zeros((ctx.N // 2, 28, 28))
    X = net.encrypt_images(ctx, None, imgs, 0)
    W = net.encrypt_weights(ctx, None, np.zeros((28, 1, 3, 3)), np.zeros((10, 4732)), (0, 0))
    Z = net.forward(ctx, rlk, {}, X, W)
    assert len(Z) == 10 and Z[0].limbs == 1
    return ctx.meter.peak


def test_dry_run_device_memory():
    GiB = 1 << 30
    peak1, peak2 = dry_run_peak(1), dry_run_peak(2)
    # images 784 x 8 MiB, conv weights 252 x 8 MiB, FC weights 47,320 x 1 MiB, relin key 160 MiB;
    # one band: conv outputs, activations, pooled maps; the pooled maps at two limbs
    fixed = (784 * 8 + 252 * 8 + 47320 * 1 + 160) * (1 << 20)
    assert fixed < peak1 < peak2
    # the library's own scratch and layer workspace: each bounded by about 2 GiB per call
    # (chunked), plus one item of at most 64 MiB at N = 2^15, 16 limbs
    library = 2 * (2 * GiB + 64 * (1 << 20))
    assert peak1 + library < 0.5 * HBM_BYTES
    assert peak2 + library < 0.5 * HBM_BYTES
    assert peak1 / GiB < 90 and peak2 / GiB < 110
