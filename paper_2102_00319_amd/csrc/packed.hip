// packed.hip -- encrypted CNN layers with images packed inside the slots.
//
// Within-image packing: a ciphertext holds one channel of a batch of images,
// each image in a frame of frame_h x frame_w slots (row-major, zero guard on the
// right and below); pixel (y, x) of image b is slot b*frame_h*frame_w +
// y*frame_w + x.  A left slot rotation (Sec. 3, Fig. 2 "rotation") by
// dy*frame_w + dx then brings pixel (y+dy, x+dx) to (y, x) in every frame at
// once, so that
//   * a k x k "same" convolution is a sum of rotated inputs times replicated
//     scalar weights, followed by one relinearisation and one rescale per output;
//   * a 2x2 average pool is two rotations and adds, then one plaintext product
//     with 0.25 on the surviving positions (it also clears everything else), and
//     the dilation of the valid positions doubles;
//   * a fully connected layer is a slot-wise product with weight ciphertexts that
//     hold the weights at the valid positions, then a rotate-and-sum over the frame.
// Every stage runs batched over all channels: one rotation batch, one tensor
// multiply-accumulate launch, one batched key switch, one batched rescale.
// Intermediates live in the context's layer workspace; the operations called
// use the scratch buffer.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "fhe_internal.h"

namespace {

const fhe_evk *find_key(const fhe_evk *keys, uint32_t nkeys, uint64_t galois)
{
    for (uint32_t i = 0; i < nkeys; ++i)
        if (keys[i].d && keys[i].galois == galois) return &keys[i];
    return nullptr;
}

fhe_status chk2(const fhe_ct *x, uint32_t l, const char *what)
{
    if (!x->d || x->polys != 2 || x->limbs != l)
        return fhe_fail(FHE_EINVAL, std::string(what) + ": ciphertexts must be 2 x limbs at the expected level");
    return FHE_OK;
}

fhe_status rescale_many(fhe_ctx *c, uint32_t l, uint32_t n, const std::vector<const uint64_t *> &in,
                        const std::vector<uint64_t *> &out)
{
    const uint32_t C = std::min<uint32_t>(65535 / 2, (uint32_t)std::max<size_t>(
                                                         1, ((size_t)2 << 30) / rescale_scratch_bytes(c, l, 2, 1)));
    uint8_t *scr;
    fhe_status s;
    if ((s = ctx_scratch(c, rescale_scratch_bytes(c, l, 2, std::min(C, n)), &scr))) return s;
    for (uint32_t t0 = 0; t0 < n; t0 += C) {
        const uint32_t cn = std::min(C, n - t0);
        if ((s = rescale_run(c, l, 2, cn, in.data() + t0, out.data() + t0, scr))) return s;
    }
    c->ops[OP_RESCALE] += n;
    return FHE_OK;
}

Consts64 zero_consts()
{
    Consts64 z;
    std::memset(&z, 0, sizeof(z));
    return z;
}

constexpr int TPB = 256;
constexpr int PW_TILE = 8;
inline uint32_t blocks_for(uint64_t n, uint32_t per) { return (uint32_t)((n + per - 1) / per); }

// Multiply-accumulate with plain weights, for up to TO outputs sharing their
// ciphertext list A: out_u = sum_p A[p] * W[u][p] (both polynomials), where W is
// a per-limb integer constant (PT = false: words are the residues as doubles,
// [u][p][limb]) or a plaintext [limbs][N] (PT = true: words are pointers, [u][p]).
// Table: [a: P][w: ...][out: n_out][tiles: 2 words: o0 | k << 32, unused]; one
// block row (blockIdx.y) per tile.
template <int TO, bool PT>
__global__ __launch_bounds__(TPB) void k_plain_mac(uint64_t *const *__restrict__ tab, uint32_t P, uint32_t nW,
                                                   uint32_t n_out, const ModQ *__restrict__ mods, uint32_t logN,
                                                   uint32_t limbs)
{
    const uint32_t N = 1u << logN;
    const uint64_t e = (uint64_t)blockIdx.x * TPB + threadIdx.x;   // limb * N + k
    if (e >= ((uint64_t)limbs << logN)) return;
    const uint64_t w0 = (uint64_t)(uintptr_t)tab[P + nW + n_out + 2 * blockIdx.y];
    const uint32_t o0 = (uint32_t)w0, k = (uint32_t)(w0 >> 32);
    const uint32_t limb = (uint32_t)(e >> logN);
    const uint64_t off1 = (uint64_t)limbs * N;
    const double q = mods[limb].q, qi = mods[limb].qinv;
    double d0[TO], d1[TO];
#pragma unroll
    for (int u = 0; u < TO; ++u) d0[u] = d1[u] = 0.0;
    for (uint32_t p = 0; p < P; ++p) {
        const gu64 *A = gview(tab[p]);
        const double a0 = u64_to_f64(A[e]), a1 = u64_to_f64(A[e + off1]);
#pragma unroll
        for (int u = 0; u < TO; ++u) {
            if (u < (int)k) {
                double w;
                if (PT) w = u64_to_f64(gview(tab[P + (size_t)(o0 + u) * P + p])[e]);
                else w = __longlong_as_double((long long)(uintptr_t)tab[P + ((size_t)(o0 + u) * P + p) * limbs + limb]);
                d0[u] += mulmod(a0, w, q, qi);
                d1[u] += mulmod(a1, w, q, qi);
            }
        }
        if ((p & 7) == 7) {   // |mulmod| <= 0.75 q + 2^46: eight terms stay below 2^53
#pragma unroll
            for (int u = 0; u < TO; ++u) {
                d0[u] = redc(d0[u], q, qi);
                d1[u] = redc(d1[u], q, qi);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < TO; ++u) {
        if (u < (int)k) {
            gu64 *out = gview(tab[P + nW + o0 + u]);
            out[e] = f64_to_u64(canon(d0[u], q, qi));
            out[e + off1] = f64_to_u64(canon(d1[u], q, qi));
        }
    }
}

// out[o] = Rescale(sum_p A[p] * W[o][p]) for all outputs (all outputs share A); W
// as constants (cst: n_out x P values, multiplied as round(value * wscale)) or as
// plaintexts (pts: n_out x P device pointers).  Writes 2 x (l-1) outputs.
fhe_status plain_mac_rescale(fhe_ctx *c, uint32_t l, const std::vector<uint64_t *> &A, const double *cst,
                             double wscale, const std::vector<const uint64_t *> &pts, uint32_t n_out,
                             const std::vector<uint64_t *> &Y)
{
    const uint32_t P = (uint32_t)A.size();
    const size_t N = c->N;
    fhe_status s;
    const bool pt = cst == nullptr;
    // accumulators (2 polys at l limbs) per output and the rescale scratch
    const size_t acc_bytes = (size_t)n_out * 2 * l * N * sizeof(uint64_t);
    const size_t rs_bytes = rescale_scratch_bytes(c, l, 2, n_out);
    uint8_t *scr;
    if ((s = ctx_scratch(c, acc_bytes + rs_bytes, &scr))) return s;
    uint64_t *acc = (uint64_t *)scr;
    std::vector<uint64_t *> tab(A.begin(), A.end());
    if (pt) {
        for (uint32_t o = 0; o < n_out; ++o)
            for (uint32_t p = 0; p < P; ++p) tab.push_back((uint64_t *)pts[(size_t)o * P + p]);
    } else {
        for (uint32_t o = 0; o < n_out; ++o)
            for (uint32_t p = 0; p < P; ++p) {
                Consts64 r;
                if ((s = const_residues(c, cst[(size_t)o * P + p] * wscale, l, &r))) return s;
                for (uint32_t i = 0; i < l; ++i) {
                    uint64_t bits;
                    std::memcpy(&bits, &r.v[i], 8);
                    tab.push_back((uint64_t *)(uintptr_t)bits);
                }
            }
    }
    const uint32_t nW = (uint32_t)(tab.size() - P);
    for (uint32_t o = 0; o < n_out; ++o) tab.push_back(acc + (size_t)o * 2 * l * N);
    uint32_t ntiles = 0;
    for (uint32_t o0 = 0; o0 < n_out; o0 += PW_TILE, ++ntiles) {
        const uint32_t k = std::min<uint32_t>(PW_TILE, n_out - o0);
        tab.push_back((uint64_t *)(uintptr_t)(o0 | ((uint64_t)k << 32)));
        tab.push_back(nullptr);
    }
    uint64_t **dt;
    if ((s = ctx_ptr_table(c, tab, &dt))) return s;
    {
        ProfScope ps(c, "tensor");
        const dim3 grid(blocks_for((uint64_t)l * N, TPB), ntiles);
        if (pt)
            hipLaunchKernelGGL((k_plain_mac<PW_TILE, true>), grid, dim3(TPB), 0, c->stream, (uint64_t *const *)dt, P,
                               nW, n_out, (const ModQ *)c->d_mod, c->logN, l);
        else
            hipLaunchKernelGGL((k_plain_mac<PW_TILE, false>), grid, dim3(TPB), 0, c->stream, (uint64_t *const *)dt, P,
                               nW, n_out, (const ModQ *)c->d_mod, c->logN, l);
    }
    std::vector<const uint64_t *> ai(n_out);
    for (uint32_t o = 0; o < n_out; ++o) ai[o] = acc + (size_t)o * 2 * l * N;
    if ((s = rescale_run(c, l, 2, n_out, ai.data(), Y.data(), scr + acc_bytes))) return s;
    c->ops[OP_PT_MULT] += (uint64_t)P * n_out;
    c->ops[OP_PT_ADD] += 0;
    c->ops[OP_CT_ADD] += (uint64_t)(P - 1) * n_out;
    c->ops[OP_RESCALE] += n_out;
    HIPCHK(hipGetLastError());
    return FHE_OK;
}

}  // namespace

// Quadratic activation at depth 1 (the paper's count for g): T = Relin(x (x) x) is read
// as c2 x^2 at scale S' = S*S/c2, so c2 costs no level; c1 x joins as the integer
// multiple round(c1 S / c2) of x, c0 as round(c0 S'), and one rescale ends it.
static size_t poly_act2_item_bytes(const fhe_ctx *c, uint32_t l)
{
    return 7 * (size_t)l * c->N * sizeof(uint64_t) + ks_scratch_bytes(c, l, 1) + rescale_scratch_bytes(c, l, 2, 1);
}
static fhe_status poly_act2(fhe_ctx *c, const fhe_evk *rlk, const fhe_ct *x, uint32_t n, const double *coef, fhe_ct *y)
{
    fhe_status s;
    const uint32_t l = x[0].limbs;
    const double S = x[0].scale;
    const size_t N = c->N, w3 = 3 * (size_t)l * N, w2 = 2 * (size_t)l * N;
    // workspace: T3 [n][3][l], U [n][2][l], B [n][2][l]
    uint8_t *ws;
    if ((s = ctx_workspace(c, (size_t)n * (w3 + 2 * w2) * sizeof(uint64_t), &ws))) return s;
    uint64_t *T3 = (uint64_t *)ws, *U = T3 + n * w3, *Bw = U + n * w2;
    std::vector<const uint64_t *> xin(n), d2(n), ad(2 * (size_t)n), Uc(n), Bc(n);
    std::vector<uint64_t *> Tp(n), Up(n), Bp(n), Yp(n);
    std::vector<uint32_t> ls(n, l);
    for (uint32_t i = 0; i < n; ++i) {
        xin[i] = x[i].d;
        Tp[i] = T3 + i * w3;
        Up[i] = U + i * w2;
        Bp[i] = Bw + i * w2;
        d2[i] = Tp[i] + 2 * (size_t)l * N;
        ad[2 * i] = Tp[i];
        ad[2 * i + 1] = Tp[i] + (size_t)l * N;
        Uc[i] = Up[i];
        Bc[i] = Bp[i];
        Yp[i] = y[i].d;
    }
    if ((s = tensor_run(c, n, ls.data(), xin.data(), xin.data(), Tp.data()))) return s;
    std::vector<const uint64_t *> ek(n, rlk->d);
    if ((s = ks_run(c, l, n, d2.data(), nullptr, ek.data(), Up.data(), ad.data(), nullptr))) return s;
    const double Sp = S * S / coef[2];
    Consts64 k1, k0;
    if ((s = const_residues(c, coef[1] * S / coef[2], l, &k1))) return s;
    if ((s = ew_batch(c, EW_MULC, l, l, 2, n, xin.data(), nullptr, Bp.data(), k1))) return s;
    if ((s = ew_batch(c, EW_ADD, l, l, 2, n, Uc.data(), Bc.data(), Up.data(), zero_consts()))) return s;
    if ((s = const_residues(c, coef[0] * Sp, l, &k0))) return s;
    if ((s = ew_batch(c, EW_ADDC, l, l, 2, n, Uc.data(), nullptr, Up.data(), k0))) return s;
    if ((s = rescale_many(c, l, n, Uc, Yp))) return s;
    for (uint32_t i = 0; i < n; ++i) y[i].scale = Sp / (double)c->mod[l - 1];
    c->ops[OP_CT_MULT] += n;
    c->ops[OP_RELIN] += n;
    c->ops[OP_PT_MULT] += n;
    c->ops[OP_PT_ADD] += n;
    c->ops[OP_CT_ADD] += n;
    return FHE_OK;
}

extern "C" {

fhe_status fhe_conv2d_packed(fhe_ctx *c, const fhe_evk *rlk, const fhe_evk *keys, uint32_t nkeys, const fhe_ct *X,
                             uint32_t Cin, const fhe_ct *Wt, uint32_t Cout, uint32_t k, uint32_t dil,
                             uint32_t frame_w, fhe_ct *Y)
{
    fhe_status s;
    if (!c || !rlk || !rlk->d || !X || !Wt || !Y || (nkeys && !keys))
        return fhe_fail(FHE_EINVAL, "fhe_conv2d_packed: null argument");
    if (!Cin || !Cout || !k || !(k & 1) || !dil || !frame_w)
        return fhe_fail(FHE_EINVAL, "fhe_conv2d_packed: zero dimension or even kernel size");
    if (rlk->galois != 0) return fhe_fail(FHE_ENOKEY, "fhe_conv2d_packed: needs the relinearisation key");
    const uint32_t l = X[0].limbs, kk = k * k;
    if (l < 2) return fhe_fail(FHE_ELEVEL, "fhe_conv2d_packed: inputs need two limbs");
    for (uint32_t i = 0; i < Cin; ++i) {
        if ((s = chk2(&X[i], l, "fhe_conv2d_packed"))) return s;
        if (!scales_match(X[i].scale, X[0].scale)) return fhe_fail(FHE_ESCALE, "fhe_conv2d_packed: input scales differ");
    }
    for (uint32_t i = 0; i < Cout * Cin * kk; ++i) {
        if ((s = chk2(&Wt[i], l, "fhe_conv2d_packed"))) return s;
        if (!scales_match(Wt[i].scale, Wt[0].scale)) return fhe_fail(FHE_ESCALE, "fhe_conv2d_packed: weight scales differ");
    }
    for (uint32_t o = 0; o < Cout; ++o)
        if ((s = chk2(&Y[o], l - 1, "fhe_conv2d_packed"))) return s;
    if (!scale_has_room(c, l - 1, X[0].scale * Wt[0].scale / (double)c->mod[l - 1]))
        return scale_room_error("fhe_conv2d_packed");
    // rotation step of tap t = (p, q), row-major
    const int64_t half = k / 2;
    std::vector<int64_t> step(kk);
    std::vector<const fhe_evk *> tapkey(kk, nullptr);
    uint32_t nz = 0;
    for (uint32_t t = 0; t < kk; ++t) {
        step[t] = (int64_t)dil * (((int64_t)(t / k) - half) * (int64_t)frame_w + ((int64_t)(t % k) - half));
        if (!step[t]) continue;
        ++nz;
        if (!(tapkey[t] = find_key(keys, nkeys, fhe_galois_elt(c, (int32_t)step[t]))))
            return fhe_fail(FHE_ENOKEY, "fhe_conv2d_packed: no Galois key for step " + std::to_string(step[t]));
    }
    const size_t ct_words = 2 * (size_t)l * c->N;
    uint8_t *ws;
    if ((s = ctx_workspace(c, (size_t)Cin * nz * ct_words * sizeof(uint64_t), &ws))) return s;
    uint64_t *rot = (uint64_t *)ws;
    // R[ci][t]: the input itself for the centre tap, else its rotation
    std::vector<uint64_t *> R((size_t)Cin * kk);
    std::vector<const uint64_t *> ri;
    std::vector<const fhe_evk *> rk;
    std::vector<uint64_t *> ro;
    for (uint32_t ci = 0; ci < Cin; ++ci)
        for (uint32_t t = 0; t < kk; ++t) {
            if (!step[t]) {
                R[(size_t)ci * kk + t] = X[ci].d;
                continue;
            }
            uint64_t *dst = rot + ro.size() * ct_words;
            R[(size_t)ci * kk + t] = dst;
            ri.push_back(X[ci].d);
            rk.push_back(tapkey[t]);
            ro.push_back(dst);
        }
    if ((s = rotate_run(c, l, (uint32_t)ro.size(), ri.data(), rk.data(), ro.data()))) return s;
    std::vector<uint64_t *> A, B, Yp;
    std::vector<uint32_t> off{0};
    for (uint32_t co = 0; co < Cout; ++co) {
        for (uint32_t ci = 0; ci < Cin; ++ci)
            for (uint32_t t = 0; t < kk; ++t) {
                A.push_back(R[(size_t)ci * kk + t]);
                B.push_back(Wt[((size_t)co * Cin + ci) * kk + t].d);
            }
        off.push_back((uint32_t)A.size());
        Yp.push_back(Y[co].d);
    }
    if ((s = mac_relin_rescale(c, rlk, l, A, B, off, Yp))) return s;
    const double so = X[0].scale * Wt[0].scale / (double)c->mod[l - 1];
    for (uint32_t o = 0; o < Cout; ++o) Y[o].scale = so;
    return FHE_OK;
}

}  // extern "C"

static size_t poly_act3_item_bytes(const fhe_ctx *c, uint32_t l)
{
    // workspace T, U, A, Bq; the products inside bound their own scratch
    return (2 * (size_t)l + 4 * ((size_t)l - 1) + 2 * ((size_t)l - 2)) * c->N * sizeof(uint64_t) +
           rescale_scratch_bytes(c, l, 2, 1);
}
// Cubic activation at depth 2: (c3 u + c2) u^2 + (c1 u + c0), each constant an integer
// multiple chosen so that the branches meet at one scale.
static fhe_status poly_act3(fhe_ctx *c, const fhe_evk *rlk, const fhe_ct *x, uint32_t n, const double *coef,
                            fhe_ct *y)
{
    fhe_status s;
    const uint32_t l = x[0].limbs;
    const double S = x[0].scale;
    const size_t N = c->N, w1 = 2 * (size_t)(l - 1) * N, w2 = 2 * (size_t)(l - 2) * N;
    // workspace: T [n][2][l], U [n][2][l-1], A [n][2][l-1], Bq [n][2][l-2]
    uint8_t *ws;
    if ((s = ctx_workspace(c, (size_t)n * (2 * (size_t)l * N + 2 * w1 + w2) * sizeof(uint64_t), &ws))) return s;
    uint64_t *T = (uint64_t *)ws, *U = T + (size_t)n * 2 * l * N, *Aw = U + n * w1, *Bq = Aw + n * w1;
    std::vector<const uint64_t *> xin(n), Tc(n), Ac(n), Bc(n);
    std::vector<uint64_t *> Tp(n), Up(n), Ap(n), Bp(n), Yp(n);
    for (uint32_t i = 0; i < n; ++i) {
        xin[i] = x[i].d;
        Tp[i] = T + (size_t)i * 2 * l * N;
        Up[i] = U + i * w1;
        Ap[i] = Aw + i * w1;
        Bp[i] = Bq + i * w2;
        Yp[i] = y[i].d;
        Tc[i] = Tp[i];
        Ac[i] = Ap[i];
        Bc[i] = Bp[i];
    }
    const double ql = (double)c->mod[l - 1], ql2 = (double)c->mod[l - 2];
    // a = Rescale(round(c3 * q_(l-1)) * x) + c2
    Consts64 k1, k2;
    if ((s = const_residues(c, coef[3] * ql, l, &k1))) return s;
    if ((s = ew_batch(c, EW_MULC, l, l, 2, n, xin.data(), nullptr, Tp.data(), k1))) return s;
    if ((s = rescale_many(c, l, n, Tc, Ap))) return s;
    const double sA = S * ql / ql;
    if ((s = const_residues(c, coef[2] * sA, l - 1, &k2))) return s;
    if ((s = ew_batch(c, EW_ADDC, l - 1, l - 1, 2, n, Ac.data(), nullptr, Ap.data(), k2))) return s;
    c->ops[OP_PT_MULT] += n;
    c->ops[OP_PT_ADD] += n;
    std::vector<uint64_t *> A1(Ap.begin(), Ap.end()), B1;
    std::vector<uint32_t> off(n + 1);
    for (uint32_t i = 0; i <= n; ++i) off[i] = i;
    // u^2, then p = Rescale(Relin(a (x) u^2))
    std::vector<uint64_t *> X2(n);
    for (uint32_t i = 0; i < n; ++i) X2[i] = x[i].d;
    if ((s = mac_relin_rescale(c, rlk, l, X2, X2, off, Up))) return s;
    const double sU = S * S / ql;
    if ((s = mac_relin_rescale(c, rlk, l - 1, A1, Up, off, Yp))) return s;
    const double sp = sA * sU / ql2;
    // b = Rescale(round(c1 * s1) * x at l-1 limbs) + c0, s1 chosen so that b lands on sp
    const double s1 = sp * ql2 / S;
    Consts64 k3, k4;
    if ((s = const_residues(c, coef[1] * s1, l - 1, &k3))) return s;
    if ((s = ew_batch(c, EW_MULC, l - 1, l, 2, n, xin.data(), nullptr, Tp.data(), k3))) return s;
    if ((s = rescale_many(c, l - 1, n, Tc, Bp))) return s;
    const double sB = S * s1 / ql2;
    if ((s = const_residues(c, coef[0] * sB, l - 2, &k4))) return s;
    if ((s = ew_batch(c, EW_ADDC, l - 2, l - 2, 2, n, Bc.data(), nullptr, Bp.data(), k4))) return s;
    std::vector<const uint64_t *> Yc(Yp.begin(), Yp.end());
    if ((s = ew_batch(c, EW_ADD, l - 2, l - 2, 2, n, Yc.data(), Bc.data(), Yp.data(), zero_consts()))) return s;
    c->ops[OP_PT_MULT] += n;
    c->ops[OP_PT_ADD] += n;
    c->ops[OP_CT_ADD] += n;
    for (uint32_t i = 0; i < n; ++i) y[i].scale = sp;
    return FHE_OK;
}

extern "C" {

// Every input is validated first; the items then go through in chunks whose layer
// workspace and scratch stay near 2 GiB, so the memory a call takes does not grow
// with the number of ciphertexts.
fhe_status fhe_poly_act(fhe_ctx *c, const fhe_evk *rlk, const fhe_ct *x, uint32_t n, const double *coef, uint32_t deg,
                        fhe_ct *y)
{
    fhe_status s;
    if (!c || !rlk || !rlk->d || !x || !y || !coef || !n) return fhe_fail(FHE_EINVAL, "fhe_poly_act: null or empty");
    if (rlk->galois != 0) return fhe_fail(FHE_ENOKEY, "fhe_poly_act: needs the relinearisation key");
    if (deg != 2 && deg != 3) return fhe_fail(FHE_EINVAL, "fhe_poly_act: degree must be 2 or 3");
    const uint32_t l = x[0].limbs, depth = deg == 2 ? 1 : 2;
    if (l < depth + 1)
        return fhe_fail(FHE_ELEVEL, deg == 2 ? "fhe_poly_act: degree 2 needs two limbs (depth 1)"
                                             : "fhe_poly_act: inputs need three limbs (depth 2)");
    if (deg == 2 && !(coef[2] > 0.0))   // it becomes a factor of the output scale
        return fhe_fail(FHE_EINVAL, "fhe_poly_act: degree 2 needs a positive quadratic coefficient");
    const double S = x[0].scale;
    for (uint32_t i = 0; i < n; ++i) {
        if ((s = chk2(&x[i], l, "fhe_poly_act")) || (s = chk2(&y[i], l - depth, "fhe_poly_act"))) return s;
        if (x[i].scale != S) return fhe_fail(FHE_ESCALE, "fhe_poly_act: input scales differ");
    }
    // output scale: depth 1, S^2 / c2 / q_(l-1); depth 2, S (S^2 / q_(l-1)) / q_(l-2)
    const double so = deg == 2 ? S * S / coef[2] / (double)c->mod[l - 1]
                               : S * (S * S / (double)c->mod[l - 1]) / (double)c->mod[l - 2];
    if (!scale_has_room(c, l - depth, so)) return scale_room_error("fhe_poly_act");
    const size_t per = deg == 2 ? poly_act2_item_bytes(c, l) : poly_act3_item_bytes(c, l);
    const uint32_t C = (uint32_t)std::max<size_t>(1, std::min<size_t>(n, ((size_t)2 << 30) / per));
    for (uint32_t t0 = 0; t0 < n; t0 += C) {
        const uint32_t cn = std::min(C, n - t0);
        s = deg == 2 ? poly_act2(c, rlk, x + t0, cn, coef, y + t0) : poly_act3(c, rlk, x + t0, cn, coef, y + t0);
        if (s) return s;
    }
    return FHE_OK;
}

fhe_status fhe_avgpool2x2(fhe_ctx *c, const fhe_evk *keys, uint32_t nkeys, const fhe_ct *x, uint32_t n,
                          uint32_t dil, uint32_t frame_w, const fhe_pt *mask, fhe_ct *y)
{
    fhe_status s;
    if (!c || !keys || !x || !y || !mask || !mask->d || !n || !dil || !frame_w)
        return fhe_fail(FHE_EINVAL, "fhe_avgpool2x2: null or empty");
    const uint32_t l = x[0].limbs;
    if (l < 2) return fhe_fail(FHE_ELEVEL, "fhe_avgpool2x2: inputs need two limbs");
    if (mask->limbs != l) return fhe_fail(FHE_ELEVEL, "fhe_avgpool2x2: mask must have the inputs' limbs");
    for (uint32_t i = 0; i < n; ++i)
        if ((s = chk2(&x[i], l, "fhe_avgpool2x2")) || (s = chk2(&y[i], l - 1, "fhe_avgpool2x2"))) return s;
    const int32_t st1 = (int32_t)dil, st2 = (int32_t)(frame_w * dil);
    const fhe_evk *k1 = find_key(keys, nkeys, fhe_galois_elt(c, st1));
    const fhe_evk *k2 = find_key(keys, nkeys, fhe_galois_elt(c, st2));
    if (!k1 || !k2) return fhe_fail(FHE_ENOKEY, "fhe_avgpool2x2: missing Galois key");
    const size_t cw = 2 * (size_t)l * c->N;
    uint8_t *ws;
    if ((s = ctx_workspace(c, 2 * (size_t)n * cw * sizeof(uint64_t), &ws))) return s;
    uint64_t *R1 = (uint64_t *)ws, *R2 = R1 + n * cw;
    std::vector<const uint64_t *> xin(n), r1c(n), r2c(n);
    std::vector<uint64_t *> r1(n), r2(n), yo(n);
    std::vector<const fhe_evk *> kv1(n, k1), kv2(n, k2);
    std::vector<const uint64_t *> mk(n, mask->d);
    for (uint32_t i = 0; i < n; ++i) {
        xin[i] = x[i].d;
        r1[i] = R1 + i * cw;
        r2[i] = R2 + i * cw;
        r1c[i] = r1[i];
        r2c[i] = r2[i];
        yo[i] = y[i].d;
    }
    const Consts64 z = zero_consts();
    // s = x + rot(x, dil); s = s + rot(s, frame_w dil); y = Rescale(s * mask)
    if ((s = rotate_run(c, l, n, xin.data(), kv1.data(), r1.data()))) return s;
    if ((s = ew_batch(c, EW_ADD, l, l, 2, n, xin.data(), r1c.data(), r1.data(), z))) return s;
    if ((s = rotate_run(c, l, n, r1c.data(), kv2.data(), r2.data()))) return s;
    if ((s = ew_batch(c, EW_ADD, l, l, 2, n, r1c.data(), r2c.data(), r2.data(), z))) return s;
    if ((s = ew_batch(c, EW_MULPT, l, l, 2, n, r2c.data(), mk.data(), r1.data(), z))) return s;
    if ((s = rescale_many(c, l, n, r1c, yo))) return s;
    c->ops[OP_CT_ADD] += 2 * (uint64_t)n;
    c->ops[OP_PT_MULT] += n;
    for (uint32_t i = 0; i < n; ++i) y[i].scale = x[i].scale * mask->scale / (double)c->mod[l - 1];
    return FHE_OK;
}

fhe_status fhe_fc_packed(fhe_ctx *c, const fhe_evk *rlk, const fhe_evk *keys, uint32_t nkeys, const fhe_ct *x,
                         uint32_t n_in, const fhe_ct *Wt, uint32_t n_out, uint32_t frame_slots, fhe_ct *y)
{
    fhe_status s;
    if (!c || !rlk || !rlk->d || !x || !Wt || !y || !n_in || !n_out || (nkeys && !keys))
        return fhe_fail(FHE_EINVAL, "fhe_fc_packed: null or empty");
    if (rlk->galois != 0) return fhe_fail(FHE_ENOKEY, "fhe_fc_packed: needs the relinearisation key");
    if (!frame_slots || (frame_slots & (frame_slots - 1)) || frame_slots > c->N / 2)
        return fhe_fail(FHE_EINVAL, "fhe_fc_packed: frame size must be a power of two up to N/2");
    const uint32_t l = x[0].limbs;
    if (l < 2) return fhe_fail(FHE_ELEVEL, "fhe_fc_packed: inputs need two limbs");
    for (uint32_t i = 0; i < n_in; ++i) {
        if ((s = chk2(&x[i], l, "fhe_fc_packed"))) return s;
        if (!scales_match(x[i].scale, x[0].scale)) return fhe_fail(FHE_ESCALE, "fhe_fc_packed: input scales differ");
    }
    for (uint32_t i = 0; i < n_in * n_out; ++i) {
        if ((s = chk2(&Wt[i], l, "fhe_fc_packed"))) return s;
        if (!scales_match(Wt[i].scale, Wt[0].scale)) return fhe_fail(FHE_ESCALE, "fhe_fc_packed: weight scales differ");
    }
    for (uint32_t o = 0; o < n_out; ++o)
        if ((s = chk2(&y[o], l - 1, "fhe_fc_packed"))) return s;
    if (!scale_has_room(c, l - 1, x[0].scale * Wt[0].scale / (double)c->mod[l - 1]))
        return scale_room_error("fhe_fc_packed");
    std::vector<const fhe_evk *> sumkey;
    for (uint32_t i = 1; i < frame_slots; i *= 2) {
        const fhe_evk *kk = find_key(keys, nkeys, fhe_galois_elt(c, (int32_t)i));
        if (!kk) return fhe_fail(FHE_ENOKEY, "fhe_fc_packed: no Galois key for step " + std::to_string(i));
        sumkey.push_back(kk);
    }
    const size_t cw = 2 * (size_t)(l - 1) * c->N;
    uint8_t *ws;
    if ((s = ctx_workspace(c, 2 * (size_t)n_out * cw * sizeof(uint64_t), &ws))) return s;
    uint64_t *Z = (uint64_t *)ws, *R = Z + n_out * cw;
    std::vector<uint64_t *> A, B, zp(n_out), rp(n_out), yp(n_out);
    std::vector<const uint64_t *> zc(n_out), rc(n_out);
    std::vector<uint32_t> off{0};
    for (uint32_t o = 0; o < n_out; ++o) {
        for (uint32_t i = 0; i < n_in; ++i) {
            A.push_back(x[i].d);
            B.push_back(Wt[(size_t)o * n_in + i].d);
        }
        off.push_back((uint32_t)A.size());
        zp[o] = Z + o * cw;
        rp[o] = R + o * cw;
        zc[o] = zp[o];
        rc[o] = rp[o];
        yp[o] = y[o].d;
    }
    if ((s = mac_relin_rescale(c, rlk, l, A, B, off, zp))) return s;
    const Consts64 zk = zero_consts();
    // z += rot(z, i) for i = 1, 2, ..., frame_slots / 2; the last sum goes to y
    for (size_t j = 0; j < sumkey.size(); ++j) {
        std::vector<const fhe_evk *> kv(n_out, sumkey[j]);
        if ((s = rotate_run(c, l - 1, n_out, zc.data(), kv.data(), rp.data()))) return s;
        const bool last = j + 1 == sumkey.size();
        if ((s = ew_batch(c, EW_ADD, l - 1, l - 1, 2, n_out, zc.data(), rc.data(), last ? yp.data() : zp.data(), zk)))
            return s;
        c->ops[OP_CT_ADD] += n_out;
    }
    if (sumkey.empty())
        if ((s = ew_batch(c, EW_COPY, l - 1, l - 1, 2, n_out, zc.data(), nullptr, yp.data(), zk))) return s;
    const double so = x[0].scale * Wt[0].scale / (double)c->mod[l - 1];
    for (uint32_t o = 0; o < n_out; ++o) y[o].scale = so;
    return FHE_OK;
}


fhe_status fhe_conv2d_packed_pw(fhe_ctx *c, const fhe_evk *keys, uint32_t nkeys, const fhe_ct *X, uint32_t Cin,
                                const double *w, uint32_t Cout, uint32_t k, uint32_t dil, uint32_t frame_w,
                                double wscale, fhe_ct *Y)
{
    fhe_status s;
    if (!c || !X || !w || !Y || (nkeys && !keys)) return fhe_fail(FHE_EINVAL, "fhe_conv2d_packed_pw: null argument");
    if (!Cin || !Cout || !k || !(k & 1) || !dil || !frame_w || !(wscale > 0.0))
        return fhe_fail(FHE_EINVAL, "fhe_conv2d_packed_pw: zero dimension, even kernel size or bad scale");
    const uint32_t l = X[0].limbs, kk = k * k;
    if (l < 2) return fhe_fail(FHE_ELEVEL, "fhe_conv2d_packed_pw: inputs need two limbs");
    for (uint32_t i = 0; i < Cin; ++i) {
        if ((s = chk2(&X[i], l, "fhe_conv2d_packed_pw"))) return s;
        if (!scales_match(X[i].scale, X[0].scale)) return fhe_fail(FHE_ESCALE, "fhe_conv2d_packed_pw: input scales differ");
    }
    for (uint32_t o = 0; o < Cout; ++o)
        if ((s = chk2(&Y[o], l - 1, "fhe_conv2d_packed_pw"))) return s;
    if (!scale_has_room(c, l - 1, X[0].scale * wscale / (double)c->mod[l - 1]))
        return scale_room_error("fhe_conv2d_packed_pw");
    const int64_t half = k / 2;
    std::vector<int64_t> step(kk);
    std::vector<const fhe_evk *> tapkey(kk, nullptr);
    uint32_t nz = 0;
    for (uint32_t t = 0; t < kk; ++t) {
        step[t] = (int64_t)dil * (((int64_t)(t / k) - half) * (int64_t)frame_w + ((int64_t)(t % k) - half));
        if (!step[t]) continue;
        ++nz;
        if (!(tapkey[t] = find_key(keys, nkeys, fhe_galois_elt(c, (int32_t)step[t]))))
            return fhe_fail(FHE_ENOKEY, "fhe_conv2d_packed_pw: no Galois key for step " + std::to_string(step[t]));
    }
    const size_t ct_words = 2 * (size_t)l * c->N;
    uint8_t *ws;
    if ((s = ctx_workspace(c, (size_t)Cin * nz * ct_words * sizeof(uint64_t), &ws))) return s;
    uint64_t *rot = (uint64_t *)ws;
    std::vector<uint64_t *> R((size_t)Cin * kk);
    std::vector<const uint64_t *> ri;
    std::vector<const fhe_evk *> rk;
    std::vector<uint64_t *> ro;
    for (uint32_t ci = 0; ci < Cin; ++ci)
        for (uint32_t t = 0; t < kk; ++t) {
            if (!step[t]) {
                R[(size_t)ci * kk + t] = X[ci].d;
                continue;
            }
            uint64_t *dst = rot + ro.size() * ct_words;
            R[(size_t)ci * kk + t] = dst;
            ri.push_back(X[ci].d);
            rk.push_back(tapkey[t]);
            ro.push_back(dst);
        }
    if ((s = rotate_run(c, l, (uint32_t)ro.size(), ri.data(), rk.data(), ro.data()))) return s;
    std::vector<uint64_t *> Yp(Cout);
    for (uint32_t o = 0; o < Cout; ++o) Yp[o] = Y[o].d;
    // weights w[(co*Cin + ci)*k*k + t] follow the A order (ci, t) per output
    if ((s = plain_mac_rescale(c, l, R, w, wscale, {}, Cout, Yp))) return s;
    const double so = X[0].scale * wscale / (double)c->mod[l - 1];
    for (uint32_t o = 0; o < Cout; ++o) Y[o].scale = so;
    return FHE_OK;
}

fhe_status fhe_fc_packed_pw(fhe_ctx *c, const fhe_evk *keys, uint32_t nkeys, const fhe_ct *x, uint32_t n_in,
                            const fhe_pt *Wt, uint32_t n_out, uint32_t frame_slots, fhe_ct *y)
{
    fhe_status s;
    if (!c || !x || !Wt || !y || !n_in || !n_out || (nkeys && !keys))
        return fhe_fail(FHE_EINVAL, "fhe_fc_packed_pw: null or empty");
    if (!frame_slots || (frame_slots & (frame_slots - 1)) || frame_slots > c->N / 2)
        return fhe_fail(FHE_EINVAL, "fhe_fc_packed_pw: frame size must be a power of two up to N/2");
    const uint32_t l = x[0].limbs;
    if (l < 2) return fhe_fail(FHE_ELEVEL, "fhe_fc_packed_pw: inputs need two limbs");
    for (uint32_t i = 0; i < n_in; ++i) {
        if ((s = chk2(&x[i], l, "fhe_fc_packed_pw"))) return s;
        if (!scales_match(x[i].scale, x[0].scale)) return fhe_fail(FHE_ESCALE, "fhe_fc_packed_pw: input scales differ");
    }
    std::vector<const uint64_t *> pts((size_t)n_in * n_out);
    for (uint32_t i = 0; i < n_in * n_out; ++i) {
        if (!Wt[i].d || Wt[i].limbs != l) return fhe_fail(FHE_ELEVEL, "fhe_fc_packed_pw: weights must have l limbs");
        if (!scales_match(Wt[i].scale, Wt[0].scale)) return fhe_fail(FHE_ESCALE, "fhe_fc_packed_pw: weight scales differ");
        pts[i] = Wt[i].d;
    }
    for (uint32_t o = 0; o < n_out; ++o)
        if ((s = chk2(&y[o], l - 1, "fhe_fc_packed_pw"))) return s;
    if (!scale_has_room(c, l - 1, x[0].scale * Wt[0].scale / (double)c->mod[l - 1]))
        return scale_room_error("fhe_fc_packed_pw");
    std::vector<const fhe_evk *> sumkey;
    for (uint32_t i = 1; i < frame_slots; i *= 2) {
        const fhe_evk *kk = find_key(keys, nkeys, fhe_galois_elt(c, (int32_t)i));
        if (!kk) return fhe_fail(FHE_ENOKEY, "fhe_fc_packed_pw: no Galois key for step " + std::to_string(i));
        sumkey.push_back(kk);
    }
    const size_t cw = 2 * (size_t)(l - 1) * c->N;
    uint8_t *ws;
    if ((s = ctx_workspace(c, 2 * (size_t)n_out * cw * sizeof(uint64_t), &ws))) return s;
    uint64_t *Z = (uint64_t *)ws, *R = Z + n_out * cw;
    std::vector<uint64_t *> A(n_in), zp(n_out), rp(n_out), yp(n_out);
    std::vector<const uint64_t *> zc(n_out), rc(n_out);
    for (uint32_t i = 0; i < n_in; ++i) A[i] = x[i].d;
    for (uint32_t o = 0; o < n_out; ++o) {
        zp[o] = Z + o * cw;
        rp[o] = R + o * cw;
        zc[o] = zp[o];
        rc[o] = rp[o];
        yp[o] = y[o].d;
    }
    if ((s = plain_mac_rescale(c, l, A, nullptr, 0.0, pts, n_out, zp))) return s;
    const Consts64 zk = zero_consts();
    for (size_t j = 0; j < sumkey.size(); ++j) {
        std::vector<const fhe_evk *> kv(n_out, sumkey[j]);
        if ((s = rotate_run(c, l - 1, n_out, zc.data(), kv.data(), rp.data()))) return s;
        const bool last = j + 1 == sumkey.size();
        if ((s = ew_batch(c, EW_ADD, l - 1, l - 1, 2, n_out, zc.data(), rc.data(), last ? yp.data() : zp.data(), zk)))
            return s;
        c->ops[OP_CT_ADD] += n_out;
    }
    if (sumkey.empty())
        if ((s = ew_batch(c, EW_COPY, l - 1, l - 1, 2, n_out, zc.data(), nullptr, yp.data(), zk))) return s;
    const double so = x[0].scale * Wt[0].scale / (double)c->mod[l - 1];
    for (uint32_t o = 0; o < n_out; ++o) y[o].scale = so;
    return FHE_OK;
}

}  // extern "C"
