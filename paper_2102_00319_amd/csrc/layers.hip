// layers.hip -- encrypted CNN layers built from batched ciphertext operations.
//
// Slot packing of the paper (Sec. 3 "Convolution Operator", Fig. 2): one
// ciphertext per pixel holding that pixel of every image of the batch in its
// slots, and one ciphertext per weight with the weight replicated in every
// slot.  A layer output is then an inner product of ciphertexts, Eq. (enc_conv):
//   Y[o] = Rescale(Relin( sum_t X[a_t] (x) W[b_t] ))
// computed for all outputs of a layer at once: one tensor multiply-accumulate
// launch over a CSR list of (input, weight) pairs, one batched key switch, one
// batched rescale, in chunks that bound the scratch memory.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>

#include "fhe_internal.h"

namespace {

constexpr int TPB = 256;
inline uint32_t blocks_for(uint64_t n, uint32_t per) { return (uint32_t)((n + per - 1) / per); }
constexpr uint64_t TAG_UNIFORM = 2, TAG_ERROR = 3, TAG_EPHEMERAL = 4;

// Tensor multiply-accumulate over tiles of outputs that share their first
// factors: tile t has P_t pairs and k_t <= TO outputs; output u of the tile
// accumulates sum_p A[p] (x) B[u][p] into a 3-poly ciphertext.  Each thread
// owns one (limb, coefficient) element and loads A[p] once for the whole tile.
// Table: [a: sum P_t][b: sum k_t P_t][out: n_out][tiles: 2 words each]
// tile words: a_off | P << 32, b_off | o0 << 32 (o0 = first output) ; k_t in the
// top 8 bits of the second word's output field (o0 < 2^24).
template <int TO>
__global__ __launch_bounds__(TPB) void k_tensor_tile(uint64_t *const *__restrict__ tab, uint32_t nA, uint32_t nB,
                                                     uint32_t n_out, const ModQ *__restrict__ mods, uint32_t logN,
                                                     uint32_t limbs)
{
    // two consecutive coefficients per thread (16-byte loads and stores)
    const uint32_t N = 1u << logN;
    // blockIdx.x = tile, blockIdx.y = coefficient block: the tiles of one block are
    // dispatched together, so their shared factors are read while still in cache
    const uint64_t e = 2 * ((uint64_t)blockIdx.y * TPB + threadIdx.x);   // limb * N + k, k even
    if (e >= ((uint64_t)limbs << logN)) return;
    const uint64_t w0 = (uint64_t)(uintptr_t)tab[nA + nB + n_out + 2 * blockIdx.x];
    const uint64_t w1 = (uint64_t)(uintptr_t)tab[nA + nB + n_out + 2 * blockIdx.x + 1];
    const uint32_t a_off = (uint32_t)w0, P = (uint32_t)(w0 >> 32), b_off = (uint32_t)w1;
    const uint32_t o0 = (uint32_t)(w1 >> 32) & 0xFFFFFF, k = (uint32_t)(w1 >> 56);
    uint64_t *const *ap = tab + a_off, *const *bp = tab + nA + b_off;
    const uint32_t limb = (uint32_t)(e >> logN);
    const uint64_t off1 = (uint64_t)limbs * N;
    const double q = mods[limb].q, qi = mods[limb].qinv;
    double d0[TO][2], d1[TO][2], d2[TO][2];
#pragma unroll
    for (int u = 0; u < TO; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h) d0[u][h] = d1[u][h] = d2[u][h] = 0.0;
    for (uint32_t p = 0; p < P; ++p) {
        const gu64 *A = gview(ap[p]);
        const double a0[2] = {u64_to_f64(A[e]), u64_to_f64(A[e + 1])};
        const double a1[2] = {u64_to_f64(A[e + off1]), u64_to_f64(A[e + off1 + 1])};
#pragma unroll
        for (int u = 0; u < TO; ++u) {
            if (u < (int)k) {
                const gu64 *Bp = gview(bp[(size_t)u * P + p]);
                const double b0[2] = {u64_to_f64(Bp[e]), u64_to_f64(Bp[e + 1])};
                const double b1[2] = {u64_to_f64(Bp[e + off1]), u64_to_f64(Bp[e + off1 + 1])};
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    d0[u][h] += mulmod(a0[h], b0[h], q, qi);
                    d1[u][h] += mulmod(a0[h], b1[h], q, qi) + mulmod(a1[h], b0[h], q, qi);
                    d2[u][h] += mulmod(a1[h], b1[h], q, qi);
                }
            }
        }
        // |mulmod| <= 0.75 q + 2^46: four pairs keep every sum below 2^53 (q < 2^50)
        if ((p & 3) == 3) {
#pragma unroll
            for (int u = 0; u < TO; ++u)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    d0[u][h] = redc(d0[u][h], q, qi);
                    d1[u][h] = redc(d1[u][h], q, qi);
                    d2[u][h] = redc(d2[u][h], q, qi);
                }
        }
    }
#pragma unroll
    for (int u = 0; u < TO; ++u) {
        if (u < (int)k) {
            gu64 *out = gview(tab[nA + nB + o0 + u]);
            out[e] = f64_to_u64(canon(d0[u][0], q, qi));
            out[e + 1] = f64_to_u64(canon(d0[u][1], q, qi));
            out[e + off1] = f64_to_u64(canon(d1[u][0], q, qi));
            out[e + off1 + 1] = f64_to_u64(canon(d1[u][1], q, qi));
            out[e + 2 * off1] = f64_to_u64(canon(d2[u][0], q, qi));
            out[e + 2 * off1 + 1] = f64_to_u64(canon(d2[u][1], q, qi));
        }
    }
}
constexpr int MAC_TILE = 8;

// Two-group tiles: TG groups whose outputs pair the same B lists with their own A
// lists (conv positions next to each other: one window each, the same weights per
// channel).  Group g has its A list at a_off + g*P; output u of every group uses the
// B list at b_off + u*P; output (g, u) is tab[nA + nB + o0 + g*k + u].  Each B
// element loaded serves all TG groups.  One coefficient per thread.  Tile words
// (after the single-group tiles, from tile0 on): a_off | P << 32 | tg << 56,
// b_off | o0 << 32 | k << 56.
template <int TG, int TO>
__global__ __launch_bounds__(TPB) void k_tensor_tile2(uint64_t *const *__restrict__ tab, uint32_t nA, uint32_t nB,
                                                      uint32_t n_out, uint32_t tile0, const ModQ *__restrict__ mods,
                                                      uint32_t logN, uint32_t limbs)
{
    const uint64_t e = (uint64_t)blockIdx.y * TPB + threadIdx.x;   // limb * N + k; blockIdx.x = tile
    if (e >= ((uint64_t)limbs << logN)) return;
    const uint64_t w0 = (uint64_t)(uintptr_t)tab[nA + nB + n_out + 2 * (tile0 + blockIdx.x)];
    const uint64_t w1 = (uint64_t)(uintptr_t)tab[nA + nB + n_out + 2 * (tile0 + blockIdx.x) + 1];
    const uint32_t a_off = (uint32_t)w0, P = (uint32_t)(w0 >> 32) & 0xFFFFFF, tg = (uint32_t)(w0 >> 56);
    const uint32_t b_off = (uint32_t)w1, o0 = (uint32_t)(w1 >> 32) & 0xFFFFFF, k = (uint32_t)(w1 >> 56);
    uint64_t *const *ap = tab + a_off, *const *bp = tab + nA + b_off;
    const uint32_t limb = (uint32_t)(e >> logN);
    const uint64_t off1 = (uint64_t)limbs << logN;
    const double q = mods[limb].q, qi = mods[limb].qinv;
    double d0[TG][TO], d1[TG][TO], d2[TG][TO];
#pragma unroll
    for (int g = 0; g < TG; ++g)
#pragma unroll
        for (int u = 0; u < TO; ++u) d0[g][u] = d1[g][u] = d2[g][u] = 0.0;
    for (uint32_t p = 0; p < P; ++p) {
        double a0[TG], a1[TG];
#pragma unroll
        for (int g = 0; g < TG; ++g) {
            a0[g] = a1[g] = 0.0;
            if (g < (int)tg) {
                const gu64 *A = gview(ap[(size_t)g * P + p]);
                a0[g] = u64_to_f64(A[e]);
                a1[g] = u64_to_f64(A[e + off1]);
            }
        }
#pragma unroll
        for (int u = 0; u < TO; ++u) {
            if (u < (int)k) {
                const gu64 *Bp = gview(bp[(size_t)u * P + p]);
                const double b0 = u64_to_f64(Bp[e]), b1 = u64_to_f64(Bp[e + off1]);
#pragma unroll
                for (int g = 0; g < TG; ++g) {
                    d0[g][u] += mulmod(a0[g], b0, q, qi);
                    d1[g][u] += mulmod(a0[g], b1, q, qi) + mulmod(a1[g], b0, q, qi);
                    d2[g][u] += mulmod(a1[g], b1, q, qi);
                }
            }
        }
        // |mulmod| <= 0.75 q + 2^46: four pairs keep every sum below 2^53 (q < 2^50)
        if ((p & 3) == 3) {
#pragma unroll
            for (int g = 0; g < TG; ++g)
#pragma unroll
                for (int u = 0; u < TO; ++u) {
                    d0[g][u] = redc(d0[g][u], q, qi);
                    d1[g][u] = redc(d1[g][u], q, qi);
                    d2[g][u] = redc(d2[g][u], q, qi);
                }
        }
    }
#pragma unroll
    for (int g = 0; g < TG; ++g)
#pragma unroll
        for (int u = 0; u < TO; ++u) {
            if (g < (int)tg && u < (int)k) {
                gu64 *out = gview(tab[nA + nB + o0 + g * k + u]);
                out[e] = f64_to_u64(canon(d0[g][u], q, qi));
                out[e + off1] = f64_to_u64(canon(d1[g][u], q, qi));
                out[e + 2 * off1] = f64_to_u64(canon(d2[g][u], q, qi));
            }
        }
}
constexpr int MAC_GROUPS = 2;

// ---- batched encryption of constant (slot-replicated) plaintexts
__global__ void k_small_batch(int64_t *out, const uint64_t *__restrict__ seeds, const uint64_t *__restrict__ cdt,
                              uint32_t ncdt, uint32_t N)
{
    // per item: v (ternary, tag 4, poly 0), e0 (tag 3, poly 0), e1 (tag 3, poly 1) -> out [item][3][N]
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    const uint32_t item = blockIdx.y;
    const uint64_t seed = seeds[item];
    int64_t *o = out + (size_t)item * 3 * N;
    {
        const uint64_t lim = 3ull * (0x100000000ull / 3);
        int64_t val = 0;
        for (uint64_t round = 0; round < 64; ++round) {
            uint64_t w[4];
            philox4x64_10(seed, TAG_EPHEMERAL, k, 0, 0, round, w);
            bool found = false;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint64_t u = w[i] & 0xffffffffull;
                if (!found && u < lim) { val = (int64_t)(u % 3) - 1; found = true; }
            }
            if (found) break;
        }
        o[k] = val;
    }
    for (uint64_t pid = 0; pid < 2; ++pid) {
        uint64_t w[4];
        philox4x64_10(seed, TAG_ERROR, k, 0, pid, 0, w);
        int64_t mag = 0;
        for (uint32_t i = 0; i < ncdt; ++i) mag += cdt[i] <= w[0];
        o[(size_t)(1 + pid) * N + k] = (mag != 0 && (w[1] & 1)) ? -mag : mag;
    }
}
// signed values [item][3][N] -> residues [item][3][l][N]
__global__ void k_small_batch_rns(const int64_t *__restrict__ in, uint64_t *out, const ModQ *__restrict__ mods,
                                  uint32_t logN, uint32_t l)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    const uint32_t limb = blockIdx.y, row = blockIdx.z;   // row = item * 3 + which
    const int64_t q = (int64_t)mods[limb].q;
    int64_t r = in[(size_t)row * N + k] % q;
    if (r < 0) r += q;
    out[((size_t)row * l + limb) * N + k] = (uint64_t)r;
}
// c0 = v*b + e0 + m, c1 = v*a + e1 with m the constant polynomial cres[item] (same value at
// every evaluation point); outp[item] is [2][l][N].
__global__ void k_encrypt_const(const uint64_t *__restrict__ pk, uint32_t L, const uint64_t *__restrict__ vee,
                                const int64_t *__restrict__ cvals, uint64_t *const *__restrict__ outp, uint32_t l,
                                const ModQ *__restrict__ mods, uint32_t logN)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    const uint32_t i = blockIdx.y, item = blockIdx.z;
    const double q = mods[i].q, qi = mods[i].qinv;
    const uint64_t *base = vee + (size_t)item * 3 * l * N;
    const double v = u64_to_f64(base[(size_t)i * N + k]);
    const double e0 = u64_to_f64(base[((size_t)l + i) * N + k]);
    const double e1 = u64_to_f64(base[((size_t)2 * l + i) * N + k]);
    int64_t mv = cvals[item] % (int64_t)q;
    if (mv < 0) mv += (int64_t)q;
    const double b = u64_to_f64(pk[(size_t)i * N + k]), a = u64_to_f64(pk[((size_t)L + i) * N + k]);
    const double c0 = mulmod(v, b, q, qi) + e0 + (double)mv;
    const double c1 = mulmod(v, a, q, qi) + e1;
    gu64 *o = gview(outp[item]);
    o[(size_t)i * N + k] = f64_to_u64(canon(c0, q, qi));
    o[((size_t)l + i) * N + k] = f64_to_u64(canon(c1, q, qi));
}

}  // namespace

// Y[o] = Rescale(Relin(sum over CSR pairs)) for every output; all inputs at l limbs, 2 polys.
// Outputs whose first factors are the same list (conv channels over one window,
// FC rows over one input vector) are grouped into tiles of up to MAC_TILE; two such
// groups next to each other whose outputs share their second factors (neighbouring
// conv windows) form one two-group tile that loads each second factor once.
fhe_status mac_relin_rescale(fhe_ctx *c, const fhe_evk *rlk, uint32_t l, const std::vector<uint64_t *> &A,
                             const std::vector<uint64_t *> &B, const std::vector<uint32_t> &off,
                             const std::vector<uint64_t *> &Y)
{
    const uint32_t n_out = (uint32_t)Y.size();
    if (l < 2) return fhe_fail(FHE_ELEVEL, "layer: inputs need at least 2 limbs (one rescale)");
    if (n_out >= (1u << 24)) return fhe_fail(FHE_EINVAL, "layer: too many outputs");
    const size_t N = c->N, LB = N * sizeof(uint64_t);
    // order outputs so that those sharing their A list are adjacent
    std::map<std::vector<uint64_t *>, std::vector<uint32_t>> groups;
    std::vector<std::vector<uint64_t *>> keys;
    for (uint32_t o = 0; o < n_out; ++o) {
        std::vector<uint64_t *> key(A.begin() + off[o], A.begin() + off[o + 1]);
        auto it = groups.find(key);
        if (it == groups.end()) {
            keys.push_back(key);
            groups[key].push_back(o);
        } else {
            it->second.push_back(o);
        }
    }
    std::vector<uint32_t> order, gid;
    for (size_t g = 0; g < keys.size(); ++g)
        for (uint32_t o : groups[keys[g]]) {
            order.push_back(o);
            gid.push_back((uint32_t)g);
        }
    // chunk size: bound the scratch of one chunk to about 2 GiB
    const size_t per_out = ks_scratch_bytes(c, l, 1) + (3 * (size_t)l + 2 * (size_t)l) * LB +
                           rescale_scratch_bytes(c, l, 2, 1);
    uint32_t C = (uint32_t)std::max<size_t>(1, std::min<size_t>(n_out, ((size_t)2 << 30) / per_out));
    C = std::min<uint32_t>(C, 4096);
    uint8_t *scr;
    fhe_status s;
    if ((s = ctx_scratch(c, per_out * C, &scr))) return s;
    uint8_t *ks_scr = scr;
    uint64_t *acc3 = (uint64_t *)(scr + ks_scratch_bytes(c, l, C));
    uint64_t *tmp2 = acc3 + (size_t)C * 3 * l * N;
    uint8_t *rs_scr = (uint8_t *)(tmp2 + (size_t)C * 2 * l * N);
    std::vector<const uint64_t *> kd(C), ke(C, rlk->d), ka(2 * (size_t)C);
    std::vector<uint64_t *> ko(C), ro(C);
    std::vector<const uint64_t *> ri(C);
    uint64_t pairs = 0;
    for (uint32_t o0 = 0; o0 < n_out; o0 += C) {
        const uint32_t cn = std::min(C, n_out - o0);
        // tiles inside this chunk: runs of one group, at most MAC_TILE outputs; two runs
        // of different groups next to each other whose outputs have the same B lists
        // (and the same pair count) form one two-group tile
        std::vector<uint64_t *> ta, tb, tout, tt, tt2;
        auto run_len = [&](uint32_t t) {
            uint32_t k = 1;
            while (t + k < cn && k < (uint32_t)MAC_TILE && gid[o0 + t + k] == gid[o0 + t]) ++k;
            return k;
        };
        auto same_b = [&](uint32_t t, uint32_t t2, uint32_t k) {
            for (uint32_t u = 0; u < k; ++u) {
                const uint32_t o = order[o0 + t + u], o2 = order[o0 + t2 + u];
                if (off[o + 1] - off[o] != off[o2 + 1] - off[o2] ||
                    !std::equal(B.begin() + off[o], B.begin() + off[o + 1], B.begin() + off[o2]))
                    return false;
            }
            return true;
        };
        for (uint32_t t = 0; t < cn;) {
            const uint32_t k = run_len(t);
            const uint32_t first = order[o0 + t];
            const uint32_t P = off[first + 1] - off[first];
            const uint32_t t2 = t + k;
            const bool pair = t2 < cn && gid[o0 + t2] != gid[o0 + t] && run_len(t2) == k && same_b(t, t2, k) &&
                              P < (1u << 24);
            const uint32_t tg = pair ? 2 : 1;
            const uint64_t a_off = ta.size(), b_off = tb.size();
            for (uint32_t g = 0; g < tg; ++g) {
                const uint32_t fg = order[o0 + t + g * k];
                ta.insert(ta.end(), A.begin() + off[fg], A.begin() + off[fg + 1]);
                for (uint32_t u = 0; u < k; ++u) pairs += P;
            }
            for (uint32_t u = 0; u < k; ++u) {
                const uint32_t o = order[o0 + t + u];
                tb.insert(tb.end(), B.begin() + off[o], B.begin() + off[o + 1]);
            }
            auto &dst = pair ? tt2 : tt;
            // single-group tile words carry P in all 32 high bits; two-group ones P < 2^24 and tg
            dst.push_back((uint64_t *)(uintptr_t)(a_off | ((uint64_t)P << 32) | (pair ? (uint64_t)tg << 56 : 0)));
            dst.push_back((uint64_t *)(uintptr_t)(b_off | ((uint64_t)t << 32) | ((uint64_t)k << 56)));
            t += tg * k;
        }
        for (uint32_t t = 0; t < cn; ++t) tout.push_back(acc3 + (size_t)t * 3 * l * N);
        std::vector<uint64_t *> tab;
        tab.reserve(ta.size() + tb.size() + tout.size() + tt.size());
        tab.insert(tab.end(), ta.begin(), ta.end());
        tab.insert(tab.end(), tb.begin(), tb.end());
        tab.insert(tab.end(), tout.begin(), tout.end());
        tab.insert(tab.end(), tt.begin(), tt.end());
        tab.insert(tab.end(), tt2.begin(), tt2.end());
        uint64_t **dt;
        if ((s = ctx_ptr_table(c, tab, &dt))) return s;
        const uint32_t ntiles = (uint32_t)(tt.size() / 2), ntiles2 = (uint32_t)(tt2.size() / 2);
        {
            ProfScope ps(c, "tensor");
            if (ntiles > 65535u || ntiles2 > 65535u) return fhe_fail(FHE_EINVAL, "layer: too many tiles in one chunk");
            if (blocks_for((uint64_t)l * N, TPB) > 65535u) return fhe_fail(FHE_EINVAL, "layer: ciphertexts too large");
            if (ntiles)
                hipLaunchKernelGGL(k_tensor_tile<MAC_TILE>, dim3(ntiles, blocks_for((uint64_t)l * N / 2, TPB)), dim3(TPB),
                                   0, c->stream, (uint64_t *const *)dt, (uint32_t)ta.size(), (uint32_t)tb.size(), cn,
                                   (const ModQ *)c->d_mod, c->logN, l);
            if (ntiles2)
                hipLaunchKernelGGL((k_tensor_tile2<MAC_GROUPS, MAC_TILE>), dim3(ntiles2, blocks_for((uint64_t)l * N, TPB)),
                                   dim3(TPB), 0, c->stream, (uint64_t *const *)dt, (uint32_t)ta.size(),
                                   (uint32_t)tb.size(), cn, ntiles, (const ModQ *)c->d_mod, c->logN, l);
        }
        for (uint32_t t = 0; t < cn; ++t) {
            uint64_t *a3 = acc3 + (size_t)t * 3 * l * N;
            kd[t] = a3 + 2 * (size_t)l * N;
            ka[2 * t] = a3;
            ka[2 * t + 1] = a3 + (size_t)l * N;
            ko[t] = tmp2 + (size_t)t * 2 * l * N;
            ri[t] = ko[t];
            ro[t] = Y[order[o0 + t]];
        }
        if ((s = ks_run(c, l, cn, kd.data(), nullptr, ke.data(), ko.data(), ka.data(), ks_scr))) return s;
        if ((s = rescale_run(c, l, 2, cn, ri.data(), ro.data(), rs_scr))) return s;
    }
    c->ops[OP_CT_MULT] += pairs;
    c->ops[OP_CT_ADD] += pairs - n_out;
    c->ops[OP_RELIN] += n_out;
    c->ops[OP_RESCALE] += n_out;
    HIPCHK(hipGetLastError());
    return FHE_OK;
}

static fhe_status chk_in(const fhe_ct *x, uint32_t l, const char *what)
{
    if (!x->d || x->polys != 2 || x->limbs != l)
        return fhe_fail(FHE_EINVAL, std::string(what) + ": every input must be a 2-poly ciphertext at the same level");
    return FHE_OK;
}

extern "C" {

fhe_status fhe_op_counts(fhe_ctx *c, uint64_t out[8])
{
    if (!c || !out) return fhe_fail(FHE_EINVAL, "fhe_op_counts: null argument");
    for (int i = 0; i < 8; ++i) out[i] = c->ops[i];
    std::memset(c->ops, 0, sizeof(c->ops));
    return FHE_OK;
}

fhe_status fhe_relin_batch(fhe_ctx *c, const fhe_evk *rlk, const fhe_ct *in3, uint32_t n, fhe_ct *out2)
{
    if (!c || !rlk || !rlk->d || !in3 || !out2 || !n) return fhe_fail(FHE_EINVAL, "fhe_relin_batch: null or empty");
    if (rlk->galois != 0) return fhe_fail(FHE_ENOKEY, "fhe_relin_batch: needs the relinearisation key");
    const uint32_t l = in3[0].limbs;
    const size_t per = (size_t)l * c->N;
    std::vector<const uint64_t *> d(n), e(n, rlk->d), a(2 * (size_t)n);
    std::vector<uint64_t *> o(n);
    for (uint32_t t = 0; t < n; ++t) {
        if (!in3[t].d || in3[t].polys != 3 || in3[t].limbs != l || !out2[t].d || out2[t].polys != 2 ||
            out2[t].limbs != l)
            return fhe_fail(FHE_EINVAL, "fhe_relin_batch: need 3-poly inputs and 2-poly outputs at one level");
        d[t] = in3[t].d + 2 * per;
        a[2 * t] = in3[t].d;
        a[2 * t + 1] = in3[t].d + per;
        o[t] = out2[t].d;
    }
    const uint32_t C = (uint32_t)std::max<size_t>(1, std::min<size_t>(n, ((size_t)2 << 30) / ks_scratch_bytes(c, l, 1)));
    uint8_t *scr;
    fhe_status s;
    if ((s = ctx_scratch(c, ks_scratch_bytes(c, l, C), &scr))) return s;
    for (uint32_t t0 = 0; t0 < n; t0 += C) {
        const uint32_t cn = std::min(C, n - t0);
        if ((s = ks_run(c, l, cn, d.data() + t0, nullptr, e.data() + t0, o.data() + t0, a.data() + 2 * t0, scr)))
            return s;
    }
    for (uint32_t t = 0; t < n; ++t) out2[t].scale = in3[t].scale;
    c->ops[OP_RELIN] += n;
    return FHE_OK;
}

fhe_status fhe_rescale_batch(fhe_ctx *c, const fhe_ct *in, uint32_t n, fhe_ct *out)
{
    if (!c || !in || !out || !n) return fhe_fail(FHE_EINVAL, "fhe_rescale_batch: null or empty");
    const uint32_t l = in[0].limbs, P = in[0].polys;
    if (l < 2) return fhe_fail(FHE_ELEVEL, "fhe_rescale_batch: one limb left");
    std::vector<const uint64_t *> ip(n);
    std::vector<uint64_t *> op(n);
    for (uint32_t t = 0; t < n; ++t) {
        if (!in[t].d || in[t].limbs != l || in[t].polys != P || !out[t].d || out[t].limbs != l - 1 ||
            out[t].polys != P)
            return fhe_fail(FHE_EINVAL, "fhe_rescale_batch: shapes differ");
        const uint64_t *ib = in[t].d, *ie = ib + (size_t)P * l * c->N;
        const uint64_t *ob = out[t].d, *oe = ob + (size_t)P * (l - 1) * c->N;
        if (ob < ie && ib < oe) return fhe_fail(FHE_EINVAL, "fhe_rescale_batch: outputs must not overlap inputs");
        ip[t] = in[t].d;
        op[t] = out[t].d;
    }
    const uint32_t C = std::min<uint32_t>(65535 / P, (uint32_t)std::max<size_t>(
                                                          1, ((size_t)2 << 30) / rescale_scratch_bytes(c, l, P, 1)));
    uint8_t *scr;
    fhe_status s;
    if ((s = ctx_scratch(c, rescale_scratch_bytes(c, l, P, std::min(C, n)), &scr))) return s;
    for (uint32_t t0 = 0; t0 < n; t0 += C) {
        const uint32_t cn = std::min(C, n - t0);
        if ((s = rescale_run(c, l, P, cn, ip.data() + t0, op.data() + t0, scr))) return s;
    }
    for (uint32_t t = 0; t < n; ++t) out[t].scale = in[t].scale / (double)c->mod[l - 1];
    c->ops[OP_RESCALE] += n;
    return FHE_OK;
}

fhe_status fhe_conv2d_slot(fhe_ctx *c, const fhe_evk *rlk, const fhe_ct *X, uint32_t H, uint32_t W, uint32_t Cin,
                           const fhe_ct *Wt, uint32_t Cout, uint32_t kh, uint32_t kw, uint32_t stride, uint32_t pad_t,
                           uint32_t pad_l, uint32_t Ho, uint32_t Wo, fhe_ct *Y)
{
    fhe_status s;
    if (!c || !rlk || !rlk->d || !X || !Wt || !Y) return fhe_fail(FHE_EINVAL, "fhe_conv2d_slot: null argument");
    if (!H || !W || !Cin || !Cout || !kh || !kw || !stride || !Ho || !Wo)
        return fhe_fail(FHE_EINVAL, "fhe_conv2d_slot: zero dimension");
    if (rlk->galois != 0) return fhe_fail(FHE_ENOKEY, "fhe_conv2d_slot: needs the relinearisation key");
    const uint32_t l = X[0].limbs;
    const double sx = X[0].scale, sw = Wt[0].scale;
    for (uint32_t i = 0; i < H * W * Cin; ++i) {
        if ((s = chk_in(&X[i], l, "fhe_conv2d_slot"))) return s;
        if (!scales_match(X[i].scale, sx)) return fhe_fail(FHE_ESCALE, "fhe_conv2d_slot: input scales differ");
    }
    for (uint32_t i = 0; i < Cout * Cin * kh * kw; ++i) {
        if ((s = chk_in(&Wt[i], l, "fhe_conv2d_slot"))) return s;
        if (!scales_match(Wt[i].scale, sw)) return fhe_fail(FHE_ESCALE, "fhe_conv2d_slot: weight scales differ");
    }
    std::vector<uint64_t *> A, B, Yp;
    std::vector<uint32_t> off{0};
    for (uint32_t co = 0; co < Cout; ++co)
        for (uint32_t i = 0; i < Ho; ++i)
            for (uint32_t j = 0; j < Wo; ++j) {
                for (uint32_t ci = 0; ci < Cin; ++ci)
                    for (uint32_t p = 0; p < kh; ++p)
                        for (uint32_t q = 0; q < kw; ++q) {
                            const int64_t y = (int64_t)i * stride + p - pad_t, x = (int64_t)j * stride + q - pad_l;
                            if (y < 0 || x < 0 || y >= (int64_t)H || x >= (int64_t)W) continue;   // zero padding
                            A.push_back(X[((size_t)ci * H + y) * W + x].d);
                            B.push_back(Wt[(((size_t)co * Cin + ci) * kh + p) * kw + q].d);
                        }
                if (A.size() == off.back()) return fhe_fail(FHE_EINVAL, "fhe_conv2d_slot: an output has no taps");
                off.push_back((uint32_t)A.size());
                fhe_ct &y = Y[((size_t)co * Ho + i) * Wo + j];
                if (!y.d || y.polys != 2 || y.limbs != l - 1)
                    return fhe_fail(FHE_EINVAL, "fhe_conv2d_slot: outputs must be 2 x (l-1)");
                Yp.push_back(y.d);
            }
    const double so = sx * sw / (double)c->mod[l - 1];
    if (!scale_has_room(c, l - 1, so)) return scale_room_error("fhe_conv2d_slot");
    if ((s = mac_relin_rescale(c, rlk, l, A, B, off, Yp))) return s;
    for (uint32_t o = 0; o < Cout * Ho * Wo; ++o) Y[o].scale = so;
    return FHE_OK;
}

fhe_status fhe_fc_slot(fhe_ctx *c, const fhe_evk *rlk, const fhe_ct *x, uint32_t n_in, const fhe_ct *Wt,
                       uint32_t n_out, fhe_ct *y)
{
    fhe_status s;
    if (!c || !rlk || !rlk->d || !x || !Wt || !y || !n_in || !n_out) return fhe_fail(FHE_EINVAL, "fhe_fc_slot: null");
    if (rlk->galois != 0) return fhe_fail(FHE_ENOKEY, "fhe_fc_slot: needs the relinearisation key");
    const uint32_t l = x[0].limbs;
    for (uint32_t i = 0; i < n_in; ++i) {
        if ((s = chk_in(&x[i], l, "fhe_fc_slot"))) return s;
        if (!scales_match(x[i].scale, x[0].scale)) return fhe_fail(FHE_ESCALE, "fhe_fc_slot: input scales differ");
    }
    std::vector<uint64_t *> A, B, Yp;
    std::vector<uint32_t> off{0};
    for (uint32_t o = 0; o < n_out; ++o) {
        for (uint32_t i = 0; i < n_in; ++i) {
            const fhe_ct &w = Wt[(size_t)o * n_in + i];
            if ((s = chk_in(&w, l, "fhe_fc_slot"))) return s;
            if (!scales_match(w.scale, Wt[0].scale)) return fhe_fail(FHE_ESCALE, "fhe_fc_slot: weight scales differ");
            A.push_back(x[i].d);
            B.push_back(w.d);
        }
        off.push_back((uint32_t)A.size());
        if (!y[o].d || y[o].polys != 2 || y[o].limbs != l - 1) return fhe_fail(FHE_EINVAL, "fhe_fc_slot: bad output");
        Yp.push_back(y[o].d);
    }
    const double so = x[0].scale * Wt[0].scale / (double)c->mod[l - 1];
    if (!scale_has_room(c, l - 1, so)) return scale_room_error("fhe_fc_slot");
    if ((s = mac_relin_rescale(c, rlk, l, A, B, off, Yp))) return s;
    for (uint32_t o = 0; o < n_out; ++o) y[o].scale = so;
    return FHE_OK;
}

fhe_status fhe_square_act(fhe_ctx *c, const fhe_evk *rlk, const fhe_ct *x, uint32_t n, fhe_ct *y)
{
    fhe_status s;
    if (!c || !rlk || !rlk->d || !x || !y || !n) return fhe_fail(FHE_EINVAL, "fhe_square_act: null");
    if (rlk->galois != 0) return fhe_fail(FHE_ENOKEY, "fhe_square_act: needs the relinearisation key");
    const uint32_t l = x[0].limbs;
    std::vector<uint64_t *> A, B, Yp;
    std::vector<uint32_t> off{0};
    for (uint32_t i = 0; i < n; ++i) {
        if ((s = chk_in(&x[i], l, "fhe_square_act"))) return s;
        if (!scale_has_room(c, l - 1, x[i].scale * x[i].scale / (double)c->mod[l - 1]))
            return scale_room_error("fhe_square_act");
        if (!y[i].d || y[i].polys != 2 || y[i].limbs != l - 1) return fhe_fail(FHE_EINVAL, "fhe_square_act: bad output");
        A.push_back(x[i].d);
        B.push_back(x[i].d);
        off.push_back(i + 1);
        Yp.push_back(y[i].d);
    }
    if ((s = mac_relin_rescale(c, rlk, l, A, B, off, Yp))) return s;
    for (uint32_t i = 0; i < n; ++i) y[i].scale = x[i].scale * x[i].scale / (double)c->mod[l - 1];
    return FHE_OK;
}

fhe_status fhe_pool2x2_sum_slot(fhe_ctx *c, const fhe_ct *x, uint32_t C, uint32_t H, uint32_t W, fhe_ct *y)
{
    fhe_status s;
    if (!c || !x || !y || !C || H < 2 || W < 2) return fhe_fail(FHE_EINVAL, "fhe_pool2x2_sum_slot: null or empty");
    const uint32_t l = x[0].limbs, Hp = H / 2, Wp = W / 2, n = C * Hp * Wp;
    for (uint32_t i = 0; i < C * H * W; ++i) {
        if ((s = chk_in(&x[i], l, "fhe_pool2x2_sum_slot"))) return s;
        if (!scales_match(x[i].scale, x[0].scale)) return fhe_fail(FHE_ESCALE, "fhe_pool2x2_sum_slot: scales differ");
    }
    std::vector<const uint64_t *> a(n), b(n), cc(n), d(n), yc(n);
    std::vector<uint64_t *> yo(n);
    for (uint32_t ch = 0; ch < C; ++ch)
        for (uint32_t i = 0; i < Hp; ++i)
            for (uint32_t j = 0; j < Wp; ++j) {
                const uint32_t o = (ch * Hp + i) * Wp + j;
                auto at = [&](uint32_t yy, uint32_t xx) { return x[((size_t)ch * H + yy) * W + xx].d; };
                if ((s = chk_in(&y[o], l, "fhe_pool2x2_sum_slot"))) return s;
                a[o] = at(2 * i, 2 * j);
                b[o] = at(2 * i, 2 * j + 1);
                cc[o] = at(2 * i + 1, 2 * j);
                d[o] = at(2 * i + 1, 2 * j + 1);
                for (const uint64_t *q : {a[o], b[o], cc[o], d[o]}) {
                    const uint64_t *ye = y[o].d + 2 * (size_t)l * c->N, *qe = q + 2 * (size_t)l * c->N;
                    if (y[o].d < qe && q < ye) return fhe_fail(FHE_EINVAL, "fhe_pool2x2_sum_slot: output overlaps an input");
                }
                yo[o] = y[o].d;
                yc[o] = y[o].d;
            }
    Consts64 z;
    std::memset(&z, 0, sizeof(z));
    if ((s = ew_batch(c, EW_ADD, l, l, 2, n, a.data(), b.data(), yo.data(), z))) return s;
    if ((s = ew_batch(c, EW_ADD, l, l, 2, n, yc.data(), cc.data(), yo.data(), z))) return s;
    if ((s = ew_batch(c, EW_ADD, l, l, 2, n, yc.data(), d.data(), yo.data(), z))) return s;
    for (uint32_t o = 0; o < n; ++o) y[o].scale = x[0].scale;
    c->ops[OP_CT_ADD] += 3 * (uint64_t)n;
    return FHE_OK;
}

fhe_status fhe_encrypt_const_batch(fhe_ctx *c, const fhe_ct *pk, const double *values, uint32_t n, double scale,
                                   const uint64_t *seeds, fhe_ct *out)
{
    if (!c || !pk || !pk->d || !values || !seeds || !out || !n)
        return fhe_fail(FHE_EINVAL, "fhe_encrypt_const_batch: null argument");
    if (pk->polys != 2 || pk->limbs != c->L) return fhe_fail(FHE_EINVAL, "fhe_encrypt_const_batch: bad public key");
    const uint32_t l = out[0].limbs, N = c->N;
    if (l < 1 || l > c->L) return fhe_fail(FHE_ELEVEL, "fhe_encrypt_const_batch: level out of range");
    for (uint32_t t = 0; t < n; ++t)
        if (!out[t].d || out[t].polys != 2 || out[t].limbs != l)
            return fhe_fail(FHE_EINVAL, "fhe_encrypt_const_batch: outputs must be 2 x limbs, all at one level");
    const size_t LB = (size_t)N * 8;
    // chunks of at most 1024 weights and about 2 GiB of scratch
    const uint32_t C = (uint32_t)std::max<size_t>(
        1, std::min<size_t>({(size_t)n, 1024, ((size_t)2 << 30) / (3 * LB * ((size_t)l + 1))}));
    // scratch: seeds [C], values [C], small [C][3][N] int64, residues [C][3][l][N]
    uint8_t *scr;
    fhe_status s;
    if ((s = ctx_scratch(c, 16 * (size_t)C + 256 + (size_t)C * 3 * LB + (size_t)C * 3 * l * LB, &scr))) return s;
    uint64_t *dseed = (uint64_t *)scr;
    int64_t *dval = (int64_t *)(dseed + C);
    int64_t *small = (int64_t *)(scr + ((16 * (size_t)C + 255) & ~(size_t)255));
    uint64_t *res = (uint64_t *)(small + (size_t)C * 3 * N);
    std::vector<int64_t> iv(C);
    std::vector<uint64_t *> optr(C);
    for (uint32_t t0 = 0; t0 < n; t0 += C) {
        const uint32_t cn = std::min(C, n - t0);
        for (uint32_t t = 0; t < cn; ++t) {
            const double v = std::nearbyint(values[t0 + t] * scale);
            if (!(std::fabs(v) < 4611686018427387904.0)) return fhe_fail(FHE_EINVAL, "constant out of range");
            iv[t] = (int64_t)v;
            optr[t] = out[t0 + t].d;
        }
        HIPCHK(hipMemcpyAsync(dseed, seeds + t0, cn * 8, hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(dval, iv.data(), cn * 8, hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));   // iv is reused by the next chunk
        uint64_t **dt;
        if ((s = ctx_ptr_table(c, std::vector<uint64_t *>(optr.begin(), optr.begin() + cn), &dt))) return s;
        hipLaunchKernelGGL(k_small_batch, dim3(blocks_for(N, TPB), cn), dim3(TPB), 0, c->stream, small,
                           (const uint64_t *)dseed, (const uint64_t *)c->d_cdt, c->ncdt, N);
        hipLaunchKernelGGL(k_small_batch_rns, dim3(blocks_for(N, TPB), l, 3 * cn), dim3(TPB), 0, c->stream,
                           (const int64_t *)small, res, (const ModQ *)c->d_mod, c->logN, l);
        uint32_t m[FHE_LIMBTAB];
        for (uint32_t i = 0; i < l; ++i) m[i] = i;
        launch_ntt_fwd(c, limbset_list(res, m, l), 3 * cn * l);
        hipLaunchKernelGGL(k_encrypt_const, dim3(blocks_for(N, TPB), l, cn), dim3(TPB), 0, c->stream,
                           (const uint64_t *)pk->d, c->L, (const uint64_t *)res, (const int64_t *)dval,
                           (uint64_t *const *)dt, l, (const ModQ *)c->d_mod, c->logN);
        for (uint32_t t = 0; t < cn; ++t) out[t0 + t].scale = scale;
    }
    HIPCHK(hipGetLastError());
    return FHE_OK;
}

}  // extern "C"
