// keyswitch.hip -- hybrid key switching (ModUp, key inner product, ModDown) for
// a batch of inputs, the operation under relinearisation and slot rotation
// (the CT-CT multiplications of Sec. 3 and the rotations of its packing).
//
// For each item b: input d_b (l_b limbs, NTT domain) read through a Galois
// permutation gal_b (0 = none), key evk_b [dnum][2][L+K][N], output out_b
// (2 polys of l_b limbs), optional addends add[2b], add[2b+1] (read through
// gal_b).  Items may sit at different levels l_b: every launch walks flat lists
// of (item, limb) or (item, digit) entries built on the host, so that one launch
// sequence serves a whole ragged batch.
//   ModUp:   digits D_j = limbs [j alpha, min((j+1) alpha, l)); each converted to
//            Q_l u P by fast basis conversion (canonical representatives);
//   inner:   u_t = sum_j D_j * evk_{j,t} over Q_l u P;
//   ModDown: ks_t = (u_t + (P-1)/2 - Conv_{P->Q}([u_t + (P-1)/2]_P)) * P^-1,
//            i.e. u_t / P rounded (up to the fast-conversion error);
//   out_t  = ks_t + add_t.
//
// Kernel sequence (every transform split into a column pass and a row pass of at
// most 2^8 elements, so that the fused row kernels run in 256-thread groups):
//   1 k_ks_intt_first   inverse row pass of d_b, gathered through gal_b  -> dc
//     inverse column pass                                               -> dc (coefficients)
//   2 k_bconv           ModUp conversion of every digit                  -> up
//   3 forward column and row passes of up
//   4 k_ks_inner        key inner product over the digits                -> uQ, uP
//   5 inverse transform of uP (coefficients)
//   6 k_bconv<true>     rounded conversion P -> Q_l                       -> z
//   7 forward column pass of z
//   8 k_ks_moddown_final forward row pass of z fused with (u - z) P^-1 + add -> out
#include <algorithm>
#include <cstring>

#include "ntt_core.h"

using namespace nttc;


namespace {

constexpr int TPB = 256;
inline uint32_t blocks_for(uint64_t n, uint32_t per) { return (uint32_t)((n + per - 1) / per); }
constexpr uint32_t GRID_Y = 65535;

// Per-item layout of one batch (device copy in the pointer table, 7 words).
struct KsItem {
    uint32_t l, nd;
    uint32_t dc_off;    // first limb of the item in dc
    uint32_t up_off;    // first limb of the item in up
    uint32_t uq_off;    // first limb of the item in uQ and z ([2][l] each)
    uint32_t pad;
    uint16_t upoff[16]; // first converted limb of digit j, relative to up_off
};
static_assert(sizeof(KsItem) == 56, "KsItem is 7 table words");
struct BcJob {          // one basis conversion: nsrc source limbs -> ndst destination limbs
    uint32_t off;       // constants in the conversion table
    uint32_t nsrc, ndst;
    uint32_t src0, dst0;   // absolute first limbs in the source and destination buffers
    uint32_t pad;
};
static_assert(sizeof(BcJob) == 24, "BcJob is 3 table words");
// Word offsets of the sections of one batch's table:
//   [d: n][evk: n][out: n][add: 2n][gal: n][items: 7n][la: sum l][upjobs: 3 sum nd]
//   [upmods: sum ups][inner: sum (l + K)][dnjobs: 3 * 2n][fl: sum 2l]
// la entries: item << 16 | limb (dc order); inner: item << 16 | x (x < l: Q limb,
// else special prime x - l); fl: item << 17 | poly << 16 | limb (z and uQ order).
struct KsTab {
    uint32_t n, K, L;
    uint32_t it, la, uj, um, il, dj, fl;
};
__device__ __forceinline__ const KsItem &tab_item(uint64_t *const *tab, const KsTab &t, uint32_t b)
{
    return reinterpret_cast<const KsItem *>(tab + t.it)[b];
}
__device__ __forceinline__ uint64_t tab_word(uint64_t *const *tab, uint32_t off, uint32_t y)
{
    return (uint64_t)(uintptr_t)tab[off + y];
}

// Fast basis conversion, one thread per coefficient, blockIdx.y + y0 = job:
//   y_t = sum_a [x_a (B/b_a)^-1]_{b_a} (B/b_a mod c_t)  mod c_t.
// ADD_HALF: sources offset by hsrc (per source limb) and results by -hdst (per
// destination limb): the rounding shift of ModDown.
template <bool ADD_HALF>
__global__ __launch_bounds__(TPB) void k_bconv(const uint64_t *__restrict__ src, uint64_t *__restrict__ dst,
                                               const double *__restrict__ ctab, const BcJob *__restrict__ jobs,
                                               uint32_t y0, uint32_t logN, const double *__restrict__ hsrc,
                                               const double *__restrict__ hdst)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    const BcJob jb = jobs[blockIdx.y + y0];
    const double *T = ctab + jb.off;
    const double *qhinv = T, *sq = T + jb.nsrc, *sqi = T + 2 * jb.nsrc, *dq = T + 3 * jb.nsrc,
                 *dqi = T + 3 * jb.nsrc + jb.ndst, *qh = T + 3 * jb.nsrc + 2 * jb.ndst;
    const uint64_t *S = src + (size_t)jb.src0 * N + k;
    uint64_t *D = dst + (size_t)jb.dst0 * N + k;
    double v[16];
#pragma unroll
    for (int a = 0; a < 16; ++a) {
        if (a < (int)jb.nsrc) {
            double x = u64_to_f64(S[(size_t)a * N]);
            if (ADD_HALF) x += hsrc[a];
            v[a] = canon(mulmod(x, qhinv[a], sq[a], sqi[a]), sq[a], sqi[a]);
        }
    }
    for (uint32_t t = 0; t < jb.ndst; ++t) {
        const double q = dq[t], qi = dqi[t];
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < 16; ++a) {
            if (a < (int)jb.nsrc) {
                acc += mulmod(v[a], qh[(size_t)a * jb.ndst + t], q, qi);
                if ((a & 3) == 3) acc = redc(acc, q, qi);
            }
        }
        if (ADD_HALF) acc -= hdst[t];
        D[(size_t)t * N] = f64_to_u64(canon(acc, q, qi));
    }
}

// 1. First (row) pass of the inverse transform of d_b, gathered through gal_b,
//    into dc as lazy FP64 bits.  blockIdx.y + y0 = entry of the la list.
template <int LOGG, int WG>
__global__ __launch_bounds__(WG) void k_ks_intt_first(uint64_t *const *__restrict__ tab, KsTab t, uint32_t y0,
                                                      uint64_t *__restrict__ dc, const ModQ *__restrict__ mods,
                                                      const double *__restrict__ itwt, uint32_t logN,
                                                      uint32_t sigma0)
{
    using Gm = Geom<LOGG, WG, false>;
    __shared__ double lds[Gm::LDS];
    const uint32_t N = 1u << logN;
    const uint32_t y = blockIdx.y + y0;
    const uint64_t e = tab_word(tab, t.la, y);
    const uint32_t b = (uint32_t)(e >> 16), i = (uint32_t)(e & 0xFFFF);
    const uint64_t *src = tab[b] + (size_t)i * N;
    const uint32_t gal = (uint32_t)tab_word(tab, 5 * t.n, b);
    const double q = mods[i].q, qinv = mods[i].qinv;
    const Gm gm(logN, blockIdx.x);
    double x[R];
#pragma unroll
    for (int k = 0; k < R; k++) x[k] = u64_to_f64(src[galois_src(gm.coal(k), gal, logN)]);
    gm.coal_to_inv_in(x, lds);
    gm.template inv<false>(x, lds, itwt + (size_t)i * N, q, qinv, 0.0, logN, sigma0);
    uint64_t *dst = dc + (size_t)y * N;
#pragma unroll
    for (int k = 0; k < R; k++) dst[gm.inv_out(k)] = f64_to_bits(x[k]);
}

// 4b. Key inner product, one thread per pair of coefficients (16-byte loads) of
//     one limb x of Q_l u P (blockIdx.y + y0 = entry of the inner list):
//     u_t[x] = sum_j D_j[x] * evk_{j,t}[x]; D_j[x] is the input limb itself
//     inside digit j, else the converted limb.
__device__ __forceinline__ void ld2(const uint64_t *p, double &a, double &b)
{
    const ulonglong2 v = *reinterpret_cast<const ulonglong2 *>(p);
    a = u64_to_f64(v.x);
    b = u64_to_f64(v.y);
}
__global__ __launch_bounds__(TPB) void k_ks_inner(uint64_t *const *__restrict__ tab, KsTab t, uint32_t y0,
                                                  const uint64_t *__restrict__ up, uint64_t *__restrict__ uQ,
                                                  uint64_t *__restrict__ uP, const ModQ *__restrict__ mods,
                                                  uint32_t alpha, uint32_t logN)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = 2 * (blockIdx.x * TPB + threadIdx.x);
    if (k >= N) return;
    const uint64_t e = tab_word(tab, t.il, blockIdx.y + y0);
    const uint32_t b = (uint32_t)(e >> 16), x = (uint32_t)(e & 0xFFFF);
    const KsItem &it = tab_item(tab, t, b);
    const uint32_t l = it.l;
    const uint32_t mx = x < l ? x : t.L + (x - l);
    const double q = mods[mx].q, qi = mods[mx].qinv;
    const uint64_t *d = tab[b], *ev = tab[t.n + b];
    const uint64_t *upb = up + (size_t)it.up_off * N;
    const size_t ML = t.L + t.K;
    double a0 = 0.0, a1 = 0.0, c0 = 0.0, c1 = 0.0;
    for (uint32_t j = 0; j < it.nd; ++j) {
        const uint32_t lo = j * alpha, hi = min(lo + alpha, l);
        double D0, D1, e00, e01, e10, e11;
        if (x >= lo && x < hi) ld2(d + (size_t)x * N + k, D0, D1);
        else {
            const uint32_t pos = x < lo ? x : x - (hi - lo);
            ld2(upb + (size_t)(it.upoff[j] + pos) * N + k, D0, D1);
        }
        ld2(ev + (((size_t)j * 2 + 0) * ML + mx) * N + k, e00, e01);
        ld2(ev + (((size_t)j * 2 + 1) * ML + mx) * N + k, e10, e11);
        a0 += mulmod(D0, e00, q, qi);
        c0 += mulmod(D1, e01, q, qi);
        a1 += mulmod(D0, e10, q, qi);
        c1 += mulmod(D1, e11, q, qi);
        if ((j & 3) == 3) {
            a0 = redc(a0, q, qi);
            c0 = redc(c0, q, qi);
            a1 = redc(a1, q, qi);
            c1 = redc(c1, q, qi);
        }
    }
    uint64_t *o0, *o1;
    if (x < l) {
        o0 = uQ + ((size_t)it.uq_off + x) * N;
        o1 = uQ + ((size_t)it.uq_off + l + x) * N;
    } else {
        o0 = uP + ((size_t)b * 2 * t.K + (x - l)) * N;
        o1 = uP + ((size_t)b * 2 * t.K + t.K + (x - l)) * N;
    }
    *reinterpret_cast<ulonglong2 *>(o0 + k) =
        make_ulonglong2(f64_to_u64(canon(a0, q, qi)), f64_to_u64(canon(c0, q, qi)));
    *reinterpret_cast<ulonglong2 *>(o1 + k) =
        make_ulonglong2(f64_to_u64(canon(a1, q, qi)), f64_to_u64(canon(c1, q, qi)));
}

// 8. Forward row pass of z fused with the ModDown finish:
//    out_t[i] = (u_t[i] - z_t[i]) * P^-1 + add_t[i].  blockIdx.y + y0 = entry of fl.
template <int LOGG, int WG>
__global__ __launch_bounds__(WG, 3) void k_ks_moddown_final(uint64_t *const *__restrict__ tab, KsTab t, uint32_t y0,
                                                         const uint64_t *__restrict__ z,
                                                         const uint64_t *__restrict__ uQ,
                                                         const ModQ *__restrict__ mods, const double *__restrict__ twt,
                                                         const double *__restrict__ pinv, uint32_t logN,
                                                         uint32_t sigma0)
{
    using Gm = Geom<LOGG, WG, false>;
    __shared__ double lds[Gm::LDS];
    const uint32_t N = 1u << logN;
    const uint32_t y = blockIdx.y + y0;
    const uint64_t e = tab_word(tab, t.fl, y);
    const uint32_t b = (uint32_t)(e >> 17), tt = (uint32_t)((e >> 16) & 1), i = (uint32_t)(e & 0xFFFF);
    const uint32_t l = tab_item(tab, t, b).l;
    const double q = mods[i].q, qinv = mods[i].qinv;
    const Gm gm(logN, blockIdx.x);
    const uint64_t *zs = z + (size_t)y * N;
    double v[R];
#pragma unroll
    for (int k = 0; k < R; k++) v[k] = bits_to_f64(zs[gm.fwd_in(k)]);
    gm.fwd(v, lds, twt + (size_t)i * N, q, qinv, logN, sigma0);
    gm.fwd_out_to_coal(v, lds);
    const uint64_t *uq = uQ + (size_t)y * N;
    const uint64_t *ad = tab[3 * t.n + 2 * b + tt];
    const uint32_t gal = (uint32_t)tab_word(tab, 5 * t.n, b);
    uint64_t *out = tab[2 * t.n + b] + ((size_t)tt * l + i) * N;
    const double pi = pinv[i];
#pragma unroll
    for (int k = 0; k < R; k++) {
        const uint32_t idx = gm.coal(k);
        double r = canon(mulmod(u64_to_f64(uq[idx]) - v[k], pi, q, qinv), q, qinv);
        if (ad) r = fold(r + u64_to_f64(ad[(size_t)i * N + galois_src(idx, gal, logN)]), q);
        out[idx] = f64_to_u64(r);
    }
}

// Column and row passes of the key-switching path (split_ks) over a flat limb
// buffer whose limb y is reduced modulo mods[lst[y] & 0xFFFF]: forward (canonical
// in, lazy bits out; row: bits in, canonical out, coalesced stores) and inverse
// column (bits in, canonical out, N^-1 folded).
template <int LOGG, int WG>
__global__ __launch_bounds__(WG) void k_col_fwd(uint64_t *__restrict__ base, const uint64_t *__restrict__ lst,
                                                uint32_t y0, const ModQ *__restrict__ mods,
                                                const double *__restrict__ twt, uint32_t logN)
{
    using Gm = Geom<LOGG, WG, true>;
    __shared__ double lds[Gm::LDS];
    const uint32_t N = 1u << logN;
    const uint32_t b = blockIdx.y + y0;
    const uint32_t m = (uint32_t)(lst[b] & 0xFFFF);
    const double q = mods[m].q, qinv = mods[m].qinv;
    uint64_t *p = base + (size_t)b * N;
    const Gm gm(logN, blockIdx.x);
    double x[R];
#pragma unroll
    for (int k = 0; k < R; k++) x[k] = u64_to_f64(p[gm.fwd_in(k)]);
    gm.fwd(x, lds, twt + (size_t)m * N, q, qinv, logN, 0);
#pragma unroll
    for (int k = 0; k < R; k++) p[gm.fwd_out(k)] = f64_to_bits(x[k]);
}
template <int LOGG, int WG>
__global__ __launch_bounds__(WG) void k_row_fwd(uint64_t *__restrict__ base, const uint64_t *__restrict__ lst,
                                                uint32_t y0, const ModQ *__restrict__ mods,
                                                const double *__restrict__ twt, uint32_t logN, uint32_t sigma0)
{
    using Gm = Geom<LOGG, WG, false>;
    __shared__ double lds[Gm::LDS];
    const uint32_t N = 1u << logN;
    const uint32_t b = blockIdx.y + y0;
    const uint32_t m = (uint32_t)(lst[b] & 0xFFFF);
    const double q = mods[m].q, qinv = mods[m].qinv;
    uint64_t *p = base + (size_t)b * N;
    const Gm gm(logN, blockIdx.x);
    double x[R];
#pragma unroll
    for (int k = 0; k < R; k++) x[k] = bits_to_f64(p[gm.fwd_in(k)]);
    gm.fwd(x, lds, twt + (size_t)m * N, q, qinv, logN, sigma0);
    gm.fwd_out_to_coal(x, lds);
#pragma unroll
    for (int k = 0; k < R; k++) p[gm.coal(k)] = f64_to_u64(canon(x[k], q, qinv));
}
template <int LOGG, int WG>
__global__ __launch_bounds__(WG) void k_col_inv(uint64_t *__restrict__ base, const uint64_t *__restrict__ lst,
                                                uint32_t y0, const ModQ *__restrict__ mods,
                                                const double *__restrict__ itwt, const double *__restrict__ ninvt,
                                                uint32_t logN)
{
    using Gm = Geom<LOGG, WG, true>;
    __shared__ double lds[Gm::LDS];
    const uint32_t N = 1u << logN;
    const uint32_t b = blockIdx.y + y0;
    const uint32_t m = (uint32_t)(lst[b] & 0xFFFF);
    const double q = mods[m].q, qinv = mods[m].qinv;
    uint64_t *p = base + (size_t)b * N;
    const Gm gm(logN, blockIdx.x);
    double x[R];
#pragma unroll
    for (int k = 0; k < R; k++) x[k] = bits_to_f64(p[gm.inv_in(k)]);
    gm.template inv<true>(x, lds, itwt + (size_t)m * N, q, qinv, ninvt[m], logN, 0);
#pragma unroll
    for (int k = 0; k < R; k++) p[gm.inv_out(k)] = f64_to_u64(canon(x[k], q, qinv));
}

// Per ring degree: column pass (LOGA stages, WA threads, GA blocks per limb) and
// row pass (LOGB stages, WB threads, GB blocks per limb), sigma0 of the row pass = LOGA.
template <int LOGN>
struct KsShape {
    static constexpr int LOGB = LOGN - 4 < 8 ? LOGN - 4 : 8, LOGA = LOGN - LOGB;
    static constexpr int TA = 1 << (LOGA - 4), NCOL = 1 << LOGB;
    static constexpr int WA = TA * NCOL < 256 ? TA * NCOL : 256, GA = NCOL / (WA / TA);
    static constexpr int TB = 1 << (LOGB - 4), NROW = 1 << LOGA;
    static constexpr int WB = TB * NROW < 256 ? TB * NROW : 256, GB = NROW / (WB / TB);
};

template <int LOGN, typename F>
void with_shape(F f)
{
    f(KsShape<LOGN>{});
}
template <typename F>
void dispatch_logn(uint32_t logN, F f)
{
    switch (logN) {
    case 10: with_shape<10>(f); break;
    case 11: with_shape<11>(f); break;
    case 12: with_shape<12>(f); break;
    case 13: with_shape<13>(f); break;
    case 14: with_shape<14>(f); break;
    case 15: with_shape<15>(f); break;
    case 16: with_shape<16>(f); break;
    default: break;
    }
}
// run f(y0, count) over [0, total) in grid-sized pieces
template <typename F>
void in_pieces(uint32_t total, F f)
{
    for (uint32_t y0 = 0; y0 < total; y0 += GRID_Y) f(y0, std::min(GRID_Y, total - y0));
}

// Host plan of one ragged batch.
struct KsPlan {
    uint32_t n, sum_l, sum_nd, sum_ups, sum_inner;
    std::vector<KsItem> items;
    std::vector<BcJob> upjobs, dnjobs;
    std::vector<uint64_t> la, upmods, inner, fl;
};

fhe_status ks_plan(const fhe_ctx *c, uint32_t n, const uint32_t *ls, KsPlan &pl)
{
    const uint32_t K = c->K, alpha = c->alpha;
    pl.n = n;
    pl.items.assign(n, KsItem{});
    uint32_t dc = 0, up = 0, uq = 0;
    for (uint32_t b = 0; b < n; ++b) {
        const uint32_t l = ls[b];
        if (l < 1 || l > c->L) return fhe_fail(FHE_ELEVEL, "key switch: limb count out of range");
        const uint32_t nd = (l + alpha - 1) / alpha;
        if (nd > 16) return fhe_fail(FHE_EPARAM, "key switching supports at most 16 digits");
        if (b >= 32768) return fhe_fail(FHE_EINVAL, "key-switch batch too large");
        KsItem &it = pl.items[b];
        it.l = l;
        it.nd = nd;
        it.dc_off = dc;
        it.up_off = up;
        it.uq_off = uq;
        uint32_t u = 0;
        for (uint32_t j = 0; j < nd; ++j) {
            const BconvTab &t = c->modup[(size_t)l * c->dnum + j];
            it.upoff[j] = (uint16_t)u;
            pl.upjobs.push_back(BcJob{t.off, t.nsrc, t.ndst, dc + j * alpha, up + u, 0});
            for (uint32_t a = 0; a < t.ndst; ++a) pl.upmods.push_back(t.dst[a]);
            u += t.ndst;
        }
        for (uint32_t i = 0; i < l; ++i) pl.la.push_back(((uint64_t)b << 16) | i);
        for (uint32_t x = 0; x < l + K; ++x) pl.inner.push_back(((uint64_t)b << 16) | x);
        for (uint32_t tt = 0; tt < 2; ++tt) {
            const BconvTab &md = c->moddown[l];
            pl.dnjobs.push_back(BcJob{md.off, md.nsrc, md.ndst, (2 * b + tt) * K, uq + tt * l, 0});
            for (uint32_t i = 0; i < l; ++i) pl.fl.push_back(((uint64_t)b << 17) | ((uint64_t)tt << 16) | i);
        }
        dc += l;
        up += u;
        uq += 2 * l;
    }
    pl.sum_l = dc;
    pl.sum_ups = up;
    pl.sum_nd = (uint32_t)pl.upjobs.size();
    pl.sum_inner = (uint32_t)pl.inner.size();
    return FHE_OK;
}

}  // namespace

// ---- launchers of the key-switching path
static void ks_col_fwd(fhe_ctx *c, uint64_t *base, const uint64_t *lst, uint32_t nlimbs)
{
    ProfScope ps(c, "ntt_fwd_col");
    dispatch_logn(c->logN, [&](auto sh) {
        using S = decltype(sh);
        in_pieces(nlimbs, [&](uint32_t y0, uint32_t cnt) {
            hipLaunchKernelGGL((k_col_fwd<S::LOGA, S::WA>), dim3(S::GA, cnt), dim3(S::WA), 0, c->stream, base, lst, y0,
                               (const ModQ *)c->d_mod, (const double *)c->d_tw, c->logN);
        });
    });
}
static void ks_col_inv(fhe_ctx *c, uint64_t *base, const uint64_t *lst, uint32_t nlimbs)
{
    ProfScope ps(c, "ntt_inv_col");
    dispatch_logn(c->logN, [&](auto sh) {
        using S = decltype(sh);
        in_pieces(nlimbs, [&](uint32_t y0, uint32_t cnt) {
            hipLaunchKernelGGL((k_col_inv<S::LOGA, S::WA>), dim3(S::GA, cnt), dim3(S::WA), 0, c->stream, base, lst, y0,
                               (const ModQ *)c->d_mod, (const double *)c->d_itw, (const double *)c->d_ninv, c->logN);
        });
    });
}
static void ks_row_fwd(fhe_ctx *c, uint64_t *base, const uint64_t *lst, uint32_t nlimbs)
{
    ProfScope ps(c, "ntt_fwd_row");
    dispatch_logn(c->logN, [&](auto sh) {
        using S = decltype(sh);
        in_pieces(nlimbs, [&](uint32_t y0, uint32_t cnt) {
            hipLaunchKernelGGL((k_row_fwd<S::LOGB, S::WB>), dim3(S::GB, cnt), dim3(S::WB), 0, c->stream, base, lst, y0,
                               (const ModQ *)c->d_mod, (const double *)c->d_tw, c->logN, (uint32_t)S::LOGA);
        });
    });
}

size_t ks_scratch_bytes_ragged(const fhe_ctx *c, uint32_t n, const uint32_t *ls)
{
    size_t limbs = 2 * (size_t)c->K * n;
    for (uint32_t b = 0; b < n; ++b) {
        const uint32_t l = ls[b], nd = (l + c->alpha - 1) / c->alpha;
        size_t ups = 0;
        for (uint32_t j = 0; j < nd; ++j) ups += c->modup[(size_t)l * c->dnum + j].ndst;
        limbs += 5 * (size_t)l + ups;
    }
    return limbs * c->N * sizeof(uint64_t);
}
size_t ks_scratch_bytes(const fhe_ctx *c, uint32_t l, uint32_t n)
{
    if (!n) return 0;
    std::vector<uint32_t> ls(n, l);
    return ks_scratch_bytes_ragged(c, n, ls.data());
}

fhe_status ks_run_ragged(fhe_ctx *c, uint32_t n, const uint32_t *ls, const uint64_t *const *d, const uint32_t *gal,
                         const uint64_t *const *evk, uint64_t *const *out, const uint64_t *const *add, uint8_t *scr_in)
{
    if (!n) return FHE_OK;
    if (!c->K) return fhe_fail(FHE_EPARAM, "key switching needs special primes");
    const uint32_t N = c->N, K = c->K, L = c->L;
    if (c->alpha > 16 || K > 16)
        return fhe_fail(FHE_EPARAM, "key switching supports at most 16 limbs per digit and 16 special primes");
    if (2ull * n > GRID_Y) return fhe_fail(FHE_EINVAL, "key-switch batch too large");
    KsPlan pl;
    fhe_status s;
    if ((s = ks_plan(c, n, ls, pl))) return s;

    // scratch: dc [sum l], up [sum ups], uQ [sum 2l], uP [n][2][K], z [sum 2l]
    uint8_t *scr = scr_in;
    if (!scr && (s = ctx_scratch(c, ks_scratch_bytes_ragged(c, n, ls), &scr))) return s;
    uint64_t *dc = (uint64_t *)scr, *up = dc + (size_t)pl.sum_l * N, *uQ = up + (size_t)pl.sum_ups * N,
             *uP = uQ + 2 * (size_t)pl.sum_l * N, *z = uP + 2 * (size_t)n * K * N;

    // one table: pointers, then the plan's lists
    std::vector<uint64_t *> tab;
    auto push_words = [&](const void *src, size_t bytes) {
        const uint64_t *w = (const uint64_t *)src;
        for (size_t i = 0; i < bytes / 8; ++i) tab.push_back((uint64_t *)(uintptr_t)w[i]);
    };
    KsTab kt;
    kt.n = n;
    kt.K = K;
    kt.L = L;
    for (uint32_t b = 0; b < n; ++b) tab.push_back((uint64_t *)d[b]);
    for (uint32_t b = 0; b < n; ++b) tab.push_back((uint64_t *)evk[b]);
    for (uint32_t b = 0; b < n; ++b) tab.push_back(out[b]);
    for (uint32_t b = 0; b < 2 * n; ++b) tab.push_back(add ? (uint64_t *)add[b] : nullptr);
    for (uint32_t b = 0; b < n; ++b) tab.push_back((uint64_t *)(uintptr_t)(gal ? gal[b] : 0u));
    kt.it = (uint32_t)tab.size();
    push_words(pl.items.data(), pl.items.size() * sizeof(KsItem));
    kt.la = (uint32_t)tab.size();
    push_words(pl.la.data(), pl.la.size() * 8);
    kt.uj = (uint32_t)tab.size();
    push_words(pl.upjobs.data(), pl.upjobs.size() * sizeof(BcJob));
    kt.um = (uint32_t)tab.size();
    push_words(pl.upmods.data(), pl.upmods.size() * 8);
    kt.il = (uint32_t)tab.size();
    push_words(pl.inner.data(), pl.inner.size() * 8);
    kt.dj = (uint32_t)tab.size();
    push_words(pl.dnjobs.data(), pl.dnjobs.size() * sizeof(BcJob));
    kt.fl = (uint32_t)tab.size();
    push_words(pl.fl.data(), pl.fl.size() * 8);
    uint64_t **dt;
    if ((s = ctx_ptr_table(c, tab, &dt))) return s;
    const uint64_t *dwords = (const uint64_t *)dt;
    hipStream_t st = c->stream;
    const uint32_t gx = blocks_for(N, TPB);
    const uint32_t sum2l = 2 * pl.sum_l;

    // 1. coefficients of the (permuted) inputs
    {
        ProfScope ps(c, "ks_intt_first");
        dispatch_logn(c->logN, [&](auto sh) {
            using S = decltype(sh);
            in_pieces(pl.sum_l, [&](uint32_t y0, uint32_t cnt) {
                hipLaunchKernelGGL((k_ks_intt_first<S::LOGB, S::WB>), dim3(S::GB, cnt), dim3(S::WB), 0, st,
                                   (uint64_t *const *)dt, kt, y0, dc, (const ModQ *)c->d_mod, (const double *)c->d_itw,
                                   c->logN, (uint32_t)S::LOGA);
            });
        });
    }
    ks_col_inv(c, dc, dwords + kt.la, pl.sum_l);
    // 2-3. ModUp conversion and the forward transform of the converted limbs
    {
        ProfScope ps(c, "bconv_up");
        in_pieces(pl.sum_nd, [&](uint32_t y0, uint32_t cnt) {
            hipLaunchKernelGGL(k_bconv<false>, dim3(gx, cnt), dim3(TPB), 0, st, (const uint64_t *)dc, up,
                               (const double *)c->d_bconv, (const BcJob *)(dwords + kt.uj), y0, c->logN,
                               (const double *)nullptr, (const double *)nullptr);
        });
    }
    ks_col_fwd(c, up, dwords + kt.um, pl.sum_ups);
    ks_row_fwd(c, up, dwords + kt.um, pl.sum_ups);
    // 4. key inner product over the digits
    {
        ProfScope ps(c, "ks_inner");
        in_pieces(pl.sum_inner, [&](uint32_t y0, uint32_t cnt) {
            hipLaunchKernelGGL(k_ks_inner, dim3(blocks_for(N / 2, TPB), cnt), dim3(TPB), 0, st, (uint64_t *const *)dt,
                               kt, y0,
                               (const uint64_t *)up, uQ, uP, (const ModQ *)c->d_mod, c->alpha, c->logN);
        });
    }
    // 5-6. ModDown: P limbs to coefficients, rounded conversion to Q_l
    {
        uint32_t m[FHE_LIMBTAB];
        for (uint32_t k = 0; k < K; ++k) m[k] = L + k;
        launch_ntt_inv(c, limbset_list(uP, m, K), n * 2 * K);
    }
    {
        ProfScope ps(c, "bconv_down");
        hipLaunchKernelGGL(k_bconv<true>, dim3(gx, 2 * n), dim3(TPB), 0, st, (const uint64_t *)uP, z,
                           (const double *)c->d_bconv, (const BcJob *)(dwords + kt.dj), 0u, c->logN,
                           (const double *)(c->d_phalf + L), (const double *)c->d_phalf);
    }
    // 7-8. column pass of z, row pass fused with the finish
    ks_col_fwd(c, z, dwords + kt.fl, sum2l);
    {
        ProfScope ps(c, "ks_moddown_final");
        dispatch_logn(c->logN, [&](auto sh) {
            using S = decltype(sh);
            in_pieces(sum2l, [&](uint32_t y0, uint32_t cnt) {
                hipLaunchKernelGGL((k_ks_moddown_final<S::LOGB, S::WB>), dim3(S::GB, cnt), dim3(S::WB), 0, st,
                                   (uint64_t *const *)dt, kt, y0, (const uint64_t *)z, (const uint64_t *)uQ,
                                   (const ModQ *)c->d_mod, (const double *)c->d_tw, (const double *)c->d_pinv,
                                   c->logN, (uint32_t)S::LOGA);
            });
        });
    }
    HIPCHK(hipGetLastError());
    return FHE_OK;
}

fhe_status ks_run(fhe_ctx *c, uint32_t l, uint32_t n, const uint64_t *const *d, const uint32_t *gal,
                  const uint64_t *const *evk, uint64_t *const *out, const uint64_t *const *add, uint8_t *scr_in)
{
    std::vector<uint32_t> ls(n, l);
    return ks_run_ragged(c, n, ls.data(), d, gal, evk, out, add, scr_in);
}
