// keyswitch.hip -- hybrid key switching (ModUp, key inner product, ModDown) for
// a batch of inputs, the operation under relinearisation and slot rotation
// (the CT-CT multiplications of Sec. 3 and the rotations of its packing).
//
// For each item b: input d_b (l limbs, NTT domain) read through a Galois
// permutation gal_b (0 = none: relinearisation; 5^r: rotation, so that the
// automorphism is never materialised), key evk_b [dnum][2][L+K][N], output
// out_b (2 polys), optional addends add[2b], add[2b+1] (read through gal_b).
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

// pointer table of one ks_run: [d: n][evk: n][out: n][add: 2n][gal: n (integers)]
__device__ __forceinline__ uint32_t tab_gal(uint64_t *const *tab, uint32_t n, uint32_t b)
{
    return (uint32_t)(uintptr_t)tab[5 * n + b];
}

struct BcJob {
    uint32_t off, nsrc, ndst;
    uint32_t src0;       // first source limb within one batch item of src
    uint32_t dst0;       // first destination limb within one batch item of dst
};
struct BcArgs {
    uint32_t njobs;
    uint32_t src_bstride, dst_bstride;   // limbs per batch item
    BcJob job[16];
};
// Fast basis conversion, one thread per coefficient, blockIdx.y = job, blockIdx.z = batch item:
//   y_t = sum_a [x_a (B/b_a)^-1]_{b_a} (B/b_a mod c_t)  mod c_t.
// ADD_HALF: sources offset by hsrc (per source limb) and results by -hdst (per
// destination limb): the rounding shift of ModDown.
template <bool ADD_HALF>
__global__ __launch_bounds__(TPB) void k_bconv(const uint64_t *__restrict__ src, uint64_t *__restrict__ dst,
                                               const double *__restrict__ tab, BcArgs args, uint32_t logN,
                                               const double *__restrict__ hsrc, const double *__restrict__ hdst)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    const BcJob jb = args.job[blockIdx.y];
    const uint64_t b = blockIdx.z;
    const double *T = tab + jb.off;
    const double *qhinv = T, *sq = T + jb.nsrc, *sqi = T + 2 * jb.nsrc, *dq = T + 3 * jb.nsrc,
                 *dqi = T + 3 * jb.nsrc + jb.ndst, *qh = T + 3 * jb.nsrc + 2 * jb.ndst;
    const uint64_t *S = src + (b * args.src_bstride + jb.src0) * N + k;
    uint64_t *D = dst + (b * args.dst_bstride + jb.dst0) * N + k;
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

struct KsDims {
    uint32_t l, K, L, alpha, nd, ups;
    uint32_t upoff[16];   // first converted limb of digit j within one batch item of `up`
};

// 1. First (row) pass of the inverse transform of d_b, gathered through gal_b,
//    into dc as lazy FP64 bits (SINGLE: the whole inverse, canonical out).
template <int LOGG, int WG, bool SINGLE>
__global__ __launch_bounds__(WG) void k_ks_intt_first(uint64_t *const *__restrict__ tab, uint32_t n,
                                                      uint64_t *__restrict__ dc, const ModQ *__restrict__ mods,
                                                      const double *__restrict__ itwt,
                                                      const double *__restrict__ ninvt, uint32_t l, uint32_t logN,
                                                      uint32_t sigma0)
{
    using Gm = Geom<LOGG, WG, false>;
    __shared__ double lds[Gm::LDS];
    const uint32_t N = 1u << logN;
    const uint32_t y = blockIdx.y, b = y / l, i = y % l;
    const uint64_t *src = tab[b] + (size_t)i * N;
    const uint32_t gal = tab_gal(tab, n, b);
    const double q = mods[i].q, qinv = mods[i].qinv;
    const Gm gm(logN, blockIdx.x);
    double x[R];
#pragma unroll
    for (int k = 0; k < R; k++) x[k] = u64_to_f64(src[galois_src(gm.coal(k), gal, logN)]);
    gm.coal_to_inv_in(x, lds);
    gm.template inv<SINGLE>(x, lds, itwt + (size_t)i * N, q, qinv, ninvt[i], logN, sigma0);
    uint64_t *dst = dc + (size_t)y * N;
#pragma unroll
    for (int k = 0; k < R; k++) dst[gm.inv_out(k)] = SINGLE ? f64_to_u64(canon(x[k], q, qinv)) : f64_to_bits(x[k]);
}

// 4b. Key inner product, one thread per coefficient of one limb x of Q_l u P:
//     u_t[x] = sum_j D_j[x] * evk_{j,t}[x]; D_j[x] is the input limb itself
//     inside digit j, else the converted limb.
__global__ __launch_bounds__(TPB) void k_ks_inner(uint64_t *const *__restrict__ tab, uint32_t n,
                                                  const uint64_t *__restrict__ up, uint64_t *__restrict__ uQ,
                                                  uint64_t *__restrict__ uP, const ModQ *__restrict__ mods,
                                                  KsDims dm, uint32_t logN)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    const uint32_t x = blockIdx.y, b = blockIdx.z;
    const uint32_t mx = x < dm.l ? x : dm.L + (x - dm.l);
    const double q = mods[mx].q, qi = mods[mx].qinv;
    const uint64_t *d = tab[b], *ev = tab[n + b];
    const uint64_t *upb = up + (size_t)b * dm.ups * N;
    const size_t ML = dm.L + dm.K;
    double a0 = 0.0, a1 = 0.0;
    for (uint32_t j = 0; j < dm.nd; ++j) {
        const uint32_t lo = j * dm.alpha, hi = min(lo + dm.alpha, dm.l);
        double D;
        if (x >= lo && x < hi) D = u64_to_f64(d[(size_t)x * N + k]);
        else {
            const uint32_t pos = x < lo ? x : x - (hi - lo);
            D = u64_to_f64(upb[(size_t)(dm.upoff[j] + pos) * N + k]);
        }
        a0 += mulmod(D, u64_to_f64(ev[(((size_t)j * 2 + 0) * ML + mx) * N + k]), q, qi);
        a1 += mulmod(D, u64_to_f64(ev[(((size_t)j * 2 + 1) * ML + mx) * N + k]), q, qi);
        if ((j & 3) == 3) { a0 = redc(a0, q, qi); a1 = redc(a1, q, qi); }
    }
    uint64_t *o0, *o1;
    if (x < dm.l) {
        o0 = uQ + ((size_t)b * 2 * dm.l + x) * N;
        o1 = uQ + ((size_t)b * 2 * dm.l + dm.l + x) * N;
    } else {
        o0 = uP + ((size_t)b * 2 * dm.K + (x - dm.l)) * N;
        o1 = uP + ((size_t)b * 2 * dm.K + dm.K + (x - dm.l)) * N;
    }
    o0[k] = f64_to_u64(canon(a0, q, qi));
    o1[k] = f64_to_u64(canon(a1, q, qi));
}

// 8. Forward row pass of z fused with the ModDown finish:
//    out_t[i] = (u_t[i] - z_t[i]) * P^-1 + add_t[i].  blockIdx.y = limb i, blockIdx.z = 2b + t.
template <int LOGG, int WG, bool IN_U64>
__global__ __launch_bounds__(WG, 3) void k_ks_moddown_final(uint64_t *const *__restrict__ tab, uint32_t n,
                                                         const uint64_t *__restrict__ z,
                                                         const uint64_t *__restrict__ uQ,
                                                         const ModQ *__restrict__ mods, const double *__restrict__ twt,
                                                         const double *__restrict__ pinv, uint32_t l, uint32_t logN,
                                                         uint32_t sigma0)
{
    using Gm = Geom<LOGG, WG, false>;
    __shared__ double lds[Gm::LDS];
    const uint32_t N = 1u << logN;
    const uint32_t i = blockIdx.y, item = blockIdx.z, b = item >> 1, t = item & 1;
    const double q = mods[i].q, qinv = mods[i].qinv;
    const Gm gm(logN, blockIdx.x);
    const uint64_t *zs = z + ((size_t)item * l + i) * N;
    double v[R];
#pragma unroll
    for (int k = 0; k < R; k++) {
        const uint64_t w = zs[gm.fwd_in(k)];
        v[k] = IN_U64 ? u64_to_f64(w) : bits_to_f64(w);
    }
    gm.fwd(v, lds, twt + (size_t)i * N, q, qinv, logN, sigma0);
    gm.fwd_out_to_coal(v, lds);
    const uint64_t *uq = uQ + ((size_t)item * l + i) * N;
    const uint64_t *ad = tab[3 * n + 2 * b + t];
    const uint32_t gal = tab_gal(tab, n, b);
    uint64_t *out = tab[2 * n + b] + ((size_t)t * l + i) * N;
    const double pi = pinv[i];
#pragma unroll
    for (int k = 0; k < R; k++) {
        const uint32_t idx = gm.coal(k);
        double r = canon(mulmod(u64_to_f64(uq[idx]) - v[k], pi, q, qinv), q, qinv);
        if (ad) r = fold(r + u64_to_f64(ad[(size_t)i * N + galois_src(idx, gal, logN)]), q);
        out[idx] = f64_to_u64(r);
    }
}

// Column passes of the key-switching path (split_ks): forward (canonical in,
// lazy bits out) and inverse (bits in, canonical out, N^-1 folded).
struct ModPat {
    uint32_t period, b0;
    uint8_t m[FHE_LIMBTAB];
};
template <int LOGG, int WG>
__global__ __launch_bounds__(WG) void k_col_fwd(uint64_t *__restrict__ base, ModPat pat, const ModQ *__restrict__ mods,
                                                const double *__restrict__ twt, uint32_t logN)
{
    using Gm = Geom<LOGG, WG, true>;
    __shared__ double lds[Gm::LDS];
    const uint32_t N = 1u << logN;
    const uint32_t b = blockIdx.y + pat.b0;
    const uint32_t m = pat.m[b % pat.period];
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
// 4a. Forward row pass of the converted limbs: lazy bits in, canonical out,
//     stores coalesced through an LDS transpose.
template <int LOGG, int WG>
__global__ __launch_bounds__(WG) void k_row_fwd(uint64_t *__restrict__ base, ModPat pat, const ModQ *__restrict__ mods,
                                                const double *__restrict__ twt, uint32_t logN, uint32_t sigma0)
{
    using Gm = Geom<LOGG, WG, false>;
    __shared__ double lds[Gm::LDS];
    const uint32_t N = 1u << logN;
    const uint32_t b = blockIdx.y + pat.b0;
    const uint32_t m = pat.m[b % pat.period];
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
__global__ __launch_bounds__(WG) void k_col_inv(uint64_t *__restrict__ base, uint32_t period, uint32_t b0,
                                                const ModQ *__restrict__ mods, const double *__restrict__ itwt,
                                                const double *__restrict__ ninvt, uint32_t logN)
{
    using Gm = Geom<LOGG, WG, true>;
    __shared__ double lds[Gm::LDS];
    const uint32_t N = 1u << logN;
    const uint32_t b = blockIdx.y + b0;
    const uint32_t m = b % period;          // limbs 0..period-1 of Q, repeated
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

}  // namespace

// ---- launchers of the key-switching path
static void ks_col_fwd(fhe_ctx *c, uint64_t *base, const uint32_t *mods, uint32_t period, uint32_t nlimbs)
{
    ProfScope ps(c, "ntt_fwd_col");
    ModPat pat;
    std::memset(&pat, 0, sizeof(pat));
    pat.period = period;
    for (uint32_t i = 0; i < period; ++i) pat.m[i] = (uint8_t)mods[i];
    dispatch_logn(c->logN, [&](auto sh) {
        using S = decltype(sh);
        for (uint32_t done = 0; done < nlimbs; done += 65535u) {
            pat.b0 = done;
            hipLaunchKernelGGL((k_col_fwd<S::LOGA, S::WA>), dim3(S::GA, std::min(65535u, nlimbs - done)), dim3(S::WA),
                               0, c->stream, base, pat, (const ModQ *)c->d_mod, (const double *)c->d_tw, c->logN);
        }
    });
}
static void ks_col_inv(fhe_ctx *c, uint64_t *base, uint32_t period, uint32_t nlimbs)
{
    ProfScope ps(c, "ntt_inv_col");
    dispatch_logn(c->logN, [&](auto sh) {
        using S = decltype(sh);
        for (uint32_t done = 0; done < nlimbs; done += 65535u)
            hipLaunchKernelGGL((k_col_inv<S::LOGA, S::WA>), dim3(S::GA, std::min(65535u, nlimbs - done)),
                               dim3(S::WA), 0, c->stream, base, period, done, (const ModQ *)c->d_mod,
                               (const double *)c->d_itw, (const double *)c->d_ninv, c->logN);
    });
}
static void run_intt_first(fhe_ctx *c, uint64_t **dt, uint32_t n, uint64_t *dc, uint32_t l)
{
    ProfScope ps(c, "ks_intt_first");
    dispatch_logn(c->logN, [&](auto sh) {
        using S = decltype(sh);
        hipLaunchKernelGGL((k_ks_intt_first<S::LOGB, S::WB, false>), dim3(S::GB, n * l), dim3(S::WB), 0, c->stream,
                           (uint64_t *const *)dt, n, dc, (const ModQ *)c->d_mod, (const double *)c->d_itw,
                           (const double *)c->d_ninv, l, c->logN, (uint32_t)S::LOGA);
    });
}
static void ks_row_fwd(fhe_ctx *c, uint64_t *base, const uint32_t *mods, uint32_t period, uint32_t nlimbs)
{
    ProfScope ps(c, "ntt_fwd_row");
    ModPat pat;
    std::memset(&pat, 0, sizeof(pat));
    pat.period = period;
    for (uint32_t i = 0; i < period; ++i) pat.m[i] = (uint8_t)mods[i];
    dispatch_logn(c->logN, [&](auto sh) {
        using S = decltype(sh);
        for (uint32_t done = 0; done < nlimbs; done += 65535u) {
            pat.b0 = done;
            hipLaunchKernelGGL((k_row_fwd<S::LOGB, S::WB>), dim3(S::GB, std::min(65535u, nlimbs - done)), dim3(S::WB),
                               0, c->stream, base, pat, (const ModQ *)c->d_mod, (const double *)c->d_tw, c->logN,
                               (uint32_t)S::LOGA);
        }
    });
}
static void run_moddown_final(fhe_ctx *c, uint64_t **dt, uint32_t n, const uint64_t *z, const uint64_t *uQ,
                              uint32_t l)
{
    ProfScope ps(c, "ks_moddown_final");
    dispatch_logn(c->logN, [&](auto sh) {
        using S = decltype(sh);
        hipLaunchKernelGGL((k_ks_moddown_final<S::LOGB, S::WB, false>), dim3(S::GB, l, 2 * n), dim3(S::WB), 0,
                           c->stream, (uint64_t *const *)dt, n, z, uQ, (const ModQ *)c->d_mod,
                           (const double *)c->d_tw, (const double *)c->d_pinv, l, c->logN, (uint32_t)S::LOGA);
    });
}

size_t ks_scratch_bytes(const fhe_ctx *c, uint32_t l, uint32_t n)
{
    const uint32_t nd = (l + c->alpha - 1) / c->alpha;
    size_t ups = 0;
    for (uint32_t j = 0; j < nd; ++j) ups += c->modup[(size_t)l * c->dnum + j].ndst;
    return (size_t)n * (5 * (size_t)l + ups + 2 * (size_t)c->K) * c->N * sizeof(uint64_t);
}

fhe_status ks_run(fhe_ctx *c, uint32_t l, uint32_t n, const uint64_t *const *d, const uint32_t *gal,
                  const uint64_t *const *evk, uint64_t *const *out, const uint64_t *const *add, uint8_t *scr_in)
{
    if (!c->K) return fhe_fail(FHE_EPARAM, "key switching needs special primes");
    const uint32_t N = c->N, K = c->K, L = c->L, alpha = c->alpha;
    const uint32_t nd = (l + alpha - 1) / alpha;
    if (nd > 16 || alpha > 16 || K > 16)
        return fhe_fail(FHE_EPARAM, "key switching supports at most 16 digits, 16 limbs per digit, 16 special primes");
    if ((uint64_t)n * l > 65535u || 2ull * n > 65535u) return fhe_fail(FHE_EINVAL, "key-switch batch too large");
    KsDims dm;
    std::memset(&dm, 0, sizeof(dm));
    dm.l = l; dm.K = K; dm.L = L; dm.alpha = alpha; dm.nd = nd;
    BcArgs up_args;
    std::memset(&up_args, 0, sizeof(up_args));
    uint32_t upmods[FHE_LIMBTAB], ups = 0;
    for (uint32_t j = 0; j < nd; ++j) {
        const BconvTab &t = c->modup[(size_t)l * c->dnum + j];
        dm.upoff[j] = ups;
        up_args.job[j] = BcJob{t.off, t.nsrc, t.ndst, j * alpha, ups};
        for (uint32_t a = 0; a < t.ndst; ++a) {
            if (ups >= FHE_LIMBTAB) return fhe_fail(FHE_EPARAM, "extended basis too large for one launch");
            upmods[ups++] = t.dst[a];
        }
    }
    dm.ups = ups;
    up_args.njobs = nd;
    up_args.src_bstride = l;
    up_args.dst_bstride = ups;
    const BconvTab &mdt = c->moddown[l];
    BcArgs dn_args;
    std::memset(&dn_args, 0, sizeof(dn_args));
    dn_args.njobs = 1;
    dn_args.src_bstride = K;   // batch item = one polynomial (2 per key switch)
    dn_args.dst_bstride = l;
    dn_args.job[0] = BcJob{mdt.off, mdt.nsrc, mdt.ndst, 0, 0};

    // scratch: dc [n][l], up [n][ups], uQ [n][2][l], uP [n][2][K], z [n][2][l]
    const size_t n_dc = (size_t)n * l, n_up = (size_t)n * ups, n_uq = (size_t)n * 2 * l, n_up2 = (size_t)n * 2 * K;
    uint8_t *scr = scr_in;
    fhe_status s = FHE_OK;
    if (!scr && (s = ctx_scratch(c, ks_scratch_bytes(c, l, n), &scr))) return s;
    uint64_t *dc = (uint64_t *)scr, *up = dc + n_dc * N, *uQ = up + n_up * N, *uP = uQ + n_uq * N, *z = uP + n_up2 * N;

    std::vector<uint64_t *> tab;
    tab.reserve(6 * (size_t)n);
    for (uint32_t b = 0; b < n; ++b) tab.push_back((uint64_t *)d[b]);
    for (uint32_t b = 0; b < n; ++b) tab.push_back((uint64_t *)evk[b]);
    for (uint32_t b = 0; b < n; ++b) tab.push_back(out[b]);
    for (uint32_t b = 0; b < 2 * n; ++b) tab.push_back(add ? (uint64_t *)add[b] : nullptr);
    for (uint32_t b = 0; b < n; ++b) tab.push_back((uint64_t *)(uintptr_t)(gal ? gal[b] : 0u));
    uint64_t **dt;
    if ((s = ctx_ptr_table(c, tab, &dt))) return s;
    hipStream_t st = c->stream;
    const uint32_t gx = blocks_for(N, TPB);
    uint32_t qm[FHE_LIMBTAB];
    for (uint32_t i = 0; i < l; ++i) qm[i] = i;

    // 1. coefficients of the (permuted) inputs
    run_intt_first(c, dt, n, dc, l);
    ks_col_inv(c, dc, l, n * l);
    // 2-3. ModUp conversion and the column pass of the converted limbs
    {
        ProfScope ps(c, "bconv_up");
        hipLaunchKernelGGL(k_bconv<false>, dim3(gx, nd, n), dim3(TPB), 0, st, (const uint64_t *)dc, up,
                           (const double *)c->d_bconv, up_args, c->logN, (const double *)nullptr,
                           (const double *)nullptr);
    }
    ks_col_fwd(c, up, upmods, ups, n * ups);
    ks_row_fwd(c, up, upmods, ups, n * ups);
    // 4. key inner product over the digits
    {
        ProfScope ps(c, "ks_inner");
        hipLaunchKernelGGL(k_ks_inner, dim3(gx, l + K, n), dim3(TPB), 0, st, (uint64_t *const *)dt, n,
                           (const uint64_t *)up, uQ, uP, (const ModQ *)c->d_mod, dm, c->logN);
    }
    // 5-6. ModDown: P limbs to coefficients, rounded conversion to Q_l
    {
        uint32_t m[FHE_LIMBTAB];
        for (uint32_t k = 0; k < K; ++k) m[k] = L + k;
        launch_ntt_inv(c, limbset_list(uP, m, K), n * 2 * K);
    }
    {
        ProfScope ps(c, "bconv_down");
        hipLaunchKernelGGL(k_bconv<true>, dim3(gx, 1, n * 2), dim3(TPB), 0, st, (const uint64_t *)uP, z,
                           (const double *)c->d_bconv, dn_args, c->logN, (const double *)(c->d_phalf + L),
                           (const double *)c->d_phalf);
    }
    // 7-8. column pass of z, row pass fused with the finish
    ks_col_fwd(c, z, qm, l, n * 2 * l);
    run_moddown_final(c, dt, n, z, uQ, l);
    HIPCHK(hipGetLastError());
    return FHE_OK;
}
