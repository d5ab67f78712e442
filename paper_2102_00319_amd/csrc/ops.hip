// ops.hip -- server-side ciphertext arithmetic on gfx950: element-wise
// add/sub/plaintext ops, tensor product and tensor multiply-accumulate,
// Galois automorphism, rescale and hybrid key switching (relinearisation,
// rotation).  Ciphertexts are in the NTT domain, [polys][limbs][N].
//
// The paper needs exactly these ciphertext operations: CT-CT and CT-PT
// add/mult (Sec. 3, Eq. (enc_conv), the cost counts after Eq. (approxReLU)
// and of mean pooling), slot rotation (Sec. 3 "Convolution Operator") and
// levelled rescaling (Sec. 2.1, Sec. 4.2).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "fhe_internal.h"

namespace {

constexpr int TPB = 256;

inline uint32_t blocks_for(uint64_t n, uint32_t per) { return (uint32_t)((n + per - 1) / per); }

// ---------------------------------------------------------------- kernels
// out = a + b or a - b (mod q), canonical in/out.  i indexes elements of [polys][limbs][N].
__global__ void k_addsub(const uint64_t *__restrict__ a, const uint64_t *__restrict__ b, uint64_t *out,
                         const ModQ *__restrict__ mods, uint32_t logN, uint32_t limbs, uint64_t total, int sub)
{
    uint64_t i = (uint64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= total) return;
    const uint32_t limb = (uint32_t)((i >> logN) % limbs);
    const uint64_t q = (uint64_t)mods[limb].q;
    const uint64_t x = a[i], y = b[i];
    uint64_t r;
    if (sub) r = x >= y ? x - y : x + q - y;
    else { r = x + y; r = r >= q ? r - q : r; }
    out[i] = r;
}
// out[p] = a[p] * pt  (pt broadcast over polys)
__global__ void k_mulpt(const uint64_t *__restrict__ a, const uint64_t *__restrict__ pt, uint64_t *out,
                        const ModQ *__restrict__ mods, uint32_t logN, uint32_t limbs, uint64_t total)
{
    uint64_t i = (uint64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= total) return;
    const uint64_t per = (uint64_t)limbs << logN;
    const uint32_t limb = (uint32_t)((i >> logN) % limbs);
    const double q = mods[limb].q, qi = mods[limb].qinv;
    const double r = mulmod(u64_to_f64(a[i]), u64_to_f64(pt[i % per]), q, qi);
    out[i] = f64_to_u64(fold(r, q));
}
// out = a * c_limb
__global__ void k_mulconst(const uint64_t *__restrict__ a, uint64_t *out, Consts64 cres,
                           const ModQ *__restrict__ mods, uint32_t logN, uint32_t limbs, uint64_t total)
{
    uint64_t i = (uint64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= total) return;
    const uint32_t limb = (uint32_t)((i >> logN) % limbs);
    const double q = mods[limb].q, qi = mods[limb].qinv;
    out[i] = f64_to_u64(fold(mulmod(u64_to_f64(a[i]), cres.v[limb], q, qi), q));
}
// acc3 = sum_t a_t (x) b_t over n pairs; a_t, b_t are 2-poly ciphertexts given
// by device pointer tables.  One thread per (limb, coefficient); the three
// accumulators stay in registers.
__global__ void k_tensor_acc(uint64_t *const *__restrict__ ap, uint64_t *const *__restrict__ bp, uint32_t n,
                             uint64_t *out, const ModQ *__restrict__ mods, uint32_t logN, uint32_t limbs)
{
    const uint32_t N = 1u << logN;
    const uint64_t e = (uint64_t)blockIdx.x * TPB + threadIdx.x;   // limb * N + k
    if (e >= ((uint64_t)limbs << logN)) return;
    const uint32_t limb = (uint32_t)(e >> logN);
    const uint64_t off1 = (uint64_t)limbs * N;
    const double q = mods[limb].q, qi = mods[limb].qinv;
    double d0 = 0, d1 = 0, d2 = 0;
    for (uint32_t t = 0; t < n; ++t) {
        const uint64_t *A = ap[t], *B = bp[t];
        const double a0 = u64_to_f64(A[e]), a1 = u64_to_f64(A[e + off1]);
        const double b0 = u64_to_f64(B[e]), b1 = u64_to_f64(B[e + off1]);
        d0 += mulmod(a0, b0, q, qi);
        d1 += mulmod(a0, b1, q, qi) + mulmod(a1, b0, q, qi);
        d2 += mulmod(a1, b1, q, qi);
        if ((t & 3) == 3) {
            d0 = redc(d0, q, qi);
            d1 = redc(d1, q, qi);
            d2 = redc(d2, q, qi);
        }
    }
    out[e] = f64_to_u64(canon(d0, q, qi));
    out[e + off1] = f64_to_u64(canon(d1, q, qi));
    out[e + 2 * off1] = f64_to_u64(canon(d2, q, qi));
}
// NTT-domain Galois automorphism: out[x] = in[y], 2 brv(y) + 1 = (2 brv(x) + 1) g mod 2N.
__global__ void k_automorph(const uint64_t *__restrict__ in, uint64_t *__restrict__ out, uint32_t logN,
                            uint64_t nlimbs_total, uint32_t g)
{
    const uint64_t i = (uint64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= (nlimbs_total << logN)) return;
    const uint32_t N = 1u << logN, x = (uint32_t)(i & (N - 1));
    const uint64_t base = i - x;
    const uint32_t ex = 2u * (__brev(x) >> (32 - logN)) + 1u;
    const uint32_t ey = (uint32_t)(((uint64_t)ex * g) & (2u * N - 1));
    const uint32_t y = __brev((ey - 1u) >> 1) >> (32 - logN);
    out[i] = in[base + y];
}
// Rescale over a batch of ciphertexts given by pointer tables (item b = ciphertext).
// Step 1: copy the last limb of every polynomial to tmp [n*P][N].
__global__ void k_gather_last(uint64_t *const *__restrict__ inp, uint64_t *__restrict__ tmp, uint32_t logN, uint32_t l,
                              uint32_t polys)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    const uint32_t item = blockIdx.y, b = item / polys, p = item % polys;
    tmp[(size_t)item * N + k] = inp[b][((size_t)p * l + (l - 1)) * N + k];
}
// Step 2: the last limb r (coefficient domain, mod q_last) lifted to (-q_last/2, q_last/2]
// and reduced mod q_i for i < l-1: dst [n*P][l-1][N].
__global__ void k_spread_centered(const uint64_t *__restrict__ r, uint64_t *__restrict__ dst,
                                  const ModQ *__restrict__ mods, uint32_t logN, uint32_t l)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    const uint32_t limb = blockIdx.y, item = blockIdx.z, lo = l - 1;
    const double ql = mods[l - 1].q;
    double v = u64_to_f64(r[(size_t)item * N + k]);
    v = v > 0.5 * ql ? v - ql : v;   // centered lift (q_last odd: no ties)
    const double q = mods[limb].q, qi = mods[limb].qinv;
    dst[((size_t)item * lo + limb) * N + k] = f64_to_u64(canon(v, q, qi));
}
// Step 3: out = (c - s) * q_last^-1 mod q_i.
__global__ void k_rescale_fin(uint64_t *const *__restrict__ inp, const uint64_t *__restrict__ s,
                              uint64_t *const *__restrict__ outp, const ModQ *__restrict__ mods,
                              const double *__restrict__ qlinv_row, uint32_t logN, uint32_t l, uint32_t polys)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    const uint32_t limb = blockIdx.y, item = blockIdx.z, b = item / polys, p = item % polys, lo = l - 1;
    const double q = mods[limb].q, qi = mods[limb].qinv;
    const double c = u64_to_f64(inp[b][((size_t)p * l + limb) * N + k]);
    const double r = mulmod(c - u64_to_f64(s[((size_t)item * lo + limb) * N + k]), qlinv_row[limb], q, qi);
    outp[b][((size_t)p * lo + limb) * N + k] = f64_to_u64(fold(r, q));
}

// ------------------------------------------------------------ key switching
struct BcJob {
    uint32_t off, nsrc, ndst;
    uint32_t src0;       // first source limb (within one batch item of src)
    uint32_t dst0;       // first destination limb (within one batch item of dst)
};
struct BcArgs {
    uint32_t njobs;
    uint32_t src_bstride, dst_bstride;   // limbs per batch item
    BcJob job[16];
};
// Fast basis conversion, one thread per coefficient, blockIdx.y = job, blockIdx.z = batch item.
// y_t = sum_a [x_a (B/b_a)^-1]_{b_a} (B/b_a mod c_t)  mod c_t.
// ADD_HALF: the sources are first offset by hsrc (per source limb) and the results
// are offset by -hdst (per destination limb): the rounding shift of ModDown.
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
    uint32_t upoff[16];   // first limb of digit j's converted limbs within one batch item of `up`
};
// u_t[x] = sum_j D_j[x] * evk_j,t[x] over the extended basis Q_l u P (x < l: Q, else P).
// D_j[x] is the input limb itself inside digit j, else the converted limb.
__global__ __launch_bounds__(TPB) void k_ks_inner(uint64_t *const *__restrict__ dptr,
                                                  uint64_t *const *__restrict__ evkptr,
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
    const uint64_t *d = dptr[b];
    const uint64_t *ev = evkptr[b];
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
        const double e0 = u64_to_f64(ev[(((size_t)j * 2 + 0) * ML + mx) * N + k]);
        const double e1 = u64_to_f64(ev[(((size_t)j * 2 + 1) * ML + mx) * N + k]);
        a0 += mulmod(D, e0, q, qi);
        a1 += mulmod(D, e1, q, qi);
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
// out_t[i] = (u_t[i] - z_t[i]) * P^-1 (+ add_t[i]) mod q_i.  blockIdx.y = limb i, blockIdx.z = 2*b + t.
// addptr (optional) holds 2 pointers per item: the addend polynomials for t = 0, 1 (each may be null).
__global__ __launch_bounds__(TPB) void k_ks_final(const uint64_t *__restrict__ uQ, const uint64_t *__restrict__ z,
                                                  uint64_t *const *__restrict__ outptr,
                                                  uint64_t *const *__restrict__ addptr, const double *__restrict__ pinv,
                                                  const ModQ *__restrict__ mods, uint32_t l, uint32_t logN)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    const uint32_t i = blockIdx.y, t = blockIdx.z & 1, b = blockIdx.z >> 1;
    const double q = mods[i].q, qi = mods[i].qinv;
    const size_t e = ((size_t)b * 2 * l + (size_t)t * l + i) * N + k;
    double r = mulmod(u64_to_f64(uQ[e]) - u64_to_f64(z[e]), pinv[i], q, qi);
    r = fold(r, q);
    const size_t oe = ((size_t)t * l + i) * N + k;
    const uint64_t *ad = addptr ? addptr[2 * b + t] : nullptr;   // addend polynomial t of item b, or none
    if (ad) r = fold(r + u64_to_f64(ad[(size_t)i * N + k]), q);
    outptr[b][oe] = f64_to_u64(r);
}
__global__ void k_copy_limbs(uint64_t *const *__restrict__ srcptr, uint64_t *__restrict__ dst, uint64_t per_item)
{
    const uint64_t i = (uint64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= per_item) return;
    dst[(uint64_t)blockIdx.y * per_item + i] = srcptr[blockIdx.y][i];
}

}  // namespace

// ============================================================ host helpers
static fhe_status chk_ct(const fhe_ctx *c, const fhe_ct *a, const char *what)
{
    if (!a || !a->d) return fhe_fail(FHE_EINVAL, std::string(what) + ": null ciphertext");
    if (a->limbs < 1 || a->limbs > c->L) return fhe_fail(FHE_ELEVEL, std::string(what) + ": limb count out of range");
    if (a->polys < 2 || a->polys > 3) return fhe_fail(FHE_EINVAL, std::string(what) + ": polys must be 2 or 3");
    return FHE_OK;
}
static bool scales_match(double a, double b) { return std::fabs(a / b - 1.0) <= 9.5367431640625e-07; }   // 2^-20

// Host-side key switch driver: n inputs (each l limbs, NTT domain), keys, outputs
// (2 polys, l limbs) and optional addends folded into the result: add[2b + t] is
// the polynomial (l limbs) added to output polynomial t of item b, or null.
size_t ks_scratch_bytes(const fhe_ctx *c, uint32_t l, uint32_t n)
{
    const uint32_t nd = (l + c->alpha - 1) / c->alpha;
    size_t ups = 0;
    for (uint32_t j = 0; j < nd; ++j) ups += c->modup[(size_t)l * c->dnum + j].ndst;
    return (size_t)n * (5 * (size_t)l + ups + 2 * (size_t)c->K) * c->N * sizeof(uint64_t);
}

fhe_status ks_run(fhe_ctx *c, uint32_t l, uint32_t n, const uint64_t *const *d, const uint64_t *const *evk,
                  uint64_t *const *out, const uint64_t *const *add, uint8_t *scr_in)
{
    if (!c->K) return fhe_fail(FHE_EPARAM, "key switching needs special primes");
    const uint32_t N = c->N, K = c->K, L = c->L, alpha = c->alpha;
    const uint32_t nd = (l + alpha - 1) / alpha;
    if (nd > 16 || alpha > 16 || K > 16)
        return fhe_fail(FHE_EPARAM, "key switching supports at most 16 digits, 16 limbs per digit, 16 special primes");
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
    const size_t LB = (size_t)N * sizeof(uint64_t);
    const size_t n_dc = (size_t)n * l, n_up = (size_t)n * ups, n_uq = (size_t)n * 2 * l, n_up2 = (size_t)n * 2 * K;
    uint8_t *scr = scr_in;
    fhe_status s = FHE_OK;
    if (!scr && (s = ctx_scratch(c, (n_dc + n_up + n_uq + n_up2 + n_uq) * LB, &scr))) return s;
    uint64_t *dc = (uint64_t *)scr, *up = dc + n_dc * N, *uQ = up + n_up * N, *uP = uQ + n_uq * N, *z = uP + n_up2 * N;

    std::vector<uint64_t *> tab;
    for (uint32_t b = 0; b < n; ++b) tab.push_back((uint64_t *)d[b]);
    for (uint32_t b = 0; b < n; ++b) tab.push_back((uint64_t *)evk[b]);
    for (uint32_t b = 0; b < n; ++b) tab.push_back(out[b]);
    for (uint32_t b = 0; b < 2 * n; ++b) tab.push_back(add ? (uint64_t *)add[b] : nullptr);
    uint64_t **dt;
    if ((s = ctx_ptr_table(c, tab, &dt))) return s;
    hipStream_t st = c->stream;
    const uint32_t gx = blocks_for(N, TPB);

    // 1. coefficient-domain copy of the inputs
    {
        ProfScope ps(c, "ks_copy");
        hipLaunchKernelGGL(k_copy_limbs, dim3(blocks_for((uint64_t)l * N, TPB), n), dim3(TPB), 0, st, dt, dc,
                           (uint64_t)l * N);
    }
    {
        uint32_t m[FHE_LIMBTAB];
        for (uint32_t i = 0; i < l; ++i) m[i] = i;
        launch_ntt_inv(c, limbset_list(dc, m, l), n * l);
    }
    // 2. ModUp basis conversion, 3. NTT of the converted limbs
    {
        ProfScope ps(c, "bconv_up");
        hipLaunchKernelGGL(k_bconv<false>, dim3(gx, nd, n), dim3(TPB), 0, st, (const uint64_t *)dc, up,
                           (const double *)c->d_bconv, up_args, c->logN, (const double *)nullptr,
                           (const double *)nullptr);
    }
    launch_ntt_fwd(c, limbset_list(up, upmods, ups), n * ups);
    // 4. inner product with the key over Q_l u P
    {
        ProfScope ps(c, "ks_inner");
        hipLaunchKernelGGL(k_ks_inner, dim3(gx, l + K, n), dim3(TPB), 0, st, (uint64_t *const *)dt,
                           (uint64_t *const *)(dt + n), (const uint64_t *)up, uQ, uP, (const ModQ *)c->d_mod, dm,
                           c->logN);
    }
    // 5. ModDown: P limbs to coefficients, rounded conversion to Q_l, NTT, finish
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
    {
        uint32_t m[FHE_LIMBTAB];
        for (uint32_t i = 0; i < l; ++i) m[i] = i;
        launch_ntt_fwd(c, limbset_list(z, m, l), n * 2 * l);
    }
    {
        ProfScope ps(c, "ks_final");
        hipLaunchKernelGGL(k_ks_final, dim3(gx, l, 2 * n), dim3(TPB), 0, st, (const uint64_t *)uQ,
                           (const uint64_t *)z, (uint64_t *const *)(dt + 2 * n),
                           add ? (uint64_t *const *)(dt + 3 * n) : nullptr, (const double *)c->d_pinv,
                           (const ModQ *)c->d_mod, l, c->logN);
    }
    HIPCHK(hipGetLastError());
    return FHE_OK;
}

size_t rescale_scratch_bytes(const fhe_ctx *c, uint32_t l, uint32_t polys, uint32_t n)
{
    return (size_t)n * polys * ((size_t)l) * c->N * sizeof(uint64_t);   // last limbs + spread limbs
}
// Rescale n ciphertexts (polys each, l limbs) into outputs (l-1 limbs); outputs must not overlap inputs.
fhe_status rescale_run(fhe_ctx *c, uint32_t l, uint32_t polys, uint32_t n, const uint64_t *const *in,
                       uint64_t *const *out, uint8_t *scr)
{
    const size_t N = c->N;
    fhe_status s;
    std::vector<uint64_t *> tab;
    for (uint32_t b = 0; b < n; ++b) tab.push_back((uint64_t *)in[b]);
    for (uint32_t b = 0; b < n; ++b) tab.push_back(out[b]);
    uint64_t **dt;
    if ((s = ctx_ptr_table(c, tab, &dt))) return s;
    uint64_t *last = (uint64_t *)scr, *spread = last + (size_t)n * polys * N;
    const uint32_t gx = blocks_for(N, TPB), items = n * polys;
    if (items > 65535u) return fhe_fail(FHE_EINVAL, "rescale batch too large for one launch");
    ProfScope ps(c, "rescale");
    hipLaunchKernelGGL(k_gather_last, dim3(gx, items), dim3(TPB), 0, c->stream, (uint64_t *const *)dt, last, c->logN,
                       l, polys);
    uint32_t m1 = l - 1;
    launch_ntt_inv(c, limbset_list(last, &m1, 1), items);
    hipLaunchKernelGGL(k_spread_centered, dim3(gx, l - 1, items), dim3(TPB), 0, c->stream, (const uint64_t *)last,
                       spread, (const ModQ *)c->d_mod, c->logN, l);
    {
        uint32_t m[FHE_LIMBTAB];
        for (uint32_t i = 0; i < l - 1; ++i) m[i] = i;
        launch_ntt_fwd(c, limbset_list(spread, m, l - 1), items * (l - 1));
    }
    hipLaunchKernelGGL(k_rescale_fin, dim3(gx, l - 1, items), dim3(TPB), 0, c->stream, (uint64_t *const *)dt,
                       (const uint64_t *)spread, (uint64_t *const *)(dt + n), (const ModQ *)c->d_mod,
                       (const double *)(c->d_qlinv + (size_t)(l - 1) * c->L), c->logN, l, polys);
    HIPCHK(hipGetLastError());
    return FHE_OK;
}

// ========================================================= C entry points
extern "C" {

fhe_status fhe_add(fhe_ctx *c, const fhe_ct *a, const fhe_ct *b, fhe_ct *out)
{
    fhe_status s;
    if (!c) return fhe_fail(FHE_EINVAL, "null context");
    if ((s = chk_ct(c, a, "fhe_add")) || (s = chk_ct(c, b, "fhe_add")) || (s = chk_ct(c, out, "fhe_add"))) return s;
    if (a->limbs != b->limbs || out->limbs != a->limbs) return fhe_fail(FHE_ELEVEL, "fhe_add: limb counts differ");
    if (a->polys != b->polys || out->polys != a->polys) return fhe_fail(FHE_EINVAL, "fhe_add: poly counts differ");
    if (!scales_match(a->scale, b->scale)) return fhe_fail(FHE_ESCALE, "fhe_add: scales differ");
    const uint64_t total = (uint64_t)a->polys * a->limbs * c->N;
    hipLaunchKernelGGL(k_addsub, dim3(blocks_for(total, TPB)), dim3(TPB), 0, c->stream, (const uint64_t *)a->d,
                       (const uint64_t *)b->d, out->d, (const ModQ *)c->d_mod, c->logN, a->limbs, total, 0);
    out->scale = a->scale;
    c->ops[OP_CT_ADD] += 1;
    HIPCHK(hipGetLastError());
    return FHE_OK;
}
fhe_status fhe_sub(fhe_ctx *c, const fhe_ct *a, const fhe_ct *b, fhe_ct *out)
{
    fhe_status s;
    if (!c) return fhe_fail(FHE_EINVAL, "null context");
    if ((s = chk_ct(c, a, "fhe_sub")) || (s = chk_ct(c, b, "fhe_sub")) || (s = chk_ct(c, out, "fhe_sub"))) return s;
    if (a->limbs != b->limbs || out->limbs != a->limbs) return fhe_fail(FHE_ELEVEL, "fhe_sub: limb counts differ");
    if (a->polys != b->polys || out->polys != a->polys) return fhe_fail(FHE_EINVAL, "fhe_sub: poly counts differ");
    if (!scales_match(a->scale, b->scale)) return fhe_fail(FHE_ESCALE, "fhe_sub: scales differ");
    const uint64_t total = (uint64_t)a->polys * a->limbs * c->N;
    hipLaunchKernelGGL(k_addsub, dim3(blocks_for(total, TPB)), dim3(TPB), 0, c->stream, (const uint64_t *)a->d,
                       (const uint64_t *)b->d, out->d, (const ModQ *)c->d_mod, c->logN, a->limbs, total, 1);
    out->scale = a->scale;
    HIPCHK(hipGetLastError());
    return FHE_OK;
}
fhe_status fhe_add_pt(fhe_ctx *c, const fhe_ct *a, const fhe_pt *p, fhe_ct *out)
{
    fhe_status s;
    if (!c || !p || !p->d) return fhe_fail(FHE_EINVAL, "fhe_add_pt: null argument");
    if ((s = chk_ct(c, a, "fhe_add_pt")) || (s = chk_ct(c, out, "fhe_add_pt"))) return s;
    if (p->limbs != a->limbs || out->limbs != a->limbs || out->polys != a->polys)
        return fhe_fail(FHE_ELEVEL, "fhe_add_pt: shapes differ");
    if (!scales_match(a->scale, p->scale)) return fhe_fail(FHE_ESCALE, "fhe_add_pt: scales differ");
    const uint64_t per = (uint64_t)a->limbs * c->N;
    hipLaunchKernelGGL(k_addsub, dim3(blocks_for(per, TPB)), dim3(TPB), 0, c->stream, (const uint64_t *)a->d,
                       (const uint64_t *)p->d, out->d, (const ModQ *)c->d_mod, c->logN, a->limbs, per, 0);
    c->ops[OP_PT_ADD] += 1;
    if (out->d != a->d)
        HIPCHK(hipMemcpyAsync(out->d + per, a->d + per, (a->polys - 1) * per * sizeof(uint64_t),
                              hipMemcpyDeviceToDevice, c->stream));
    out->scale = a->scale;
    HIPCHK(hipGetLastError());
    return FHE_OK;
}
fhe_status fhe_mul_pt(fhe_ctx *c, const fhe_ct *a, const fhe_pt *p, fhe_ct *out)
{
    fhe_status s;
    if (!c || !p || !p->d) return fhe_fail(FHE_EINVAL, "fhe_mul_pt: null argument");
    if ((s = chk_ct(c, a, "fhe_mul_pt")) || (s = chk_ct(c, out, "fhe_mul_pt"))) return s;
    if (p->limbs != a->limbs || out->limbs != a->limbs || out->polys != a->polys)
        return fhe_fail(FHE_ELEVEL, "fhe_mul_pt: shapes differ");
    const uint64_t total = (uint64_t)a->polys * a->limbs * c->N;
    hipLaunchKernelGGL(k_mulpt, dim3(blocks_for(total, TPB)), dim3(TPB), 0, c->stream, (const uint64_t *)a->d,
                       (const uint64_t *)p->d, out->d, (const ModQ *)c->d_mod, c->logN, a->limbs, total);
    out->scale = a->scale * p->scale;
    c->ops[OP_PT_MULT] += 1;
    HIPCHK(hipGetLastError());
    return FHE_OK;
}
fhe_status fhe_mul_const(fhe_ctx *c, const fhe_ct *a, double value, double const_scale, fhe_ct *out)
{
    fhe_status s;
    if (!c) return fhe_fail(FHE_EINVAL, "null context");
    if ((s = chk_ct(c, a, "fhe_mul_const")) || (s = chk_ct(c, out, "fhe_mul_const"))) return s;
    if (out->limbs != a->limbs || out->polys != a->polys) return fhe_fail(FHE_EINVAL, "fhe_mul_const: shapes differ");
    const double v = std::nearbyint(value * const_scale);
    if (!(std::fabs(v) < 9.0e15)) return fhe_fail(FHE_EINVAL, "fhe_mul_const: constant out of range");
    Consts64 cres;
    std::memset(&cres, 0, sizeof(cres));
    const int64_t iv = (int64_t)v;
    for (uint32_t i = 0; i < a->limbs; ++i) {
        int64_t r = iv % (int64_t)c->mod[i];
        cres.v[i] = (double)(r < 0 ? r + (int64_t)c->mod[i] : r);
    }
    const uint64_t total = (uint64_t)a->polys * a->limbs * c->N;
    hipLaunchKernelGGL(k_mulconst, dim3(blocks_for(total, TPB)), dim3(TPB), 0, c->stream, (const uint64_t *)a->d,
                       out->d, cres, (const ModQ *)c->d_mod, c->logN, a->limbs, total);
    out->scale = a->scale * const_scale;
    c->ops[OP_PT_MULT] += 1;
    HIPCHK(hipGetLastError());
    return FHE_OK;
}
fhe_status fhe_mul_acc(fhe_ctx *c, const fhe_ct *a, const fhe_ct *b, uint32_t n, fhe_ct *acc3)
{
    fhe_status s;
    if (!c || !a || !b || !acc3 || !acc3->d || n == 0) return fhe_fail(FHE_EINVAL, "fhe_mul_acc: null or empty");
    const uint32_t l = a[0].limbs;
    if (acc3->polys != 3 || acc3->limbs != l) return fhe_fail(FHE_EINVAL, "fhe_mul_acc: accumulator must be 3 x l");
    const double sc = a[0].scale * b[0].scale;
    std::vector<uint64_t *> tab(2 * (size_t)n);
    for (uint32_t t = 0; t < n; ++t) {
        if ((s = chk_ct(c, &a[t], "fhe_mul_acc")) || (s = chk_ct(c, &b[t], "fhe_mul_acc"))) return s;
        if (a[t].limbs != l || b[t].limbs != l) return fhe_fail(FHE_ELEVEL, "fhe_mul_acc: limb counts differ");
        if (a[t].polys != 2 || b[t].polys != 2) return fhe_fail(FHE_EINVAL, "fhe_mul_acc: inputs must be 2-poly");
        if (!scales_match(a[t].scale * b[t].scale, sc)) return fhe_fail(FHE_ESCALE, "fhe_mul_acc: product scales differ");
        tab[t] = a[t].d;
        tab[n + t] = b[t].d;
    }
    uint64_t **dt;
    if ((s = ctx_ptr_table(c, tab, &dt))) return s;
    hipLaunchKernelGGL(k_tensor_acc, dim3(blocks_for((uint64_t)l * c->N, TPB)), dim3(TPB), 0, c->stream,
                       (uint64_t *const *)dt, (uint64_t *const *)(dt + n), n, acc3->d, (const ModQ *)c->d_mod, c->logN,
                       l);
    acc3->scale = sc;
    c->ops[OP_CT_MULT] += n;
    c->ops[OP_CT_ADD] += n - 1;
    HIPCHK(hipGetLastError());
    return FHE_OK;
}
fhe_status fhe_mul(fhe_ctx *c, const fhe_ct *a, const fhe_ct *b, fhe_ct *out3)
{
    return fhe_mul_acc(c, a, b, 1, out3);
}
fhe_status fhe_drop_level(fhe_ctx *c, const fhe_ct *in, uint32_t limbs, fhe_ct *out)
{
    fhe_status s;
    if (!c) return fhe_fail(FHE_EINVAL, "null context");
    if ((s = chk_ct(c, in, "fhe_drop_level")) || (s = chk_ct(c, out, "fhe_drop_level"))) return s;
    if (limbs < 1 || limbs > in->limbs || out->limbs != limbs || out->polys != in->polys)
        return fhe_fail(FHE_ELEVEL, "fhe_drop_level: bad target level");
    const size_t N = c->N;
    for (uint32_t p = 0; p < in->polys; ++p)
        if (out->d + p * limbs * N != in->d + p * in->limbs * N)
            HIPCHK(hipMemcpyAsync(out->d + p * limbs * N, in->d + p * in->limbs * N, limbs * N * sizeof(uint64_t),
                                  hipMemcpyDeviceToDevice, c->stream));
    out->scale = in->scale;
    return FHE_OK;
}
fhe_status fhe_rescale(fhe_ctx *c, const fhe_ct *in, fhe_ct *out)
{
    fhe_status s;
    if (!c) return fhe_fail(FHE_EINVAL, "null context");
    if ((s = chk_ct(c, in, "fhe_rescale")) || (s = chk_ct(c, out, "fhe_rescale"))) return s;
    const uint32_t l = in->limbs, P = in->polys;
    if (l < 2) return fhe_fail(FHE_ELEVEL, "fhe_rescale: one limb left");
    if (out->limbs != l - 1 || out->polys != P) return fhe_fail(FHE_EINVAL, "fhe_rescale: output must have l-1 limbs");
    const size_t N = c->N;
    // the output layout [P][l-1] overlaps an aliased input [P][l] at other offsets:
    // then write to scratch and copy back
    const uint64_t *ib = in->d, *ie = in->d + (size_t)P * l * N, *ob = out->d, *oe = out->d + (size_t)P * (l - 1) * N;
    const bool overlap = ob < ie && ib < oe;
    const size_t need = rescale_scratch_bytes(c, l, P, 1);
    uint8_t *scr;
    if ((s = ctx_scratch(c, need + (overlap ? (size_t)P * (l - 1) * N * 8 : 0), &scr))) return s;
    uint64_t *dst = overlap ? (uint64_t *)(scr + need) : out->d;
    const uint64_t *ip[1] = {in->d};
    uint64_t *op[1] = {dst};
    if ((s = rescale_run(c, l, P, 1, ip, op, scr))) return s;
    if (overlap)
        HIPCHK(hipMemcpyAsync(out->d, dst, (size_t)P * (l - 1) * N * sizeof(uint64_t), hipMemcpyDeviceToDevice,
                              c->stream));
    out->scale = in->scale / (double)c->mod[l - 1];
    c->ops[OP_RESCALE] += 1;
    return FHE_OK;
}
fhe_status fhe_keyswitch(fhe_ctx *c, const fhe_evk *evk, const uint64_t *d, uint32_t limbs, fhe_ct *out)
{
    fhe_status s;
    if (!c || !evk || !evk->d || !d) return fhe_fail(FHE_EINVAL, "fhe_keyswitch: null argument");
    if ((s = chk_ct(c, out, "fhe_keyswitch"))) return s;
    if (out->limbs != limbs || out->polys != 2) return fhe_fail(FHE_EINVAL, "fhe_keyswitch: output must be 2 x limbs");
    const uint64_t *dd[1] = {d};
    const uint64_t *ek[1] = {evk->d};
    uint64_t *oo[1] = {out->d};
    return ks_run(c, limbs, 1, dd, ek, oo, nullptr, nullptr);
}
fhe_status fhe_keyswitch_batch(fhe_ctx *c, const fhe_evk *evk, const uint64_t *const *d, uint32_t limbs, uint32_t n,
                               fhe_ct *out)
{
    fhe_status s;
    if (!c || !evk || !d || !out || !n) return fhe_fail(FHE_EINVAL, "fhe_keyswitch_batch: null or empty");
    std::vector<const uint64_t *> dd(n), ek(n);
    std::vector<uint64_t *> oo(n);
    for (uint32_t b = 0; b < n; ++b) {
        if (!evk[b].d || !d[b]) return fhe_fail(FHE_EINVAL, "fhe_keyswitch_batch: null entry");
        if ((s = chk_ct(c, &out[b], "fhe_keyswitch_batch"))) return s;
        if (out[b].limbs != limbs || out[b].polys != 2) return fhe_fail(FHE_EINVAL, "fhe_keyswitch_batch: bad output");
        dd[b] = d[b]; ek[b] = evk[b].d; oo[b] = out[b].d;
    }
    return ks_run(c, limbs, n, dd.data(), ek.data(), oo.data(), nullptr, nullptr);
}
fhe_status fhe_relin(fhe_ctx *c, const fhe_evk *rlk, const fhe_ct *in3, fhe_ct *out2)
{
    fhe_status s;
    if (!c || !rlk || !rlk->d) return fhe_fail(FHE_EINVAL, "fhe_relin: null argument");
    if ((s = chk_ct(c, in3, "fhe_relin")) || (s = chk_ct(c, out2, "fhe_relin"))) return s;
    if (in3->polys != 3 || out2->polys != 2 || out2->limbs != in3->limbs)
        return fhe_fail(FHE_EINVAL, "fhe_relin: need 3-poly input and 2-poly output at the same level");
    if (rlk->galois != 0) return fhe_fail(FHE_ENOKEY, "fhe_relin: key is a rotation key");
    const size_t per = (size_t)in3->limbs * c->N;
    const uint64_t *dd[1] = {in3->d + 2 * per};
    const uint64_t *ek[1] = {rlk->d};
    uint64_t *oo[1] = {out2->d};
    const uint64_t *ad[2] = {in3->d, in3->d + per};   // (d0, d1) + (ks0, ks1)
    fhe_status r = ks_run(c, in3->limbs, 1, dd, ek, oo, ad, nullptr);
    out2->scale = in3->scale;
    c->ops[OP_RELIN] += 1;
    return r;
}
fhe_status fhe_rotate(fhe_ctx *c, const fhe_evk *gk, const fhe_ct *in, int32_t step, fhe_ct *out)
{
    fhe_status s;
    if (!c || !gk || !gk->d) return fhe_fail(FHE_EINVAL, "fhe_rotate: null argument");
    if ((s = chk_ct(c, in, "fhe_rotate")) || (s = chk_ct(c, out, "fhe_rotate"))) return s;
    if (in->polys != 2 || out->polys != 2 || out->limbs != in->limbs) return fhe_fail(FHE_EINVAL, "fhe_rotate: shapes");
    const uint64_t g = fhe_galois_elt(c, step);
    if (gk->galois != g) return fhe_fail(FHE_ENOKEY, "fhe_rotate: Galois key is for another step");
    const uint32_t l = in->limbs;
    const size_t per = (size_t)l * c->N;
    // sigma_g of both polys into scratch tail; key switch of sigma_g(c1), add sigma_g(c0)
    uint8_t *scr;
    // the key-switch scratch is taken first; the permuted input lives past it
    const uint32_t nd = (l + c->alpha - 1) / c->alpha;
    size_t ups = 0;
    for (uint32_t j = 0; j < nd; ++j) ups += c->modup[(size_t)l * c->dnum + j].ndst;
    const size_t ks_limbs = l + ups + 4 * (size_t)l + 2 * c->K;
    if ((s = ctx_scratch(c, (ks_limbs + 2 * (size_t)l) * c->N * sizeof(uint64_t), &scr))) return s;
    uint64_t *perm = (uint64_t *)scr + ks_limbs * c->N;
    hipLaunchKernelGGL(k_automorph, dim3(blocks_for(2 * per, TPB)), dim3(TPB), 0, c->stream, (const uint64_t *)in->d,
                       perm, c->logN, (uint64_t)2 * l, (uint32_t)g);
    const uint64_t *dd[1] = {perm + per};
    const uint64_t *ek[1] = {gk->d};
    uint64_t *oo[1] = {out->d};
    const uint64_t *ad[2] = {perm, nullptr};   // (sigma_g(c0) + ks0, ks1)
    fhe_status r = ks_run(c, l, 1, dd, ek, oo, ad, scr);
    out->scale = in->scale;
    c->ops[OP_ROTATE] += 1;
    return r;
}

fhe_status fhe_rotate_batch(fhe_ctx *c, const fhe_evk *gk, const fhe_ct *in, const int32_t *steps, uint32_t n,
                            fhe_ct *out)
{
    fhe_status s;
    if (!c || !gk || !in || !steps || !out || !n) return fhe_fail(FHE_EINVAL, "fhe_rotate_batch: null or empty");
    const uint32_t l = in[0].limbs;
    for (uint32_t b = 0; b < n; ++b) {
        if (!gk[b].d) return fhe_fail(FHE_EINVAL, "fhe_rotate_batch: null key");
        if ((s = chk_ct(c, &in[b], "fhe_rotate_batch")) || (s = chk_ct(c, &out[b], "fhe_rotate_batch"))) return s;
        if (in[b].limbs != l || in[b].polys != 2 || out[b].polys != 2 || out[b].limbs != l)
            return fhe_fail(FHE_EINVAL, "fhe_rotate_batch: all inputs and outputs must be 2 x l");
        if (gk[b].galois != fhe_galois_elt(c, steps[b]))
            return fhe_fail(FHE_ENOKEY, "fhe_rotate_batch: Galois key is for another step");
    }
    const size_t per = (size_t)l * c->N;
    const uint32_t nd = (l + c->alpha - 1) / c->alpha;
    size_t ups = 0;
    for (uint32_t j = 0; j < nd; ++j) ups += c->modup[(size_t)l * c->dnum + j].ndst;
    const size_t ks_limbs = (size_t)n * (l + ups + 4 * (size_t)l + 2 * c->K);
    uint8_t *scr;
    if ((s = ctx_scratch(c, (ks_limbs + 2 * (size_t)n * l) * c->N * sizeof(uint64_t), &scr))) return s;
    uint64_t *perm = (uint64_t *)scr + ks_limbs * c->N;
    std::vector<const uint64_t *> dd(n), ek(n), ad(2 * (size_t)n, nullptr);
    std::vector<uint64_t *> oo(n);
    {
        ProfScope ps(c, "automorph");
        for (uint32_t b = 0; b < n; ++b) {
            uint64_t *pb = perm + (size_t)b * 2 * per;
            hipLaunchKernelGGL(k_automorph, dim3(blocks_for(2 * per, TPB)), dim3(TPB), 0, c->stream,
                               (const uint64_t *)in[b].d, pb, c->logN, (uint64_t)2 * l, (uint32_t)gk[b].galois);
            dd[b] = pb + per;
            ad[2 * b] = pb;
            ek[b] = gk[b].d;
            oo[b] = out[b].d;
        }
    }
    fhe_status r = ks_run(c, l, n, dd.data(), ek.data(), oo.data(), ad.data(), scr);
    for (uint32_t b = 0; b < n; ++b) out[b].scale = in[b].scale;
    c->ops[OP_ROTATE] += n;
    return r;
}

}  // extern "C"

// Used by the client code (keygen): NTT-domain automorphism of nlimbs limbs.
void launch_automorph(fhe_ctx *c, const uint64_t *in, uint64_t *out, uint32_t nlimbs, uint64_t g)
{
    hipLaunchKernelGGL(k_automorph, dim3(blocks_for((uint64_t)nlimbs * c->N, TPB)), dim3(TPB), 0, c->stream, in, out,
                       c->logN, (uint64_t)nlimbs, (uint32_t)g);
}
