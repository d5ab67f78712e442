// client.hip -- the end user's side of the protocol (the paper's MLaaS setting,
// Sec. 1 and Fig. 1: the user generates the keys, encrypts its images, and
// the model owner encrypts the weights under the same public key; the user
// decrypts the class scores, Sec. 4.3): Philox4x64-10 samplers, key
// generation, encryption, decryption and slot encoding/decoding, all on the GPU.
//
// Random streams (rejection loops stop after 64 rounds, a probability below
// 2^-256 that the definition below never reaches).  Philox4x64-10 with key (seed, tag), counter
// (coefficient, modulus index or 0, polynomial id, round):
//   tag 1 secret s, tag 2 uniform polynomials, tag 3 errors, tag 4 the
//   encryption mask v.
//   uniform mod q: each word of the block masked to bitlen(q), the first one
//     below q is taken, a fully rejected block moves to the next round;
//   ternary: low 32 bits u of each word, rejected if u >= 3 floor(2^32/3),
//     value (u mod 3) - 1;
//   error: |e| = #{i : cdt[i] <= w0}, negative when nonzero and w1 is odd.
// Key material (secret key polys 0; public key poly 0; key-switching key of
// digit j: poly j; encryption: v poly 0, e0 poly 0, e1 poly 1).
//
// Encoding.  Slot j is the evaluation at zeta^(5^j mod 2N), zeta = e^(i pi/N);
//   m_k = rint( (sum_j re_j cos(pi e/N) + im_j sin(pi e/N)) * (2/N) * scale ),
//   e = k 5^j mod 2N, summed in slot order; decoding sums m_k cos / sin in
//   coefficient order and divides by the scale.  Both use direct O(N n) sums in
//   FP64 without contraction, one thread per output.
#include <cmath>
#include <cstring>

#include "fhe_internal.h"

#pragma clang fp contract(off)

void launch_automorph(fhe_ctx *c, const uint64_t *in, uint64_t *out, uint32_t nlimbs, uint64_t g);

namespace {

constexpr int TPB = 256;
constexpr uint64_t TAG_SECRET = 1, TAG_UNIFORM = 2, TAG_ERROR = 3, TAG_EPHEMERAL = 4;

inline uint32_t blocks_for(uint64_t n, uint32_t per) { return (uint32_t)((n + per - 1) / per); }

struct ModList {
    uint32_t n;
    uint8_t m[FHE_LIMBTAB];
};

__global__ void k_sample_uniform(uint64_t *out, ModList ml, const ModQ *__restrict__ mods, uint64_t seed,
                                 uint64_t poly_id, uint32_t logN)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    const uint32_t li = blockIdx.y, mi = ml.m[li];
    const uint64_t q = (uint64_t)mods[mi].q;
    const uint32_t bits = 64 - __clzll(q);
    const uint64_t mask = bits >= 64 ? ~0ull : ((1ull << bits) - 1);
    uint64_t val = 0;
    // a block is rejected with probability < 1/16; 64 rounds bound the loop
    for (uint64_t round = 0; round < 64; ++round) {
        uint64_t w[4];
        philox4x64_10(seed, TAG_UNIFORM, k, mi, poly_id, round, w);
        bool found = false;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (!found && (w[i] & mask) < q) { val = w[i] & mask; found = true; }
        if (found) break;
    }
    out[(size_t)li * N + k] = val;
}
__global__ void k_sample_ternary(int64_t *out, uint64_t seed, uint64_t tag, uint64_t poly_id, uint32_t N)
{
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    const uint64_t lim = 3ull * (0x100000000ull / 3);
    int64_t val = 0;
    for (uint64_t round = 0; round < 64; ++round) {
        uint64_t w[4];
        philox4x64_10(seed, tag, k, 0, poly_id, round, w);
        bool found = false;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint64_t u = w[i] & 0xffffffffull;
            if (!found && u < lim) { val = (int64_t)(u % 3) - 1; found = true; }
        }
        if (found) break;
    }
    out[k] = val;
}
__global__ void k_sample_gauss(int64_t *out, const uint64_t *__restrict__ cdt, uint32_t ncdt, uint64_t seed,
                               uint64_t poly_id, uint32_t N)
{
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    uint64_t w[4];
    philox4x64_10(seed, TAG_ERROR, k, 0, poly_id, 0, w);
    int64_t mag = 0;
    for (uint32_t i = 0; i < ncdt; ++i) mag += cdt[i] <= w[0];
    out[k] = (mag != 0 && (w[1] & 1)) ? -mag : mag;
}
// signed small coefficients -> residues on the listed limbs
__global__ void k_small_to_rns(const int64_t *__restrict__ a, uint64_t *out, ModList ml,
                               const ModQ *__restrict__ mods, uint32_t logN)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    const uint32_t li = blockIdx.y;
    const int64_t q = (int64_t)mods[ml.m[li]].q;
    int64_t r = a[k] % q;
    if (r < 0) r += q;
    out[(size_t)li * N + k] = (uint64_t)r;
}
__global__ void k_i8_to_i64(const int8_t *__restrict__ a, int64_t *out, uint32_t N)
{
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k < N) out[k] = a[k];
}
// b = e - a*s (+ g * t) on limb li (modulus ml.m[li]); g per limb (0 = none), all NTT domain.
__global__ void k_rlwe_b(const uint64_t *__restrict__ a, const uint64_t *__restrict__ s, const uint64_t *__restrict__ e,
                         const uint64_t *__restrict__ t, Consts64 gadget, uint64_t *b, ModList ml,
                         const ModQ *__restrict__ mods, uint32_t logN)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    const uint32_t li = blockIdx.y;
    const size_t i = (size_t)li * N + k;
    const double q = mods[ml.m[li]].q, qi = mods[ml.m[li]].qinv;
    double r = u64_to_f64(e[i]) - mulmod(u64_to_f64(a[i]), u64_to_f64(s[i]), q, qi);
    if (t && gadget.v[li] != 0.0) r += mulmod(gadget.v[li], u64_to_f64(t[i]), q, qi);
    b[i] = f64_to_u64(canon(r, q, qi));
}
// pointwise product out = x * y (limbs ml)
__global__ void k_pmul(const uint64_t *__restrict__ x, const uint64_t *__restrict__ y, uint64_t *out, ModList ml,
                       const ModQ *__restrict__ mods, uint32_t logN)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    const size_t i = (size_t)blockIdx.y * N + k;
    const double q = mods[ml.m[blockIdx.y]].q, qi = mods[ml.m[blockIdx.y]].qinv;
    out[i] = f64_to_u64(fold(mulmod(u64_to_f64(x[i]), u64_to_f64(y[i]), q, qi), q));
}
// encryption: c0 = v*b + e0 + m, c1 = v*a + e1 on limbs 0..l-1 (pk has L limbs per poly)
__global__ void k_encrypt(const uint64_t *__restrict__ pk, uint32_t L, const uint64_t *__restrict__ v,
                          const uint64_t *__restrict__ e0, const uint64_t *__restrict__ e1,
                          const uint64_t *__restrict__ m, uint64_t *ct, uint32_t l, const ModQ *__restrict__ mods,
                          uint32_t logN)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    const uint32_t i = blockIdx.y;
    const size_t x = (size_t)i * N + k;
    const double q = mods[i].q, qi = mods[i].qinv;
    const double vv = u64_to_f64(v[x]);
    const double b = u64_to_f64(pk[x]), a = u64_to_f64(pk[(size_t)(L + i) * N + k]);
    const double c0 = mulmod(vv, b, q, qi) + u64_to_f64(e0[x]) + u64_to_f64(m[x]);
    const double c1 = mulmod(vv, a, q, qi) + u64_to_f64(e1[x]);
    ct[x] = f64_to_u64(canon(c0, q, qi));
    ct[(size_t)l * N + x] = f64_to_u64(canon(c1, q, qi));
}
// decryption: m = c0 + c1 s (+ c2 s^2)
__global__ void k_decrypt(const uint64_t *__restrict__ ct, uint32_t polys, const uint64_t *__restrict__ s,
                          uint64_t *m, uint32_t l, const ModQ *__restrict__ mods, uint32_t logN)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    const uint32_t i = blockIdx.y;
    const size_t x = (size_t)i * N + k, per = (size_t)l * N;
    const double q = mods[i].q, qi = mods[i].qinv;
    const double sv = u64_to_f64(s[x]);
    double r = u64_to_f64(ct[x]) + mulmod(u64_to_f64(ct[per + x]), sv, q, qi);
    if (polys == 3) {
        const double s2 = fold(mulmod(sv, sv, q, qi), q);
        r += mulmod(u64_to_f64(ct[2 * per + x]), s2, q, qi);
    }
    m[x] = f64_to_u64(canon(r, q, qi));
}
// encoding: one thread per coefficient k
__global__ void k_encode(const double *__restrict__ re, const double *__restrict__ im, uint32_t n,
                         const double *__restrict__ cs, const double *__restrict__ sn, const uint32_t *__restrict__ g5,
                         double scale, uint32_t logN, int64_t *coeff, int *overflow)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    const uint32_t mask = 2u * N - 1u;
    double acc = 0.0;
    for (uint32_t j = 0; j < n; ++j) {
        const uint32_t e = (k * g5[j]) & mask;
        acc += re[j] * cs[e];
        if (im) acc += im[j] * sn[e];
    }
    double v = __builtin_rint(acc * (2.0 / (double)N) * scale);
    if (!(fabs(v) < 4611686018427387904.0)) {
        *overflow = 1;
        v = 0.0;
    }
    coeff[k] = (int64_t)v;
}
// Correctly rounded conversion of an unsigned 128-bit integer (hi, lo) to double:
// the top 64 significant bits with the discarded bits folded into a sticky bit,
// then one rounding of that 64-bit integer and an exact scaling by 2^s.
__device__ __forceinline__ double u128_to_f64(uint64_t hi, uint64_t lo)
{
    if (hi == 0) return (double)lo;
    const int s = 64 - __clzll(hi);
    uint64_t m = (hi << (64 - s)) | (lo >> s);
    if (lo & ((1ull << s) - 1)) m |= 1ull;
    return ldexp((double)m, s);
}
// centered lift of the plaintext from limb 0 (l == 1) or limbs 0, 1 by CRT
__global__ void k_lift(const uint64_t *__restrict__ m, uint32_t l, uint64_t q0, uint64_t q1, uint64_t q0inv_mod_q1,
                       double *out, uint32_t logN)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    if (l == 1) {
        const uint64_t x = m[k];
        out[k] = x > q0 / 2 ? -(double)(q0 - x) : (double)x;
    } else {
        typedef unsigned __int128 u128;
        const uint64_t x0 = m[k], x1 = m[(size_t)N + k];
        const uint64_t d = (x1 + q1 - x0 % q1) % q1;
        const uint64_t t = (uint64_t)(((u128)d * q0inv_mod_q1) % q1);
        const u128 Q = (u128)q0 * q1, x = (u128)x0 + (u128)q0 * t;
        if (x > Q / 2) {
            const u128 y = Q - x;
            out[k] = -u128_to_f64((uint64_t)(y >> 64), (uint64_t)y);
        } else {
            out[k] = u128_to_f64((uint64_t)(x >> 64), (uint64_t)x);
        }
    }
}
__global__ void k_narrow_u32(const uint64_t *__restrict__ w, uint32_t n, uint32_t *out)
{
    const uint32_t t = blockIdx.x * TPB + threadIdx.x;
    if (t < n) out[t] = (uint32_t)w[t];
}
// Decoding: slot j = sum_k m_k zeta^(k 5^j), one 256-thread block per slot
// (blockIdx.x = output index, slot idx[blockIdx.x] or the index itself): thread t
// sums the terms k = t mod 256, then a tree reduction in LDS.
__global__ __launch_bounds__(TPB) void k_decode(const double *__restrict__ mv, const double *__restrict__ cs,
                                               const double *__restrict__ sn, const uint32_t *__restrict__ g5,
                                               const uint32_t *__restrict__ idx, double scale, uint32_t logN,
                                               double *re, double *im)
{
    __shared__ double sr[TPB], si[TPB];
    const uint32_t N = 1u << logN;
    const uint32_t o = blockIdx.x, j = idx ? idx[o] : o;
    const uint32_t mask = 2u * N - 1u, g = g5[j];
    double ar = 0.0, ai = 0.0;
    for (uint32_t k = threadIdx.x; k < N; k += TPB) {
        const uint32_t e = (k * g) & mask;
        ar += mv[k] * cs[e];
        ai += mv[k] * sn[e];
    }
    sr[threadIdx.x] = ar;
    si[threadIdx.x] = ai;
    __syncthreads();
    for (uint32_t h = TPB / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            sr[threadIdx.x] += sr[threadIdx.x + h];
            si[threadIdx.x] += si[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        re[o] = sr[0] / scale;
        im[o] = si[0] / scale;
    }
}

ModList modlist_range(uint32_t first, uint32_t count)
{
    ModList ml;
    std::memset(&ml, 0, sizeof(ml));
    ml.n = count;
    for (uint32_t i = 0; i < count; ++i) ml.m[i] = (uint8_t)(first + i);
    return ml;
}
ModList modlist_qp(const fhe_ctx *c)   // all L + K moduli
{
    return modlist_range(0, c->L + c->K);
}
void ntt_list(fhe_ctx *c, uint64_t *d, const ModList &ml, bool inverse)
{
    uint32_t m[FHE_LIMBTAB];
    for (uint32_t i = 0; i < ml.n; ++i) m[i] = ml.m[i];
    LimbSet ls = limbset_list(d, m, ml.n);
    if (inverse) launch_ntt_inv(c, ls, ml.n);
    else launch_ntt_fwd(c, ls, ml.n);
}
// s (host int8) -> NTT-domain residues on the listed limbs
void upload_secret_ntt(fhe_ctx *c, const int8_t *s_dev, int64_t *tmp, uint64_t *out, const ModList &ml)
{
    const uint32_t gx = blocks_for(c->N, TPB);
    hipLaunchKernelGGL(k_i8_to_i64, dim3(gx), dim3(TPB), 0, c->stream, s_dev, tmp, c->N);
    hipLaunchKernelGGL(k_small_to_rns, dim3(gx, ml.n), dim3(TPB), 0, c->stream, (const int64_t *)tmp, out, ml,
                       (const ModQ *)c->d_mod, c->logN);
    ntt_list(c, out, ml, false);
}

}  // namespace

// ===================================================================== API
extern "C" {

fhe_status fhe_keygen_secret(fhe_ctx *c, uint64_t seed, int8_t *s_host)
{
    if (!c || !s_host) return fhe_fail(FHE_EINVAL, "fhe_keygen_secret: null argument");
    uint8_t *scr;
    fhe_status s = ctx_scratch(c, (size_t)c->N * sizeof(int64_t), &scr);
    if (s) return s;
    hipLaunchKernelGGL(k_sample_ternary, dim3(blocks_for(c->N, TPB)), dim3(TPB), 0, c->stream, (int64_t *)scr, seed,
                       TAG_SECRET, (uint64_t)0, c->N);
    std::vector<int64_t> h(c->N);
    HIPCHK(hipMemcpyAsync(h.data(), scr, c->N * sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (uint32_t k = 0; k < c->N; ++k) s_host[k] = (int8_t)h[k];
    return FHE_OK;
}

// Scratch layout for key generation / encryption: [s8 (N bytes, padded)] [i64 N] [limb buffers...]
static fhe_status client_scratch(fhe_ctx *c, uint32_t nlimbs, int8_t **s8, int64_t **i64, uint64_t **limbs)
{
    const size_t N = c->N;
    uint8_t *scr;
    fhe_status s = ctx_scratch(c, ((N + 255) & ~(size_t)255) + N * 8 + (size_t)nlimbs * N * 8, &scr);
    if (s) return s;
    *s8 = (int8_t *)scr;
    *i64 = (int64_t *)(scr + ((N + 255) & ~(size_t)255));
    *limbs = (uint64_t *)(*i64 + N);
    return FHE_OK;
}

fhe_status fhe_keygen_pk(fhe_ctx *c, const int8_t *s_host, uint64_t seed, fhe_ct *pk)
{
    if (!c || !s_host || !pk || !pk->d) return fhe_fail(FHE_EINVAL, "fhe_keygen_pk: null argument");
    if (pk->polys != 2 || pk->limbs != c->L) return fhe_fail(FHE_EINVAL, "fhe_keygen_pk: pk must be 2 x n_q limbs");
    const uint32_t L = c->L, N = c->N;
    int8_t *s8; int64_t *i64; uint64_t *lb;
    fhe_status s = client_scratch(c, 2 * L, &s8, &i64, &lb);
    if (s) return s;
    uint64_t *s_ntt = lb, *e_ntt = lb + (size_t)L * N;
    HIPCHK(hipMemcpyAsync(s8, s_host, N, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));   // s_host may be reused by the caller
    ModList ml = modlist_range(0, L);
    upload_secret_ntt(c, s8, i64, s_ntt, ml);
    const uint32_t gx = blocks_for(N, TPB);
    uint64_t *a = pk->d + (size_t)L * N;
    hipLaunchKernelGGL(k_sample_uniform, dim3(gx, L), dim3(TPB), 0, c->stream, a, ml, (const ModQ *)c->d_mod, seed,
                       (uint64_t)0, c->logN);
    ntt_list(c, a, ml, false);
    hipLaunchKernelGGL(k_sample_gauss, dim3(gx), dim3(TPB), 0, c->stream, i64, (const uint64_t *)c->d_cdt, c->ncdt,
                       seed, (uint64_t)0, N);
    hipLaunchKernelGGL(k_small_to_rns, dim3(gx, L), dim3(TPB), 0, c->stream, (const int64_t *)i64, e_ntt, ml,
                       (const ModQ *)c->d_mod, c->logN);
    ntt_list(c, e_ntt, ml, false);
    Consts64 none;
    std::memset(&none, 0, sizeof(none));
    hipLaunchKernelGGL(k_rlwe_b, dim3(gx, L), dim3(TPB), 0, c->stream, (const uint64_t *)a, (const uint64_t *)s_ntt,
                       (const uint64_t *)e_ntt, (const uint64_t *)nullptr, none, pk->d, ml, (const ModQ *)c->d_mod,
                       c->logN);
    pk->scale = 0.0;
    HIPCHK(hipGetLastError());
    return FHE_OK;
}

// Key-switching key from s_from (given NTT-domain on all L+K limbs) to s.
static fhe_status keygen_evk(fhe_ctx *c, const uint64_t *s_ntt, const uint64_t *sf_ntt, int64_t *i64, uint64_t *e_ntt,
                             uint64_t seed, uint64_t *evk)
{
    const uint32_t L = c->L, K = c->K, M = L + K, N = c->N;
    const uint32_t gx = blocks_for(N, TPB);
    ModList ml = modlist_qp(c);
    for (uint32_t j = 0; j < c->dnum; ++j) {
        uint64_t *b = evk + (size_t)j * 2 * M * N, *a = b + (size_t)M * N;
        hipLaunchKernelGGL(k_sample_uniform, dim3(gx, M), dim3(TPB), 0, c->stream, a, ml, (const ModQ *)c->d_mod, seed,
                           (uint64_t)j, c->logN);
        ntt_list(c, a, ml, false);
        hipLaunchKernelGGL(k_sample_gauss, dim3(gx), dim3(TPB), 0, c->stream, i64, (const uint64_t *)c->d_cdt, c->ncdt,
                           seed, (uint64_t)j, N);
        hipLaunchKernelGGL(k_small_to_rns, dim3(gx, M), dim3(TPB), 0, c->stream, (const int64_t *)i64, e_ntt, ml,
                           (const ModQ *)c->d_mod, c->logN);
        ntt_list(c, e_ntt, ml, false);
        Consts64 g;
        std::memset(&g, 0, sizeof(g));
        const uint32_t lo = j * c->alpha, hi = std::min(lo + c->alpha, L);
        for (uint32_t i = lo; i < hi; ++i) {
            // P mod q_i
            unsigned __int128 pm = 1;
            for (uint32_t t = 0; t < K; ++t) pm = pm * (c->mod[L + t] % c->mod[i]) % c->mod[i];
            g.v[i] = (double)(uint64_t)pm;
        }
        hipLaunchKernelGGL(k_rlwe_b, dim3(gx, M), dim3(TPB), 0, c->stream, (const uint64_t *)a, s_ntt,
                           (const uint64_t *)e_ntt, sf_ntt, g, b, ml, (const ModQ *)c->d_mod, c->logN);
    }
    HIPCHK(hipGetLastError());
    return FHE_OK;
}

fhe_status fhe_keygen_relin(fhe_ctx *c, const int8_t *s_host, uint64_t seed, fhe_evk *out)
{
    if (!c || !s_host || !out || !out->d) return fhe_fail(FHE_EINVAL, "fhe_keygen_relin: null argument");
    if (!c->K) return fhe_fail(FHE_EPARAM, "key switching needs special primes");
    const uint32_t M = c->L + c->K, N = c->N;
    int8_t *s8; int64_t *i64; uint64_t *lb;
    fhe_status s = client_scratch(c, 3 * M, &s8, &i64, &lb);
    if (s) return s;
    uint64_t *s_ntt = lb, *s2 = lb + (size_t)M * N, *e_ntt = lb + (size_t)2 * M * N;
    HIPCHK(hipMemcpyAsync(s8, s_host, N, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    ModList ml = modlist_qp(c);
    upload_secret_ntt(c, s8, i64, s_ntt, ml);
    hipLaunchKernelGGL(k_pmul, dim3(blocks_for(N, TPB), M), dim3(TPB), 0, c->stream, (const uint64_t *)s_ntt,
                       (const uint64_t *)s_ntt, s2, ml, (const ModQ *)c->d_mod, c->logN);
    out->galois = 0;
    return keygen_evk(c, s_ntt, s2, i64, e_ntt, seed, out->d);
}

fhe_status fhe_keygen_rot(fhe_ctx *c, const int8_t *s_host, int32_t step, uint64_t seed, fhe_evk *out)
{
    if (!c || !s_host || !out || !out->d) return fhe_fail(FHE_EINVAL, "fhe_keygen_rot: null argument");
    if (!c->K) return fhe_fail(FHE_EPARAM, "key switching needs special primes");
    const uint32_t M = c->L + c->K, N = c->N;
    int8_t *s8; int64_t *i64; uint64_t *lb;
    fhe_status s = client_scratch(c, 3 * M, &s8, &i64, &lb);
    if (s) return s;
    uint64_t *s_ntt = lb, *sg = lb + (size_t)M * N, *e_ntt = lb + (size_t)2 * M * N;
    HIPCHK(hipMemcpyAsync(s8, s_host, N, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    ModList ml = modlist_qp(c);
    upload_secret_ntt(c, s8, i64, s_ntt, ml);
    const uint64_t g = fhe_galois_elt(c, step);
    launch_automorph(c, s_ntt, sg, M, g);
    out->galois = g;
    return keygen_evk(c, s_ntt, sg, i64, e_ntt, seed, out->d);
}

fhe_status fhe_encrypt(fhe_ctx *c, const fhe_ct *pk, const fhe_pt *m, uint64_t seed, fhe_ct *out)
{
    if (!c || !pk || !pk->d || !m || !m->d || !out || !out->d) return fhe_fail(FHE_EINVAL, "fhe_encrypt: null argument");
    if (pk->polys != 2 || pk->limbs != c->L) return fhe_fail(FHE_EINVAL, "fhe_encrypt: bad public key");
    const uint32_t l = m->limbs, N = c->N;
    if (l < 1 || l > c->L) return fhe_fail(FHE_ELEVEL, "fhe_encrypt: plaintext level out of range");
    if (out->polys != 2 || out->limbs != l) return fhe_fail(FHE_EINVAL, "fhe_encrypt: output must be 2 x limbs");
    int8_t *s8; int64_t *i64; uint64_t *lb;
    fhe_status s = client_scratch(c, 3 * l, &s8, &i64, &lb);
    if (s) return s;
    uint64_t *v = lb, *e0 = lb + (size_t)l * N, *e1 = lb + (size_t)2 * l * N;
    const uint32_t gx = blocks_for(N, TPB);
    ModList ml = modlist_range(0, l);
    hipLaunchKernelGGL(k_sample_ternary, dim3(gx), dim3(TPB), 0, c->stream, i64, seed, TAG_EPHEMERAL, (uint64_t)0, N);
    hipLaunchKernelGGL(k_small_to_rns, dim3(gx, l), dim3(TPB), 0, c->stream, (const int64_t *)i64, v, ml,
                       (const ModQ *)c->d_mod, c->logN);
    hipLaunchKernelGGL(k_sample_gauss, dim3(gx), dim3(TPB), 0, c->stream, i64, (const uint64_t *)c->d_cdt, c->ncdt,
                       seed, (uint64_t)0, N);
    hipLaunchKernelGGL(k_small_to_rns, dim3(gx, l), dim3(TPB), 0, c->stream, (const int64_t *)i64, e0, ml,
                       (const ModQ *)c->d_mod, c->logN);
    hipLaunchKernelGGL(k_sample_gauss, dim3(gx), dim3(TPB), 0, c->stream, i64, (const uint64_t *)c->d_cdt, c->ncdt,
                       seed, (uint64_t)1, N);
    hipLaunchKernelGGL(k_small_to_rns, dim3(gx, l), dim3(TPB), 0, c->stream, (const int64_t *)i64, e1, ml,
                       (const ModQ *)c->d_mod, c->logN);
    {
        uint32_t mm[FHE_LIMBTAB];
        for (uint32_t i = 0; i < l; ++i) mm[i] = i;
        launch_ntt_fwd(c, limbset_list(lb, mm, l), 3 * l);
    }
    hipLaunchKernelGGL(k_encrypt, dim3(gx, l), dim3(TPB), 0, c->stream, (const uint64_t *)pk->d, c->L,
                       (const uint64_t *)v, (const uint64_t *)e0, (const uint64_t *)e1, (const uint64_t *)m->d, out->d,
                       l, (const ModQ *)c->d_mod, c->logN);
    out->scale = m->scale;
    HIPCHK(hipGetLastError());
    return FHE_OK;
}

fhe_status fhe_decrypt(fhe_ctx *c, const int8_t *s_host, const fhe_ct *ct, fhe_pt *out)
{
    if (!c || !s_host || !ct || !ct->d || !out || !out->d) return fhe_fail(FHE_EINVAL, "fhe_decrypt: null argument");
    const uint32_t l = ct->limbs, N = c->N;
    if (l < 1 || l > c->L || out->limbs != l) return fhe_fail(FHE_ELEVEL, "fhe_decrypt: level mismatch");
    if (ct->polys < 2 || ct->polys > 3) return fhe_fail(FHE_EINVAL, "fhe_decrypt: polys must be 2 or 3");
    int8_t *s8; int64_t *i64; uint64_t *lb;
    fhe_status s = client_scratch(c, l, &s8, &i64, &lb);
    if (s) return s;
    HIPCHK(hipMemcpyAsync(s8, s_host, N, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    ModList ml = modlist_range(0, l);
    upload_secret_ntt(c, s8, i64, lb, ml);
    hipLaunchKernelGGL(k_decrypt, dim3(blocks_for(N, TPB), l), dim3(TPB), 0, c->stream, (const uint64_t *)ct->d,
                       ct->polys, (const uint64_t *)lb, out->d, l, (const ModQ *)c->d_mod, c->logN);
    out->scale = ct->scale;
    HIPCHK(hipGetLastError());
    return FHE_OK;
}

fhe_status fhe_encode_coeffs(fhe_ctx *c, const int64_t *coeff_host, fhe_pt *out)
{
    if (!c || !coeff_host || !out || !out->d) return fhe_fail(FHE_EINVAL, "fhe_encode_coeffs: null argument");
    const uint32_t l = out->limbs, N = c->N;
    if (l < 1 || l > c->L) return fhe_fail(FHE_ELEVEL, "fhe_encode_coeffs: level out of range");
    int8_t *s8; int64_t *i64; uint64_t *lb;
    fhe_status s = client_scratch(c, 0, &s8, &i64, &lb);
    if (s) return s;
    HIPCHK(hipMemcpyAsync(i64, coeff_host, (size_t)N * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    ModList ml = modlist_range(0, l);
    hipLaunchKernelGGL(k_small_to_rns, dim3(blocks_for(N, TPB), l), dim3(TPB), 0, c->stream, (const int64_t *)i64,
                       out->d, ml, (const ModQ *)c->d_mod, c->logN);
    ntt_list(c, out->d, ml, false);
    HIPCHK(hipGetLastError());
    return FHE_OK;
}

fhe_status fhe_encode(fhe_ctx *c, const double *re, const double *im, uint32_t n, double scale, fhe_pt *out)
{
    if (!c || !re || !out || !out->d) return fhe_fail(FHE_EINVAL, "fhe_encode: null argument");
    const uint32_t l = out->limbs, N = c->N;
    if (n > N / 2) return fhe_fail(FHE_EINVAL, "fhe_encode: more values than slots");
    if (l < 1 || l > c->L) return fhe_fail(FHE_ELEVEL, "fhe_encode: level out of range");
    if (!(scale > 0.0)) return fhe_fail(FHE_EINVAL, "fhe_encode: scale must be positive");
    uint8_t *scr;
    const size_t nn = n ? n : 1;
    fhe_status s = ctx_scratch(c, (size_t)N * 8 + 2 * nn * 8 + 256, &scr);
    if (s) return s;
    int64_t *coeff = (int64_t *)scr;
    double *dre = (double *)(coeff + N), *dim = dre + nn;
    int *flag = (int *)(dim + nn);
    HIPCHK(hipMemcpyAsync(dre, re, (size_t)n * 8, hipMemcpyHostToDevice, c->stream));
    if (im) HIPCHK(hipMemcpyAsync(dim, im, (size_t)n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), c->stream));
    hipLaunchKernelGGL(k_encode, dim3(blocks_for(N, TPB)), dim3(TPB), 0, c->stream, (const double *)dre,
                       im ? (const double *)dim : nullptr, n, (const double *)c->d_cos, (const double *)c->d_sin,
                       (const uint32_t *)c->d_g5, scale, c->logN, coeff, flag);
    int hflag = 0;
    HIPCHK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (hflag) return fhe_fail(FHE_EINVAL, "fhe_encode: a coefficient exceeds 2^62");
    ModList ml = modlist_range(0, l);
    hipLaunchKernelGGL(k_small_to_rns, dim3(blocks_for(N, TPB), l), dim3(TPB), 0, c->stream, (const int64_t *)coeff,
                       out->d, ml, (const ModQ *)c->d_mod, c->logN);
    ntt_list(c, out->d, ml, false);
    out->scale = scale;
    HIPCHK(hipGetLastError());
    return FHE_OK;
}

static fhe_status decode_common(fhe_ctx *c, const fhe_pt *pt, const uint32_t *slots, double *re, double *im,
                                uint32_t n)
{
    const uint32_t N = c->N;
    if (pt->limbs < 1 || pt->limbs > c->L) return fhe_fail(FHE_ELEVEL, "fhe_decode: level out of range");
    const uint32_t lu = pt->limbs >= 2 ? 2 : 1;
    const size_t nn = n ? n : 1;
    uint8_t *scr;
    fhe_status s = ctx_scratch(c, (size_t)lu * N * 8 + (size_t)N * 8 + 2 * nn * 8 + nn * 4 + 256, &scr);
    if (s) return s;
    uint64_t *limbs = (uint64_t *)scr;
    double *mv = (double *)(limbs + (size_t)lu * N), *dre = mv + N, *dim = dre + nn;
    uint32_t *didx = nullptr;
    if (slots) {   // the slot list travels as a pointer table, narrowed to 32-bit words
        std::vector<uint64_t *> tab(n);
        for (uint32_t t = 0; t < n; ++t) tab[t] = (uint64_t *)(uintptr_t)slots[t];
        uint64_t **dt;
        if ((s = ctx_ptr_table(c, tab, &dt))) return s;
        didx = (uint32_t *)(dim + nn);
        hipLaunchKernelGGL(k_narrow_u32, dim3(blocks_for(n, TPB)), dim3(TPB), 0, c->stream, (const uint64_t *)dt, n,
                           didx);
    }
    HIPCHK(hipMemcpyAsync(limbs, pt->d, (size_t)lu * N * 8, hipMemcpyDeviceToDevice, c->stream));
    ModList ml = modlist_range(0, lu);
    ntt_list(c, limbs, ml, true);
    const uint64_t q0 = c->mod[0], q1 = lu == 2 ? c->mod[1] : 1;
    uint64_t q0inv = 0;
    if (lu == 2) {   // q0^-1 mod q1 (q1 prime)
        unsigned __int128 r = 1, b = q0 % q1;
        for (uint64_t e = q1 - 2; e; e >>= 1, b = b * b % q1)
            if (e & 1) r = r * b % q1;
        q0inv = (uint64_t)r;
    }
    hipLaunchKernelGGL(k_lift, dim3(blocks_for(N, TPB)), dim3(TPB), 0, c->stream, (const uint64_t *)limbs, lu, q0, q1,
                       q0inv, mv, c->logN);
    if (n) {
        hipLaunchKernelGGL(k_decode, dim3(n), dim3(TPB), 0, c->stream, (const double *)mv, (const double *)c->d_cos,
                           (const double *)c->d_sin, (const uint32_t *)c->d_g5, (const uint32_t *)didx, pt->scale,
                           c->logN, dre, dim);
        HIPCHK(hipMemcpyAsync(re, dre, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
        if (im) HIPCHK(hipMemcpyAsync(im, dim, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    return FHE_OK;
}

fhe_status fhe_decode(fhe_ctx *c, const fhe_pt *pt, double *re, double *im, uint32_t n)
{
    if (!c || !pt || !pt->d || !re) return fhe_fail(FHE_EINVAL, "fhe_decode: null argument");
    if (n > c->N / 2) return fhe_fail(FHE_EINVAL, "fhe_decode: more values than slots");
    return decode_common(c, pt, nullptr, re, im, n);
}

fhe_status fhe_decode_slots(fhe_ctx *c, const fhe_pt *pt, const uint32_t *slots, uint32_t n, double *re, double *im)
{
    if (!c || !pt || !pt->d || !re || (n && !slots)) return fhe_fail(FHE_EINVAL, "fhe_decode_slots: null argument");
    for (uint32_t t = 0; t < n; ++t)
        if (slots[t] >= c->N / 2) return fhe_fail(FHE_EINVAL, "fhe_decode_slots: slot index out of range");
    return decode_common(c, pt, slots, re, im, n);
}

}  // extern "C"
