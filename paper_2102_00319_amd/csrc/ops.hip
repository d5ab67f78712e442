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
        const gu64 *A = gview(ap[t]), *B = gview(bp[t]);
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
}  // namespace

// ============================================================ host helpers
static fhe_status chk_ct(const fhe_ctx *c, const fhe_ct *a, const char *what)
{
    if (!a || !a->d) return fhe_fail(FHE_EINVAL, std::string(what) + ": null ciphertext");
    if (a->limbs < 1 || a->limbs > c->L) return fhe_fail(FHE_ELEVEL, std::string(what) + ": limb count out of range");
    if (a->polys < 2 || a->polys > 3) return fhe_fail(FHE_EINVAL, std::string(what) + ": polys must be 2 or 3");
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
    return ks_run(c, limbs, 1, dd, nullptr, ek, oo, nullptr, nullptr);
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
    return ks_run(c, limbs, n, dd.data(), nullptr, ek.data(), oo.data(), nullptr, nullptr);
}
// The same key switches with the scratch in this GPU's static array: nothing is
// allocated (the pointer table goes through the ring made with the context).
fhe_status fhe_keyswitch_batch_static(fhe_ctx *c, const fhe_evk *evk, const uint64_t *const *d, uint32_t limbs,
                                      uint32_t n, fhe_ct *out)
{
    fhe_status s;
    if (!c || !evk || !d || !out || !n) return fhe_fail(FHE_EINVAL, "fhe_keyswitch_batch_static: null or empty");
    if (!c->static_scr) return fhe_fail(FHE_EDEVICE, "fhe_keyswitch_batch_static: static scratch not resolved");
    if (limbs < 1 || limbs > c->L) return fhe_fail(FHE_ELEVEL, "fhe_keyswitch_batch_static: limb count out of range");
    std::vector<const uint64_t *> dd(n), ek(n);
    std::vector<uint64_t *> oo(n);
    for (uint32_t b = 0; b < n; ++b) {
        if (!evk[b].d || !d[b]) return fhe_fail(FHE_EINVAL, "fhe_keyswitch_batch_static: null entry");
        if ((s = chk_ct(c, &out[b], "fhe_keyswitch_batch_static"))) return s;
        if (out[b].limbs != limbs || out[b].polys != 2)
            return fhe_fail(FHE_EINVAL, "fhe_keyswitch_batch_static: bad output");
        dd[b] = d[b]; ek[b] = evk[b].d; oo[b] = out[b].d;
    }
    const size_t need = ks_scratch_bytes(c, limbs, n);
    if (need > FHE_STATIC_SCRATCH_BYTES)
        return fhe_fail(FHE_ENOMEM, "fhe_keyswitch_batch_static: the batch needs " + std::to_string(need) +
                                        " bytes of scratch, the static array holds " +
                                        std::to_string(FHE_STATIC_SCRATCH_BYTES) + " (split the batch)");
    struct NoAlloc {
        fhe_ctx *c;
        explicit NoAlloc(fhe_ctx *cc) : c(cc) { c->no_alloc = true; }
        ~NoAlloc() { c->no_alloc = false; }
    } guard(c);
    return ks_run(c, limbs, n, dd.data(), nullptr, ek.data(), oo.data(), nullptr, c->static_scr);
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
    fhe_status r = ks_run(c, in3->limbs, 1, dd, nullptr, ek, oo, ad, nullptr);
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
    // the input copied to scratch first, so that out may alias in; then the key switch
    // of sigma_g(c1) (c1's digits extended, read through the permutation) adds
    // sigma_g(c0), read through the permutation as well
    const size_t ksb = ks_scratch_bytes(c, l, 1);
    uint8_t *scr;
    if ((s = ctx_scratch(c, ksb + 2 * per * sizeof(uint64_t), &scr))) return s;
    uint64_t *cp = (uint64_t *)(scr + ksb);
    HIPCHK(hipMemcpyAsync(cp, in->d, 2 * per * sizeof(uint64_t), hipMemcpyDeviceToDevice, c->stream));
    const uint64_t *dd[1] = {cp + per};
    const uint32_t ga[1] = {(uint32_t)g};
    const uint64_t *ek[1] = {gk->d};
    uint64_t *oo[1] = {out->d};
    const uint64_t *ad[2] = {cp, nullptr};   // (sigma_g(c0) + ks0, ks1)
    fhe_status r = ks_run(c, l, 1, dd, ga, ek, oo, ad, scr);
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
    for (uint32_t b = 0; b < n; ++b)
        for (uint32_t b2 = 0; b2 < n; ++b2)
            if (out[b].d < in[b2].d + 2 * per && in[b2].d < out[b].d + 2 * per)
                return fhe_fail(FHE_EINVAL, "fhe_rotate_batch: outputs must not overlap inputs");
    std::vector<const uint64_t *> ip(n);
    std::vector<const fhe_evk *> kp(n);
    std::vector<uint64_t *> op(n);
    for (uint32_t b = 0; b < n; ++b) {
        ip[b] = in[b].d;
        kp[b] = &gk[b];
        op[b] = out[b].d;
    }
    if ((s = rotate_run(c, l, n, ip.data(), kp.data(), op.data()))) return s;
    for (uint32_t b = 0; b < n; ++b) out[b].scale = in[b].scale;
    return FHE_OK;
}

// ct + value: the constant polynomial round(value * scale) (the same value at
// every evaluation point) added to c0.
fhe_status fhe_add_const(fhe_ctx *c, const fhe_ct *a, double value, fhe_ct *out)
{
    fhe_status s;
    if (!c) return fhe_fail(FHE_EINVAL, "null context");
    if ((s = chk_ct(c, a, "fhe_add_const")) || (s = chk_ct(c, out, "fhe_add_const"))) return s;
    if (out->limbs != a->limbs || out->polys != a->polys) return fhe_fail(FHE_EINVAL, "fhe_add_const: shapes differ");
    Consts64 cres;
    if ((s = const_residues(c, value * a->scale, a->limbs, &cres))) return s;
    const uint64_t *ap = a->d;
    uint64_t *optr = out->d;
    if ((s = ew_batch(c, EW_ADDC, a->limbs, a->limbs, a->polys, 1, &ap, nullptr, &optr, cres))) return s;
    out->scale = a->scale;
    c->ops[OP_PT_ADD] += 1;
    return FHE_OK;
}

}  // extern "C"

// Used by the client code (keygen): NTT-domain automorphism of nlimbs limbs.
void launch_automorph(fhe_ctx *c, const uint64_t *in, uint64_t *out, uint32_t nlimbs, uint64_t g)
{
    hipLaunchKernelGGL(k_automorph, dim3(blocks_for((uint64_t)nlimbs * c->N, TPB)), dim3(TPB), 0, c->stream, in, out,
                       c->logN, (uint64_t)nlimbs, (uint32_t)g);
}

// n rotations (a key switch of sigma_g(c1) with sigma_g(c0) as addend, both read
// through the permutation; rotations of one input share its digit extension), items
// at levels ls[b], in chunks whose scratch stays near 4 GiB.  Outputs must not
// overlap inputs.
fhe_status rotate_run_ragged(fhe_ctx *c, uint32_t n, const uint32_t *ls, const uint64_t *const *in,
                             const fhe_evk *const *keys, uint64_t *const *out)
{
    // The key switch extends the digits of c1 itself, reads them through the Galois
    // permutation in its inner product and adds sigma_g(c0) in its last pass: a
    // wavefront's 64 consecutive outputs gather from one aligned block of 64 inputs
    // (the permutation is affine in bit-reversed index order), so the gathers stay
    // coalesced and no permuted copy is made.
    const size_t N = c->N, cap = (size_t)4 << 30;
    fhe_status s;
    for (uint32_t b0 = 0; b0 < n;) {
        // grow the chunk while it fits
        uint32_t cn = 0;
        size_t bytes = 0;
        const uint32_t lim = c->tune_chunk ? c->tune_chunk : 16384;
        while (b0 + cn < n && cn < lim) {
            const size_t item = ks_scratch_bytes(c, ls[b0 + cn], 1);
            if (cn && bytes + item > cap) break;
            bytes += item;
            ++cn;
        }
        uint8_t *scr;
        if ((s = ctx_scratch(c, ks_scratch_bytes_ragged(c, cn, ls + b0), &scr))) return s;
        std::vector<const uint64_t *> dd(cn), ek(cn), ad(2 * (size_t)cn, nullptr);
        std::vector<uint64_t *> oo(cn);
        std::vector<uint32_t> gal(cn);
        for (uint32_t b = 0; b < cn; ++b) {
            const uint64_t *x = in[b0 + b];
            gal[b] = (uint32_t)keys[b0 + b]->galois;
            dd[b] = x + (size_t)ls[b0 + b] * N;   // c1
            ad[2 * b] = x;                         // c0
            ek[b] = keys[b0 + b]->d;
            oo[b] = out[b0 + b];
        }
        if ((s = ks_run_ragged(c, cn, ls + b0, dd.data(), gal.data(), ek.data(), oo.data(), ad.data(), scr))) return s;
        b0 += cn;
    }
    c->ops[OP_ROTATE] += n;
    return FHE_OK;
}
fhe_status rotate_run(fhe_ctx *c, uint32_t l, uint32_t n, const uint64_t *const *in, const fhe_evk *const *keys,
                      uint64_t *const *out)
{
    std::vector<uint32_t> ls(n, l);
    return rotate_run_ragged(c, n, ls.data(), in, keys, out);
}

// Residues of the integer round(v) (|round(v)| < 2^62) on limbs 0..limbs-1.
// Residues of the integer nearest to v (ties to even).  Beyond 2^62 the double is an
// integer m * 2^e with m < 2^53: its residues are (m mod q) (2^e mod q) mod q, exact.
fhe_status const_residues(const fhe_ctx *c, double v, uint32_t limbs, Consts64 *out)
{
    const double r = std::nearbyint(v);
    if (!std::isfinite(r)) return fhe_fail(FHE_EINVAL, "constant out of range");
    std::memset(out, 0, sizeof(*out));
    if (std::fabs(r) < 4611686018427387904.0) {
        const int64_t iv = (int64_t)r;
        for (uint32_t i = 0; i < limbs; ++i) {
            int64_t m = iv % (int64_t)c->mod[i];
            out->v[i] = (double)(m < 0 ? m + (int64_t)c->mod[i] : m);
        }
        return FHE_OK;
    }
    int ex;
    const double f = std::frexp(std::fabs(r), &ex);                 // |r| = f 2^ex, f in [0.5, 1)
    const uint64_t m = (uint64_t)std::ldexp(f, 53);                  // exact: 53 significant bits
    const int e = ex - 53;                                           // > 0 here
    for (uint32_t i = 0; i < limbs; ++i) {
        const uint64_t q = c->mod[i];
        unsigned __int128 p2 = 1, b = 2 % q;
        for (int k = e; k; k >>= 1) {
            if (k & 1) p2 = p2 * b % q;
            b = b * b % q;
        }
        uint64_t res = (uint64_t)((unsigned __int128)(m % q) * p2 % q);
        if (r < 0 && res) res = q - res;
        out->v[i] = (double)res;
    }
    return FHE_OK;
}

namespace {
// Batched elementwise operations.  Item t (blockIdx.y) reads a[t] (layout
// [polys][la][N], of which limbs 0..l-1 are used: la > l drops levels) and, for
// EW_ADD, b[t] ([polys][l][N]); for EW_MULPT, b[t] is a plaintext [l][N].
// Writes out[t] ([polys][l][N]).  EW_MULC multiplies by the per-limb constant,
// EW_ADDC adds it to poly 0, EW_COPY copies.  Pointer table: [a: n][b: n][out: n].
template <int OP>
__global__ __launch_bounds__(TPB) void k_ew_batch(uint64_t *const *__restrict__ tab, uint32_t n, uint32_t logN,
                                                  uint32_t l, uint32_t la, uint32_t polys, Consts64 cst,
                                                  const ModQ *__restrict__ mods)
{
    const uint64_t per = (uint64_t)l << logN;
    const uint64_t e = (uint64_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= per * polys) return;
    const uint32_t t = blockIdx.y;
    const uint32_t p = (uint32_t)(e / per);
    const uint64_t r = e - (uint64_t)p * per;
    const uint32_t limb = (uint32_t)(r >> logN);
    const uint64_t a = gview(tab[t])[(uint64_t)p * ((uint64_t)la << logN) + r];
    const uint64_t qq = (uint64_t)mods[limb].q;
    uint64_t o;
    if (OP == EW_ADD) {
        o = a + gview(tab[n + t])[e];
        o = o >= qq ? o - qq : o;
    } else if (OP == EW_COPY) {
        o = a;
    } else if (OP == EW_ADDC) {
        o = a;
        if (p == 0) {
            o = a + (uint64_t)cst.v[limb];
            o = o >= qq ? o - qq : o;
        }
    } else {
        const double q = mods[limb].q, qi = mods[limb].qinv;
        const double m = OP == EW_MULC ? cst.v[limb] : u64_to_f64(gview(tab[n + t])[r]);
        o = f64_to_u64(canon(mulmod(u64_to_f64(a), m, q, qi), q, qi));
    }
    gview(tab[2 * n + t])[e] = o;
}
}  // namespace

fhe_status ew_batch(fhe_ctx *c, int op, uint32_t l, uint32_t la, uint32_t polys, uint32_t n,
                    const uint64_t *const *a, const uint64_t *const *b, uint64_t *const *out, const Consts64 &cst)
{
    if (!n) return FHE_OK;
    for (uint32_t t0 = 0; t0 < n; t0 += 65535) {
        const uint32_t cn = std::min<uint32_t>(65535, n - t0);
        std::vector<uint64_t *> tab(3 * (size_t)cn);
        for (uint32_t t = 0; t < cn; ++t) {
            tab[t] = (uint64_t *)a[t0 + t];
            tab[cn + t] = b ? (uint64_t *)b[t0 + t] : nullptr;
            tab[2 * cn + t] = out[t0 + t];
        }
        uint64_t **dt;
        fhe_status s;
        if ((s = ctx_ptr_table(c, tab, &dt))) return s;
        const dim3 grid(blocks_for((uint64_t)polys * l * c->N, TPB), cn);
        ProfScope ps(c, "elementwise");
        switch (op) {
        case EW_ADD:
            hipLaunchKernelGGL(k_ew_batch<EW_ADD>, grid, dim3(TPB), 0, c->stream, (uint64_t *const *)dt, cn, c->logN,
                               l, la, polys, cst, (const ModQ *)c->d_mod);
            break;
        case EW_MULC:
            hipLaunchKernelGGL(k_ew_batch<EW_MULC>, grid, dim3(TPB), 0, c->stream, (uint64_t *const *)dt, cn,
                               c->logN, l, la, polys, cst, (const ModQ *)c->d_mod);
            break;
        case EW_ADDC:
            hipLaunchKernelGGL(k_ew_batch<EW_ADDC>, grid, dim3(TPB), 0, c->stream, (uint64_t *const *)dt, cn,
                               c->logN, l, la, polys, cst, (const ModQ *)c->d_mod);
            break;
        case EW_MULPT:
            hipLaunchKernelGGL(k_ew_batch<EW_MULPT>, grid, dim3(TPB), 0, c->stream, (uint64_t *const *)dt, cn,
                               c->logN, l, la, polys, cst, (const ModQ *)c->d_mod);
            break;
        case EW_COPY:
            hipLaunchKernelGGL(k_ew_batch<EW_COPY>, grid, dim3(TPB), 0, c->stream, (uint64_t *const *)dt, cn,
                               c->logN, l, la, polys, cst, (const ModQ *)c->d_mod);
            break;
        default: return fhe_fail(FHE_EINVAL, "ew_batch: unknown operation");
        }
        HIPCHK(hipGetLastError());
    }
    return FHE_OK;
}
