// batch.hip -- work lists of ciphertext operations at mixed levels, run as a
// few ragged launch sequences.
//
// The paper parallelises its CPU evaluation by splitting independent work
// (channels, output positions) over threads (Sec. 4.2); on the GPU the same
// independence is taken further: every operation of one kind whose inputs are
// ready runs in one launch sequence, whatever its level, through kernels that
// walk flat (item, limb) lists.  A work list is split into stages by data
// dependence (an operation reading another's output runs in a later stage);
// within a stage, operations are grouped by kind.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>

#include "fhe_internal.h"

namespace {

constexpr int TPB = 256;
inline uint32_t blocks_for(uint64_t n, uint32_t per) { return (uint32_t)((n + per - 1) / per); }

// out_b = a_b (x) b_b at l_b limbs.  Table: [a: n][b: n][out: n][lvl: n][list: sum l_b]
// with list entries b << 16 | limb.
__global__ __launch_bounds__(TPB) void k_tensor_batch(uint64_t *const *__restrict__ tab, uint32_t n, uint32_t lst,
                                                      const ModQ *__restrict__ mods, uint32_t logN, uint32_t y0)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    const uint64_t e = (uint64_t)(uintptr_t)tab[lst + blockIdx.y + y0];
    const uint32_t b = (uint32_t)(e >> 16), limb = (uint32_t)(e & 0xFFFF);
    const uint32_t l = (uint32_t)(uintptr_t)tab[3 * n + b];
    const size_t off1 = (size_t)l * N, x = (size_t)limb * N + k;
    const gu64 *A = gview(tab[b]), *B = gview(tab[n + b]);
    gu64 *out = gview(tab[2 * n + b]);
    const double q = mods[limb].q, qi = mods[limb].qinv;
    const double a0 = u64_to_f64(A[x]), a1 = u64_to_f64(A[x + off1]);
    const double b0 = u64_to_f64(B[x]), b1 = u64_to_f64(B[x + off1]);
    out[x] = f64_to_u64(canon(mulmod(a0, b0, q, qi), q, qi));
    out[x + off1] = f64_to_u64(canon(mulmod(a0, b1, q, qi) + mulmod(a1, b0, q, qi), q, qi));
    out[x + 2 * off1] = f64_to_u64(canon(mulmod(a1, b1, q, qi), q, qi));
}

}  // namespace

fhe_status tensor_run(fhe_ctx *c, uint32_t n, const uint32_t *ls, const uint64_t *const *a, const uint64_t *const *b,
                      uint64_t *const *out)
{
    std::vector<uint64_t *> tab;
    for (uint32_t t = 0; t < n; ++t) tab.push_back((uint64_t *)a[t]);
    for (uint32_t t = 0; t < n; ++t) tab.push_back((uint64_t *)b[t]);
    for (uint32_t t = 0; t < n; ++t) tab.push_back(out[t]);
    for (uint32_t t = 0; t < n; ++t) tab.push_back((uint64_t *)(uintptr_t)ls[t]);
    const uint32_t lst = (uint32_t)tab.size();
    for (uint32_t t = 0; t < n; ++t)
        for (uint32_t i = 0; i < ls[t]; ++i) tab.push_back((uint64_t *)(uintptr_t)(((uint64_t)t << 16) | i));
    const uint32_t cnt = (uint32_t)tab.size() - lst;
    uint64_t **dt;
    fhe_status s;
    if ((s = ctx_ptr_table(c, tab, &dt))) return s;
    ProfScope ps(c, "tensor");
    for (uint32_t y0 = 0; y0 < cnt; y0 += 65535u)
        hipLaunchKernelGGL(k_tensor_batch, dim3(blocks_for(c->N, TPB), std::min(65535u, cnt - y0)), dim3(TPB), 0,
                           c->stream, (uint64_t *const *)dt, n, lst, (const ModQ *)c->d_mod, c->logN, y0);
    HIPCHK(hipGetLastError());
    return FHE_OK;
}

namespace {

bool overlaps(const fhe_ct *x, const fhe_ct *y, size_t N)
{
    const uint64_t *xb = x->d, *xe = xb + (size_t)x->polys * x->limbs * N;
    const uint64_t *yb = y->d, *ye = yb + (size_t)y->polys * y->limbs * N;
    return xb < ye && yb < xe;
}

// a (x) b -> relin -> rescale for a group of operations (ragged), in chunks
// whose scratch stays near 4 GiB.
fhe_status run_mrr(fhe_ctx *c, const std::vector<const fhe_op *> &g)
{
    const size_t N = c->N, LB = N * sizeof(uint64_t), cap = (size_t)4 << 30;
    fhe_status s;
    for (size_t t0 = 0; t0 < g.size();) {
        size_t cn = 0, bytes = 0;
        const size_t lim = c->tune_chunk ? c->tune_chunk : 16384;
        while (t0 + cn < g.size() && cn < lim) {
            const uint32_t l = g[t0 + cn]->a->limbs;
            const size_t item = ks_scratch_bytes(c, l, 1) + 5 * (size_t)l * LB + rescale_scratch_bytes(c, l, 2, 1);
            if (cn && bytes + item > cap) break;
            bytes += item;
            ++cn;
        }
        std::vector<uint32_t> ls(cn);
        for (size_t t = 0; t < cn; ++t) ls[t] = g[t0 + t]->a->limbs;
        const size_t ksb = ks_scratch_bytes_ragged(c, (uint32_t)cn, ls.data());
        uint8_t *scr;
        if ((s = ctx_scratch(c, bytes, &scr))) return s;
        uint64_t *acc3 = (uint64_t *)(scr + ksb);
        size_t sum_l = 0;
        for (uint32_t l : ls) sum_l += l;
        uint64_t *tmp2 = acc3 + 3 * sum_l * N;
        uint8_t *rs = (uint8_t *)(tmp2 + 2 * sum_l * N);
        std::vector<const uint64_t *> A(cn), B(cn), kd(cn), ke(cn), ka(2 * cn), ri(cn);
        std::vector<uint64_t *> T3(cn), ko(cn), ro(cn);
        size_t off = 0;
        for (size_t t = 0; t < cn; ++t) {
            const fhe_op *op = g[t0 + t];
            const size_t l = ls[t];
            A[t] = op->a->d;
            B[t] = op->b->d;
            T3[t] = acc3 + 3 * off * N;
            kd[t] = T3[t] + 2 * l * N;
            ka[2 * t] = T3[t];
            ka[2 * t + 1] = T3[t] + l * N;
            ke[t] = op->key->d;
            ko[t] = tmp2 + 2 * off * N;
            ri[t] = ko[t];
            ro[t] = op->out->d;
            off += l;
        }
        if ((s = tensor_run(c, (uint32_t)cn, ls.data(), A.data(), B.data(), T3.data()))) return s;
        if ((s = ks_run_ragged(c, (uint32_t)cn, ls.data(), kd.data(), nullptr, ke.data(), ko.data(), ka.data(), scr)))
            return s;
        if ((s = rescale_run_ragged(c, 2, (uint32_t)cn, ls.data(), ri.data(), ro.data(), rs))) return s;
        t0 += cn;
    }
    return FHE_OK;
}

}  // namespace

extern "C" {

fhe_status fhe_batch_run(fhe_ctx *c, const fhe_op *ops, uint32_t n_ops)
{
    fhe_status s;
    if (!c || (!ops && n_ops)) return fhe_fail(FHE_EINVAL, "fhe_batch_run: null argument");
    const size_t N = c->N;
    // validate, and stage by dependence: an input written by an earlier operation
    std::vector<uint32_t> stage(n_ops, 0);
    for (uint32_t i = 0; i < n_ops; ++i) {
        const fhe_op &op = ops[i];
        if (!op.a || !op.a->d || !op.out || !op.out->d) return fhe_fail(FHE_EINVAL, "fhe_batch_run: null operand");
        const uint32_t l = op.a->limbs;
        if (l < 1 || l > c->L || op.a->polys != 2) return fhe_fail(FHE_EINVAL, "fhe_batch_run: bad input");
        switch (op.kind) {
        case FHE_OP_MUL_RELIN_RESCALE:
            if (!op.b || !op.b->d || op.b->limbs != l || op.b->polys != 2)
                return fhe_fail(FHE_EINVAL, "fhe_batch_run: multiplication operands differ in shape");
            if (!op.key || !op.key->d || op.key->galois != 0)
                return fhe_fail(FHE_ENOKEY, "fhe_batch_run: multiplication needs the relinearisation key");
            if (l < 2) return fhe_fail(FHE_ELEVEL, "fhe_batch_run: multiplication needs two limbs");
            if (op.out->limbs != l - 1 || op.out->polys != 2)
                return fhe_fail(FHE_EINVAL, "fhe_batch_run: product output must be 2 x (l - 1)");
            break;
        case FHE_OP_ROTATE:
            if (!op.key || !op.key->d || op.key->galois != fhe_galois_elt(c, op.step))
                return fhe_fail(FHE_ENOKEY, "fhe_batch_run: Galois key is for another step");
            if (op.out->limbs != l || op.out->polys != 2)
                return fhe_fail(FHE_EINVAL, "fhe_batch_run: rotation output must be 2 x l");
            break;
        default: return fhe_fail(FHE_EINVAL, "fhe_batch_run: unknown operation kind");
        }
        for (uint32_t j = 0; j < n_ops; ++j) {
            const fhe_op &o2 = ops[j];
            if (j != i && overlaps(op.out, o2.out, N))
                return fhe_fail(FHE_EINVAL, "fhe_batch_run: two outputs overlap");
            const bool reads = overlaps(op.out, o2.a, N) || (o2.kind == FHE_OP_MUL_RELIN_RESCALE && overlaps(op.out, o2.b, N));
            if (!reads) continue;
            if (j <= i) return fhe_fail(FHE_EINVAL, "fhe_batch_run: an output overlaps an input of itself or an earlier operation");
        }
        for (uint32_t j = 0; j < i; ++j) {
            const bool dep = overlaps(ops[j].out, op.a, N) ||
                             (op.kind == FHE_OP_MUL_RELIN_RESCALE && overlaps(ops[j].out, op.b, N));
            if (dep) stage[i] = std::max(stage[i], stage[j] + 1);
        }
    }
    const uint32_t nst = n_ops ? *std::max_element(stage.begin(), stage.end()) + 1 : 0;
    for (uint32_t st = 0; st < nst; ++st) {
        std::vector<const fhe_op *> mrr, rot;
        for (uint32_t i = 0; i < n_ops; ++i)
            if (stage[i] == st) (ops[i].kind == FHE_OP_MUL_RELIN_RESCALE ? mrr : rot).push_back(&ops[i]);
        if (!mrr.empty()) {
            if ((s = run_mrr(c, mrr))) return s;
            c->ops[OP_CT_MULT] += mrr.size();
            c->ops[OP_RELIN] += mrr.size();
            c->ops[OP_RESCALE] += mrr.size();
        }
        if (!rot.empty()) {
            std::vector<uint32_t> ls(rot.size());
            std::vector<const uint64_t *> in(rot.size());
            std::vector<const fhe_evk *> keys(rot.size());
            std::vector<uint64_t *> out(rot.size());
            for (size_t t = 0; t < rot.size(); ++t) {
                ls[t] = rot[t]->a->limbs;
                in[t] = rot[t]->a->d;
                keys[t] = rot[t]->key;
                out[t] = rot[t]->out->d;
            }
            if ((s = rotate_run_ragged(c, (uint32_t)rot.size(), ls.data(), in.data(), keys.data(), out.data())))
                return s;
        }
    }
    // scales (host bookkeeping in list order): an input written by an earlier
    // operation takes that operation's output scale
    std::vector<double> outsc(n_ops);
    auto in_scale = [&](uint32_t i, const fhe_ct *x) {
        double sc = x->scale;
        for (uint32_t j = 0; j < i; ++j)
            if (overlaps(ops[j].out, x, N)) sc = outsc[j];
        return sc;
    };
    for (uint32_t i = 0; i < n_ops; ++i) {
        const fhe_op &op = ops[i];
        double sc = in_scale(i, op.a);
        if (op.kind == FHE_OP_MUL_RELIN_RESCALE) sc = sc * in_scale(i, op.b) / (double)c->mod[op.a->limbs - 1];
        outsc[i] = sc;
    }
    for (uint32_t i = 0; i < n_ops; ++i) ops[i].out->scale = outsc[i];
    return FHE_OK;
}

}  // extern "C"
