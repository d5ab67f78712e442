// ntt.hip -- negacyclic NTT / inverse NTT over batches of RNS limbs (gfx950).
//
// Forward transform: Cooley-Tukey butterflies with the table psi^brv(i), natural
// order in, bit-reversed order out, so that A[x] = a(psi^(2 brv(x) + 1)).
// Inverse: Gentleman-Sande butterflies with psi^-brv(i), the factor N^-1
// folded into the last stage.  (Standard negacyclic NTT; the paper's ring is
// Z[X]/(Phi_m(X)) with m = 2^16, Sec. 4.2.)
//
// N <= 2^14 is one pass (a whole limb per workgroup, up to 139 KB of LDS);
// N = 2^15, 2^16 are a column pass over the first stages (strided, coalesced
// across columns) and a row pass over contiguous blocks.  Between the two
// passes values stay in lazily reduced FP64 form (|x| < 2q); the last pass
// writes canonical residues.  The round structure is in ntt_core.h.
#include "ntt_core.h"

using namespace nttc;

namespace {

template <int LOGG, int WG, bool COL, bool IN_U64, bool OUT_U64>
__global__ __launch_bounds__(WG) void k_ntt_fwd(LimbSet ls, const ModQ *__restrict__ mods,
                                                const double *__restrict__ twt, uint32_t logN, uint32_t sigma0)
{
    using Gm = Geom<LOGG, WG, COL>;
    __shared__ double lds[Gm::LDS];
    const uint32_t N = 1u << logN;
    const uint32_t b = blockIdx.y + ls.b0;
    gu64 *p = gview(limb_ptr(ls, b, N));
    const uint32_t m = limb_mod(ls, b);
    const double q = mods[m].q, qinv = mods[m].qinv;
    const Gm gm(logN, blockIdx.x);
    double x[R];
#pragma unroll
    for (int k = 0; k < R; k++) {
        const uint64_t v = p[gm.fwd_in(k)];
        x[k] = IN_U64 ? u64_to_f64(v) : bits_to_f64(v);
    }
    gm.fwd(x, lds, twt + (size_t)m * N, q, qinv, logN, sigma0);
    if (!COL) {
        gm.fwd_out_to_coal(x, lds);
#pragma unroll
        for (int k = 0; k < R; k++) p[gm.coal(k)] = OUT_U64 ? f64_to_u64(canon(x[k], q, qinv)) : f64_to_bits(x[k]);
    } else {
#pragma unroll
        for (int k = 0; k < R; k++) p[gm.fwd_out(k)] = OUT_U64 ? f64_to_u64(canon(x[k], q, qinv)) : f64_to_bits(x[k]);
    }
}

template <int LOGG, int WG, bool COL, bool IN_U64, bool OUT_U64, bool LASTSTAGE>
__global__ __launch_bounds__(WG) void k_ntt_inv(LimbSet ls, const ModQ *__restrict__ mods,
                                                const double *__restrict__ itwt, const double *__restrict__ ninvt,
                                                uint32_t logN, uint32_t sigma0)
{
    using Gm = Geom<LOGG, WG, COL>;
    __shared__ double lds[Gm::LDS];
    const uint32_t N = 1u << logN;
    const uint32_t b = blockIdx.y + ls.b0;
    gu64 *p = gview(limb_ptr(ls, b, N));
    const uint32_t m = limb_mod(ls, b);
    const double q = mods[m].q, qinv = mods[m].qinv;
    const Gm gm(logN, blockIdx.x);
    double x[R];
    if (!COL) {
#pragma unroll
        for (int k = 0; k < R; k++) {
            const uint64_t v = p[gm.coal(k)];
            x[k] = IN_U64 ? u64_to_f64(v) : bits_to_f64(v);
        }
        gm.coal_to_inv_in(x, lds);
    } else {
#pragma unroll
        for (int k = 0; k < R; k++) {
            const uint64_t v = p[gm.inv_in(k)];
            x[k] = IN_U64 ? u64_to_f64(v) : bits_to_f64(v);
        }
    }
    gm.template inv<LASTSTAGE>(x, lds, itwt + (size_t)m * N, q, qinv, ninvt[m], logN, sigma0);
#pragma unroll
    for (int k = 0; k < R; k++) p[gm.inv_out(k)] = OUT_U64 ? f64_to_u64(canon(x[k], q, qinv)) : f64_to_bits(x[k]);
}

template <typename F>
void chunked(uint32_t nlimbs, const LimbSet &ls, F launch)
{
    for (uint32_t done = 0; done < nlimbs; done += 65535u) {
        LimbSet l2 = ls;
        l2.b0 = ls.b0 + done;
        launch(l2, nlimbs - done < 65535u ? nlimbs - done : 65535u);
    }
}

}  // namespace

void launch_ntt_fwd(fhe_ctx *c, const LimbSet &ls, uint32_t nlimbs)
{
    if (!nlimbs) return;
    const uint32_t logN = c->logN;
    hipStream_t st = c->stream;
    auto go = [&](auto kern, uint32_t gx, int wg, uint32_t sig0, const char *cat) {
        ProfScope ps(c, cat);
        chunked(nlimbs, ls, [&](const LimbSet &l2, uint32_t cnt) {
            hipLaunchKernelGGL(kern, dim3(gx, cnt), dim3(wg), 0, st, l2, (const ModQ *)c->d_mod,
                               (const double *)c->d_tw, logN, sig0);
        });
    };
    switch (logN) {
    case 10: go(k_ntt_fwd<10, 64, false, true, true>, 1, 64, 0, "ntt_fwd"); break;
    case 11: go(k_ntt_fwd<11, 128, false, true, true>, 1, 128, 0, "ntt_fwd"); break;
    case 12: go(k_ntt_fwd<12, 256, false, true, true>, 1, 256, 0, "ntt_fwd"); break;
    case 13: go(k_ntt_fwd<13, 512, false, true, true>, 1, 512, 0, "ntt_fwd"); break;
    case 14: go(k_ntt_fwd<14, 1024, false, true, true>, 1, 1024, 0, "ntt_fwd"); break;
    case 15:
        go(k_ntt_fwd<7, 256, true, true, false>, (1u << 8) / 32, 256, 0, "ntt_fwd_col");
        go(k_ntt_fwd<8, 256, false, false, true>, (1u << 7) / 16, 256, 7, "ntt_fwd_row");
        break;
    case 16:
        go(k_ntt_fwd<8, 256, true, true, false>, (1u << 8) / 16, 256, 0, "ntt_fwd_col");
        go(k_ntt_fwd<8, 256, false, false, true>, (1u << 8) / 16, 256, 8, "ntt_fwd_row");
        break;
    default: break;
    }
}

void launch_ntt_inv(fhe_ctx *c, const LimbSet &ls, uint32_t nlimbs)
{
    if (!nlimbs) return;
    const uint32_t logN = c->logN;
    hipStream_t st = c->stream;
    auto go = [&](auto kern, uint32_t gx, int wg, uint32_t sig0, const char *cat) {
        ProfScope ps(c, cat);
        chunked(nlimbs, ls, [&](const LimbSet &l2, uint32_t cnt) {
            hipLaunchKernelGGL(kern, dim3(gx, cnt), dim3(wg), 0, st, l2, (const ModQ *)c->d_mod,
                               (const double *)c->d_itw, (const double *)c->d_ninv, logN, sig0);
        });
    };
    switch (logN) {
    case 10: go(k_ntt_inv<10, 64, false, true, true, true>, 1, 64, 0, "ntt_inv"); break;
    case 11: go(k_ntt_inv<11, 128, false, true, true, true>, 1, 128, 0, "ntt_inv"); break;
    case 12: go(k_ntt_inv<12, 256, false, true, true, true>, 1, 256, 0, "ntt_inv"); break;
    case 13: go(k_ntt_inv<13, 512, false, true, true, true>, 1, 512, 0, "ntt_inv"); break;
    case 14: go(k_ntt_inv<14, 1024, false, true, true, true>, 1, 1024, 0, "ntt_inv"); break;
    case 15:
        go(k_ntt_inv<8, 256, false, true, false, false>, (1u << 7) / 16, 256, 7, "ntt_inv_row");
        go(k_ntt_inv<7, 256, true, false, true, true>, (1u << 8) / 32, 256, 0, "ntt_inv_col");
        break;
    case 16:
        go(k_ntt_inv<8, 256, false, true, false, false>, (1u << 8) / 16, 256, 8, "ntt_inv_row");
        go(k_ntt_inv<8, 256, true, false, true, true>, (1u << 8) / 16, 256, 0, "ntt_inv_col");
        break;
    default: break;
    }
}
