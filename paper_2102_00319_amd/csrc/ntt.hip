// ntt.hip -- negacyclic NTT / inverse NTT over batches of RNS limbs (gfx950).
//
// Forward transform: Cooley-Tukey butterflies with the table psi^brv(i), natural
// order in, bit-reversed order out, so that A[x] = a(psi^(2 brv(x) + 1)).
// Inverse: Gentleman-Sande butterflies with psi^-brv(i), the factor N^-1
// folded into the last stage.  (Standard negacyclic NTT; the paper's ring is
// Z[X]/(Phi_m(X)) with m = 2^16, Sec. 4.2.)
//
// Data path: one limb is split into groups of G = 2^LOGG elements that are
// independent for LOGG consecutive stages.  Each thread holds R = 16 of a
// group's elements in registers and runs 4 stages on them (radix 16); groups
// exchange through padded LDS between rounds.  N <= 2^14 is one pass (a whole
// limb per workgroup, up to 139 KB of LDS); N = 2^15, 2^16 are a column pass
// (the first log2(N1) stages over strided columns, coalesced across columns)
// and a row pass over contiguous blocks.  Between the two passes values stay
// in lazily reduced FP64 form (|x| < 2q); the last pass writes canonical
// residues.
#include "fhe_internal.h"

namespace {

constexpr int LOGR = 4;
constexpr int R = 1 << LOGR;

// Local index of register k of lane tau in a round that covers bits [blo, blo+rho).
template <int LOGT>
__device__ __forceinline__ int elem_local(int tau, int k, int blo, int rho)
{
    int fr = ((k >> rho) << LOGT) | tau;
    return ((fr >> blo) << (blo + rho)) | ((k & ((1 << rho) - 1)) << blo) | (fr & ((1 << blo) - 1));
}
__device__ __forceinline__ int lds_pad(int g) { return g + (g >> LOGR); }

template <int LOGG, int WG, bool COL, bool IN_U64, bool OUT_U64>
__global__ __launch_bounds__(WG) void k_ntt_fwd(LimbSet ls, const ModQ *__restrict__ mods,
                                                const double *__restrict__ twt, uint32_t logN, uint32_t sigma0)
{
    constexpr int G = 1 << LOGG, LOGT = LOGG - LOGR, T = 1 << LOGT, GPW = WG / T;
    constexpr int GS = G + G / R + 1;                 // padded group stride in LDS
    constexpr int NR = (LOGG + LOGR - 1) / LOGR;
    __shared__ double lds[NR > 1 ? GPW * GS : 1];
    const uint32_t N = 1u << logN;
    const uint32_t b = blockIdx.y + ls.b0;
    uint64_t *p = limb_ptr(ls, b, N);
    const uint32_t m = limb_mod(ls, b);
    const double q = mods[m].q, qinv = mods[m].qinv;
    const double *tw = twt + (size_t)m * N;
    const int tid = threadIdx.x;
    const int grp = COL ? (tid % GPW) : (tid / T);
    const int tau = COL ? (tid / GPW) : (tid % T);
    const uint32_t gi = blockIdx.x * GPW + grp;
    const uint32_t N2 = N >> LOGG;
    auto gidx = [&](int g) -> uint32_t { return COL ? gi + (uint32_t)g * N2 : (gi << LOGG) + (uint32_t)g; };

    double x[R];
#pragma unroll
    for (int k = 0; k < R; k++) {
        const int g = elem_local<LOGT>(tau, k, LOGG - LOGR, LOGR);
        const uint64_t v = p[gidx(g)];
        x[k] = IN_U64 ? u64_to_f64(v) : bits_to_f64(v);
    }
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const int bhi = LOGG - r * LOGR;
        const int rho = bhi < LOGR ? bhi : LOGR;
        const int blo = bhi - rho;
        if (r > 0) {
            const int pblo = bhi, prho = LOGR;
#pragma unroll
            for (int k = 0; k < R; k++) lds[grp * GS + lds_pad(elem_local<LOGT>(tau, k, pblo, prho))] = x[k];
            __syncthreads();
#pragma unroll
            for (int k = 0; k < R; k++) x[k] = lds[grp * GS + lds_pad(elem_local<LOGT>(tau, k, blo, rho))];
            __syncthreads();
        }
#pragma unroll
        for (int s = 0; s < rho; s++) {
            const int bit = rho - 1 - s;
            const int lb = blo + bit;
            const uint32_t sigma = sigma0 + (uint32_t)(LOGG - 1 - lb);
#pragma unroll
            for (int k = 0; k < R; k++) {
                if (k & (1 << bit)) continue;
                const int kt = k & ~((2 << bit) - 1);
                const uint32_t j = gidx(elem_local<LOGT>(tau, kt, blo, rho));
                const double W = tw[(1u << sigma) + (j >> (logN - sigma))];
                const double X = redc(x[k], q, qinv);
                const double V = mulmod(x[k | (1 << bit)], W, q, qinv);
                x[k] = X + V;
                x[k | (1 << bit)] = X - V;
            }
        }
    }
    {
        constexpr int rl = LOGG - (NR - 1) * LOGR;
#pragma unroll
        for (int k = 0; k < R; k++) {
            const uint32_t idx = gidx(elem_local<LOGT>(tau, k, 0, rl));
            p[idx] = OUT_U64 ? f64_to_u64(canon(x[k], q, qinv)) : f64_to_bits(x[k]);
        }
    }
}

template <int LOGG, int WG, bool COL, bool IN_U64, bool OUT_U64, bool LASTSTAGE>
__global__ __launch_bounds__(WG) void k_ntt_inv(LimbSet ls, const ModQ *__restrict__ mods,
                                                const double *__restrict__ itwt, const double *__restrict__ ninvt,
                                                uint32_t logN, uint32_t sigma0)
{
    constexpr int G = 1 << LOGG, LOGT = LOGG - LOGR, T = 1 << LOGT, GPW = WG / T;
    constexpr int GS = G + G / R + 1;
    constexpr int NR = (LOGG + LOGR - 1) / LOGR;
    __shared__ double lds[NR > 1 ? GPW * GS : 1];
    const uint32_t N = 1u << logN;
    const uint32_t b = blockIdx.y + ls.b0;
    uint64_t *p = limb_ptr(ls, b, N);
    const uint32_t m = limb_mod(ls, b);
    const double q = mods[m].q, qinv = mods[m].qinv;
    const double *tw = itwt + (size_t)m * N;
    const int tid = threadIdx.x;
    const int grp = COL ? (tid % GPW) : (tid / T);
    const int tau = COL ? (tid / GPW) : (tid % T);
    const uint32_t gi = blockIdx.x * GPW + grp;
    const uint32_t N2 = N >> LOGG;
    auto gidx = [&](int g) -> uint32_t { return COL ? gi + (uint32_t)g * N2 : (gi << LOGG) + (uint32_t)g; };

    double x[R];
    {
        constexpr int r0 = LOGG < LOGR ? LOGG : LOGR;
#pragma unroll
        for (int k = 0; k < R; k++) {
            const uint64_t v = p[gidx(elem_local<LOGT>(tau, k, 0, r0))];
            x[k] = IN_U64 ? u64_to_f64(v) : bits_to_f64(v);
        }
    }
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const int blo = r * LOGR;
        const int rho = (LOGG - blo) < LOGR ? (LOGG - blo) : LOGR;
        if (r > 0) {
            const int pblo = blo - LOGR, prho = LOGR;
#pragma unroll
            for (int k = 0; k < R; k++) lds[grp * GS + lds_pad(elem_local<LOGT>(tau, k, pblo, prho))] = x[k];
            __syncthreads();
#pragma unroll
            for (int k = 0; k < R; k++) x[k] = lds[grp * GS + lds_pad(elem_local<LOGT>(tau, k, blo, rho))];
            __syncthreads();
        }
#pragma unroll
        for (int s = 0; s < rho; s++) {
            const int bit = s;
            const int lb = blo + bit;
            const uint32_t sigma = sigma0 + (uint32_t)(LOGG - 1 - lb);
            const bool fold_ninv = LASTSTAGE && (lb == LOGG - 1);   // global stage 0
#pragma unroll
            for (int k = 0; k < R; k++) {
                if (k & (1 << bit)) continue;
                const int kt = k & ~((2 << bit) - 1);
                const uint32_t j = gidx(elem_local<LOGT>(tau, kt, blo, rho));
                double W = tw[(1u << sigma) + (j >> (logN - sigma))];
                const double U = x[k], V = x[k | (1 << bit)];
                if (fold_ninv) {
                    const double ni = ninvt[m];
                    W = canon(mulmod(W, ni, q, qinv), q, qinv);
                    x[k] = mulmod(U + V, ni, q, qinv);
                } else {
                    x[k] = redc(U + V, q, qinv);
                }
                x[k | (1 << bit)] = mulmod(U - V, W, q, qinv);
            }
        }
    }
    {
        constexpr int rl = LOGG - (NR - 1) * LOGR;
        constexpr int blo_last = (NR - 1) * LOGR;
#pragma unroll
        for (int k = 0; k < R; k++) {
            const uint32_t idx = gidx(elem_local<LOGT>(tau, k, blo_last, rl));
            p[idx] = OUT_U64 ? f64_to_u64(canon(x[k], q, qinv)) : f64_to_bits(x[k]);
        }
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
        for (uint32_t done = 0; done < nlimbs; done += 65535u) {
            LimbSet l2 = ls;
            l2.b0 = ls.b0 + done;
            const uint32_t cnt = nlimbs - done < 65535u ? nlimbs - done : 65535u;
            hipLaunchKernelGGL(kern, dim3(gx, cnt), dim3(wg), 0, st, l2, (const ModQ *)c->d_mod,
                               (const double *)c->d_tw, logN, sig0);
        }
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
        for (uint32_t done = 0; done < nlimbs; done += 65535u) {
            LimbSet l2 = ls;
            l2.b0 = ls.b0 + done;
            const uint32_t cnt = nlimbs - done < 65535u ? nlimbs - done : 65535u;
            hipLaunchKernelGGL(kern, dim3(gx, cnt), dim3(wg), 0, st, l2, (const ModQ *)c->d_mod,
                               (const double *)c->d_itw, (const double *)c->d_ninv, logN, sig0);
        }
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
