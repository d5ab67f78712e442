// ntt_core.h -- register/LDS round structure of the negacyclic NTT, shared by
// the plain transforms (ntt.hip) and the fused key-switching kernels.
//
// A group of G = 2^LOGG elements, independent for LOGG consecutive stages, is
// held by T = G/16 lanes, 16 elements each.  A round runs up to 4 stages in
// registers (radix 16); rounds exchange through padded LDS.  COL groups are
// strided columns (element g of group gi at gi + g*N/G, lanes of a wavefront
// spread over consecutive columns); ROW groups are contiguous blocks.
#pragma once
#include "fhe_internal.h"

namespace nttc {

constexpr int LOGR = 4;
constexpr int R = 1 << LOGR;

// Local index of register k of lane tau in a round covering bits [blo, blo+rho).
template <int LOGT>
__host__ __device__ constexpr int elem_local(int tau, int k, int blo, int rho)
{
    const int fr = ((k >> rho) << LOGT) | tau;
    return ((fr >> blo) << (blo + rho)) | ((k & ((1 << rho) - 1)) << blo) | (fr & ((1 << blo) - 1));
}
// The lane's part and the register's part of elem_local have disjoint bits, so
// elem_local(tau, k) = elem_local(tau, 0) + elem_local(0, k), and the same holds for
// their right shifts and for lds_pad: a lane computes its part once per round and
// every register adds a compile-time constant (an immediate offset of its load).
__host__ __device__ constexpr int lds_pad(int g) { return g + (g >> LOGR); }

template <int LOGG, int WG, bool COL>
struct Geom {
    static constexpr int G = 1 << LOGG, LOGT = LOGG - LOGR, T = 1 << LOGT, GPW = WG / T;
    static constexpr int GS = G + G / R + 1;                  // padded group stride in LDS
    static constexpr int NR = (LOGG + LOGR - 1) / LOGR;
    static constexpr int RL = LOGG - (NR - 1) * LOGR;         // bits of the last round
    static constexpr int LDS = GPW * GS;
    int grp, tau;
    uint32_t gi, N2;
    __device__ __forceinline__ Geom(uint32_t logN, uint32_t block) : Geom(logN, block, threadIdx.x) {}
    // tid: this lane's thread index (passed through an opaque copy, it keeps the compiler
    // from holding every derived address across an outer loop)
    __device__ __forceinline__ Geom(uint32_t logN, uint32_t block, uint32_t tid_)
    {
        const int tid = (int)tid_;
        grp = COL ? (tid % GPW) : (tid / T);
        tau = COL ? (tid / GPW) : (tid % T);
        gi = block * GPW + grp;
        N2 = (1u << logN) >> LOGG;
    }
    __device__ __forceinline__ uint32_t gidx(int g) const
    {
        return COL ? gi + (uint32_t)g * N2 : (gi << LOGG) + (uint32_t)g;
    }
    __device__ __forceinline__ uint32_t gidx2(int gt, int gk) const   // gidx(gt + gk), disjoint bits
    {
        return COL ? gi + (uint32_t)gt * N2 + (uint32_t)gk * N2 : (gi << LOGG) + (uint32_t)gt + (uint32_t)gk;
    }
    __device__ __forceinline__ int lt(int blo, int rho) const { return elem_local<LOGT>(tau, 0, blo, rho); }
    static constexpr int lk(int k, int blo, int rho) { return elem_local<LOGT>(0, k, blo, rho); }
    // forward: registers hold round-0 elements on entry, last-round elements on exit
    __device__ __forceinline__ uint32_t fwd_in(int k) const
    {
        return gidx2(lt(LOGG - LOGR, LOGR), lk(k, LOGG - LOGR, LOGR));
    }
    __device__ __forceinline__ uint32_t fwd_out(int k) const { return gidx2(lt(0, RL), lk(k, 0, RL)); }
    // inverse: the opposite round order
    __device__ __forceinline__ uint32_t inv_in(int k) const
    {
        constexpr int r0 = LOGG < LOGR ? LOGG : LOGR;
        return gidx2(lt(0, r0), lk(k, 0, r0));
    }
    __device__ __forceinline__ uint32_t inv_out(int k) const
    {
        return gidx2(lt((NR - 1) * LOGR, RL), lk(k, (NR - 1) * LOGR, RL));
    }

    // Coalesced order: register k of lane tau holds local element k*T + tau, so that
    // for a fixed k consecutive lanes touch consecutive addresses (ROW groups).
    __device__ __forceinline__ uint32_t coal(int k) const { return gidx2(tau, k << LOGT); }
    // Exchange through LDS: register k goes to the slot of round (wb, wr) and comes
    // back from the slot of round (rb, rr).
    __device__ __forceinline__ void exchange(double (&x)[R], double *lds, int wb, int wr, int rb, int rr) const
    {
        double *w = lds + grp * GS + lds_pad(lt(wb, wr));
#pragma unroll
        for (int k = 0; k < R; k++) w[lds_pad(lk(k, wb, wr))] = x[k];
        __syncthreads();
        const double *r = lds + grp * GS + lds_pad(lt(rb, rr));
#pragma unroll
        for (int k = 0; k < R; k++) x[k] = r[lds_pad(lk(k, rb, rr))];
        __syncthreads();
    }
    // coalesced order <-> the slot of a round (the coalesced index k*T + tau is the
    // local index of register k in round (LOGT, 4) when the group has LOGT + 4 bits)
    __device__ __forceinline__ void fwd_out_to_coal(double (&x)[R], double *lds) const
    {
        double *w = lds + grp * GS + lds_pad(lt(0, RL));
#pragma unroll
        for (int k = 0; k < R; k++) w[lds_pad(lk(k, 0, RL))] = x[k];
        __syncthreads();
        const double *r = lds + grp * GS + lds_pad(tau);
#pragma unroll
        for (int k = 0; k < R; k++) x[k] = r[lds_pad(k << LOGT)];
        __syncthreads();
    }
    // From the coalesced order to the inverse input order.
    __device__ __forceinline__ void coal_to_inv_in(double (&x)[R], double *lds) const
    {
        constexpr int r0 = LOGG < LOGR ? LOGG : LOGR;
        double *w = lds + grp * GS + lds_pad(tau);
#pragma unroll
        for (int k = 0; k < R; k++) w[lds_pad(k << LOGT)] = x[k];
        __syncthreads();
        const double *r = lds + grp * GS + lds_pad(lt(0, r0));
#pragma unroll
        for (int k = 0; k < R; k++) x[k] = r[lds_pad(lk(k, 0, r0))];
        __syncthreads();
    }
    // Twiddle base of a stage on local bit lb (sigma = sigma0 + LOGG - 1 - lb).  A ROW
    // pass holds the last LOGG stages (sigma0 = logN - LOGG) and a COL pass the first
    // (sigma0 = 0), so in both the table index (1 << sigma) + (j >> (logN - sigma))
    // of element j = gidx(local) is (1 << sigma) + [ROW: gi << (LOGG - lb - 1)] +
    // (local >> (lb + 1)), and local >> (lb + 1) splits into the lane's part and the
    // register's constant.
    __device__ __forceinline__ const double *tw_stage(const double *tw, uint32_t sigma0, int lb, int blo,
                                                      int rho) const
    {
        const uint32_t sigma = sigma0 + (uint32_t)(LOGG - 1 - lb);
        uint32_t base = (1u << sigma) + ((uint32_t)lt(blo, rho) >> (lb + 1));
        if (!COL) base += gi << (LOGG - lb - 1);
        return tw + base;
    }

    // Cooley-Tukey stages sigma0 .. sigma0 + LOGG - 1 (table psi^brv).  The upper input
    // of a butterfly is reduced to [-q/2-1, q/2+1] on every other stage only (the first,
    // third, ... of each round): with q < 2^50 and inputs |x| < 2.7q the values stay
    // below 2.7q (< 2^51.5), where every operation is exact.  Out: |x| < 2.7q.
    __device__ __forceinline__ void fwd(double (&x)[R], double *lds, const double *__restrict__ tw, double q,
                                        double qinv, uint32_t logN, uint32_t sigma0) const
    {
#pragma unroll
        for (int r = 0; r < NR; r++) {
            const int bhi = LOGG - r * LOGR;
            const int rho = bhi < LOGR ? bhi : LOGR;
            const int blo = bhi - rho;
            if (r > 0) exchange(x, lds, bhi, LOGR, blo, rho);
#pragma unroll
            for (int s = 0; s < rho; s++) {
                const int bit = rho - 1 - s;
                const int lb = blo + bit;
                const double *tws = tw_stage(tw, sigma0, lb, blo, rho);
#pragma unroll
                for (int k = 0; k < R; k++) {
                    if (k & (1 << bit)) continue;
                    const int kt = k & ~((2 << bit) - 1);
                    const double W = tws[lk(kt, blo, rho) >> (lb + 1)];
                    const double X = (s & 1) ? x[k] : redc(x[k], q, qinv);
                    const double V = mulmod(x[k | (1 << bit)], W, q, qinv);
                    x[k] = X + V;
                    x[k | (1 << bit)] = X - V;
                }
            }
        }
    }

    // Gentleman-Sande stages (table psi^-brv); LASTSTAGE folds N^-1 into global stage 0.
    template <bool LASTSTAGE>
    __device__ __forceinline__ void inv(double (&x)[R], double *lds, const double *__restrict__ tw, double q,
                                        double qinv, double ninv, uint32_t logN, uint32_t sigma0) const
    {
#pragma unroll
        for (int r = 0; r < NR; r++) {
            const int blo = r * LOGR;
            const int rho = (LOGG - blo) < LOGR ? (LOGG - blo) : LOGR;
            if (r > 0) exchange(x, lds, blo - LOGR, LOGR, blo, rho);
#pragma unroll
            for (int s = 0; s < rho; s++) {
                const int bit = s;
                const int lb = blo + bit;
                const bool fold_ninv = LASTSTAGE && (lb == LOGG - 1);
                const double *tws = tw_stage(tw, sigma0, lb, blo, rho);
#pragma unroll
                for (int k = 0; k < R; k++) {
                    if (k & (1 << bit)) continue;
                    const int kt = k & ~((2 << bit) - 1);
                    double W = tws[lk(kt, blo, rho) >> (lb + 1)];
                    const double U = x[k], V = x[k | (1 << bit)];
                    if (fold_ninv) {
                        W = canon(mulmod(W, ninv, q, qinv), q, qinv);
                        x[k] = mulmod(U + V, ninv, q, qinv);
                    } else {
                        x[k] = redc(U + V, q, qinv);
                    }
                    x[k | (1 << bit)] = mulmod(U - V, W, q, qinv);
                }
            }
        }
    }
};

// NTT-domain Galois permutation: the element that lands at x under X -> X^g
// (out[x] = in[perm(x)], 2 brv(perm(x)) + 1 = (2 brv(x) + 1) g mod 2N).  g = 0: identity.
__device__ __forceinline__ uint32_t galois_src(uint32_t x, uint32_t g, uint32_t logN)
{
    if (!g) return x;
    const uint32_t N = 1u << logN;
    const uint32_t ex = 2u * (__brev(x) >> (32 - logN)) + 1u;
    const uint32_t ey = (uint32_t)(((uint64_t)ex * g) & (2u * N - 1));
    return __brev((ey - 1u) >> 1) >> (32 - logN);
}

// Split of a transform into passes: N <= 2^14 one ROW pass of G = N; 2^15 and
// 2^16 a COL pass over the first LOGA stages and a ROW pass over the rest.
struct Split {
    uint32_t logA, logB;   // logA = 0: single pass of LOGG = logB
};
inline Split split_of(uint32_t logN)
{
    if (logN <= 14) return {0, logN};
    if (logN == 15) return {7, 8};
    return {8, 8};
}
// The key-switching path always uses two passes with a row pass of at most 2^8
// elements, so that its fused row kernels run in 256-thread workgroups.
inline Split split_ks(uint32_t logN)
{
    const uint32_t b = logN - 4 < 8 ? logN - 4 : 8;
    return {logN - b, b};
}

}  // namespace nttc
