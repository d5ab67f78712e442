// keyswitch.hip -- hybrid key switching (ModUp, key inner product, ModDown) for
// a batch of inputs, the operation under relinearisation and slot rotation
// (the CT-CT multiplications of Sec. 3 and the rotations of its packing).
//
// For each item b: input d_b (l_b limbs, NTT domain), Galois element gal_b (0 =
// none), key evk_b [dnum][2][L+K][N], output out_b (2 polys of l_b limbs), optional
// addends add[2b], add[2b+1] (read through gal_b).  Items may sit at different
// levels l_b: every launch walks flat lists of (item, limb) or (item, digit) entries
// built on the host, so that one launch sequence serves a whole ragged batch.
// Items with the same input and level share one ModUp (rotations of one ciphertext
// by several steps).
//   ModUp:   digits D_j = limbs [j alpha, min((j+1) alpha, l)) of d_b itself; each
//            converted to Q_l u P by fast basis conversion (canonical representatives);
//   inner:   u_t = sum_j sigma_g(D_j) * evk_{j,t} over Q_l u P, every limb of D_j read
//            through the permutation of gal_b (the key switch of sigma_g(d_b) that a
//            rotation needs, with the extension done once for all g);
//   ModDown: ks_t = (u_t + (P-1)/2 - Conv_{P->Q}([u_t + (P-1)/2]_P)) * P^-1,
//            i.e. u_t / P rounded (up to the fast-conversion error);
//   out_t  = ks_t + add_t.
//
// Transforms are split into rows of N/8 elements (the last logN - 3 forward stages,
// the first inverse ones: one workgroup per row, radix-16 register rounds through
// LDS) and columns of 8 elements at stride N/8 (the other 3 stages).  A column fits
// in one thread's registers, so the column stages run inside the basis conversions:
// a conversion thread finishes the inverse transform of its digit's sources on its
// column, converts, and starts the forward transform of every target on it.
// Kernel sequence:
//   1 k_ks_intt_first   inverse row pass of d_b                         -> dc
//   2 k_conv_cols<up>   inverse column stages of the digit's limbs, times
//                       (Q_j/q_a)^-1, conversion to every other limb of Q_l u P,
//                       forward column stages                          -> up
// then, for items with their own key (the default):
//   3 k_ks_row_inner_pinv  forward row passes of the converted special-prime limbs,
//                       key inner product, inverse row pass of the sum      -> uP
//   4 k_conv_cols<down> inverse column stages, plus (P-1)/2, times (P/p_a)^-1,
//                       conversion P -> Q_l minus (P-1)/2, forward column stages -> z
//   5 k_ks_final_q      forward row passes of the converted Q limbs, key inner
//                       product, forward row pass of z, (u - z) P^-1 + add   -> out
// or, when items share a key (read once per group) or the fusion is off:
//   3 k_row_fwd, k_ks_inner   forward row passes, then the inner product -> uQ, uP
//   4 k_row_inv         inverse row pass of uP
//   5 k_conv_cols<down> as above                                          -> z
//   6 k_ks_moddown_final forward row pass of z fused with (u - z) P^-1 + add -> out
#include <algorithm>
#include <cstring>
#include <map>
#include <type_traits>

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
    uint32_t ginv;      // inverse of the item's Galois element mod 2N (0: none)
    uint16_t upoff[16]; // first converted limb of digit j, relative to up_off
};
static_assert(sizeof(KsItem) == 56, "KsItem is 7 table words");
// One basis conversion with its column stages: nsrc source limbs (moduli smod0 ..)
// -> ndst target limbs; target t has modulus t (t < glo), t + gn (t < l - gn) or
// L + t - (l - gn) (the special primes): Q_l u P without the digit's own limbs.
struct CvJob {
    uint32_t off;          // constants in the conversion table (BconvTab layout)
    uint16_t nsrc, ndst;
    uint32_t src0, dst0;   // first source / target limb in their buffers
    uint8_t smod0, glo, gn, l;
    uint32_t pad;
};
static_assert(sizeof(CvJob) == 24, "CvJob is 3 table words");
// Items of one batch that use the same key at the same level share the key reads
// of the inner product: up to KS_GRP of them form a group.
constexpr uint32_t KS_GRP = 8;
struct KsGrp {
    uint32_t m;              // members
    uint16_t it[KS_GRP];     // item indices
    uint32_t pad;
};
static_assert(sizeof(KsGrp) == 24, "KsGrp is 3 table words");
// Word offsets of the sections of one batch's table:
//   [d: n][evk: n][out: n][add: 2n][gal: n][items: 7n][la: sum l][upjobs: 3 sum nd]
//   [upmods: sum ups][inner: sum over groups (l + K)][dnjobs: 3 * 2n][fl: sum 2l]
//   [pl: 2nK][groups: 3 per group]
// la entries: item << 16 | limb (dc order); inner: group << 16 | x (x < l: Q limb,
// else special prime x - l); fl: item << 17 | poly << 16 | limb (z and uQ order);
// pl (uP limbs): modulus.  upmods and fl also carry the limb of up / z (and uQ) in
// bits 32..; upmods is sorted by modulus.
struct KsTab {
    uint32_t n, K, L;
    uint32_t it, la, uj, um, il, dj, fl, pl, gr;
    uint32_t ip, iq;   // the inner list's special-prime entries, and its Q entries
};
__device__ __forceinline__ const KsItem &tab_item(uint64_t *const *tab, const KsTab &t, uint32_t b)
{
    return reinterpret_cast<const KsItem *>(tab + t.it)[b];
}
__device__ __forceinline__ uint64_t tab_word(uint64_t *const *tab, uint32_t off, uint32_t y)
{
    return (uint64_t)(uintptr_t)tab[off + y];
}

// Loads and stores of data read or written once (NT: non-temporal, so that they pass
// through the caches without evicting the twiddle rows that every pass re-reads).
template <bool NT, typename P>
__device__ __forceinline__ uint64_t ld1(const P *p)
{
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}
template <bool NT, typename P>
__device__ __forceinline__ void st1(P *p, uint64_t v)
{
    if (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}
// 1. First (row) pass of the inverse transform of d_b into dc as lazy FP64 bits.
//    blockIdx.y + y0 = entry of the la list.
template <int LOGG, int WG, bool NT>
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
    const uint32_t b = (uint32_t)((e >> 16) & 0xFFFF), i = (uint32_t)(e & 0xFFFF);
    const gu64 *src = gview(tab[b] + (size_t)i * N);
    const double q = mods[i].q, qinv = mods[i].qinv;
    const Gm gm(logN, blockIdx.x);
    double x[R];
#pragma unroll
    for (int k = 0; k < R; k++) x[k] = u64_to_f64(ld1<NT>(src + gm.coal(k)));
    gm.coal_to_inv_in(x, lds);
    gm.template inv<false>(x, lds, itwt + (size_t)i * N, q, qinv, 0.0, logN, sigma0);
    uint64_t *dst = dc + (size_t)y * N;
#pragma unroll
    for (int k = 0; k < R; k++) st1<NT>(dst + gm.inv_out(k), f64_to_bits(x[k]));
}

// 4b. Key inner product, one thread per pair of coefficients (16-byte loads) of
//     one limb x of Q_l u P for the TI (or fewer) items of one group, which share
//     the key: u_t[x] = sum_j sigma_g(D_j[x]) * evk_{j,t}[x]; D_j[x] is the item's input
//     limb itself inside digit j, else its converted limb, both read through the
//     group's Galois permutation.  blockIdx.y + y0 = entry of the inner list.
__device__ __forceinline__ void ld2(const uint64_t *p, double &a, double &b)
{
    // p comes from the pointer table: a generic pointer to device memory, loaded as
    // global memory (a flat load would also wait on the scalar loads of the table)
    const gu64 *g = gview(p);
    a = u64_to_f64(g[0]);
    b = u64_to_f64(g[1]);
}
template <int TI>
__global__ __launch_bounds__(TPB) void k_ks_inner(uint64_t *const *__restrict__ tab, KsTab t, uint32_t y0,
                                                  const uint64_t *__restrict__ up, uint64_t *__restrict__ uQ,
                                                  uint64_t *__restrict__ uP, const ModQ *__restrict__ mods,
                                                  uint32_t alpha, uint32_t logN)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = 2 * (blockIdx.x * TPB + threadIdx.x);
    if (k >= N) return;
    const uint64_t e = tab_word(tab, t.il, blockIdx.y + y0);
    const uint32_t g = (uint32_t)(e >> 16), x = (uint32_t)(e & 0xFFFF);
    const KsGrp &gr = reinterpret_cast<const KsGrp *>(tab + t.gr)[g];
    const uint32_t m = TI == 1 ? 1u : gr.m;
    const KsItem &i0 = tab_item(tab, t, gr.it[0]);
    const uint32_t l = i0.l, nd = i0.nd;
    const uint32_t mx = x < l ? x : t.L + (x - l);
    const double q = mods[mx].q, qi = mods[mx].qinv;
    const uint64_t *ev = tab[t.n + gr.it[0]];
    const size_t ML = t.L + t.K;
    // every limb is read through the Galois permutation of the group's key, which maps
    // the pair (k, k+1) onto the pair (y, y^1): one 16-byte load, swapped when y is odd
    const uint32_t gal = (uint32_t)tab_word(tab, 5 * t.n, gr.it[0]);
    const uint32_t ys = galois_src(k, gal, logN), yk = ys & ~1u;
    const bool swp = ys & 1u;
    double a0[TI], a1[TI], c0[TI], c1[TI];
#pragma unroll
    for (int u = 0; u < TI; ++u) a0[u] = a1[u] = c0[u] = c1[u] = 0.0;
    for (uint32_t j = 0; j < nd; ++j) {
        const uint32_t lo = j * alpha, hi = min(lo + alpha, l);
        const bool inside = x >= lo && x < hi;
        const uint32_t pos = x < lo ? x : x - (hi - lo);
        double e00, e01, e10, e11;
        ld2(ev + (((size_t)j * 2 + 0) * ML + mx) * N + k, e00, e01);
        ld2(ev + (((size_t)j * 2 + 1) * ML + mx) * N + k, e10, e11);
#pragma unroll
        for (int u = 0; u < TI; ++u) {
            if (u < (int)m) {
                const uint32_t b = gr.it[u];
                double D0, D1;
                if (inside) {
                    ld2(tab[b] + (size_t)x * N + yk, D0, D1);
                } else {
                    const KsItem &it = tab_item(tab, t, b);
                    ld2(up + ((size_t)it.up_off + it.upoff[j] + pos) * N + yk, D0, D1);
                }
                if (swp) {
                    const double t0 = D0;
                    D0 = D1;
                    D1 = t0;
                }
                a0[u] += mulmod(D0, e00, q, qi);
                c0[u] += mulmod(D1, e01, q, qi);
                a1[u] += mulmod(D0, e10, q, qi);
                c1[u] += mulmod(D1, e11, q, qi);
            }
        }
        if ((j & 3) == 3) {
#pragma unroll
            for (int u = 0; u < TI; ++u) {
                a0[u] = redc(a0[u], q, qi);
                c0[u] = redc(c0[u], q, qi);
                a1[u] = redc(a1[u], q, qi);
                c1[u] = redc(c1[u], q, qi);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < TI; ++u) {
        if (u < (int)m) {
            const uint32_t b = gr.it[u];
            uint64_t *o0, *o1;
            if (x < l) {
                const uint32_t uq = tab_item(tab, t, b).uq_off;
                o0 = uQ + ((size_t)uq + x) * N;
                o1 = uQ + ((size_t)uq + l + x) * N;
            } else {
                o0 = uP + ((size_t)b * 2 * t.K + (x - l)) * N;
                o1 = uP + ((size_t)b * 2 * t.K + t.K + (x - l)) * N;
            }
            *reinterpret_cast<ulonglong2 *>(o0 + k) =
                make_ulonglong2(f64_to_u64(canon(a0[u], q, qi)), f64_to_u64(canon(c0[u], q, qi)));
            *reinterpret_cast<ulonglong2 *>(o1 + k) =
                make_ulonglong2(f64_to_u64(canon(a1[u], q, qi)), f64_to_u64(canon(c1[u], q, qi)));
        }
    }
}

// 3 (items with their own key). The forward row pass of the converted limbs fused
//     with the key inner product: one block per row of limb x of Q_l u P.  Per digit
//     j, D_j[x] is the item's input limb (x inside the digit, already in the NTT
//     domain) or its converted limb, whose row stages run here; both are taken at
//     positions y' in coalesced order.  With Galois element g (permutation pi of the
//     NTT positions, out[y] = in[pi(y)]) the sum lands at y = pi^-1(y'):
//       u_t[y] = sum_j D_j[pi(y)] evk_{j,t}[y],
//     so the key is read at y and u stored at y; pi^-1 maps an aligned block of 64
//     positions onto another one, so both stay coalesced.  Lazy values below 2.7 q
//     enter the products (|v e / q| < 2^52) and three digits' products sum below 2^53
//     (the sums are reduced every four digits).
//     pi^-1 also maps the whole row of N/8 positions that a block reads onto one row
//     (the row is fixed by the low 3 bits of the bit-reversed position, and those of
//     pi^-1's image depend only on them), so a block holds a complete row of u: the
//     fused forms below finish that row in the same block.
struct InnerRow {
    uint32_t b, x, l, nd, ginv, mx;
    double q, qi;
};
// 16-byte access of the adjacent pair (p, p + 1), p even.
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) u64x2 gu64x2;
template <bool NT>
__device__ __forceinline__ u64x2 ld2w(const gu64 *p)
{
    const gu64x2 *v = reinterpret_cast<const gu64x2 *>(p);
    if (NT) return __builtin_nontemporal_load(v);
    return *v;
}
template <bool NT>
__device__ __forceinline__ void st2w(gu64 *p, uint64_t a, uint64_t b)
{
    gu64x2 *v = reinterpret_cast<gu64x2 *>(p);
    u64x2 w = {a, b};
    if (NT) __builtin_nontemporal_store(w, v);
    else *v = w;
}
// Where register k of a row sits after a forward row pass.  When the pass's last round
// covers one bit (RL = 1), registers 2m and 2m + 1 hold the adjacent positions 2p and
// 2p + 1 and the lanes' pairs are consecutive: the row is used in that order directly
// (16-byte accesses; the Galois map sends the pair onto a pair, possibly swapped).
// Otherwise the row goes through LDS into coalesced order first.
template <int LOGG, int WG>
struct RowOrder {
    using Gm = Geom<LOGG, WG, false>;
    static constexpr bool DIRECT = Gm::RL == 1;
    static __device__ __forceinline__ uint32_t pos(const Gm &g, int k) { return DIRECT ? g.fwd_out(k) : g.coal(k); }
    // LDS slot (in the lane's group) of register k's position
    static __device__ __forceinline__ int slot_base(const Gm &g)
    {
        return DIRECT ? lds_pad(g.lt(0, Gm::RL)) : lds_pad(g.tau);
    }
    static constexpr int slot_k(int k) { return DIRECT ? lds_pad(Gm::lk(k, 0, Gm::RL)) : lds_pad(k << Gm::LOGT); }
};
template <int LOGG, int WG, bool NT>
__device__ __forceinline__ InnerRow inner_row(uint64_t *const *__restrict__ tab, const KsTab &t, uint32_t entry,
                                              const uint64_t *__restrict__ up, const ModQ *__restrict__ mods,
                                              const double *__restrict__ twt, uint32_t alpha, uint32_t logN,
                                              uint32_t sigma0, double *lds, double (&a0)[R], double (&a1)[R])
{
    using Gm = Geom<LOGG, WG, false>;
    const uint32_t N = 1u << logN;
    const uint64_t e = tab_word(tab, t.il, entry);
    const uint32_t g = (uint32_t)(e >> 16), x = (uint32_t)(e & 0xFFFF);
    const uint32_t b = reinterpret_cast<const KsGrp *>(tab + t.gr)[g].it[0];
    const KsItem &it = tab_item(tab, t, b);
    InnerRow r;
    r.b = b;
    r.x = x;
    r.l = it.l;
    r.nd = it.nd;
    r.ginv = it.ginv;
    r.mx = x < r.l ? x : t.L + (x - r.l);
    r.q = mods[r.mx].q;
    r.qi = mods[r.mx].qinv;
    const uint32_t l = r.l, nd = r.nd, ginv = r.ginv, mx = r.mx;
    const double q = r.q, qi = r.qi;
    const uint64_t *ev = tab[t.n + b];
    const size_t ML = t.L + t.K;
    using RO = RowOrder<LOGG, WG>;
    // the row of digit jj: the item's own limb (NTT domain, in the order of RO) inside
    // the digit, else its converted limb (column-stage form, forward-pass input order)
    auto load_row = [&](const Gm &gj, uint32_t jj, uint64_t (&w)[R]) {
        const uint32_t lo = jj * alpha, hi = min(lo + alpha, l);
        if (x >= lo && x < hi) {
            const gu64 *src = gview(tab[b] + (size_t)x * N);
            if (RO::DIRECT) {
#pragma unroll
                for (int k = 0; k < R; k += 2) {
                    const u64x2 p = ld2w<NT>(src + RO::pos(gj, k));
                    w[k] = p.x;
                    w[k + 1] = p.y;
                }
            } else {
#pragma unroll
                for (int k = 0; k < R; k++) w[k] = ld1<NT>(src + RO::pos(gj, k));
            }
        } else {
            const uint32_t pos = x < lo ? x : x - (hi - lo);
            const uint64_t *src = up + ((size_t)it.up_off + it.upoff[jj] + pos) * N;
#pragma unroll
            for (int k = 0; k < R; k++) w[k] = ld1<NT>(src + gj.fwd_in(k));
        }
    };
#pragma unroll
    for (int k = 0; k < R; k++) a0[k] = a1[k] = 0.0;
#pragma unroll 1
    for (uint32_t j = 0; j < nd; ++j) {
        // every address below is the same for every digit: an opaque copy of the thread
        // index keeps the compiler from computing all of them once before the loop and
        // holding them in registers
        uint32_t tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const Gm gj(logN, blockIdx.x, tid);
        const uint32_t lo = j * alpha, hi = min(lo + alpha, l);
        const bool own = x >= lo && x < hi;   // block-uniform
        uint64_t w[R];
        load_row(gj, j, w);
        double v[R];
#pragma unroll
        for (int k = 0; k < R; k++) v[k] = own ? u64_to_f64(w[k]) : bits_to_f64(w[k]);
        if (!own) {
            gj.fwd(v, lds, twt + (size_t)mx * N, q, qi, logN, sigma0);
            if (!RO::DIRECT) gj.fwd_out_to_coal(v, lds);
        }
        const gu64 *e0 = gview(ev + (((size_t)j * 2 + 0) * ML + mx) * N);
        const gu64 *e1 = gview(ev + (((size_t)j * 2 + 1) * ML + mx) * N);
        if (RO::DIRECT) {
#pragma unroll
            for (int k = 0; k < R; k += 2) {
                const uint32_t y = galois_src(RO::pos(gj, k), ginv, logN);
                const u64x2 p0 = ld2w<NT>(e0 + (y & ~1u)), p1 = ld2w<NT>(e1 + (y & ~1u));
                const bool sw = y & 1u;
                a0[k] += mulmod(v[k], u64_to_f64(sw ? p0.y : p0.x), q, qi);
                a0[k + 1] += mulmod(v[k + 1], u64_to_f64(sw ? p0.x : p0.y), q, qi);
                a1[k] += mulmod(v[k], u64_to_f64(sw ? p1.y : p1.x), q, qi);
                a1[k + 1] += mulmod(v[k + 1], u64_to_f64(sw ? p1.x : p1.y), q, qi);
            }
        } else {
#pragma unroll
            for (int k = 0; k < R; k++) {
                const uint32_t y = galois_src(RO::pos(gj, k), ginv, logN);
                a0[k] += mulmod(v[k], u64_to_f64(ld1<NT>(e0 + y)), q, qi);
                a1[k] += mulmod(v[k], u64_to_f64(ld1<NT>(e1 + y)), q, qi);
            }
        }
        if ((j & 3) == 3) {
#pragma unroll
            for (int k = 0; k < R; k++) {
                a0[k] = redc(a0[k], q, qi);
                a1[k] = redc(a1[k], q, qi);
            }
        }
    }
    return r;
}
// This lane's place in the image of its row: the same group slot of the block (and
// of LDS), the row's image under pi^-1 as the row index.
template <int LOGG, int WG>
__device__ __forceinline__ Geom<LOGG, WG, false> image_geom(uint32_t logN, uint32_t tid, uint32_t ginv)
{
    Geom<LOGG, WG, false> g(logN, blockIdx.x, tid);
    g.gi = galois_src(g.gi << LOGG, ginv, logN) >> LOGG;
    return g;
}
// The sums of both key polynomials, canonical, from registers (a_t[k] belongs at
// position pi^-1(p) of the image row, p: register k's position in RowOrder) into two row buffers of LDS, each value in
// the slot of its own position (slot: lds_pad of the offset in the row); the caller
// reads them back in the order it needs, so the sums leave the registers before the
// next transforms.
template <int LOGG, int WG>
__device__ __forceinline__ void scatter_rows(const Geom<LOGG, WG, false> &gm, const double (&a0)[R],
                                             const double (&a1)[R], double q, double qi, double *lds0, double *lds1,
                                             uint32_t ginv, uint32_t logN)
{
    constexpr uint32_t G = 1u << LOGG;
    constexpr int GS = Geom<LOGG, WG, false>::GS;
    double *w0 = lds0 + gm.grp * GS, *w1 = lds1 + gm.grp * GS;
#pragma unroll
    for (int k = 0; k < R; k++) {
        const int y = (int)(galois_src(RowOrder<LOGG, WG>::pos(gm, k), ginv, logN) & (G - 1));
        w0[lds_pad(y)] = canon(a0[k], q, qi);
        w1[lds_pad(y)] = canon(a1[k], q, qi);
    }
    __syncthreads();
}

// The special-prime entries (blockIdx.y + y0 = entry of the ip list) with the inverse
// row pass of uP in the same block: the row of u_t is gathered in LDS in its own
// positions, read in the inverse pass's order, transformed and stored as lazy bits
// (what k_row_inv stores from the canonical uP).
template <int LOGG, int WG, bool NT>
__global__ __launch_bounds__(WG) void k_ks_row_inner_pinv(uint64_t *const *__restrict__ tab, KsTab t, uint32_t y0,
                                                          const uint64_t *__restrict__ up, uint64_t *__restrict__ uP,
                                                          const ModQ *__restrict__ mods,
                                                          const double *__restrict__ twt,
                                                          const double *__restrict__ itwt, uint32_t alpha,
                                                          uint32_t logN, uint32_t sigma0)
{
    using Gm = Geom<LOGG, WG, false>;
    constexpr int r0 = LOGG < LOGR ? LOGG : LOGR;
    __shared__ double lds[2 * Gm::LDS];
    const uint32_t N = 1u << logN;
    const uint32_t entry = (uint32_t)tab_word(tab, t.ip, blockIdx.y + y0);
    InnerRow r;
    {
        double a0[R], a1[R];
        r = inner_row<LOGG, WG, NT>(tab, t, entry, up, mods, twt, alpha, logN, sigma0, lds, a0, a1);
        scatter_rows(Gm(logN, blockIdx.x), a0, a1, r.q, r.qi, lds, lds + Gm::LDS, r.ginv, logN);
    }
#pragma unroll 1
    for (int tt = 0; tt < 2; ++tt) {
        uint32_t tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const Gm go = image_geom<LOGG, WG>(logN, tid, r.ginv);
        double *buf = lds + tt * Gm::LDS;
        double v[R];
        const double *rd = buf + go.grp * Gm::GS + lds_pad(go.lt(0, r0));
#pragma unroll
        for (int k = 0; k < R; k++) v[k] = rd[lds_pad(Gm::lk(k, 0, r0))];
        __syncthreads();
        go.template inv<false>(v, buf, itwt + (size_t)r.mx * N, r.q, r.qi, 0.0, logN, sigma0);
        uint64_t *dst = uP + ((size_t)r.b * 2 * t.K + tt * t.K + (r.x - r.l)) * N;
#pragma unroll
        for (int k = 0; k < R; k++) st1<NT>(dst + go.inv_out(k), f64_to_bits(v[k]));
    }
}

// The Q entries (blockIdx.y + y0 = entry of the iq list) fused with the ModDown finish:
// the block's row of u_t (both t) is gathered in LDS in its own positions and read
// back in coalesced order, the same row of z_t gets its forward row pass, and
//   out_t[x] = (u_t[x] - z_t[x]) * P^-1 + add_t[x]
// is stored; uQ is never written.
template <int LOGG, int WG, bool NT>
__global__ __launch_bounds__(WG) void k_ks_final_q(uint64_t *const *__restrict__ tab, KsTab t, uint32_t y0,
                                                   const uint64_t *__restrict__ up, const uint64_t *__restrict__ z,
                                                   const ModQ *__restrict__ mods, const double *__restrict__ twt,
                                                   const double *__restrict__ pinv, uint32_t alpha, uint32_t logN,
                                                   uint32_t sigma0)
{
    using Gm = Geom<LOGG, WG, false>;
    __shared__ double lds[2 * Gm::LDS];
    const uint32_t N = 1u << logN;
    const uint32_t entry = (uint32_t)tab_word(tab, t.iq, blockIdx.y + y0);
    InnerRow r;
    {
        double a0[R], a1[R];
        r = inner_row<LOGG, WG, NT>(tab, t, entry, up, mods, twt, alpha, logN, sigma0, lds, a0, a1);
        scatter_rows(Gm(logN, blockIdx.x), a0, a1, r.q, r.qi, lds, lds + Gm::LDS, r.ginv, logN);
    }
    // z_t's row of this Q limb: the item's z rows follow its uQ offset
    const uint64_t *z0 = z + ((size_t)tab_item(tab, t, r.b).uq_off + r.x) * N;
    const uint32_t gal = (uint32_t)tab_word(tab, 5 * t.n, r.b);
    const double pi = pinv[r.x];
#pragma unroll 1
    for (int tt = 0; tt < 2; ++tt) {
        uint32_t tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const Gm go = image_geom<LOGG, WG>(logN, tid, r.ginv);
        double *buf = lds + tt * Gm::LDS;
        // u_t in the order z_t's row has after its pass, then buffer t serves that pass
        using RO = RowOrder<LOGG, WG>;
        double u[R], v[R];
        const double *rd = buf + go.grp * Gm::GS + RO::slot_base(go);
#pragma unroll
        for (int k = 0; k < R; k++) u[k] = rd[RO::slot_k(k)];
        const uint64_t *zs = z0 + (size_t)tt * r.l * N;
#pragma unroll
        for (int k = 0; k < R; k++) v[k] = bits_to_f64(ld1<NT>(zs + go.fwd_in(k)));
        const uint64_t *adp = tab[3 * t.n + 2 * r.b + tt];
        const gu64 *ad = gview(adp) + (size_t)r.x * N;
        __syncthreads();
        go.fwd(v, buf, twt + (size_t)r.x * N, r.q, r.qi, logN, sigma0);
        if (!RO::DIRECT) go.fwd_out_to_coal(v, buf);
        gu64 *out = gview(tab[2 * t.n + r.b] + ((size_t)tt * r.l + r.x) * N);
        double o[R];
#pragma unroll
        for (int k = 0; k < R; k++) o[k] = canon(mulmod(u[k] - v[k], pi, r.q, r.qi), r.q, r.qi);
        if (RO::DIRECT) {
#pragma unroll
            for (int k = 0; k < R; k += 2) {
                const uint32_t idx = RO::pos(go, k);
                if (adp) {
                    const uint32_t y = galois_src(idx, gal, logN);
                    const u64x2 a = ld2w<NT>(ad + (y & ~1u));
                    const bool sw = y & 1u;
                    o[k] = fold(o[k] + u64_to_f64(sw ? a.y : a.x), r.q);
                    o[k + 1] = fold(o[k + 1] + u64_to_f64(sw ? a.x : a.y), r.q);
                }
                st2w<NT>(out + idx, f64_to_u64(o[k]), f64_to_u64(o[k + 1]));
            }
        } else {
#pragma unroll
            for (int k = 0; k < R; k++) {
                const uint32_t idx = RO::pos(go, k);
                if (adp) o[k] = fold(o[k] + u64_to_f64(ld1<NT>(ad + galois_src(idx, gal, logN))), r.q);
                st1<NT>(out + idx, f64_to_u64(o[k]));
            }
        }
    }
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
    const uint32_t b = (uint32_t)((e >> 17) & 0x7FFF), tt = (uint32_t)((e >> 16) & 1), i = (uint32_t)(e & 0xFFFF);
    const size_t row = (size_t)(e >> 32);   // limb of z and uQ
    const uint32_t l = tab_item(tab, t, b).l;
    const double q = mods[i].q, qinv = mods[i].qinv;
    const Gm gm(logN, blockIdx.x);
    const uint64_t *zs = z + row * N;
    double v[R];
#pragma unroll
    for (int k = 0; k < R; k++) v[k] = bits_to_f64(zs[gm.fwd_in(k)]);
    gm.fwd(v, lds, twt + (size_t)i * N, q, qinv, logN, sigma0);
    gm.fwd_out_to_coal(v, lds);
    const uint64_t *uq = uQ + row * N;
    const uint64_t *adp = tab[3 * t.n + 2 * b + tt];
    const gu64 *ad = gview(adp);
    const uint32_t gal = (uint32_t)tab_word(tab, 5 * t.n, b);
    gu64 *out = gview(tab[2 * t.n + b] + ((size_t)tt * l + i) * N);
    const double pi = pinv[i];
#pragma unroll
    for (int k = 0; k < R; k++) {
        const uint32_t idx = gm.coal(k);
        double r = canon(mulmod(u64_to_f64(uq[idx]) - v[k], pi, q, qinv), q, qinv);
        if (adp) r = fold(r + u64_to_f64(ad[(size_t)i * N + galois_src(idx, gal, logN)]), q);
        out[idx] = f64_to_u64(r);
    }
}

// Row passes of the key-switching path over a flat limb buffer.  The inverse pass
// treats entry y of lst as limb y, reduced modulo mods[lst[y] & 0xFFFF]; the forward
// pass reads the limb index from bits 32.. of the entry, so that its list can be
// ordered by modulus (consecutive blocks then share the row-pass twiddles in L2).
// The forward row pass: lazy bits in, canonical out, coalesced stores.
template <int LOGG, int WG>
__global__ __launch_bounds__(WG) void k_row_fwd(uint64_t *__restrict__ base, const uint64_t *__restrict__ lst,
                                                uint32_t y0, const ModQ *__restrict__ mods,
                                                const double *__restrict__ twt, uint32_t logN, uint32_t sigma0)
{
    using Gm = Geom<LOGG, WG, false>;
    __shared__ double lds[Gm::LDS];
    const uint32_t N = 1u << logN;
    const uint64_t e = lst[blockIdx.y + y0];
    const uint32_t m = (uint32_t)(e & 0xFFFF);
    const double q = mods[m].q, qinv = mods[m].qinv;
    uint64_t *p = base + (size_t)(e >> 32) * N;
    const Gm gm(logN, blockIdx.x);
    double x[R];
#pragma unroll
    for (int k = 0; k < R; k++) x[k] = bits_to_f64(p[gm.fwd_in(k)]);
    gm.fwd(x, lds, twt + (size_t)m * N, q, qinv, logN, sigma0);
    gm.fwd_out_to_coal(x, lds);
#pragma unroll
    for (int k = 0; k < R; k++) p[gm.coal(k)] = f64_to_u64(canon(x[k], q, qinv));
}
// Inverse row pass over a flat buffer (canonical in, coalesced loads; lazy bits out).
template <int LOGG, int WG>
__global__ __launch_bounds__(WG) void k_row_inv(uint64_t *__restrict__ base, const uint64_t *__restrict__ lst,
                                                uint32_t y0, const ModQ *__restrict__ mods,
                                                const double *__restrict__ itwt, uint32_t logN, uint32_t sigma0)
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
    for (int k = 0; k < R; k++) x[k] = u64_to_f64(p[gm.coal(k)]);
    gm.coal_to_inv_in(x, lds);
    gm.template inv<false>(x, lds, itwt + (size_t)m * N, q, qinv, 0.0, logN, sigma0);
#pragma unroll
    for (int k = 0; k < R; k++) p[gm.inv_out(k)] = f64_to_bits(x[k]);
}
// 2 and 5. Fast basis conversion with the column stages of its transforms.  One thread
//     per column {c + i N/8 : i < 8} of one job (blockIdx.y + y0); lazy FP64 bits of the
//     row-inverted sources in, lazy bits of the column-transformed targets out.
//   * each source a (modulus smod0 + a): the last three inverse stages on the column
//     (Gentleman-Sande, twiddles itw[1..7] of its modulus), N^-1 and the conversion
//     factor (B/b_a)^-1 folded into the last stage, DOWN: plus ((P-1)/2) (B/b_a)^-1,
//     then canonical: v_a = [x_a (B/b_a)^-1]_{b_a} (of x_a + (P-1)/2 for ModDown);
//   * each target t: y = sum_a v_a (B/b_a mod c_t) reduced every four terms, DOWN: minus
//     (P-1)/2, canonical, then the first three forward stages (Cooley-Tukey, twiddles
//     tw[1..7] of c_t; the upper inputs reduced on the first and third) .
//   NS > 0: every job of the launch has NS sources; NS < 0: at most -NS (else 16).
constexpr int CV_WG = 128;
template <int NS, bool DOWN>
__global__ __launch_bounds__(CV_WG) void k_conv_cols(const uint64_t *__restrict__ src, uint64_t *__restrict__ dst,
                                                     const CvJob *__restrict__ jobs, uint32_t y0,
                                                     const ModQ *__restrict__ mods, const double *__restrict__ twt,
                                                     const double *__restrict__ itwt, const double *__restrict__ ninvt,
                                                     const double *__restrict__ ctab, const double *__restrict__ half,
                                                     uint32_t L, uint32_t logN)
{
    const uint32_t N = 1u << logN, S = N >> 3;
    const uint32_t c = blockIdx.x * CV_WG + threadIdx.x;
    if (c >= S) return;
    const CvJob jb = jobs[blockIdx.y + y0];
    const uint32_t ns = NS > 0 ? (uint32_t)NS : jb.nsrc, nt = jb.ndst;
    const double *T = ctab + jb.off;
    const double *hq = T + 3 * ns + 2 * nt;   // [nt][ns] (B/b_a) mod c_t
    constexpr int NV = NS > 0 ? NS : (NS < 0 ? -NS : 16);
    double v[NV][8];
#pragma unroll
    for (int a = 0; a < NV; ++a) {
        if (a >= (int)ns) break;
        const uint32_t m = jb.smod0 + a;
        const double q = mods[m].q, qi = mods[m].qinv;
        const double *w = itwt + (size_t)m * N;
        const uint64_t *s = src + (size_t)(jb.src0 + a) * N + c;
        double x[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = bits_to_f64(s[(size_t)i * S]);
        // inverse stage on bit 0 (pairs i, i+1), then bit 1 (i, i+2)
#pragma unroll
        for (int i = 0; i < 8; i += 2) {
            const double U = x[i], V = x[i + 1];
            x[i] = redc(U + V, q, qi);
            x[i + 1] = mulmod(U - V, w[4 + (i >> 1)], q, qi);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (i & 2) continue;
            const double U = x[i], V = x[i + 2];
            x[i] = redc(U + V, q, qi);
            x[i + 2] = mulmod(U - V, w[2 + (i >> 2)], q, qi);
        }
        // last stage (bit 2) with N^-1 (B/b_a)^-1 folded in
        const double f = canon(mulmod(ninvt[m], T[a], q, qi), q, qi);
        const double fw = canon(mulmod(w[1], f, q, qi), q, qi);
        double h = 0.0;
        if (DOWN) h = canon(mulmod(half[m], T[a], q, qi), q, qi);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double U = x[i], V = x[i + 4];
            double r0 = mulmod(U + V, f, q, qi), r1 = mulmod(U - V, fw, q, qi);
            if (DOWN) {
                r0 += h;
                r1 += h;
            }
            v[a][i] = canon(r0, q, qi);
            v[a][i + 4] = canon(r1, q, qi);
        }
    }
    for (uint32_t tt = 0; tt < nt; ++tt) {
        const uint32_t m = tt < jb.glo ? tt : (tt < (uint32_t)jb.l - jb.gn ? tt + jb.gn : L + tt - (jb.l - jb.gn));
        const double q = mods[m].q, qi = mods[m].qinv;
        const double *h = hq + (size_t)tt * ns;
        double y[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) y[i] = 0.0;
#pragma unroll
        for (int a = 0; a < NV; ++a) {
            if (a >= (int)ns) break;
            const double ha = h[a];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                y[i] += mulmod(v[a][i], ha, q, qi);
                if ((a & 3) == 3) y[i] = redc(y[i], q, qi);
            }
        }
        const double hd = DOWN ? half[m] : 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i) y[i] = canon(DOWN ? y[i] - hd : y[i], q, qi);
        // forward stages on bit 2 (pairs i, i+4), bit 1 (i, i+2), bit 0 (i, i+1)
        const double *w = twt + (size_t)m * N;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double X = redc(y[i], q, qi), V = mulmod(y[i + 4], w[1], q, qi);
            y[i] = X + V;
            y[i + 4] = X - V;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (i & 2) continue;
            const double X = y[i], V = mulmod(y[i + 2], w[2 + (i >> 2)], q, qi);
            y[i] = X + V;
            y[i + 2] = X - V;
        }
#pragma unroll
        for (int i = 0; i < 8; i += 2) {
            const double X = redc(y[i], q, qi), V = mulmod(y[i + 1], w[4 + (i >> 1)], q, qi);
            y[i] = X + V;
            y[i + 1] = X - V;
        }
        uint64_t *o = dst + (size_t)(jb.dst0 + tt) * N + c;
#pragma unroll
        for (int i = 0; i < 8; ++i) o[(size_t)i * S] = f64_to_bits(y[i]);
    }
}

// ---- rescale over a ragged batch (item b: l_b limbs, P polys).  Table:
// [in: n][out: n][lvl: n][last: n*P][spread: sum P (l_b - 1)]; a last entry
// j = b*P + p holds j << 16 | (l_b - 1), a spread entry j << 16 | i.
// Step 1: copy the last limb of every polynomial to tmp [n*P][N].
__global__ __launch_bounds__(TPB) void k_rs_gather_last(uint64_t *const *__restrict__ tab, uint32_t n,
                                                        uint32_t polys, uint64_t *__restrict__ last, uint32_t logN,
                                                        uint32_t y0)
{
    const uint32_t N = 1u << logN;
    const uint32_t k = blockIdx.x * TPB + threadIdx.x;
    if (k >= N) return;
    const uint32_t j = blockIdx.y + y0, b = j / polys, p = j % polys;
    const uint32_t l = (uint32_t)(uintptr_t)tab[2 * n + b];
    last[(size_t)j * N + k] = gview(tab[b])[((size_t)p * l + (l - 1)) * N + k];
}
// Step 2 (after the inverse transform of the last limbs): per spread entry y, the
// last limb's coefficients r lifted to (-q_last/2, q_last/2] and reduced mod q_i,
// then the forward column pass (lazy bits out into s[y]).
template <int LOGG, int WG>
__global__ __launch_bounds__(WG) void k_rs_spread_col(uint64_t *const *__restrict__ tab, uint32_t n, uint32_t polys,
                                                      uint32_t sp, const uint64_t *__restrict__ last,
                                                      uint64_t *__restrict__ sbuf, const ModQ *__restrict__ mods,
                                                      const double *__restrict__ twt, uint32_t logN, uint32_t y0)
{
    using Gm = Geom<LOGG, WG, true>;
    __shared__ double lds[Gm::LDS];
    const uint32_t N = 1u << logN;
    const uint32_t y = blockIdx.y + y0;
    const uint64_t e = (uint64_t)(uintptr_t)tab[sp + y];
    const uint32_t j = (uint32_t)(e >> 16), i = (uint32_t)(e & 0xFFFF);
    const uint32_t l = (uint32_t)(uintptr_t)tab[2 * n + j / polys];
    const double ql = mods[l - 1].q;
    const double q = mods[i].q, qinv = mods[i].qinv;
    const uint64_t *r = last + (size_t)j * N;
    const Gm gm(logN, blockIdx.x);
    double x[R];
#pragma unroll
    for (int k = 0; k < R; k++) {
        double v = u64_to_f64(r[gm.fwd_in(k)]);
        v = v > 0.5 * ql ? v - ql : v;   // centered lift (q_last odd: no ties)
        x[k] = canon(v, q, qinv);
    }
    gm.fwd(x, lds, twt + (size_t)i * N, q, qinv, logN, 0);
    uint64_t *o = sbuf + (size_t)y * N;
#pragma unroll
    for (int k = 0; k < R; k++) o[gm.fwd_out(k)] = f64_to_bits(x[k]);
}
// Step 3: the forward row pass of s fused with out = (c - s) * q_last^-1 mod q_i.
template <int LOGG, int WG>
__global__ __launch_bounds__(WG) void k_rs_row_fin(uint64_t *const *__restrict__ tab, uint32_t n, uint32_t polys,
                                                   uint32_t sp, const uint64_t *__restrict__ sbuf,
                                                   const ModQ *__restrict__ mods, const double *__restrict__ twt,
                                                   const double *__restrict__ qlinv, uint32_t L, uint32_t logN,
                                                   uint32_t sigma0, uint32_t y0)
{
    using Gm = Geom<LOGG, WG, false>;
    __shared__ double lds[Gm::LDS];
    const uint32_t N = 1u << logN;
    const uint32_t y = blockIdx.y + y0;
    const uint64_t e = (uint64_t)(uintptr_t)tab[sp + y];
    const uint32_t j = (uint32_t)(e >> 16), i = (uint32_t)(e & 0xFFFF), b = j / polys, p = j % polys;
    const uint32_t l = (uint32_t)(uintptr_t)tab[2 * n + b];
    const double q = mods[i].q, qinv = mods[i].qinv;
    const Gm gm(logN, blockIdx.x);
    const uint64_t *sv = sbuf + (size_t)y * N;
    double x[R];
#pragma unroll
    for (int k = 0; k < R; k++) x[k] = bits_to_f64(sv[gm.fwd_in(k)]);
    gm.fwd(x, lds, twt + (size_t)i * N, q, qinv, logN, sigma0);
    gm.fwd_out_to_coal(x, lds);
    const gu64 *cin = gview(tab[b] + ((size_t)p * l + i) * N);
    gu64 *out = gview(tab[n + b] + ((size_t)p * (l - 1) + i) * N);
    const double w = qlinv[(size_t)(l - 1) * L + i];
#pragma unroll
    for (int k = 0; k < R; k++) {
        const uint32_t idx = gm.coal(k);
        const double sval = canon(x[k], q, qinv);
        const double r = mulmod(u64_to_f64(cin[idx]) - sval, w, q, qinv);
        out[idx] = f64_to_u64(fold(r, q));
    }
}

// Per ring degree: column pass (LOGA stages, WA threads, GA blocks per limb) and
// row pass (LOGB stages, WB threads, GB blocks per limb), sigma0 of the row pass = LOGA.
// RW caps the row-pass workgroup: 128 (the default: half the LDS per block, twice the
// resident blocks per CU for the latency-bound row kernels; the ModDown finish runs
// 9% faster) or 256.
template <int LOGN, int RW>
struct KsShape {
    static constexpr int LOGB = LOGN - 4 < 8 ? LOGN - 4 : 8, LOGA = LOGN - LOGB;
    static constexpr int TA = 1 << (LOGA - 4), NCOL = 1 << LOGB;
    static constexpr int WA = TA * NCOL < 256 ? TA * NCOL : 256, GA = NCOL / (WA / TA);
    static constexpr int TB = 1 << (LOGB - 4), NROW = 1 << LOGA;
    static constexpr int WB = TB * NROW < RW ? TB * NROW : RW, GB = NROW / (WB / TB);
};

template <int LOGN, typename F>
void with_shape(uint32_t row_wg, F f)
{
    if (row_wg == 128) f(KsShape<LOGN, 128>{});
    else f(KsShape<LOGN, 256>{});
}
template <typename F>
void dispatch_logn(const fhe_ctx *c, F f)
{
    const uint32_t rw = c->tune_row_wg;
    switch (c->logN) {
    case 10: with_shape<10>(rw, f); break;
    case 11: with_shape<11>(rw, f); break;
    case 12: with_shape<12>(rw, f); break;
    case 13: with_shape<13>(rw, f); break;
    case 14: with_shape<14>(rw, f); break;
    case 15: with_shape<15>(rw, f); break;
    case 16: with_shape<16>(rw, f); break;
    default: break;
    }
}
// run f(y0, count) over [0, total) in grid-sized pieces
template <typename F>
void in_pieces(uint32_t total, F f)
{
    for (uint32_t y0 = 0; y0 < total; y0 += GRID_Y) f(y0, std::min(GRID_Y, total - y0));
}

// Geometry of the key-switching transforms: rows of 2^LOGW = N/8 elements (T lanes
// each, RPB rows per WG-thread block, GB blocks per limb) and the 3 column stages in
// the conversions.  A row of 2^13 elements takes one 512-thread block and 69.6 KB of LDS.
template <int LOGN>
struct KsRow {
    static constexpr int LOGW = LOGN - 3, T = 1 << (LOGW - 4);
    static constexpr int WG0 = T < 256 ? 256 : T;
    static constexpr int WG = WG0 < T * 8 ? WG0 : T * 8;
    static constexpr int GB = 8 * T / WG;
};
template <typename F>
void dispatch_row(const fhe_ctx *c, F f)
{
    switch (c->logN) {
    case 10: f(KsRow<10>{}); break;
    case 11: f(KsRow<11>{}); break;
    case 12: f(KsRow<12>{}); break;
    case 13: f(KsRow<13>{}); break;
    case 14: f(KsRow<14>{}); break;
    case 15: f(KsRow<15>{}); break;
    case 16: f(KsRow<16>{}); break;
    default: break;
    }
}

// Host plan of one ragged batch.
struct KsPlan {
    uint32_t n, sum_l, sum_dc, sum_nd, sum_ups, sum_inner, max_grp;
    uint32_t up_ns, dn_ns;   // sources of every ModUp (ModDown) conversion job, 0 if they differ
    uint32_t up_max, dn_max; // most sources of a job
    std::vector<KsItem> items;
    std::vector<CvJob> upjobs, dnjobs;
    std::vector<KsGrp> groups;
    std::vector<uint64_t> la, upmods, inner, fl, pl;
    std::vector<uint64_t> ip, iq;   // indices into inner of its special-prime and Q entries
};

// g^-1 mod 2N for odd g (the units mod 2N form a group of order N, so g^-1 = g^(N-1))
uint32_t galois_inverse(uint32_t g, uint32_t N)
{
    if (!g) return 0;
    const uint64_t m = 2ull * N;
    uint64_t r = 1, b = g % m;
    for (uint64_t e = N - 1; e; e >>= 1, b = b * b % m)
        if (e & 1) r = r * b % m;
    return (uint32_t)r;
}

fhe_status ks_plan(const fhe_ctx *c, uint32_t n, const uint32_t *ls, const uint64_t *const *d, const uint32_t *gal,
                   const uint64_t *const *evk, KsPlan &pl)
{
    const uint32_t K = c->K, L = c->L, alpha = c->alpha;
    pl.n = n;
    pl.items.assign(n, KsItem{});
    uint32_t dc = 0, up = 0, uq = 0;
    // items with the same input and level share the first one's ModUp (dc and up rows)
    std::map<std::pair<const uint64_t *, uint32_t>, uint32_t> first;
    for (uint32_t b = 0; b < n; ++b) {
        const uint32_t l = ls[b];
        if (l < 1 || l > L) return fhe_fail(FHE_ELEVEL, "key switch: limb count out of range");
        const uint32_t nd = (l + alpha - 1) / alpha;
        if (nd > 16) return fhe_fail(FHE_EPARAM, "key switching supports at most 16 digits");
        if (b >= 32768) return fhe_fail(FHE_EINVAL, "key-switch batch too large");
        KsItem &it = pl.items[b];
        it.l = l;
        it.nd = nd;
        it.uq_off = uq;
        it.ginv = galois_inverse(gal ? gal[b] : 0u, c->N);
        for (uint32_t tt = 0; tt < 2; ++tt) {
            const BconvTab &md = c->moddown[l];
            pl.dnjobs.push_back(CvJob{md.off, (uint16_t)md.nsrc, (uint16_t)md.ndst, (2 * b + tt) * K, uq + tt * l,
                                      (uint8_t)L, (uint8_t)l, 0, (uint8_t)l, 0});
            for (uint32_t i = 0; i < l; ++i)
                pl.fl.push_back(((uint64_t)b << 17) | ((uint64_t)tt << 16) | i | ((uint64_t)(uq + tt * l + i) << 32));
            for (uint32_t k = 0; k < K; ++k) pl.pl.push_back((uint64_t)(L + k));
        }
        uq += 2 * l;
        const auto key = std::make_pair(d[b], l);
        const auto f = first.find(key);
        if (f != first.end()) {
            const KsItem &src = pl.items[f->second];
            it.dc_off = src.dc_off;
            it.up_off = src.up_off;
            for (uint32_t j = 0; j < nd; ++j) it.upoff[j] = src.upoff[j];
            continue;
        }
        first.emplace(key, b);
        it.dc_off = dc;
        it.up_off = up;
        uint32_t u = 0;
        for (uint32_t j = 0; j < nd; ++j) {
            const BconvTab &t = c->modup[(size_t)l * c->dnum + j];
            const uint32_t lo = j * alpha;
            it.upoff[j] = (uint16_t)u;
            pl.upjobs.push_back(CvJob{t.off, (uint16_t)t.nsrc, (uint16_t)t.ndst, dc + lo, up + u, (uint8_t)lo,
                                      (uint8_t)lo, (uint8_t)t.nsrc, (uint8_t)l, 0});
            for (uint32_t a = 0; a < t.ndst; ++a) pl.upmods.push_back(t.dst[a] | ((uint64_t)(up + u + a) << 32));
            u += t.ndst;
        }
        for (uint32_t i = 0; i < l; ++i) pl.la.push_back(((uint64_t)b << 16) | i);
        dc += l;
        up += u;
    }
    auto common_ns = [](const std::vector<CvJob> &js) {
        const uint32_t ns = js.empty() ? 0u : js[0].nsrc;
        for (const CvJob &j : js)
            if (j.nsrc != ns) return 0u;
        return ns;
    };
    auto max_ns = [](const std::vector<CvJob> &js) {
        uint32_t m = 0;
        for (const CvJob &j : js) m = std::max<uint32_t>(m, j.nsrc);
        return m;
    };
    pl.up_ns = common_ns(pl.upjobs);
    pl.dn_ns = common_ns(pl.dnjobs);
    pl.up_max = max_ns(pl.upjobs);
    pl.dn_max = max_ns(pl.dnjobs);
    // the ModUp digits' forward row passes (grouped path) in modulus order: their
    // twiddles are then read once per modulus
    std::stable_sort(pl.upmods.begin(), pl.upmods.end(),
                     [](uint64_t a, uint64_t b) { return (a & 0xFFFF) < (b & 0xFFFF); });
    // groups of items with the same key and level, in order of first appearance
    std::map<std::pair<const uint64_t *, uint32_t>, uint32_t> open;
    pl.max_grp = 0;
    for (uint32_t b = 0; b < n; ++b) {
        const auto key = std::make_pair(evk[b], ls[b]);
        auto f = open.find(key);
        if (f == open.end() || pl.groups[f->second].m == KS_GRP) {
            open[key] = (uint32_t)pl.groups.size();
            pl.groups.push_back(KsGrp{});
            f = open.find(key);
        }
        KsGrp &g = pl.groups[f->second];
        g.it[g.m++] = (uint16_t)b;
        pl.max_grp = std::max(pl.max_grp, g.m);
    }
    if (pl.groups.size() >= 65536) return fhe_fail(FHE_EINVAL, "key-switch batch too large");
    for (uint32_t g = 0; g < pl.groups.size(); ++g) {
        const uint32_t l = ls[pl.groups[g].it[0]];
        for (uint32_t x = 0; x < l + K; ++x) {
            (x < l ? pl.iq : pl.ip).push_back(pl.inner.size());
            pl.inner.push_back(((uint64_t)g << 16) | x);
        }
    }
    pl.sum_l = uq / 2;
    pl.sum_dc = dc;
    pl.sum_ups = up;
    pl.sum_nd = (uint32_t)pl.upjobs.size();
    pl.sum_inner = (uint32_t)pl.inner.size();
    return FHE_OK;
}

}  // namespace

// ---- launchers of the key-switching path
// The fused kernels' variant from the context's knob: f(NT) as an integral constant.
template <typename F>
static void ks_fused_variant(const fhe_ctx *c, F f)
{
    if (c->tune_ks_nt) f(std::true_type{});
    else f(std::false_type{});
}
static void ks_row_fwd(fhe_ctx *c, uint64_t *base, const uint64_t *lst, uint32_t nlimbs)
{
    ProfScope ps(c, "ntt_fwd_row");
    dispatch_row(c, [&](auto sh) {
        using S = decltype(sh);
        in_pieces(nlimbs, [&](uint32_t y0, uint32_t cnt) {
            hipLaunchKernelGGL((k_row_fwd<S::LOGW, S::WG>), dim3(S::GB, cnt), dim3(S::WG), 0, c->stream, base, lst, y0,
                               (const ModQ *)c->d_mod, (const double *)c->d_tw, c->logN, 3u);
        });
    });
}
static void ks_row_inv(fhe_ctx *c, uint64_t *base, const uint64_t *lst, uint32_t nlimbs)
{
    ProfScope ps(c, "ntt_inv_row");
    dispatch_row(c, [&](auto sh) {
        using S = decltype(sh);
        in_pieces(nlimbs, [&](uint32_t y0, uint32_t cnt) {
            hipLaunchKernelGGL((k_row_inv<S::LOGW, S::WG>), dim3(S::GB, cnt), dim3(S::WG), 0, c->stream, base, lst, y0,
                               (const ModQ *)c->d_mod, (const double *)c->d_itw, c->logN, 3u);
        });
    });
}
// ns: the number of sources of every job, or 0 when they differ (then mx: the most)
template <bool DOWN>
static void ks_conv(fhe_ctx *c, const uint64_t *src, uint64_t *dst, const uint64_t *jobs, uint32_t njobs,
                    uint32_t ns, uint32_t mx, const char *cat)
{
    ProfScope ps(c, cat);
    in_pieces(njobs, [&](uint32_t y0, uint32_t cnt) {
        const dim3 grid(blocks_for(c->N / 8, CV_WG), cnt);
#define CONV_GO(NSV)                                                                                          \
    hipLaunchKernelGGL((k_conv_cols<NSV, DOWN>), grid, dim3(CV_WG), 0, c->stream, src, dst, (const CvJob *)jobs, \
                       y0, (const ModQ *)c->d_mod, (const double *)c->d_tw, (const double *)c->d_itw,          \
                       (const double *)c->d_ninv, (const double *)c->d_bconv, (const double *)c->d_phalf, c->L,   \
                       c->logN)
        switch (ns) {
        case 1: CONV_GO(1); break;
        case 2: CONV_GO(2); break;
        case 3: CONV_GO(3); break;
        case 4: CONV_GO(4); break;
        case 8: CONV_GO(8); break;
        default:
            if (mx <= 8) CONV_GO(-8);
            else CONV_GO(0);
            break;
        }
#undef CONV_GO
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
    if ((s = ks_plan(c, n, ls, d, gal, evk, pl))) return s;

    // scratch: dc [sum l of distinct inputs], up [their ups], uQ [sum 2l], uP [n][2][K],
    // z [sum 2l] (ks_scratch_bytes_ragged counts every input as distinct)
    uint8_t *scr = scr_in;
    if (!scr && (s = ctx_scratch(c, ks_scratch_bytes_ragged(c, n, ls), &scr))) return s;
    uint64_t *dc = (uint64_t *)scr, *up = dc + (size_t)pl.sum_dc * N, *uQ = up + (size_t)pl.sum_ups * N,
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
    push_words(pl.upjobs.data(), pl.upjobs.size() * sizeof(CvJob));
    kt.um = (uint32_t)tab.size();
    push_words(pl.upmods.data(), pl.upmods.size() * 8);
    kt.il = (uint32_t)tab.size();
    push_words(pl.inner.data(), pl.inner.size() * 8);
    kt.dj = (uint32_t)tab.size();
    push_words(pl.dnjobs.data(), pl.dnjobs.size() * sizeof(CvJob));
    kt.fl = (uint32_t)tab.size();
    push_words(pl.fl.data(), pl.fl.size() * 8);
    kt.pl = (uint32_t)tab.size();
    push_words(pl.pl.data(), pl.pl.size() * 8);
    kt.gr = (uint32_t)tab.size();
    push_words(pl.groups.data(), pl.groups.size() * sizeof(KsGrp));
    kt.ip = (uint32_t)tab.size();
    push_words(pl.ip.data(), pl.ip.size() * 8);
    kt.iq = (uint32_t)tab.size();
    push_words(pl.iq.data(), pl.iq.size() * 8);
    uint64_t **dt;
    if ((s = ctx_ptr_table(c, tab, &dt))) return s;
    const uint64_t *dwords = (const uint64_t *)dt;
    hipStream_t st = c->stream;
    const uint32_t sum2l = 2 * pl.sum_l;

    // 1. inverse row pass of the distinct inputs
    {
        ProfScope ps(c, "ks_intt_first");
        dispatch_row(c, [&](auto sh) {
            using S = decltype(sh);
            in_pieces(pl.sum_dc, [&](uint32_t y0, uint32_t cnt) {
                if (c->tune_ks_nt)
                    hipLaunchKernelGGL((k_ks_intt_first<S::LOGW, S::WG, true>), dim3(S::GB, cnt), dim3(S::WG), 0, st,
                                       (uint64_t *const *)dt, kt, y0, dc, (const ModQ *)c->d_mod,
                                       (const double *)c->d_itw, c->logN, 3u);
                else
                    hipLaunchKernelGGL((k_ks_intt_first<S::LOGW, S::WG, false>), dim3(S::GB, cnt), dim3(S::WG), 0,
                                       st, (uint64_t *const *)dt, kt, y0, dc, (const ModQ *)c->d_mod,
                                       (const double *)c->d_itw, c->logN, 3u);
            });
        });
    }
    // 2. ModUp: column stages and conversion of every digit
    ks_conv<false>(c, dc, up, dwords + kt.uj, pl.sum_nd, pl.up_ns, pl.up_max, "bconv_up");
    if (pl.max_grp == 1 && c->tune_fuse_row_inner) {
        // items with their own keys: 3+4. forward row passes and the key inner product
        // of the special-prime limbs with the inverse row pass of uP, 5. ModDown's
        // conversion, 6. forward row passes and the inner product of the Q limbs with
        // the ModDown finish (uQ stays on chip)
        {
            ProfScope ps(c, "ks_inner");
            dispatch_row(c, [&](auto sh) {
                using S = decltype(sh);
                in_pieces((uint32_t)pl.ip.size(), [&](uint32_t y0, uint32_t cnt) {
                    auto go = [&](auto nt) {
                        hipLaunchKernelGGL((k_ks_row_inner_pinv<S::LOGW, S::WG, decltype(nt)::value>),
                                           dim3(S::GB, cnt), dim3(S::WG), 0, st, (uint64_t *const *)dt, kt, y0,
                                           (const uint64_t *)up, uP, (const ModQ *)c->d_mod,
                                           (const double *)c->d_tw, (const double *)c->d_itw, c->alpha, c->logN, 3u);
                    };
                    ks_fused_variant(c, go);
                });
            });
        }
        ks_conv<true>(c, uP, z, dwords + kt.dj, 2 * n, pl.dn_ns, pl.dn_max, "bconv_down");
        {
            ProfScope ps(c, "ks_moddown_final");
            dispatch_row(c, [&](auto sh) {
                using S = decltype(sh);
                in_pieces((uint32_t)pl.iq.size(), [&](uint32_t y0, uint32_t cnt) {
                    auto go = [&](auto nt) {
                        hipLaunchKernelGGL((k_ks_final_q<S::LOGW, S::WG, decltype(nt)::value>),
                                           dim3(S::GB, cnt),
                                           dim3(S::WG), 0, st, (uint64_t *const *)dt, kt, y0, (const uint64_t *)up,
                                           (const uint64_t *)z, (const ModQ *)c->d_mod, (const double *)c->d_tw,
                                           (const double *)c->d_pinv, c->alpha, c->logN, 3u);
                    };
                    ks_fused_variant(c, go);
                });
            });
        }
        HIPCHK(hipGetLastError());
        return FHE_OK;
    }
    // 3. forward row pass of the converted limbs and the key inner product
    {
        ks_row_fwd(c, up, dwords + kt.um, pl.sum_ups);
        ProfScope ps(c, "ks_inner");
        in_pieces(pl.sum_inner, [&](uint32_t y0, uint32_t cnt) {
            if (pl.max_grp > 1)
                hipLaunchKernelGGL(k_ks_inner<KS_GRP>, dim3(blocks_for(N / 2, TPB), cnt), dim3(TPB), 0, st,
                                   (uint64_t *const *)dt, kt, y0, (const uint64_t *)up, uQ, uP,
                                   (const ModQ *)c->d_mod, c->alpha, c->logN);
            else
                hipLaunchKernelGGL(k_ks_inner<1>, dim3(blocks_for(N / 2, TPB), cnt), dim3(TPB), 0, st,
                                   (uint64_t *const *)dt, kt, y0, (const uint64_t *)up, uQ, uP,
                                   (const ModQ *)c->d_mod, c->alpha, c->logN);
        });
    }
    // 4-5. ModDown: inverse row pass of the P limbs, then their column stages and the
    //      rounded conversion to Q_l with the first forward column stages of z
    ks_row_inv(c, uP, dwords + kt.pl, n * 2 * K);
    ks_conv<true>(c, uP, z, dwords + kt.dj, 2 * n, pl.dn_ns, pl.dn_max, "bconv_down");
    // 6. row pass of z fused with the finish
    {
        ProfScope ps(c, "ks_moddown_final");
        dispatch_row(c, [&](auto sh) {
            using S = decltype(sh);
            in_pieces(sum2l, [&](uint32_t y0, uint32_t cnt) {
                hipLaunchKernelGGL((k_ks_moddown_final<S::LOGW, S::WG>), dim3(S::GB, cnt), dim3(S::WG), 0, st,
                                   (uint64_t *const *)dt, kt, y0, (const uint64_t *)z, (const uint64_t *)uQ,
                                   (const ModQ *)c->d_mod, (const double *)c->d_tw, (const double *)c->d_pinv,
                                   c->logN, 3u);
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

size_t rescale_scratch_bytes(const fhe_ctx *c, uint32_t l, uint32_t polys, uint32_t n)
{
    return (size_t)n * polys * ((size_t)l) * c->N * sizeof(uint64_t);   // last limbs + spread limbs
}
size_t rescale_scratch_bytes_ragged(const fhe_ctx *c, uint32_t polys, uint32_t n, const uint32_t *ls)
{
    size_t limbs = 0;
    for (uint32_t b = 0; b < n; ++b) limbs += (size_t)polys * ls[b];
    return limbs * c->N * sizeof(uint64_t);
}
// Rescale a ragged batch into outputs (l_b - 1 limbs); outputs must not overlap inputs.
fhe_status rescale_run_ragged(fhe_ctx *c, uint32_t polys, uint32_t n, const uint32_t *ls, const uint64_t *const *in,
                              uint64_t *const *out, uint8_t *scr)
{
    if (!n) return FHE_OK;
    const size_t N = c->N;
    fhe_status s;
    std::vector<uint64_t *> tab;
    for (uint32_t b = 0; b < n; ++b) tab.push_back((uint64_t *)in[b]);
    for (uint32_t b = 0; b < n; ++b) tab.push_back(out[b]);
    for (uint32_t b = 0; b < n; ++b) {
        if (ls[b] < 2 || ls[b] > c->L) return fhe_fail(FHE_ELEVEL, "rescale: limb count out of range");
        tab.push_back((uint64_t *)(uintptr_t)ls[b]);
    }
    const uint32_t items = n * polys;
    if (items >= (1u << 16) * 1024u) return fhe_fail(FHE_EINVAL, "rescale batch too large");
    const uint32_t lastoff = (uint32_t)tab.size();
    for (uint32_t b = 0; b < n; ++b)
        for (uint32_t p = 0; p < polys; ++p)
            tab.push_back((uint64_t *)(uintptr_t)((((uint64_t)(b * polys + p)) << 16) | (ls[b] - 1)));
    const uint32_t sp = (uint32_t)tab.size();
    for (uint32_t b = 0; b < n; ++b)
        for (uint32_t p = 0; p < polys; ++p)
            for (uint32_t i = 0; i + 1 < ls[b]; ++i)
                tab.push_back((uint64_t *)(uintptr_t)((((uint64_t)(b * polys + p)) << 16) | i));
    const uint32_t nsp = (uint32_t)tab.size() - sp;
    uint64_t **dt;
    if ((s = ctx_ptr_table(c, tab, &dt))) return s;
    const uint64_t *dw = (const uint64_t *)dt;
    uint64_t *last = (uint64_t *)scr, *sbuf = last + (size_t)items * N;
    ProfScope ps(c, "rescale");
    in_pieces(items, [&](uint32_t y0, uint32_t cnt) {
        hipLaunchKernelGGL(k_rs_gather_last, dim3(blocks_for(N, TPB), cnt), dim3(TPB), 0, c->stream,
                           (uint64_t *const *)dt, n, polys, last, c->logN, y0);
    });
    {
        LimbSet ls_last;
        std::memset((void *)&ls_last, 0, sizeof(ls_last));
        ls_last.base = last;
        ls_last.period = 1;
        ls_last.modlist = dw + lastoff;
        launch_ntt_inv(c, ls_last, items);
    }
    dispatch_logn(c, [&](auto sh) {
        using S = decltype(sh);
        in_pieces(nsp, [&](uint32_t y0, uint32_t cnt) {
            hipLaunchKernelGGL((k_rs_spread_col<S::LOGA, S::WA>), dim3(S::GA, cnt), dim3(S::WA), 0, c->stream,
                               (uint64_t *const *)dt, n, polys, sp, (const uint64_t *)last, sbuf,
                               (const ModQ *)c->d_mod, (const double *)c->d_tw, c->logN, y0);
        });
        in_pieces(nsp, [&](uint32_t y0, uint32_t cnt) {
            hipLaunchKernelGGL((k_rs_row_fin<S::LOGB, S::WB>), dim3(S::GB, cnt), dim3(S::WB), 0, c->stream,
                               (uint64_t *const *)dt, n, polys, sp, (const uint64_t *)sbuf, (const ModQ *)c->d_mod,
                               (const double *)c->d_tw, (const double *)c->d_qlinv, c->L, c->logN, (uint32_t)S::LOGA,
                               y0);
        });
    });
    HIPCHK(hipGetLastError());
    return FHE_OK;
}
fhe_status rescale_run(fhe_ctx *c, uint32_t l, uint32_t polys, uint32_t n, const uint64_t *const *in,
                       uint64_t *const *out, uint8_t *scr)
{
    std::vector<uint32_t> ls(n, l);
    return rescale_run_ragged(c, polys, n, ls.data(), in, out, scr);
}
