// fhe_internal.h -- shared definitions of the gfx950 RNS-CKKS library.
//
// Residue arithmetic runs on the FP64 vector ALU.  Every modulus is below
// 2^50, so a residue is an integer held exactly in a double, and so is the
// remainder of a product: for |a|, |b| with |a*b/q| < 2^52 the product
// a*b = h + l is split exactly with one FMA, the quotient estimate
// rint(h * (1/q)) is off by less than 2, and h - qt*q + l is computed
// exactly (it is an integer below 2^53 in magnitude).  CDNA runs FP64 FMA at
// the full vector rate, whereas 64-bit integer multiplies are built from
// quarter-rate 32-bit ones, so this is the cheap form of modular arithmetic
// on this GPU.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <cmath>
#include <string>
#include <deque>
#include <vector>

#include "fhe.h"

#define FHE_MAXMOD 64
#define FHE_LIMBTAB 128
#define TBL_ARENA_BYTES ((size_t)16 << 20)   // pointer-table ring per context

enum { OP_CT_MULT = 0, OP_CT_ADD, OP_PT_MULT, OP_PT_ADD, OP_RELIN, OP_RESCALE, OP_ROTATE, OP_KEYSWITCH };

struct Consts64 {
    double v[FHE_MAXMOD];
};

struct ModQ {
    double q;
    double qinv;   // 1/q rounded to nearest
};

// A batch of residue limbs.  Limb b lives at units[b / lpu] + (b % lpu) * N
// (or base + b * N when units is null) and is reduced modulo
// mods[mod[b % period]].
struct LimbSet {
    uint64_t *base;
    uint64_t *const *units;
    uint32_t lpu;
    uint32_t period;
    uint32_t b0;                  // limb number of blockIdx.y == 0 (large batches are split)
    uint8_t mod[FHE_LIMBTAB];
    const uint64_t *modlist;      // if set (device): limb b is reduced modulo mods[modlist[b] & 0xFFFF]
};

// ------------------------------------------------------------------ device
__device__ __forceinline__ double u64_to_f64(uint64_t x)   // x < 2^52
{
    return __hiloint2double((int)((uint32_t)(x >> 32) | 0x43300000u), (int)(uint32_t)x) -
           4503599627370496.0;
}
__device__ __forceinline__ uint64_t f64_to_u64(double x)   // integer x in [0, 2^52)
{
    return (uint64_t)__double_as_longlong(x + 4503599627370496.0) & 0x000FFFFFFFFFFFFFull;
}
__device__ __forceinline__ double bits_to_f64(uint64_t x) { return __longlong_as_double((long long)x); }
__device__ __forceinline__ uint64_t f64_to_bits(double x) { return (uint64_t)__double_as_longlong(x); }

// a*b mod q, |result| < 2q, valid when |a*b/q| < 2^52 and |a|,|b| < 2^52.
__device__ __forceinline__ double mulmod(double a, double b, double q, double qinv)
{
    double h = a * b;
    double l = __fma_rn(a, b, -h);
    double qt = __builtin_rint(h * qinv);
    double r = __fma_rn(-qt, q, h);
    return r + l;
}
// x mod q into [-q/2 - 1, q/2 + 1], valid for |x| < 2^52.
__device__ __forceinline__ double redc(double x, double q, double qinv)
{
    return __fma_rn(-__builtin_rint(x * qinv), q, x);
}
// x mod q into [0, q), valid for |x| < 2^52.
__device__ __forceinline__ double canon(double x, double q, double qinv)
{
    double r = redc(x, q, qinv);
    return r < 0.0 ? r + q : r;
}
// x in (-q, 2q) into [0, q)
__device__ __forceinline__ double fold(double x, double q)
{
    x = x < 0.0 ? x + q : x;
    return x >= q ? x - q : x;
}

// Device memory reached through a pointer table arrives as generic pointers, which the
// compiler accesses with flat instructions (those also count against the scalar-load
// counter, so every wait for a table word waits for them too): these views make the
// accesses global.
typedef __attribute__((address_space(1))) uint64_t gu64;
__device__ __forceinline__ const gu64 *gview(const uint64_t *p) { return (const gu64 *)p; }
__device__ __forceinline__ gu64 *gview(uint64_t *p) { return (gu64 *)p; }

__device__ __forceinline__ uint64_t *limb_ptr(const LimbSet &ls, uint32_t b, uint32_t N)
{
    return ls.units ? ls.units[b / ls.lpu] + (size_t)(b % ls.lpu) * N : ls.base + (size_t)b * N;
}
__device__ __forceinline__ uint32_t limb_mod(const LimbSet &ls, uint32_t b)
{
    return ls.modlist ? (uint32_t)(ls.modlist[b] & 0xFFFF) : ls.mod[b % ls.period];
}

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11).
__device__ __forceinline__ void philox4x64_10(uint64_t k0, uint64_t k1, uint64_t c0, uint64_t c1, uint64_t c2,
                                              uint64_t c3, uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; r++) {
        uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// --------------------------------------------------------------------- host
struct BconvTab {                 // one fast basis conversion S -> T
    uint32_t nsrc, ndst;
    uint32_t off;                 // offset into ctx->d_bconv (doubles)
    // layout at off: [nsrc] (B/b_i)^-1 mod b_i, [nsrc] b_i, [nsrc] 1/b_i, [ndst] c_t,
    // [ndst] 1/c_t, then [ndst][nsrc] (B/b_i) mod c_t (one target's constants adjacent)
    uint8_t src[FHE_MAXMOD], dst[FHE_MAXMOD];
};

struct fhe_ctx {
    uint32_t logN, N, L, K, dnum, alpha;
    uint64_t mod[FHE_MAXMOD];
    hipStream_t stream;
    uint64_t budget, used;
    int device;
    // device tables
    ModQ *d_mod;          // [L+K]
    double *d_tw;         // [L+K][N]  psi^brv(i)
    double *d_itw;        // [L+K][N]  psi^-brv(i)
    double *d_ninv;       // [L+K]     N^-1 mod q
    uint64_t *d_cdt;
    uint32_t ncdt;
    double *d_cos, *d_sin;   // [2N] cos/sin(pi e / N)
    uint32_t *d_g5;          // [N/2] 5^j mod 2N
    double *d_bconv;         // all basis-conversion constants
    BconvTab *modup;         // [L+1][dnum] host: level l, digit j
    BconvTab *moddown;       // [L+1] host: P -> Q_l
    double *d_pinv;          // [L]      P^-1 mod q_i
    double *d_phalf;         // [L+K]    (P-1)/2 mod m
    double *d_pmod;          // [L]      P mod q_i
    double *d_qlinv;         // [L][L]   q_l^-1 mod q_i  (row l)
    // scratch (device), grown on demand within the budget
    uint8_t *scratch;
    size_t scratch_bytes;
    // layer workspace (device): intermediates a layer keeps across the batched
    // operations it calls, which themselves use the scratch above
    uint8_t *wksp;
    size_t wksp_bytes;
    // pointer tables for batched launches: a ring over a device arena and its
    // pinned staging; a table's region is reused once the work enqueued up to the
    // next table request has completed (its release event)
    uint8_t *tbl_dev, *tbl_host;
    struct TblAlloc {
        size_t off, len;
        hipEvent_t ev;
        bool recorded;
    };
    std::deque<TblAlloc> tbl_live;
    std::vector<hipEvent_t> tbl_pool;
    uint64_t **d_big;        // oversize table (synchronous path)
    size_t d_big_cap;
    // HIP graph capture (fhe_graph_begin .. fhe_graph_end): pointer tables go to a
    // pinned arena whose device copy the graph owns; scratch may not grow
    bool capturing;
    int cap_error;
    uint8_t *cap_host, *cap_dev;
    size_t cap_bytes, cap_used;
    fhe_alloc_fn alloc_fn;   // caller's allocator for scratch and workspace (null: hipMalloc)
    fhe_free_fn free_fn;
    void *alloc_user;
    uint8_t *static_scr;     // this device's static scratch array (fhe_keyswitch_batch_static)
    bool no_alloc;           // set while a call that may not allocate runs: growth paths fail instead
    uint32_t tune_chunk;     // most items per ragged launch sequence (0: no limit)
    uint32_t tune_fuse_row_inner;   // key switch: fuse the converted limbs' row pass into the inner product
    uint32_t tune_ks_nt;            // fused key switch: non-temporal loads and stores of streamed data
    uint32_t tune_row_wg;    // rescale: row-pass workgroup cap (128 or 256)
    struct Prof *prof;       // kernel timing (HIP events), null until enabled
    uint64_t ops[8];         // operation counters, see OP_* (read and reset by fhe_op_counts)
};

// error handling
fhe_status fhe_fail(fhe_status code, const std::string &msg);
fhe_status fhe_hip_check(hipError_t e, const char *what);
#define HIPCHK(x)                                                                  \
    do {                                                                           \
        hipError_t _e = (x);                                                       \
        if (_e != hipSuccess) return fhe_hip_check(_e, #x);                        \
    } while (0)

// Scales of operands that are added must agree to 2^-40 relative (doubles carry
// 53 bits; scales computed along different branches differ by a few ulps).
inline bool scales_match(double a, double b) { return std::fabs(a / b - 1.0) <= 0x1p-40; }
// A layer output at `limbs` limbs and scale `scale` must leave FHE_SCALE_ROOM_BITS bits
// between the scale and Q_limbs / 2, so that slot values of magnitude below
// 2^(FHE_SCALE_ROOM_BITS - 1) decrypt without wrapping around the modulus.
inline bool scale_has_room(const fhe_ctx *c, uint32_t limbs, double scale)
{
    double lq = 0.0;
    for (uint32_t i = 0; i < limbs; ++i) lq += std::log2((double)c->mod[i]);
    return std::log2(scale) <= lq - 1.0 - FHE_SCALE_ROOM_BITS;
}
fhe_status scale_room_error(const char *what);

// scratch / pointer tables
fhe_status ctx_scratch(fhe_ctx *c, size_t bytes, uint8_t **out);
fhe_status ctx_workspace(fhe_ctx *c, size_t bytes, uint8_t **out);

// batched building blocks shared by the layer entry points
enum { EW_ADD = 0, EW_MULC, EW_ADDC, EW_MULPT, EW_COPY };
fhe_status ew_batch(fhe_ctx *c, int op, uint32_t l, uint32_t la, uint32_t polys, uint32_t n,
                    const uint64_t *const *a, const uint64_t *const *b, uint64_t *const *out, const Consts64 &cst);
fhe_status const_residues(const fhe_ctx *c, double v, uint32_t limbs, Consts64 *out);
fhe_status rotate_run(fhe_ctx *c, uint32_t l, uint32_t n, const uint64_t *const *in, const fhe_evk *const *keys,
                      uint64_t *const *out);
fhe_status rotate_run_ragged(fhe_ctx *c, uint32_t n, const uint32_t *ls, const uint64_t *const *in,
                             const fhe_evk *const *keys, uint64_t *const *out);
fhe_status mac_relin_rescale(fhe_ctx *c, const fhe_evk *rlk, uint32_t l, const std::vector<uint64_t *> &A,
                             const std::vector<uint64_t *> &B, const std::vector<uint32_t> &off,
                             const std::vector<uint64_t *> &Y);
fhe_status ctx_ptr_table(fhe_ctx *c, const std::vector<uint64_t *> &ptrs, uint64_t ***dev);
// Tensor products a[t] (x) b[t] -> out[t] = (a0 b0, a0 b1 + a1 b0, a1 b1), item t at ls[t] limbs.
fhe_status tensor_run(fhe_ctx *c, uint32_t n, const uint32_t *ls, const uint64_t *const *a, const uint64_t *const *b,
                      uint64_t *const *out);

// Kernel timing: when enabled for a category (or "*"), launches of that
// category are bracketed by HIP events on the context's stream.
int prof_begin(fhe_ctx *c, const char *cat);
void prof_end(fhe_ctx *c, int slot);
struct ProfScope {
    fhe_ctx *c;
    int slot;
    ProfScope(fhe_ctx *cc, const char *cat) : c(cc), slot(cc->prof ? prof_begin(cc, cat) : -1) {}
    ~ProfScope()
    {
        if (slot >= 0) prof_end(c, slot);
    }
};

// shared drivers (ops.hip)
size_t ks_scratch_bytes(const fhe_ctx *c, uint32_t l, uint32_t n);
// n key switches: inputs d[b] read through the Galois permutation gal[b] (gal null or
// 0: none), keys evk[b], outputs out[b] (2 polys), addends add[2b + t] (null or a
// polynomial read through gal[b]) added to output polynomial t.  scr: scratch of
// ks_scratch_bytes(l, n) bytes, or null to take the context's.
fhe_status ks_run(fhe_ctx *c, uint32_t l, uint32_t n, const uint64_t *const *d, const uint32_t *gal,
                  const uint64_t *const *evk, uint64_t *const *out, const uint64_t *const *add, uint8_t *scr);
// The same for items at different levels: item b has ls[b] limbs (input, output,
// addends); scratch of ks_scratch_bytes_ragged(n, ls) bytes.
size_t ks_scratch_bytes_ragged(const fhe_ctx *c, uint32_t n, const uint32_t *ls);
fhe_status ks_run_ragged(fhe_ctx *c, uint32_t n, const uint32_t *ls, const uint64_t *const *d, const uint32_t *gal,
                         const uint64_t *const *evk, uint64_t *const *out, const uint64_t *const *add, uint8_t *scr);
size_t rescale_scratch_bytes(const fhe_ctx *c, uint32_t l, uint32_t polys, uint32_t n);
fhe_status rescale_run(fhe_ctx *c, uint32_t l, uint32_t polys, uint32_t n, const uint64_t *const *in,
                       uint64_t *const *out, uint8_t *scr);
// Rescale of items at different levels (item b: ls[b] limbs in, ls[b] - 1 out).
size_t rescale_scratch_bytes_ragged(const fhe_ctx *c, uint32_t polys, uint32_t n, const uint32_t *ls);
fhe_status rescale_run_ragged(fhe_ctx *c, uint32_t polys, uint32_t n, const uint32_t *ls, const uint64_t *const *in,
                              uint64_t *const *out, uint8_t *scr);
void launch_automorph(fhe_ctx *c, const uint64_t *in, uint64_t *out, uint32_t nlimbs, uint64_t g);

// launchers (ntt.hip)
void launch_ntt_fwd(fhe_ctx *c, const LimbSet &ls, uint32_t nlimbs);
void launch_ntt_inv(fhe_ctx *c, const LimbSet &ls, uint32_t nlimbs);
LimbSet limbset_range(uint64_t *base, uint32_t first_mod, uint32_t count, uint32_t period_mods);
LimbSet limbset_list(uint64_t *base, const uint32_t *mods, uint32_t period);
