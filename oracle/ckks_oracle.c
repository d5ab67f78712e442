/*
 * ckks_oracle.c -- plain, slow, single-threaded CPU reference of full-RNS CKKS.
 *
 * TEST INFRASTRUCTURE ONLY (test suite, smoke check, CPU-baseline timing).
 * It is deliberately naive: every modular product goes through a 128-bit
 * integer and `%`, the NTT is the textbook radix-2 transform, and the basis
 * conversion is the defining sum written out.  No blocking, fusion or lazy
 * reduction.  Pinned by the Python tests in tests/test_oracle_*.py.
 */
#include "ckks_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
typedef __int128 i128;
typedef uint64_t u64;

struct or_ctx {
    uint32_t logN, N, L, K, dnum, alpha;
    u64 mod[OR_MAXMOD];
    u64 psi[OR_MAXMOD];
    double *cosv, *sinv;        /* cos/sin(pi*e/N), e in [0, 2N) */
};

/* ---------------------------------------------------------------- helpers */
static u64 mulm(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }
static u64 addm(u64 a, u64 b, u64 q) { u128 s = (u128)a + b; return (u64)(s % q); }
static u64 subm(u64 a, u64 b, u64 q) { return (u64)(((u128)a + q - (b % q)) % q); }
static u64 powm(u64 a, u64 e, u64 q)
{
    u64 r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = mulm(r, a, q);
        a = mulm(a, a, q);
        e >>= 1;
    }
    return r;
}
static u64 invm(u64 a, u64 q) { return powm(a, q - 2, q); }   /* q prime */
static u64 smod(int64_t v, u64 q)                            /* signed -> [0,q) */
{
    i128 r = (i128)v % (i128)q;
    if (r < 0) r += q;
    return (u64)r;
}

/* ------------------------------------------------------------- primality */
int or_is_prime(u64 n)
{
    static const u64 bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (n == bases[i]) return 1;
        if (n % bases[i] == 0) return 0;
    }
    u64 d = n - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; s++; }
    for (int i = 0; i < 12; i++) {
        u64 x = powm(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int comp = 1;
        for (int r = 1; r < s; r++) {
            x = mulm(x, x, n);
            if (x == n - 1) { comp = 0; break; }
        }
        if (comp) return 0;
    }
    return 1;
}

/* Smallest primitive 2N-th root of unity mod q: find one root w of order 2N
 * (w^N == -1), then take the minimum over its odd powers (all the others). */
u64 or_min_psi(u64 q, uint32_t N)
{
    u64 w = 0;
    for (u64 x = 2; x < q; x++) {
        u64 c = powm(x, (q - 1) / (2 * (u64)N), q);
        if (powm(c, N, q) == q - 1) { w = c; break; }
    }
    if (!w) return 0;
    u64 best = w, w2 = mulm(w, w, q), cur = w;
    for (uint32_t k = 1; k < N; k++) {      /* w^(2k+1) */
        cur = mulm(cur, w2, q);
        if (cur < best) best = cur;
    }
    return best;
}

/* ---------------------------------------------------------------- context */
or_ctx *or_ctx_new(uint32_t logN, const u64 *q, uint32_t L, const u64 *p, uint32_t K, uint32_t dnum)
{
    if (logN < 1 || logN > 17 || L < 1 || L + K > OR_MAXMOD || dnum < 1 || dnum > L) return NULL;
    or_ctx *c = (or_ctx *)calloc(1, sizeof(or_ctx));
    c->logN = logN; c->N = 1u << logN; c->L = L; c->K = K; c->dnum = dnum;
    c->alpha = (L + dnum - 1) / dnum;
    for (uint32_t i = 0; i < L; i++) c->mod[i] = q[i];
    for (uint32_t j = 0; j < K; j++) c->mod[L + j] = p[j];
    for (uint32_t i = 0; i < L + K; i++) {
        u64 m = c->mod[i];
        int bad = m >= (1ull << 62) || !or_is_prime(m) || (m - 1) % (2ull * c->N) != 0;
        for (uint32_t j = 0; j < i; j++) bad |= c->mod[j] == m;
        if (bad) { free(c); return NULL; }
        c->psi[i] = or_min_psi(m, c->N);
    }
    c->cosv = (double *)malloc(sizeof(double) * 2 * c->N);
    c->sinv = (double *)malloc(sizeof(double) * 2 * c->N);
    for (uint32_t e = 0; e < 2 * c->N; e++) {
        double ang = M_PI * (double)e / (double)c->N;
        c->cosv[e] = cos(ang);
        c->sinv[e] = sin(ang);
    }
    return c;
}
void or_ctx_free(or_ctx *c)
{
    if (!c) return;
    free(c->cosv); free(c->sinv); free(c);
}
u64 or_modulus(const or_ctx *c, uint32_t idx) { return c->mod[idx]; }
u64 or_psi(const or_ctx *c, uint32_t idx) { return c->psi[idx]; }
uint32_t or_alpha(const or_ctx *c) { return c->alpha; }

/* -------------------------------------------------------------------- NTT */
static uint32_t bitrev(uint32_t x, uint32_t bits)
{
    uint32_t r = 0;
    for (uint32_t i = 0; i < bits; i++) { r = (r << 1) | (x & 1); x >>= 1; }
    return r;
}
/* In-place cyclic DFT of length N with root w (textbook iterative radix-2). */
static void dft_cyclic(u64 *a, uint32_t N, uint32_t logN, u64 w, u64 q)
{
    for (uint32_t i = 0; i < N; i++) {
        uint32_t j = bitrev(i, logN);
        if (i < j) { u64 t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    for (uint32_t len = 2; len <= N; len <<= 1) {
        u64 wl = powm(w, N / len, q);
        for (uint32_t i = 0; i < N; i += len) {
            u64 wk = 1;
            for (uint32_t j = 0; j < len / 2; j++) {
                u64 u = a[i + j], v = mulm(a[i + j + len / 2], wk, q);
                a[i + j] = addm(u, v, q);
                a[i + j + len / 2] = subm(u, v, q);
                wk = mulm(wk, wl, q);
            }
        }
    }
}
/* Negacyclic evaluation: out[k] = sum_i a_i psi^(i(2k+1)) = a(psi^(2k+1)). */
void or_ntt(const or_ctx *c, uint32_t m, const u64 *a, u64 *out)
{
    u64 q = c->mod[m], psi = c->psi[m], pw = 1;
    for (uint32_t i = 0; i < c->N; i++) { out[i] = mulm(a[i], pw, q); pw = mulm(pw, psi, q); }
    dft_cyclic(out, c->N, c->logN, mulm(psi, psi, q), q);
}
void or_intt(const or_ctx *c, uint32_t m, const u64 *a, u64 *out)
{
    u64 q = c->mod[m], psii = invm(c->psi[m], q);
    memcpy(out, a, sizeof(u64) * c->N);
    dft_cyclic(out, c->N, c->logN, mulm(psii, psii, q), q);
    u64 ninv = invm(c->N % q, q), pw = ninv;
    for (uint32_t i = 0; i < c->N; i++) { out[i] = mulm(out[i], pw, q); pw = mulm(pw, psii, q); }
}
void or_polymul(const or_ctx *c, uint32_t m, const u64 *a, const u64 *b, u64 *out)
{
    u64 q = c->mod[m];
    u64 *A = (u64 *)malloc(sizeof(u64) * c->N), *B = (u64 *)malloc(sizeof(u64) * c->N);
    or_ntt(c, m, a, A);
    or_ntt(c, m, b, B);
    for (uint32_t i = 0; i < c->N; i++) A[i] = mulm(A[i], B[i], q);
    or_intt(c, m, A, out);
    free(A); free(B);
}

/* ----------------------------------------------------------------- Philox */
#define PH_M0 0xD2E7470EE14C6C93ull
#define PH_M1 0xCA5A826395121157ull
#define PH_W0 0x9E3779B97F4A7C15ull
#define PH_W1 0xBB67AE8584CAA73Bull
void or_philox4x64_10(const u64 key[2], const u64 ctr[4], u64 out[4])
{
    u64 x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3], k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r) { k0 += PH_W0; k1 += PH_W1; }
        u128 p0 = (u128)PH_M0 * x0, p1 = (u128)PH_M1 * x2;
        u64 y0 = (u64)(p1 >> 64) ^ x1 ^ k0;
        u64 y1 = (u64)p1;
        u64 y2 = (u64)(p0 >> 64) ^ x3 ^ k1;
        u64 y3 = (u64)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ---------------------------------------------------------------- samplers
 * Key = (seed, tag).  Counter = (coefficient, modulus index or 0, poly id, round).
 * Uniform mod q: each 64-bit word of the block, masked to bitlen(q), is tried
 * in order; the first one below q is taken; a fully rejected block moves to
 * the next round.
 * Ternary: the low 32 bits u of each word, rejected if u >= 3*floor(2^32/3);
 * value (u mod 3) - 1.
 * Gaussian (sigma = 3.2, |e| <= ncdt): magnitude = #{i : cdt[i] <= w0} with
 * cdt[i] = floor(2^64 * P(|e| <= i)); negative when nonzero and w1 is odd. */
static uint32_t bitlen(u64 x) { uint32_t b = 0; while (x) { b++; x >>= 1; } return b; }

void or_sample_uniform(const or_ctx *c, u64 seed, u64 tag, u64 poly_id, uint32_t nlimbs,
                       const uint32_t *modidx, u64 *out)
{
    u64 key[2] = {seed, tag}, blk[4];
    for (uint32_t li = 0; li < nlimbs; li++) {
        u64 q = c->mod[modidx[li]];
        uint32_t b = bitlen(q);
        u64 mask = b >= 64 ? ~0ull : ((1ull << b) - 1);
        for (uint32_t k = 0; k < c->N; k++) {
            u64 val = 0;
            int found = 0;
            for (u64 round = 0; !found; round++) {
                u64 ctr[4] = {k, modidx[li], poly_id, round};
                or_philox4x64_10(key, ctr, blk);
                for (int w = 0; w < 4 && !found; w++) {
                    u64 x = blk[w] & mask;
                    if (x < q) { val = x; found = 1; }
                }
            }
            out[(size_t)li * c->N + k] = val;
        }
    }
}
void or_sample_ternary(const or_ctx *c, u64 seed, u64 tag, u64 poly_id, int64_t *out)
{
    u64 key[2] = {seed, tag}, blk[4];
    const u64 lim = 3ull * (0x100000000ull / 3);
    for (uint32_t k = 0; k < c->N; k++) {
        int found = 0;
        for (u64 round = 0; !found; round++) {
            u64 ctr[4] = {k, 0, poly_id, round};
            or_philox4x64_10(key, ctr, blk);
            for (int w = 0; w < 4 && !found; w++) {
                u64 u = blk[w] & 0xffffffffull;
                if (u < lim) { out[k] = (int64_t)(u % 3) - 1; found = 1; }
            }
        }
    }
}
void or_sample_gauss(const or_ctx *c, u64 seed, u64 tag, u64 poly_id, const u64 *cdt,
                     uint32_t ncdt, int64_t *out)
{
    u64 key[2] = {seed, tag}, blk[4];
    for (uint32_t k = 0; k < c->N; k++) {
        u64 ctr[4] = {k, 0, poly_id, 0};
        or_philox4x64_10(key, ctr, blk);
        int64_t mag = 0;
        for (uint32_t i = 0; i < ncdt; i++) mag += cdt[i] <= blk[0];
        out[k] = (mag != 0 && (blk[1] & 1)) ? -mag : mag;
    }
}
void or_small_to_rns(const or_ctx *c, const int64_t *a, uint32_t nlimbs, const uint32_t *modidx, u64 *out)
{
    for (uint32_t li = 0; li < nlimbs; li++)
        for (uint32_t k = 0; k < c->N; k++) out[(size_t)li * c->N + k] = smod(a[k], c->mod[modidx[li]]);
}

/* ------------------------------------------------------------------- keys */
void or_keygen_secret(const or_ctx *c, u64 seed, int64_t *s)
{
    or_sample_ternary(c, seed, OR_TAG_SECRET, 0, s);
}
void or_square_small(const or_ctx *c, const int64_t *s, int64_t *out)
{
    uint32_t N = c->N;
    for (uint32_t k = 0; k < N; k++) out[k] = 0;
    for (uint32_t i = 0; i < N; i++)
        for (uint32_t j = 0; j < N; j++) {
            int64_t v = s[i] * s[j];
            if (i + j < N) out[i + j] += v; else out[i + j - N] -= v;
        }
}
void or_automorph_small(const or_ctx *c, const int64_t *s, u64 g, int64_t *out)
{
    uint32_t N = c->N;
    for (uint32_t i = 0; i < N; i++) {
        u64 t = ((u64)i * g) % (2ull * N);
        if (t < N) out[t] = s[i]; else out[t - N] = -s[i];
    }
}
u64 or_galois_elt(const or_ctx *c, int64_t r)
{
    int64_t n = c->N / 2;
    int64_t rr = ((r % n) + n) % n;
    return powm(5, (u64)rr, 2ull * c->N);
}
/* b = -a*s + e on every listed limb (coefficient domain). */
static void rlwe_sample(const or_ctx *c, const int64_t *s, const int64_t *e, const u64 *a,
                        uint32_t nlimbs, const uint32_t *modidx, u64 *b)
{
    uint32_t N = c->N;
    u64 *sr = (u64 *)malloc(sizeof(u64) * N), *t = (u64 *)malloc(sizeof(u64) * N);
    for (uint32_t li = 0; li < nlimbs; li++) {
        uint32_t m = modidx[li];
        u64 q = c->mod[m];
        for (uint32_t k = 0; k < N; k++) sr[k] = smod(s[k], q);
        or_polymul(c, m, a + (size_t)li * N, sr, t);
        for (uint32_t k = 0; k < N; k++) b[(size_t)li * N + k] = subm(smod(e[k], q), t[k], q);
    }
    free(sr); free(t);
}
void or_keygen_pk(const or_ctx *c, const int64_t *s, u64 seed, const u64 *cdt, uint32_t ncdt, u64 *pk)
{
    uint32_t N = c->N, L = c->L, idx[OR_MAXMOD];
    for (uint32_t i = 0; i < L; i++) idx[i] = i;
    int64_t *e = (int64_t *)malloc(sizeof(int64_t) * N);
    u64 *a = pk + (size_t)L * N;
    or_sample_uniform(c, seed, OR_TAG_UNIFORM, 0, L, idx, a);
    or_sample_gauss(c, seed, OR_TAG_ERROR, 0, cdt, ncdt, e);
    rlwe_sample(c, s, e, a, L, idx, pk);
    free(e);
}
/* Hybrid key-switching key from s_from to s: for digit j (limbs D_j of Q),
 * evk_j = (-a_j s + e_j + P * [Q^_j (Q^_j)^-1]_{Q_j} * s_from, a_j) over Q u P.
 * Mod q_i the gadget factor is P mod q_i for i in D_j and 0 elsewhere;
 * mod every special prime it is 0. */
void or_keygen_evk(const or_ctx *c, const int64_t *s, const int64_t *s_from, u64 seed,
                   const u64 *cdt, uint32_t ncdt, u64 *evk)
{
    uint32_t N = c->N, L = c->L, K = c->K, n = L + K, idx[OR_MAXMOD];
    for (uint32_t i = 0; i < n; i++) idx[i] = i;
    int64_t *e = (int64_t *)malloc(sizeof(int64_t) * N);
    for (uint32_t j = 0; j < c->dnum; j++) {
        u64 *b = evk + (size_t)j * 2 * n * N, *a = b + (size_t)n * N;
        or_sample_uniform(c, seed, OR_TAG_UNIFORM, j, n, idx, a);
        or_sample_gauss(c, seed, OR_TAG_ERROR, j, cdt, ncdt, e);
        rlwe_sample(c, s, e, a, n, idx, b);
        uint32_t lo = j * c->alpha, hi = lo + c->alpha < L ? lo + c->alpha : L;
        for (uint32_t i = lo; i < hi; i++) {
            u64 q = c->mod[i], pm = 1;
            for (uint32_t t = 0; t < K; t++) pm = mulm(pm, c->mod[L + t] % q, q);
            for (uint32_t k = 0; k < N; k++)
                b[(size_t)i * N + k] = addm(b[(size_t)i * N + k], mulm(pm, smod(s_from[k], q), q), q);
        }
    }
    free(e);
}

/* ---------------------------------------------------- encrypt / decrypt */
void or_encrypt(const or_ctx *c, const u64 *pk, const u64 *m, uint32_t l, u64 seed,
                const u64 *cdt, uint32_t ncdt, u64 *ct)
{
    uint32_t N = c->N, L = c->L;
    int64_t *v = (int64_t *)malloc(sizeof(int64_t) * N), *e0 = (int64_t *)malloc(sizeof(int64_t) * N),
            *e1 = (int64_t *)malloc(sizeof(int64_t) * N);
    u64 *vr = (u64 *)malloc(sizeof(u64) * N), *t = (u64 *)malloc(sizeof(u64) * N);
    or_sample_ternary(c, seed, OR_TAG_EPHEMERAL, 0, v);
    or_sample_gauss(c, seed, OR_TAG_ERROR, 0, cdt, ncdt, e0);
    or_sample_gauss(c, seed, OR_TAG_ERROR, 1, cdt, ncdt, e1);
    for (uint32_t i = 0; i < l; i++) {
        u64 q = c->mod[i];
        for (uint32_t k = 0; k < N; k++) vr[k] = smod(v[k], q);
        or_polymul(c, i, pk + (size_t)i * N, vr, t);                       /* v*b */
        for (uint32_t k = 0; k < N; k++)
            ct[(size_t)i * N + k] = addm(addm(t[k], smod(e0[k], q), q), m[(size_t)i * N + k], q);
        or_polymul(c, i, pk + (size_t)(L + i) * N, vr, t);                 /* v*a */
        for (uint32_t k = 0; k < N; k++)
            ct[(size_t)(l + i) * N + k] = addm(t[k], smod(e1[k], q), q);
    }
    free(v); free(e0); free(e1); free(vr); free(t);
}
/* m = c0 + c1*s (+ c2*s^2). */
void or_decrypt(const or_ctx *c, const u64 *ct, uint32_t npolys, uint32_t l, const int64_t *s, u64 *m)
{
    uint32_t N = c->N;
    u64 *sr = (u64 *)malloc(sizeof(u64) * N), *s2 = (u64 *)malloc(sizeof(u64) * N),
        *t = (u64 *)malloc(sizeof(u64) * N);
    for (uint32_t i = 0; i < l; i++) {
        u64 q = c->mod[i];
        for (uint32_t k = 0; k < N; k++) sr[k] = smod(s[k], q);
        for (uint32_t k = 0; k < N; k++) m[(size_t)i * N + k] = ct[(size_t)i * N + k];
        or_polymul(c, i, ct + (size_t)(l + i) * N, sr, t);
        for (uint32_t k = 0; k < N; k++) m[(size_t)i * N + k] = addm(m[(size_t)i * N + k], t[k], q);
        if (npolys == 3) {
            or_polymul(c, i, sr, sr, s2);
            or_polymul(c, i, ct + (size_t)(2 * l + i) * N, s2, t);
            for (uint32_t k = 0; k < N; k++) m[(size_t)i * N + k] = addm(m[(size_t)i * N + k], t[k], q);
        }
    }
    free(sr); free(s2); free(t);
}

/* --------------------------------------------------------------- encoding
 * Slot j <-> evaluation at zeta^(5^j mod 2N), zeta = exp(i*pi/N), j < N/2.
 * The real polynomial m with m(zeta_j) = scale*z_j (and conjugates) has
 *   m_k = (2/N) * sum_j Re(scale * z_j * zeta^(-k*5^j))
 *       = (2*scale/N) * sum_j (re_j cos(pi e/N) + im_j sin(pi e/N)),  e = k*5^j mod 2N,
 * rounded to the nearest integer (ties to even).  Direct O(N*n) sums. */
int or_encode(const or_ctx *c, const double *re, const double *im, uint32_t n, double scale, int64_t *coeff)
{
    uint32_t N = c->N, twoN = 2 * N, nslots = N / 2;
    if (n > nslots) return -1;
    u64 *g = (u64 *)malloc(sizeof(u64) * (n ? n : 1));
    u64 gj = 1;
    for (uint32_t j = 0; j < n; j++) { g[j] = gj; gj = (gj * 5) % twoN; }
    int rc = 0;
    for (uint32_t k = 0; k < N; k++) {
        double acc = 0.0;
        for (uint32_t j = 0; j < n; j++) {
            u64 e = ((u64)k * g[j]) % twoN;
            acc += re[j] * c->cosv[e];
            if (im) acc += im[j] * c->sinv[e];
        }
        double v = rint(acc * (2.0 / (double)N) * scale);
        if (!(fabs(v) < 4611686018427387904.0)) { rc = -1; v = 0; }
        coeff[k] = (int64_t)v;
    }
    free(g);
    return rc;
}
/* Centered lift from limb 0 alone (l == 1) or limbs 0,1 by CRT (l >= 2), then
 *   re_j = (1/scale) sum_k m_k cos(pi e/N),  im_j = (1/scale) sum_k m_k sin(pi e/N),  e = k*5^j mod 2N. */
void or_decode(const or_ctx *c, const u64 *m, uint32_t l, double scale, double *re, double *im, uint32_t n)
{
    uint32_t N = c->N, twoN = 2 * N;
    double *mv = (double *)malloc(sizeof(double) * N);
    u64 q0 = c->mod[0];
    for (uint32_t k = 0; k < N; k++) {
        if (l == 1) {
            u64 x = m[k];
            mv[k] = x > q0 / 2 ? -(double)(q0 - x) : (double)x;
        } else {
            u64 q1 = c->mod[1], x0 = m[k], x1 = m[(size_t)N + k];
            /* x = x0 + q0 * [(x1 - x0) * q0^-1 mod q1] */
            u64 t = mulm(subm(x1, x0 % q1, q1), invm(q0 % q1, q1), q1);
            u128 Q = (u128)q0 * q1, x = (u128)x0 + (u128)q0 * t;
            mv[k] = x > Q / 2 ? -(double)(Q - x) : (double)x;
        }
    }
    u64 gj = 1;
    for (uint32_t j = 0; j < n; j++) {
        double ar = 0.0, ai = 0.0;
        for (uint32_t k = 0; k < N; k++) {
            u64 e = ((u64)k * gj) % twoN;
            ar += mv[k] * c->cosv[e];
            ai += mv[k] * c->sinv[e];
        }
        re[j] = ar / scale;
        if (im) im[j] = ai / scale;
        gj = (gj * 5) % twoN;
    }
    free(mv);
}

/* ------------------------------------------------------ homomorphic ops */
void or_add(const or_ctx *c, const u64 *a, const u64 *b, uint32_t np, uint32_t l, u64 *out)
{
    for (uint32_t p = 0; p < np; p++)
        for (uint32_t i = 0; i < l; i++)
            for (uint32_t k = 0; k < c->N; k++) {
                size_t x = ((size_t)p * l + i) * c->N + k;
                out[x] = addm(a[x], b[x], c->mod[i]);
            }
}
void or_sub(const or_ctx *c, const u64 *a, const u64 *b, uint32_t np, uint32_t l, u64 *out)
{
    for (uint32_t p = 0; p < np; p++)
        for (uint32_t i = 0; i < l; i++)
            for (uint32_t k = 0; k < c->N; k++) {
                size_t x = ((size_t)p * l + i) * c->N + k;
                out[x] = subm(a[x], b[x], c->mod[i]);
            }
}
void or_mul_pt(const or_ctx *c, const u64 *ct, const u64 *pt, uint32_t l, u64 *out)
{
    for (uint32_t p = 0; p < 2; p++)
        for (uint32_t i = 0; i < l; i++)
            or_polymul(c, i, ct + ((size_t)p * l + i) * c->N, pt + (size_t)i * c->N,
                       out + ((size_t)p * l + i) * c->N);
}
void or_add_pt(const or_ctx *c, const u64 *ct, const u64 *pt, uint32_t l, u64 *out)
{
    size_t n = (size_t)l * c->N;
    for (uint32_t i = 0; i < l; i++)
        for (uint32_t k = 0; k < c->N; k++) {
            size_t x = (size_t)i * c->N + k;
            out[x] = addm(ct[x], pt[x], c->mod[i]);
            out[n + x] = ct[n + x];
        }
}
void or_mul_const(const or_ctx *c, const u64 *ct, uint32_t np, uint32_t l, const u64 *cres, u64 *out)
{
    for (uint32_t p = 0; p < np; p++)
        for (uint32_t i = 0; i < l; i++)
            for (uint32_t k = 0; k < c->N; k++) {
                size_t x = ((size_t)p * l + i) * c->N + k;
                out[x] = mulm(ct[x], cres[i], c->mod[i]);
            }
}
/* (a0 b0, a0 b1 + a1 b0, a1 b1) */
void or_tensor(const or_ctx *c, const u64 *a, const u64 *b, uint32_t l, u64 *out3)
{
    uint32_t N = c->N;
    u64 *t = (u64 *)malloc(sizeof(u64) * N);
    for (uint32_t i = 0; i < l; i++) {
        u64 q = c->mod[i];
        const u64 *a0 = a + (size_t)i * N, *a1 = a + (size_t)(l + i) * N;
        const u64 *b0 = b + (size_t)i * N, *b1 = b + (size_t)(l + i) * N;
        u64 *d0 = out3 + (size_t)i * N, *d1 = out3 + (size_t)(l + i) * N, *d2 = out3 + (size_t)(2 * l + i) * N;
        or_polymul(c, i, a0, b0, d0);
        or_polymul(c, i, a0, b1, d1);
        or_polymul(c, i, a1, b0, t);
        for (uint32_t k = 0; k < N; k++) d1[k] = addm(d1[k], t[k], q);
        or_polymul(c, i, a1, b1, d2);
    }
    free(t);
}
/* acc3 = sum_t a_t (x) b_t, in list order. */
void or_mul_acc(const or_ctx *c, const u64 *const *a, const u64 *const *b, uint32_t n, uint32_t l, u64 *acc3)
{
    size_t sz = (size_t)3 * l * c->N;
    u64 *t = (u64 *)malloc(sizeof(u64) * sz);
    memset(acc3, 0, sizeof(u64) * sz);
    for (uint32_t j = 0; j < n; j++) {
        or_tensor(c, a[j], b[j], l, t);
        or_add(c, acc3, t, 3, l, acc3);
    }
    free(t);
}

/* Fast basis conversion without correction (full-RNS CKKS):
 *   y_c = sum_i [x_i * (B/b_i)^-1]_{b_i} * (B/b_i mod c)   mod c. */
void or_bconv(const or_ctx *c, const u64 *x, const uint32_t *src, uint32_t nsrc, const uint32_t *dst,
              uint32_t ndst, u64 *y)
{
    uint32_t N = c->N;
    for (uint32_t d = 0; d < ndst; d++) {
        u64 cm = c->mod[dst[d]];
        for (uint32_t k = 0; k < N; k++) y[(size_t)d * N + k] = 0;
        for (uint32_t i = 0; i < nsrc; i++) {
            u64 bi = c->mod[src[i]], bhat_i = 1, bhat_c = 1;
            for (uint32_t t = 0; t < nsrc; t++)
                if (t != i) {
                    bhat_i = mulm(bhat_i, c->mod[src[t]] % bi, bi);
                    bhat_c = mulm(bhat_c, c->mod[src[t]] % cm, cm);
                }
            u64 binv = invm(bhat_i, bi);
            for (uint32_t k = 0; k < N; k++) {
                u64 v = mulm(x[(size_t)i * N + k], binv, bi);
                y[(size_t)d * N + k] = addm(y[(size_t)d * N + k], mulm(v % cm, bhat_c, cm), cm);
            }
        }
    }
}

/* X -> X^g on one coefficient-domain polynomial modulo q (g odd): coefficient i moves
 * to i*g mod 2N, negated when that lands in [N, 2N). */
static void automorph_mod(uint32_t N, const u64 *a, u64 q, u64 g, u64 *out)
{
    for (uint32_t i = 0; i < N; i++) {
        u64 t = ((u64)i * g) % (2ull * N), v = a[i];
        if (t < N) out[t] = v;
        else out[t - N] = v ? q - v : 0;
    }
}

/* Hybrid key switch of d (l limbs) with evk [dnum][2][L+K][N]:
 *   ModUp:  D_j = [d]_{Q_j} extended to Q_l u P by basis conversion (original limbs kept);
 *           with g != 1 every limb of D_j then goes through X -> X^g (see or_keyswitch_galois);
 *   inner:  u_t = sum_j D_j * evk_{j,t}  over Q_l u P;
 *   ModDown: ks_t = (u'_t - Conv_{P->Q_l}([u'_t]_P)) * P^-1 mod q_i,  u'_t = u_t + (P-1)/2,
 *            i.e. u_t / P rounded (up to the fast-conversion error). */
static void keyswitch_core(const or_ctx *c, const u64 *d, uint32_t l, const u64 *evk, u64 g, u64 *ks)
{
    uint32_t N = c->N, L = c->L, K = c->K, nx = l + K, nevk = L + K;
    uint32_t ext[OR_MAXMOD], pidx[OR_MAXMOD], qidx[OR_MAXMOD];
    for (uint32_t i = 0; i < l; i++) ext[i] = qidx[i] = i;
    for (uint32_t t = 0; t < K; t++) ext[l + t] = pidx[t] = L + t;
    u64 *u = (u64 *)calloc((size_t)2 * nx * N, sizeof(u64));
    u64 *D = (u64 *)malloc(sizeof(u64) * (size_t)nx * N), *tmp = (u64 *)malloc(sizeof(u64) * (size_t)nx * N);
    uint32_t nd = (l + c->alpha - 1) / c->alpha;
    for (uint32_t j = 0; j < nd; j++) {
        uint32_t lo = j * c->alpha, hi = lo + c->alpha < l ? lo + c->alpha : l;
        uint32_t src[OR_MAXMOD], dst[OR_MAXMOD], dpos[OR_MAXMOD], ns = 0, ndst = 0;
        for (uint32_t i = lo; i < hi; i++) src[ns++] = i;
        for (uint32_t x = 0; x < nx; x++)
            if (!(ext[x] >= lo && ext[x] < hi)) { dst[ndst] = ext[x]; dpos[ndst++] = x; }
        or_bconv(c, d + (size_t)lo * N, src, ns, dst, ndst, tmp);
        for (uint32_t i = lo; i < hi; i++) memcpy(D + (size_t)i * N, d + (size_t)i * N, sizeof(u64) * N);
        for (uint32_t t = 0; t < ndst; t++) memcpy(D + (size_t)dpos[t] * N, tmp + (size_t)t * N, sizeof(u64) * N);
        if (g != 1)
            for (uint32_t x = 0; x < nx; x++) {
                automorph_mod(N, D + (size_t)x * N, c->mod[ext[x]], g, tmp);
                memcpy(D + (size_t)x * N, tmp, sizeof(u64) * N);
            }
        const u64 *ej = evk + (size_t)j * 2 * nevk * N;
        for (uint32_t t = 0; t < 2; t++)
            for (uint32_t x = 0; x < nx; x++) {
                uint32_t m = ext[x];
                or_polymul(c, m, D + (size_t)x * N, ej + ((size_t)t * nevk + m) * N, tmp);
                u64 *ut = u + ((size_t)t * nx + x) * N;
                for (uint32_t k = 0; k < N; k++) ut[k] = addm(ut[k], tmp[k], c->mod[m]);
            }
    }
    /* Rounded ModDown: work on u' = u + (P-1)/2 so that the floor of u'/P is the
     * nearest integer to u/P (exactly so when K = 1). */
    for (uint32_t x = 0; x < nx; x++) {
        u64 m = c->mod[ext[x]], h = 1;
        for (uint32_t s = 0; s < K; s++) h = mulm(h, c->mod[L + s] % m, m);
        h = mulm(subm(h, 1, m), invm(2 % m, m), m);              /* (P-1)/2 mod m */
        for (uint32_t t = 0; t < 2; t++)
            for (uint32_t k = 0; k < N; k++) {
                u64 *v = u + ((size_t)t * nx + x) * N + k;
                *v = addm(*v, h, m);
            }
    }
    for (uint32_t t = 0; t < 2; t++) {
        u64 *ut = u + (size_t)t * nx * N;
        or_bconv(c, ut + (size_t)l * N, pidx, K, qidx, l, tmp);
        for (uint32_t i = 0; i < l; i++) {
            u64 q = c->mod[i], pm = 1;
            for (uint32_t s = 0; s < K; s++) pm = mulm(pm, c->mod[L + s] % q, q);
            u64 pinv = invm(pm, q);
            for (uint32_t k = 0; k < N; k++)
                ks[((size_t)t * l + i) * N + k] = mulm(subm(ut[(size_t)i * N + k], tmp[(size_t)i * N + k], q), pinv, q);
        }
    }
    free(u); free(D); free(tmp);
}
void or_keyswitch(const or_ctx *c, const u64 *d, uint32_t l, const u64 *evk, u64 *ks)
{
    keyswitch_core(c, d, l, evk, 1, ks);
}
/* The key switch of sigma_g(d) that a rotation uses: the digits of d itself are
 * extended, and X -> X^g is applied to every extended digit limb before the inner
 * product.  The automorphism commutes with the digit decomposition, but the fast
 * conversion of a negated coefficient differs from the negated conversion by a
 * multiple of Q_j, so the result is another valid key switch of sigma_g(d) than
 * or_keyswitch(sigma_g(d)); its extension does not depend on g, so rotations of
 * one ciphertext by several steps can share it. */
void or_keyswitch_galois(const or_ctx *c, const u64 *d, uint32_t l, const u64 *evk, u64 g, u64 *ks)
{
    keyswitch_core(c, d, l, evk, g, ks);
}
void or_relin(const or_ctx *c, const u64 *ct3, uint32_t l, const u64 *rlk, u64 *out2)
{
    size_t n = (size_t)l * c->N;
    u64 *ks = (u64 *)malloc(sizeof(u64) * 2 * n);
    or_keyswitch(c, ct3 + 2 * n, l, rlk, ks);
    or_add(c, ct3, ks, 2, l, out2);
    free(ks);
}
/* Divide by the last prime with rounding: r = [c]_{q_last} lifted to
 * (-q_last/2, q_last/2];  c'_i = (c_i - r) * q_last^-1 mod q_i. */
int or_rescale(const or_ctx *c, const u64 *ct, uint32_t np, uint32_t l, u64 *out)
{
    if (l < 2) return -1;
    uint32_t N = c->N;
    u64 ql = c->mod[l - 1];
    for (uint32_t p = 0; p < np; p++) {
        const u64 *last = ct + ((size_t)p * l + l - 1) * N;
        for (uint32_t i = 0; i < l - 1; i++) {
            u64 q = c->mod[i], qinv = invm(ql % q, q);
            for (uint32_t k = 0; k < N; k++) {
                int64_t r = last[k] > ql / 2 ? -(int64_t)(ql - last[k]) : (int64_t)last[k];
                out[((size_t)p * (l - 1) + i) * N + k] = mulm(subm(ct[((size_t)p * l + i) * N + k], smod(r, q), q), qinv, q);
            }
        }
    }
    return 0;
}
/* sigma_g: X^i -> X^(i g mod 2N), with X^N = -1. */
void or_automorph(const or_ctx *c, const u64 *a, uint32_t nlimbs, u64 g, u64 *out)
{
    uint32_t N = c->N;
    for (uint32_t li = 0; li < nlimbs; li++) {
        u64 q = c->mod[li];
        for (uint32_t i = 0; i < N; i++) {
            u64 t = ((u64)i * g) % (2ull * N), v = a[(size_t)li * N + i];
            if (t < N) out[(size_t)li * N + t] = v;
            else out[(size_t)li * N + t - N] = v ? q - v : 0;
        }
    }
}
/* Left rotation by r slots: (sigma_g c0 + ks0, ks1), ks = KS_{sigma_g(s) -> s}(sigma_g c1)
 * in the form of or_keyswitch_galois (c1's digits extended, then permuted). */
void or_rotate(const or_ctx *c, const u64 *ct, uint32_t l, int64_t r, const u64 *gk, u64 *out)
{
    size_t n = (size_t)l * c->N;
    u64 g = or_galois_elt(c, r);
    u64 *a0 = (u64 *)malloc(sizeof(u64) * n), *ks = (u64 *)malloc(sizeof(u64) * 2 * n);
    or_automorph(c, ct, l, g, a0);
    keyswitch_core(c, ct + n, l, gk, g, ks);
    for (uint32_t i = 0; i < l; i++)
        for (uint32_t k = 0; k < c->N; k++) {
            size_t x = (size_t)i * c->N + k;
            out[x] = addm(a0[x], ks[x], c->mod[i]);
            out[n + x] = ks[n + x];
        }
    free(a0); free(ks);
}
