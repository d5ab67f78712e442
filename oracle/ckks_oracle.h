/*
 * ckks_oracle.h -- plain, slow, single-threaded CPU reference of full-RNS CKKS.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the GPU library.
 *
 * The paper (Jain et al., "Efficient CNN Building Blocks for Encrypted Data",
 * Sec. 2.1 "Homomorphic Encryption" and Sec. 3 "Proposed Approach") uses the
 * CKKS scheme of Cheon-Kim-Kim-Song (2017) as a black box: ciphertext-ciphertext
 * and ciphertext-plaintext add/mult, slot rotation and levelled rescaling.
 * Every definition below is the standard one from that scheme, in its full-RNS
 * form (Cheon-Han-Kim-Kim-Song, SAC 2018) with hybrid key switching
 * (Han-Ki, CT-RSA 2020).  The readings taken where the paper is silent are
 * listed next to each function.
 *
 * Conventions
 *   - All residues are canonical, in [0, q).
 *   - Polynomials live in the COEFFICIENT domain, limb-major: [limb][N].
 *   - Modulus indices are global: 0..L-1 are the ciphertext primes q_i,
 *     L..L+K-1 the special primes p_j.
 *   - A ciphertext at level l has l limbs (moduli 0..l-1).
 */
#ifndef CKKS_ORACLE_H
#define CKKS_ORACLE_H
#include <stdint.h>

#define OR_MAXMOD 64

/* Philox key word 1 ("domain tag") for each random stream. */
#define OR_TAG_SECRET    1u
#define OR_TAG_UNIFORM   2u
#define OR_TAG_ERROR     3u
#define OR_TAG_EPHEMERAL 4u

typedef struct or_ctx or_ctx;

/* Philox4x64-10 (Salmon et al., SC'11): 4x64-bit counter, 2x64-bit key. */
void or_philox4x64_10(const uint64_t key[2], const uint64_t ctr[4], uint64_t out[4]);

int      or_is_prime(uint64_t n);
uint64_t or_min_psi(uint64_t q, uint32_t N);     /* smallest primitive 2N-th root of unity */

/* Context: returns NULL when a prime is invalid (not prime, not 1 mod 2N, >= 2^62, duplicate). */
or_ctx  *or_ctx_new(uint32_t logN, const uint64_t *q, uint32_t L, const uint64_t *p,
                    uint32_t K, uint32_t dnum);
void     or_ctx_free(or_ctx *c);
uint64_t or_modulus(const or_ctx *c, uint32_t idx);
uint64_t or_psi(const or_ctx *c, uint32_t idx);
uint32_t or_alpha(const or_ctx *c);

/* Ring arithmetic on one limb (modulus index m).  NTT: out[k] = a(psi^(2k+1)). */
void or_ntt(const or_ctx *c, uint32_t m, const uint64_t *a, uint64_t *out);
void or_intt(const or_ctx *c, uint32_t m, const uint64_t *a, uint64_t *out);
void or_polymul(const or_ctx *c, uint32_t m, const uint64_t *a, const uint64_t *b, uint64_t *out);

/* Samplers (see the .c file for the exact stream layout). */
void or_sample_uniform(const or_ctx *c, uint64_t seed, uint64_t tag, uint64_t poly_id,
                       uint32_t nlimbs, const uint32_t *modidx, uint64_t *out);
void or_sample_ternary(const or_ctx *c, uint64_t seed, uint64_t tag, uint64_t poly_id, int64_t *out);
void or_sample_gauss(const or_ctx *c, uint64_t seed, uint64_t tag, uint64_t poly_id,
                     const uint64_t *cdt, uint32_t ncdt, int64_t *out);

/* Signed small polynomial -> residues on limbs modidx[0..nlimbs). */
void or_small_to_rns(const or_ctx *c, const int64_t *a, uint32_t nlimbs, const uint32_t *modidx,
                     uint64_t *out);

/* Keys. s: ternary int64[N].  pk: [2][L][N].  evk: [dnum][2][L+K][N]. */
void or_keygen_secret(const or_ctx *c, uint64_t seed, int64_t *s);
void or_keygen_pk(const or_ctx *c, const int64_t *s, uint64_t seed, const uint64_t *cdt,
                  uint32_t ncdt, uint64_t *pk);
void or_keygen_evk(const or_ctx *c, const int64_t *s, const int64_t *s_from, uint64_t seed,
                   const uint64_t *cdt, uint32_t ncdt, uint64_t *evk);
void or_square_small(const or_ctx *c, const int64_t *s, int64_t *out);      /* s*s in Z[X]/(X^N+1) */
void or_automorph_small(const or_ctx *c, const int64_t *s, uint64_t g, int64_t *out);
uint64_t or_galois_elt(const or_ctx *c, int64_t r);                          /* 5^(r mod N/2) mod 2N */

/* Encryption / decryption.  m: [l][N]; ct: [2][l][N]; decrypt accepts 2 or 3 polys. */
void or_encrypt(const or_ctx *c, const uint64_t *pk, const uint64_t *m, uint32_t l, uint64_t seed,
                const uint64_t *cdt, uint32_t ncdt, uint64_t *ct);
void or_decrypt(const or_ctx *c, const uint64_t *ct, uint32_t npolys, uint32_t l, const int64_t *s,
                uint64_t *m);

/* Encoding.  coeff: int64[N].  Returns 0 on success, -1 if a coefficient overflows 2^62. */
int  or_encode(const or_ctx *c, const double *re, const double *im, uint32_t n, double scale,
               int64_t *coeff);
void or_decode(const or_ctx *c, const uint64_t *m, uint32_t l, double scale, double *re, double *im,
               uint32_t n);

/* Homomorphic arithmetic (l limbs each). */
void or_add(const or_ctx *c, const uint64_t *a, const uint64_t *b, uint32_t npolys, uint32_t l, uint64_t *out);
void or_sub(const or_ctx *c, const uint64_t *a, const uint64_t *b, uint32_t npolys, uint32_t l, uint64_t *out);
void or_mul_pt(const or_ctx *c, const uint64_t *ct, const uint64_t *pt, uint32_t l, uint64_t *out);
void or_add_pt(const or_ctx *c, const uint64_t *ct, const uint64_t *pt, uint32_t l, uint64_t *out);
void or_mul_const(const or_ctx *c, const uint64_t *ct, uint32_t npolys, uint32_t l,
                  const uint64_t *cres, uint64_t *out);
void or_tensor(const or_ctx *c, const uint64_t *a, const uint64_t *b, uint32_t l, uint64_t *out3);
void or_mul_acc(const or_ctx *c, const uint64_t *const *a, const uint64_t *const *b, uint32_t n,
                uint32_t l, uint64_t *acc3);
void or_bconv(const or_ctx *c, const uint64_t *x, const uint32_t *src, uint32_t nsrc,
              const uint32_t *dst, uint32_t ndst, uint64_t *y);
void or_keyswitch(const or_ctx *c, const uint64_t *d, uint32_t l, const uint64_t *evk, uint64_t *ks);
void or_keyswitch_galois(const or_ctx *c, const uint64_t *d, uint32_t l, const uint64_t *evk, uint64_t g,
                         uint64_t *ks);
void or_relin(const or_ctx *c, const uint64_t *ct3, uint32_t l, const uint64_t *rlk, uint64_t *out2);
int  or_rescale(const or_ctx *c, const uint64_t *ct, uint32_t npolys, uint32_t l, uint64_t *out);
void or_automorph(const or_ctx *c, const uint64_t *a, uint32_t nlimbs, uint64_t g, uint64_t *out);
void or_rotate(const or_ctx *c, const uint64_t *ct, uint32_t l, int64_t r, const uint64_t *gk,
               uint64_t *out);

#endif
