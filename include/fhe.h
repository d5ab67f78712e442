/*
 * fhe.h -- C ABI of the MI355X (gfx950) RNS-CKKS library.
 *
 * The operations follow the setting of Jain et al., "Efficient CNN Building
 * Blocks for Encrypted Data": the end user holds the secret key and encrypts
 * both the images and (through the model owner) the weights under its public
 * key; the untrusted cloud evaluates ciphertext-ciphertext and
 * ciphertext-plaintext additions and multiplications, rotations and the CNN
 * layers built from them; the user decrypts the class scores (Sec. 1,
 * Fig. 1; Sec. 2.1 "Homomorphic Encryption"; Sec. 3, Eq. (enc_conv),
 * Eq. (approxReLU), Eq. (ActPool); Sec. 4.3).  The paper uses CKKS as a black
 * box; the arithmetic is full-RNS CKKS with hybrid key switching.
 *
 * Conventions for every entry point
 *   - Ciphertext, plaintext and key buffers are DEVICE memory owned by the
 *     caller, 64-bit residues, limb-major [polys][limbs][N], evaluation (NTT)
 *     domain in the library's internal order.  The context owns only its
 *     precomputed tables and its scratch memory.
 *   - Arrays documented as "host" are host memory; everything else is device.
 *   - All work is enqueued on the HIP stream given to fhe_ctx_create (or
 *     fhe_set_stream) and is asynchronous, except calls that return host data
 *     (fhe_keygen_secret, fhe_decode, fhe_export_limbs), which synchronise it.
 *   - Output buffers may alias inputs for the element-wise operations,
 *     rescale, relinearisation and rotation.
 *   - Errors are negative fhe_status codes; fhe_last_error() returns a
 *     thread-local message.  On error no output buffer has been written.
 */
#ifndef FHE_H
#define FHE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fhe_status;
#define FHE_OK 0
#define FHE_EINVAL (-1)   /* null pointer, shape or size mismatch */
#define FHE_ELEVEL (-2)   /* limb-count mismatch, or rescale at one limb */
#define FHE_ESCALE (-3)   /* add of operands whose scales differ by more than 2^-40 relative, or a layer
                             output whose scale leaves fewer than FHE_SCALE_ROOM_BITS bits below Q/2 */
#define FHE_ENOKEY (-4)   /* evaluation key does not match the requested rotation */
#define FHE_EPARAM (-5)   /* invalid parameter set */
#define FHE_ENOMEM (-6)   /* the context's HBM budget would be exceeded */
#define FHE_EDEVICE (-7)  /* HIP runtime error */

/* Layer entry points (convolution, activation, fully connected) refuse outputs whose
 * scale S at l limbs has log2(S) > log2(q_0 ... q_(l-1)) - 1 - FHE_SCALE_ROOM_BITS:
 * slot values up to 2^(FHE_SCALE_ROOM_BITS - 1) in magnitude must decrypt without
 * wrapping around the modulus. */
#define FHE_SCALE_ROOM_BITS 4

/* Parameter set (all arrays host memory, copied by fhe_ctx_create).
 * Requirements: 10 <= log_n <= 16; every prime is distinct, below 2^50 and
 * = 1 mod 2N; n_q + n_p <= 64; 1 <= dnum <= n_q.  The key-switching digit
 * size is alpha = ceil(n_q / dnum).  cdt holds the cumulative thresholds of
 * the error distribution: |e| = #{i : cdt[i] <= u} for a uniform 64-bit u. */
typedef struct {
    uint32_t log_n;
    uint32_t n_q;
    uint32_t n_p;
    uint32_t dnum;
    const uint64_t *q;
    const uint64_t *p;
    const uint64_t *cdt;
    uint32_t n_cdt;
} fhe_params;

typedef struct fhe_ctx fhe_ctx;

/* Ciphertext: polys (2, or 3 after a tensor product) x limbs x N residues. */
typedef struct {
    uint64_t *d;
    uint32_t limbs;
    uint32_t polys;
    double scale;
} fhe_ct;

/* Plaintext: limbs x N residues. */
typedef struct {
    uint64_t *d;
    uint32_t limbs;
    double scale;
} fhe_pt;

/* Key-switching key: [dnum][2][n_q + n_p][N]; galois = 0 for the
 * relinearisation key, else the Galois element 5^r mod 2N of the rotation. */
typedef struct {
    uint64_t *d;
    uint64_t galois;
} fhe_evk;

/* ---------------------------------------------------------------- context */
fhe_status fhe_ctx_create(const fhe_params *params, void *hip_stream, uint64_t hbm_budget_bytes,
                          fhe_ctx **out);
void fhe_ctx_destroy(fhe_ctx *ctx);
fhe_status fhe_set_stream(fhe_ctx *ctx, void *hip_stream);
const char *fhe_last_error(void);
uint32_t fhe_ring_degree(const fhe_ctx *ctx);
uint64_t fhe_modulus(const fhe_ctx *ctx, uint32_t idx);          /* 0..n_q-1: q_i; n_q..: p_j */
size_t fhe_evk_bytes(const fhe_ctx *ctx);
size_t fhe_ct_bytes(const fhe_ctx *ctx, uint32_t limbs, uint32_t polys);   /* device bytes of a ciphertext (0: null ctx) */
uint64_t fhe_galois_elt(const fhe_ctx *ctx, int32_t step);        /* 5^(step mod N/2) mod 2N */
uint64_t fhe_scratch_bytes(const fhe_ctx *ctx);                   /* scratch currently held */
uint64_t fhe_workspace_bytes(const fhe_ctx *ctx);                 /* layer workspace currently held */

/* Device memory for the context's growable scratch and layer workspace (the only
 * device memory it allocates after creation) from the caller's allocator instead of
 * hipMalloc, e.g. a framework's caching allocator, so that one budget and one cache
 * cover the caller's buffers and the library's.  alloc_fn(bytes, stream, user)
 * returns device memory usable on `stream` (the context's) or null (the call that
 * needed it fails with FHE_ENOMEM before any work); free_fn(ptr, user) returns it,
 * called once the context's stream has drained.  Both or neither (null, null:
 * hipMalloc again).  Buffers held from the previous allocator are released first;
 * fhe_ctx_destroy releases the rest.  Not while capturing (FHE_EINVAL). */
typedef void *(*fhe_alloc_fn)(size_t bytes, void *hip_stream, void *user);
typedef void (*fhe_free_fn)(void *ptr, void *user);
fhe_status fhe_ctx_set_allocator(fhe_ctx *ctx, fhe_alloc_fn alloc_fn, fhe_free_fn free_fn, void *user);
/* Return the context's scratch and layer workspace (after its stream drains); the
 * next call that needs them allocates again.  Not while capturing (FHE_EINVAL). */
fhe_status fhe_ctx_release_buffers(fhe_ctx *ctx);

/* Kernel timing for measurement: after fhe_profile_enable(ctx, cat) every
 * launch of kernel category cat ("*" = all; categories: ntt_fwd, ntt_fwd_col,
 * ntt_fwd_row, ntt_inv, ntt_inv_col, ntt_inv_row, bconv_up, bconv_down,
 * ks_intt_first, ks_inner, ks_moddown_final, automorph, rescale, tensor,
 * elementwise) is bracketed by HIP events on the context's stream.
 * fhe_profile_read synchronises the stream and returns the summed event time
 * and launch count of a category since enabling.  fhe_profile_enable(ctx,
 * NULL) switches timing off. */
fhe_status fhe_profile_enable(fhe_ctx *ctx, const char *category);
fhe_status fhe_profile_read(fhe_ctx *ctx, const char *category, double *total_ms, uint64_t *count);

/* --------------------------------------------------- limb transforms / IO
 * Residue limbs are identified by a host list of modulus indices, one per
 * limb (e.g. 0..l-1 repeated per polynomial of a ciphertext at l limbs).
 * fhe_ntt / fhe_intt transform nlimbs consecutive limbs of d in place
 * (negacyclic NTT, the evaluation at the odd powers of a 2N-th root).
 * fhe_export_limbs writes the canonical coefficient-domain residues in
 * [0, q) to host memory (d is left unchanged); fhe_import_limbs reads them
 * from host memory and leaves the evaluation form in d. */
fhe_status fhe_ntt(fhe_ctx *ctx, uint64_t *d, uint32_t nlimbs, const uint32_t *modidx);
fhe_status fhe_intt(fhe_ctx *ctx, uint64_t *d, uint32_t nlimbs, const uint32_t *modidx);
fhe_status fhe_export_limbs(fhe_ctx *ctx, const uint64_t *d, uint32_t nlimbs, const uint32_t *modidx,
                            uint64_t *host_out);
fhe_status fhe_import_limbs(fhe_ctx *ctx, const uint64_t *host_in, uint32_t nlimbs, const uint32_t *modidx,
                            uint64_t *d);

/* -------------------------------------------------------- client side
 * The only calls that take the secret key s (host, N ternary coefficients).
 * Random polynomials come from Philox4x64-10 with key (seed, stream tag) and
 * counter (coefficient, modulus index, polynomial id, round); see the
 * sampler notes in the library sources for the exact stream layout. */
fhe_status fhe_keygen_secret(fhe_ctx *ctx, uint64_t seed, int8_t *s_host);
fhe_status fhe_keygen_pk(fhe_ctx *ctx, const int8_t *s_host, uint64_t seed, fhe_ct *pk);   /* polys 2, limbs n_q */
fhe_status fhe_keygen_relin(fhe_ctx *ctx, const int8_t *s_host, uint64_t seed, fhe_evk *out);
fhe_status fhe_keygen_rot(fhe_ctx *ctx, const int8_t *s_host, int32_t step, uint64_t seed, fhe_evk *out);
/* Slots (host re/im, im may be NULL; n <= N/2) -> round(scale * inverse
 * canonical embedding) -> residues on limbs 0..limbs-1. */
fhe_status fhe_encode(fhe_ctx *ctx, const double *re, const double *im, uint32_t n, double scale,
                      fhe_pt *out);
/* Integer coefficients (host, N values) -> plaintext on out->limbs limbs. */
fhe_status fhe_encode_coeffs(fhe_ctx *ctx, const int64_t *coeff_host, fhe_pt *out);
fhe_status fhe_encrypt(fhe_ctx *ctx, const fhe_ct *pk, const fhe_pt *m, uint64_t seed, fhe_ct *out);
fhe_status fhe_decrypt(fhe_ctx *ctx, const int8_t *s_host, const fhe_ct *ct, fhe_pt *out);
/* Plaintext -> n slots (host re/im, im may be NULL), dividing by pt->scale. */
fhe_status fhe_decode(fhe_ctx *ctx, const fhe_pt *pt, double *re, double *im, uint32_t n);
/* The same for the n slots listed in slots (host array, each < N/2): re[t], im[t]
 * hold slot slots[t] (e.g. one score per image frame). */
fhe_status fhe_decode_slots(fhe_ctx *ctx, const fhe_pt *pt, const uint32_t *slots, uint32_t n, double *re,
                            double *im);

/* --------------------------------------------------------- server side */
fhe_status fhe_add(fhe_ctx *ctx, const fhe_ct *a, const fhe_ct *b, fhe_ct *out);
fhe_status fhe_sub(fhe_ctx *ctx, const fhe_ct *a, const fhe_ct *b, fhe_ct *out);
fhe_status fhe_add_pt(fhe_ctx *ctx, const fhe_ct *a, const fhe_pt *p, fhe_ct *out);
fhe_status fhe_mul_pt(fhe_ctx *ctx, const fhe_ct *a, const fhe_pt *p, fhe_ct *out);
/* Multiply by the integer round(value * const_scale); out->scale = a->scale * const_scale. */
fhe_status fhe_mul_const(fhe_ctx *ctx, const fhe_ct *a, double value, double const_scale, fhe_ct *out);
/* Add the constant polynomial round(value * a->scale) (every slot + value);
 * out->scale = a->scale.  |round(value * scale)| must stay below 2^62. */
fhe_status fhe_add_const(fhe_ctx *ctx, const fhe_ct *a, double value, fhe_ct *out);
/* Tensor product (a0 b0, a0 b1 + a1 b0, a1 b1); out has 3 polys. */
fhe_status fhe_mul(fhe_ctx *ctx, const fhe_ct *a, const fhe_ct *b, fhe_ct *out3);
/* acc3 = sum_t a[t] (x) b[t]; a, b: host arrays of n descriptors. */
fhe_status fhe_mul_acc(fhe_ctx *ctx, const fhe_ct *a, const fhe_ct *b, uint32_t n, fhe_ct *acc3);
fhe_status fhe_relin(fhe_ctx *ctx, const fhe_evk *rlk, const fhe_ct *in3, fhe_ct *out2);
fhe_status fhe_rescale(fhe_ctx *ctx, const fhe_ct *in, fhe_ct *out);
fhe_status fhe_drop_level(fhe_ctx *ctx, const fhe_ct *in, uint32_t limbs, fhe_ct *out);
/* Left rotation by step slots with the Galois key of that step (the slot rotation of
 * Sec. 3 / Fig. 2, computed as sigma_g(c0) + KS(sigma_g(c1)) with g = 5^step mod 2N).
 * The key switch extends the digits of c1 itself and applies sigma_g to the extended
 * digits before the key inner product, the same result the oracle defines; out may
 * equal in (the input is copied to the context's scratch first). */
fhe_status fhe_rotate(fhe_ctx *ctx, const fhe_evk *gk, const fhe_ct *in, int32_t step, fhe_ct *out);
/* n independent rotations in one launch sequence: out[t] = rotate(in[t], steps[t])
 * with Galois key gk[t]; gk, in, steps, out are host arrays of n entries.  Entries
 * with the same input ciphertext share one extension of its digits.  Outputs must
 * not overlap any input (FHE_EINVAL). */
fhe_status fhe_rotate_batch(fhe_ctx *ctx, const fhe_evk *gk, const fhe_ct *in, const int32_t *steps, uint32_t n,
                            fhe_ct *out);
/* Hybrid key switch of d (limbs x N, evaluation form): out = (ks0, ks1), polys 2. */
fhe_status fhe_keyswitch(fhe_ctx *ctx, const fhe_evk *evk, const uint64_t *d, uint32_t limbs, fhe_ct *out);
/* Batched key switch: n independent inputs d[t] (each limbs x N) with keys evk[t];
 * d, evk, out are host arrays of n entries.  One launch sequence for all. */
fhe_status fhe_keyswitch_batch(fhe_ctx *ctx, const fhe_evk *evk, const uint64_t *const *d, uint32_t limbs,
                               uint32_t n, fhe_ct *out);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): fhe_keyswitch_batch with
 * its scratch in a library-owned static device array of FHE_STATIC_SCRATCH_BYTES on
 * each GPU (held until the process ends) instead of the context's growable scratch.
 * Same arguments, layout, results and errors as fhe_keyswitch_batch, plus FHE_ENOMEM
 * (nothing enqueued) when the batch needs more than FHE_STATIC_SCRATCH_BYTES of
 * scratch (a key switch at N = 2^16 and 24 limbs with 8 special primes and dnum 3
 * takes 104 MiB, so two fit; at N = 2^15 and 16 limbs, seven) or more pointer-table
 * space than the context's table ring.  The call allocates nothing: the ring and
 * its events are made when the context is created.  Every call on one GPU shares
 * that GPU's array and leaves its last contents there (the key switch writes every
 * scratch word it reads, so nothing needs clearing); calls that overlap on one GPU
 * (on different streams or host threads) race and must be serialised by the caller. */
#define FHE_STATIC_SCRATCH_BYTES (256ull << 20)
fhe_status fhe_keyswitch_batch_static(fhe_ctx *ctx, const fhe_evk *evk, const uint64_t *const *d, uint32_t limbs,
                                      uint32_t n, fhe_ct *out);

/* Work list of independent or chained operations at mixed levels (one ring).
 * Operations run as if in list order; those whose inputs are ready are grouped
 * by kind and run as one ragged launch sequence (the GPU analogue of the paper's
 * split of independent work over threads, Sec. 4.2).  An input may be the
 * output of an earlier operation in the list; outputs must not overlap each
 * other, nor any input of their own or an earlier operation (FHE_EINVAL).
 *   FHE_OP_MUL_RELIN_RESCALE: out = Rescale(Relin(a (x) b)) with key (relin),
 *     a and b at one level l >= 2, out at l - 1;
 *   FHE_OP_ROTATE: out = rotate(a, step) with key (Galois key of step), out at l.
 * Output scales are set on the out descriptors. */
enum { FHE_OP_MUL_RELIN_RESCALE = 1, FHE_OP_ROTATE = 2 };
typedef struct {
    uint32_t kind;
    int32_t step;
    const fhe_ct *a, *b;
    const fhe_evk *key;
    fhe_ct *out;
} fhe_op;
fhe_status fhe_batch_run(fhe_ctx *ctx, const fhe_op *ops, uint32_t n_ops);

/* ------------------------------------------------------------ HIP graphs
 * Capture the work that library calls enqueue on the streams of ctxs[0..n)
 * (distinct contexts, e.g. one per ring degree, each on its own stream) into one
 * graph, then replay it with fhe_graph_launch.  Between begin and end calls only
 * enqueue work: the pointer tables they build go to an arena of table_bytes per
 * context (0: 16 MiB) that the graph owns, and their scratch must already have
 * been sized by the same calls run once eagerly (else FHE_ENOMEM and the capture
 * fails at fhe_graph_end).  At fhe_graph_end the contexts' scratch buffers pass
 * to the graph.  Replays read and write the device buffers of the captured
 * calls; operation counters count the capture, not the replays.  Profiling must
 * be off.  On any failure fhe_graph_end frees the graph and returns the error. */
typedef struct fhe_graph fhe_graph;
fhe_status fhe_graph_begin(fhe_ctx *const *ctxs, uint32_t n, uint64_t table_bytes, fhe_graph **out);
fhe_status fhe_graph_end(fhe_ctx *const *ctxs, uint32_t n, fhe_graph *g);
fhe_status fhe_graph_launch(fhe_graph *g, void *hip_stream);   /* null: the first context's stream */
void fhe_graph_destroy(fhe_graph *g);                          /* waits for the device first */

/* Tuning knobs read by the batched drivers; the Python runtime's autotuner measures
 * their combinations on a workload and keeps the fastest.  None changes a result.
 *   "chunk_items": most items per ragged launch sequence (0 = no limit);
 *   "ks_fuse_row_inner": 1 (default) fuses, when every item of a key switch has its
 *     own key, the forward row passes of the converted limbs into the key inner
 *     product, the inverse row pass of the special-prime part into the same kernel and
 *     the Q part into the ModDown finish (five kernels); 0 runs the seven-kernel form;
 *   "ks_nt": 1 (default) makes the loads and stores of data used once in the first
 *     inverse pass and the fused kernels non-temporal, so that they do not evict the
 *     twiddle rows the passes re-read; 0 makes them ordinary;
 *   "row_wg": 128 (default) or 256, the workgroup size of the rescale's row pass. */
fhe_status fhe_ctx_set_tuning(fhe_ctx *ctx, const char *key, uint64_t value);

/* Batched relinearisation and rescale of n ciphertexts (host descriptor arrays;
 * one key; rescale outputs must not overlap their inputs). */
fhe_status fhe_relin_batch(fhe_ctx *ctx, const fhe_evk *rlk, const fhe_ct *in3, uint32_t n, fhe_ct *out2);
fhe_status fhe_rescale_batch(fhe_ctx *ctx, const fhe_ct *in, uint32_t n, fhe_ct *out);

/* --------------------------------------------------------- CNN layers
 * Slot packing (Sec. 3 "Convolution Operator", Fig. 2): each input ciphertext
 * holds one pixel of every image of the batch; each weight ciphertext holds one
 * weight replicated in all slots.  All arrays are host arrays of descriptors.
 *
 * fhe_conv2d_slot, Eq. (enc_conv) with stride and zero padding:
 *   Y[co][i][j] = Rescale(Relin( sum over ci, p, q with (y, x) inside the image of
 *                 X[ci][y][x] (x) W[co][ci][p][q] )),  y = i*stride + p - pad_t,
 *                 x = j*stride + q - pad_l;  padded taps are skipped.
 * Layouts: X[(ci*H + y)*W + x], W[((co*Cin + ci)*kh + p)*kw + q], Y[(co*Ho + i)*Wo + j].
 * Inputs and weights at one level l >= 2, outputs (caller-allocated) at l - 1.
 * fhe_fc_slot: y[o] = Rescale(Relin(sum_i x[i] (x) W[o*n_in + i])) (Sec. 2.3, Z = f(WX), no bias).
 * fhe_square_act: y[i] = Rescale(Relin(x[i] (x) x[i])) (the x^2 activation). */
fhe_status fhe_conv2d_slot(fhe_ctx *ctx, const fhe_evk *rlk, const fhe_ct *X, uint32_t H, uint32_t W, uint32_t Cin,
                           const fhe_ct *Wt, uint32_t Cout, uint32_t kh, uint32_t kw, uint32_t stride, uint32_t pad_t,
                           uint32_t pad_l, uint32_t Ho, uint32_t Wo, fhe_ct *Y);
fhe_status fhe_fc_slot(fhe_ctx *ctx, const fhe_evk *rlk, const fhe_ct *x, uint32_t n_in, const fhe_ct *Wt,
                       uint32_t n_out, fhe_ct *y);
fhe_status fhe_square_act(fhe_ctx *ctx, const fhe_evk *rlk, const fhe_ct *x, uint32_t n, fhe_ct *y);
/* --------------------------------------------- within-image packed CNN layers
 * One ciphertext per channel; each image of the batch sits in its own frame of
 * frame_w-wide rows of slots, zero beyond the image (pixel (y, x) of image b at
 * slot b*frame_slots + y*frame_w + x).  Rotations (Sec. 3, Fig. 2) move
 * neighbouring pixels into place in every frame at once; keys is a host array of
 * Galois keys searched by Galois element (FHE_ENOKEY if a needed one is absent).
 * The caller keeps the layout valid: the zero guard must cover dilation * (k/2)
 * rows and columns, and positions outside the valid grid hold values that later
 * masks clear.
 *
 * fhe_conv2d_packed: Y[co] = Rescale(Relin( sum_ci sum_(p,q) rot(X[ci], s_pq) (x) W[co][ci][p][q] )),
 *   s_pq = dilation * ((p - k/2) * frame_w + (q - k/2)), taps row-major, k odd;
 *   W[(co*Cin + ci)*k*k + p*k + q] are slot-replicated weights (Eq. (enc_conv)
 *   with the window sum done by rotations); X, W at level l, Y at l - 1.
 * fhe_poly_act: polynomial activation (Sec. 3 "Activation", Eq. (approxReLU)),
 *   coef = {c0, c1, c2, c3}; constants c multiply as the integer round(c * s).
 *   deg 3, depth 2: y = (c3 u + c2) u^2 + (c1 u + c0), c3 at s = q_(l-1), the
 *   linear term at the scale that lands on the product's scale; inputs at l >= 3,
 *   outputs at l - 2, output scale S^3 / (q_(l-1) q_(l-2)) up to the constants.
 *   deg 2, depth 1 (the paper's count): Relin(u (x) u) is taken as c2 u^2 at scale
 *   S' = S^2 / c2, plus round(c1 S / c2) u and round(c0 S'), then one rescale;
 *   c2 must be positive (FHE_EINVAL otherwise: it becomes a factor of the scale);
 *   inputs at l >= 2, outputs at l - 1, scale S' / q_(l-1).
 *   Inputs share one scale S.
 * fhe_avgpool2x2 (Sec. 3 "Pooling", mean of a 2x2 window): t = x + rot(x, d);
 *   t = t + rot(t, frame_w d); y = Rescale(t * mask).  mask is a plaintext at
 *   level l (0.25 on the positions that survive, zero elsewhere; its scale sets
 *   the output scale); outputs at l - 1, valid positions now at dilation 2d.
 * fhe_fc_packed (Sec. 2.3, Z = WX without bias): z[o] = Rescale(Relin(sum_i x[i] (x) W[o*n_in + i]))
 *   then z += rot(z, j) for j = 1, 2, 4, ..., frame_slots/2, so that slot 0 of
 *   every frame holds the class score; W[o*n_in + i] holds the weights of input
 *   channel i at its valid positions, zero elsewhere.  Outputs at l - 1. */
fhe_status fhe_conv2d_packed(fhe_ctx *ctx, const fhe_evk *rlk, const fhe_evk *keys, uint32_t nkeys, const fhe_ct *X,
                             uint32_t Cin, const fhe_ct *Wt, uint32_t Cout, uint32_t k, uint32_t dilation,
                             uint32_t frame_w, fhe_ct *Y);
fhe_status fhe_poly_act(fhe_ctx *ctx, const fhe_evk *rlk, const fhe_ct *x, uint32_t n, const double *coef,
                        uint32_t deg, fhe_ct *y);
fhe_status fhe_avgpool2x2(fhe_ctx *ctx, const fhe_evk *keys, uint32_t nkeys, const fhe_ct *x, uint32_t n,
                          uint32_t dilation, uint32_t frame_w, const fhe_pt *mask, fhe_ct *y);
fhe_status fhe_fc_packed(fhe_ctx *ctx, const fhe_evk *rlk, const fhe_evk *keys, uint32_t nkeys, const fhe_ct *x,
                         uint32_t n_in, const fhe_ct *Wt, uint32_t n_out, uint32_t frame_slots, fhe_ct *y);

/* The same layers with a plain (unencrypted) model, for the low-latency setting of
 * one image per ciphertext (Sec. 4.4, last paragraph: model parameters not encrypted):
 * fhe_conv2d_packed_pw: Y[co] = Rescale( sum_ci sum_(p,q) rot(X[ci], s_pq) * round(w[co][ci][p][q] * wscale) ),
 *   w a host array [Cout][Cin][k][k]; no relinearisation; Y scale = X scale * wscale / q_(l-1).
 * fhe_fc_packed_pw: z[o] = Rescale( sum_i x[i] * W[o*n_in + i] ) with plaintext weights (slot
 *   vectors at the valid positions, at the inputs' level), then the rotate-and-sum of fhe_fc_packed. */
fhe_status fhe_conv2d_packed_pw(fhe_ctx *ctx, const fhe_evk *keys, uint32_t nkeys, const fhe_ct *X, uint32_t Cin,
                                const double *w, uint32_t Cout, uint32_t k, uint32_t dilation, uint32_t frame_w,
                                double wscale, fhe_ct *Y);
fhe_status fhe_fc_packed_pw(fhe_ctx *ctx, const fhe_evk *keys, uint32_t nkeys, const fhe_ct *x, uint32_t n_in,
                            const fhe_pt *Wt, uint32_t n_out, uint32_t frame_slots, fhe_ct *y);
/* Sum pooling over 2x2 windows of slot-packed maps (Eq. (ActPool) without the 1/4,
 * which a recipe folds into the activation's coefficients):
 *   y[c][i][j] = x[c][2i][2j] + x[c][2i][2j+1] + x[c][2i+1][2j] + x[c][2i+1][2j+1],
 * x[(c*H + yy)*W + xx], y[(c*(H/2) + i)*(W/2) + j], all at one level; no level used. */
fhe_status fhe_pool2x2_sum_slot(fhe_ctx *ctx, const fhe_ct *x, uint32_t C, uint32_t H, uint32_t W, fhe_ct *y);
/* Model owner: encrypt n weights, each replicated in every slot (a constant
 * polynomial round(value * scale)), under the user's public key; per-weight
 * seeds (host array); outputs at out[0].limbs limbs. */
fhe_status fhe_encrypt_const_batch(fhe_ctx *ctx, const fhe_ct *pk, const double *values, uint32_t n, double scale,
                                   const uint64_t *seeds, fhe_ct *out);
/* Operation counters since the last call (then reset): ct-ct mult, ct-ct add,
 * ct-pt mult, ct-pt add, relinearise, rescale, rotate, (reserved). */
fhe_status fhe_op_counts(fhe_ctx *ctx, uint64_t out[8]);

#ifdef __cplusplus
}
#endif
#endif
