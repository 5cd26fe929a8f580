/*
 * pencil.h -- C ABI of the MI355X encrypted linear-layer product.
 *
 * Pencil (Liu et al., NDSS 2024) trains a network between a data owner (DO),
 * who holds the data, and a model owner (MO), who holds the weights.  Every
 * linear layer is evaluated on additive shares over Z_t (Sec. II.C) with one
 * BFV plaintext-ciphertext product (Sec. II.B):
 *   - forward, Alg. 1: the DO encrypts its share <X>_1; the MO adds <X>_0,
 *     multiplies by W, masks with s and returns the ciphertext; the DO's share
 *     of Y is the decryption, the MO's share is s + b;
 *   - input gradient by the same pattern with the transposed operator
 *     (Sec. III.B.2);
 *   - weight gradient, Alg. 2: the MO evaluates the cross terms
 *     <dY>_0 o [[<X>_1]] + [[<dY>_1]] o <X>_0 and masks them.
 * Tensors are packed into polynomials of degree N by the batched encodings of
 * App. A and multiplied as RNS negacyclic NTT -> pointwise multiply-accumulate
 * -> inverse NTT (Sec. V), then re-randomised, noise-flooded and masked.
 *
 * Conventions
 *   Layouts  Z_t tensors are int64 in [0, t), contiguous, PyTorch layout:
 *            FC activations (B, c_in), weights (c_out, c_in); Conv2d
 *            activations (B, C, H, W), weights (c_out, c_in, k, k); Conv1d
 *            activations (B, C, W), weights (c_out, c_in, k).
 *            A ciphertext is uint64 [2][L][N] (component, RNS limb,
 *            residue): the DO's input ciphertexts (pencil_encrypt) are in the
 *            NTT domain with residues in a split form, the products' outputs
 *            in the coefficient domain; a
 *            ciphertext buffer holds pencil_sizes.n_ct[...] (or n_out[...]) of
 *            them back to back, in the tile order of the plan.
 *   Memory   Every tensor, ciphertext and workspace pointer is DEVICE memory
 *            owned by the caller, sized with pencil_layout; ciphertext,
 *            polynomial and workspace pointers must be 16-byte aligned
 *            (EINVAL otherwise).  The context owns only its keys and tables,
 *            allocated once in pencil_ctx_create.  Functions marked (host)
 *            take host pointers.
 *   Streams  `stream` is a hipStream_t (NULL = default stream).  Calls enqueue
 *            their kernels and return without synchronising, except where
 *            noted.  Buffers must stay valid until the stream reaches them.
 *   Errors   Every call returns a pencil_status; nothing is thrown across the
 *            ABI.  Arguments are validated on the host before any launch.
 *            pencil_last_error(ctx) (or pencil_last_error(NULL) after a failed
 *            create) returns a message for the last failure on that context.
 *   Randomness  All random values (keys, encryption, re-randomisation, flood,
 *            masks) come from Philox-4x64-10 keyed by (seed, nonce); a nonce
 *            must not be reused with the same seed for different data.
 */
#ifndef PENCIL_H
#define PENCIL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pencil_ctx pencil_ctx;

typedef enum {
    PENCIL_OK = 0,
    PENCIL_EINVAL = 1,       /* bad argument, shape or plan                         */
    PENCIL_ENOMEM = 2,       /* device allocation failed (create only)              */
    PENCIL_EHIP = 3,         /* a HIP runtime call or kernel launch failed          */
    PENCIL_ENOISE = 4,       /* decryption noise check failed                       */
    PENCIL_EUNSUPPORTED = 5  /* valid request this library does not implement       */
} pencil_status;

/* BFV parameter set {N, t, q = q_1...q_L} (Sec. II.B; RNS limbs, Sec. V). */
typedef struct {
    uint32_t log2_n;      /* N = 2^log2_n, 10 <= log2_n <= 14                        */
    uint32_t num_limbs;   /* L, 1..4                                                 */
    uint32_t prime_bits;  /* limb size when primes[0] == 0: the L largest primes     */
                          /* below 2^prime_bits that are 1 mod 2^15, descending;     */
                          /* 40 <= prime_bits <= 60                                  */
    uint32_t flood_bits;  /* 0 = floor(log2 Delta) - 3, Delta = floor(q / t)        */
    uint64_t primes[4];   /* explicit limbs (each prime, = 1 mod 2N, < 2^60) or 0   */
    uint64_t t;           /* plaintext modulus, odd prime < 2^48; 0 = the largest   */
                          /* prime below 2^41                                        */
    uint64_t seed;        /* key for every random value                              */
} pencil_params;

/* One linear layer (Sec. II.D).  kind 0 = FC (h = w = k = 1, pad = 0);
 * 1 = Conv2d with a square k x k kernel and zero padding pad <= k - 1 on every
 * side; 2 = Conv1d (h = 1, a 1 x k kernel, padding pad at both ends of the
 * length; App. D evaluates Conv1d as this specialisation of Conv2d).  stride
 * (0 or 1 = stride 1) applies to both axes of a Conv2d and to the length of a
 * Conv1d.  The homomorphic entry points take stride-1 layers; a strided layer
 * runs as its stride-1 equivalent (pencil_stride_map, pencil_stride_relayout).
 * Tensors use PyTorch layouts: X (batch, c_in, h, w), Y (batch, c_out, h_out,
 * w_out), W (c_out, c_in, k, k); for FC and Conv1d the unit axes drop out. */
typedef struct {
    int32_t kind, batch, c_in, c_out, h, w, k, pad, stride;
} pencil_layer;

/* Partition of one product into N-slot tiles (App. A allows operands larger
 * than N to be split into pieces).  The product is the packed correlation
 *   out[m, r, y, x] = sum_{c, dy, dx} A[m, c, y+dy, x+dx] * K[r, c, dy, dx];
 * a tile takes m x r x k of the (M, R, K) channels, an oh x ow output window and a
 * kh x kw kernel window, and needs m*r*k*(oh+kh-1)*(ow+kw-1) <= N slots. */
typedef struct {
    int32_t m, r, k, oh, ow, kh, kw;
} pencil_tile;

typedef struct {
    pencil_tile fwd, dx, dw;
    /* Schedule of each product's multiply-accumulate, 0..8.  Each wave of a
     * 512-lane workgroup accumulates a 2 x 2 block of (input row, weight row)
     * outputs for 64 NTT slots.  v / 3 is the kind: 0 stages operands in LDS,
     * 1 loads them directly (both ciphertext components per wave), 2 loads
     * them directly for one component per wave.  v mod 3 is the workgroup's
     * chunk: 4 x 8, 2 x 16 or 8 x 4 rows (kinds 0 and 1), 4 x 4, 2 x 8 or 8 x 2
     * (kind 2).  Results do not depend on it; pencil_plan_auto picks a kind-1
     * chunk by a cost model, pencil_autotune by measurement. */
    int32_t sched[3];
} pencil_plan;

/* Ciphertext operands the DO encrypts (the four layouts of one layer-step). */
typedef enum {
    PENCIL_X_FWD = 0,  /* <X>_1,  forward-encoded A side of the forward product    */
    PENCIL_DY_DX = 1,  /* <dY>_1, A side of the input-gradient product             */
    PENCIL_X_DW = 2,   /* <X>_1,  A side of the weight-gradient product            */
    PENCIL_DY_DW = 3   /* <dY>_1, reverse-encoded K side of the weight gradient    */
} pencil_operand;

typedef enum { PENCIL_OP_FWD = 0, PENCIL_OP_DX = 1, PENCIL_OP_DW = 2 } pencil_op;

typedef struct {
    uint64_t ct_bytes;       /* one ciphertext, 2 * L * N * 8                        */
    uint64_t n_ct[4];        /* ciphertexts per pencil_operand                       */
    uint64_t n_out[3];       /* output ciphertexts per pencil_op                     */
    uint64_t n_pt[3];        /* plaintext polynomials per pencil_op (both dw terms)  */
    uint64_t n_products[3];  /* plaintext x ciphertext products per pencil_op        */
    uint64_t ws_fwd_bytes;   /* workspace of pencil_linear_fwd                       */
    uint64_t ws_bwd_bytes;   /* workspace of pencil_linear_bwd                       */
    uint64_t ws_dec_bytes;   /* workspace of pencil_decrypt (largest op)             */
    uint64_t ws_enc_bytes;   /* workspace of pencil_encrypt (largest operand)        */
} pencil_sizes;

/* Resolved parameters of a context (host). */
typedef struct {
    uint32_t log2_n, num_limbs, flood_bits;
    uint32_t ntt_loge;       /* log2 of the residues each NTT thread keeps (the     */
                             /* schedule pencil_autotune chose; 4 or 5)             */
    uint64_t primes[4];
    uint64_t psi[4];         /* the smallest primitive 2N-th root of unity per limb  */
    uint64_t t;
    uint64_t seed;
} pencil_info;

/* Create a context: resolve parameters, build NTT tables, and generate the key
 * pair on the GPU (KeyGen of BFV: s ternary, pk = (-(a s + e), a)).
 * Synchronous.  The current HIP device is used and must stay current for
 * every later call on the context. */
pencil_status pencil_ctx_create(const pencil_params* params, pencil_ctx** out);
pencil_status pencil_ctx_destroy(pencil_ctx* ctx);
const char* pencil_last_error(const pencil_ctx* ctx);
pencil_status pencil_ctx_info(const pencil_ctx* ctx, pencil_info* out /* host */);

/* Secret key (N int64 in {-1, 0, 1}) and public key ([2][L][N] uint64,
 * coefficient domain) copied to host memory.  The secret key belongs to the
 * DO role; this call exists for tests and for a DO that persists its key.
 * Synchronous. */
pencil_status pencil_export_keys(const pencil_ctx* ctx, int64_t* sk /* host */, uint64_t* pk /* host */);

/* Choose a partition for each product of `layer` (deterministic cost model;
 * host only). */
pencil_status pencil_plan_auto(const pencil_ctx* ctx, const pencil_layer* layer, pencil_plan* plan /* host */);

/* The same choice without a context, for a degree N = 2^log2_n (host only,
 * no GPU needed). */
pencil_status pencil_plan_auto_n(uint32_t log2_n, const pencil_layer* layer, pencil_plan* plan /* host */);

/* Buffer sizes for `layer` under `plan` (host): how many ciphertexts each
 * operand and product needs once the operands are partitioned into N-slot
 * tiles (App. A allows operands larger than N to be split into N-slot pieces;
 * the plan fixes that split), plus the workspaces.  A product whose tile is
 * all zero is treated as not planned and reported with zero sizes.  EINVAL for
 * a layer or plan that does not fit the context's N. */
pencil_status pencil_layout(const pencil_ctx* ctx, const pencil_layer* layer, const pencil_plan* plan,
                            pencil_sizes* sizes /* host */);

/* DO: the encryption that opens Alg. 1 and Alg. 2 (the DO sends [[<X>_1]] or
 * [[<dY>_1]]; BFV encryption of Sec. II.B).  Encode its share (int64 [0,t),
 * the tensor the operand is built from: X for X_FWD / X_DW, dY for DY_DX /
 * DY_DW) with the operand's layout (App. A's encodings) and encrypt it under
 * the public key (ct = (p0 u + e0 + round(q m / t), p1 u + e1)).  EINVAL for a
 * bad operand, layer, plan or pointer (nothing is launched).
 * ct receives n_ct[operand] ciphertexts in the NTT domain, the form the
 * products consume: residue i of each [limb] polynomial is its evaluation
 * v = a(psi_l^(2 rev(i) + 1)) (the order of pencil_ntt_forward), stored in the
 * split form (v mod 2^30) + 2^32 floor(v / 2^30) that the products'
 * multiply-accumulate reads directly.  Output ciphertexts of the products are
 * plain residues in the coefficient domain.  ws: ws_enc_bytes of device
 * memory. */
pencil_status pencil_encrypt(pencil_ctx* ctx, const pencil_layer* layer, const pencil_plan* plan,
                             int operand, const int64_t* share, uint64_t* ct, void* ws, uint64_t nonce,
                             void* stream);

/* MO: forward product of Alg. 1.  ct_x1: n_ct[X_FWD] ciphertexts of <X>_1 in
 * the NTT domain, split form (as pencil_encrypt writes them; read only);
 * x0: the MO's share of X; w: weights; bias: int64 [c_out] at the output's
 * scale, or NULL.  Writes ct_y (n_out[FWD] ciphertexts for the DO) and y0, the
 * MO's share of Y (same shape as Y).  ws: ws_fwd_bytes of device memory. */
pencil_status pencil_linear_fwd(pencil_ctx* ctx, const pencil_layer* layer, const pencil_plan* plan,
                                const uint64_t* ct_x1, const int64_t* x0, const int64_t* w, const int64_t* bias,
                                uint64_t* ct_y, int64_t* y0, void* ws, uint64_t nonce, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the forward
 * product of pencil_linear_fwd without the ws argument.  Its staging lives in
 * a scratch array inside the library's code object, 128 MiB per GPU, held from
 * the first context created on that GPU until the process ends; layers whose
 * ws_fwd_bytes exceed 128 MiB are refused with PENCIL_EUNSUPPORTED.  Nothing is
 * allocated, no event is recorded (kernel timing does not cover it), and the
 * results equal pencil_linear_fwd's bit for bit.  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (several streams, threads or
 * contexts) race and must be serialised by the caller. */
pencil_status pencil_linear_fwd_noalloc(pencil_ctx* ctx, const pencil_layer* layer, const pencil_plan* plan,
                                        const uint64_t* ct_x1, const int64_t* x0, const int64_t* w,
                                        const int64_t* bias, uint64_t* ct_y, int64_t* y0, uint64_t nonce,
                                        void* stream);

/* MO: backward products.  Input gradient (Sec. III.B.2): ct_dy_dx holds <dY>_1
 * in DY_DX layout, dy0 is the MO's share; writes ct_dx (for the DO) and dx0.
 * Weight-gradient cross terms (Alg. 2): ct_x_dw (<X>_1, X_DW layout) and
 * ct_dy_dw (<dY>_1, DY_DW layout) with the MO's shares dy0 and x0; writes
 * ct_dw and dw_mask, the MO's mask s shaped like W.  After decryption,
 * dec(ct_dw) + dw_mask = <dY>_0 o <X>_1 + <dY>_1 o <X>_0 (mod t).
 * Input ciphertexts are in the NTT domain, outputs in the coefficient domain.
 * Either product may be skipped by passing NULL for its outputs. */
pencil_status pencil_linear_bwd(pencil_ctx* ctx, const pencil_layer* layer, const pencil_plan* plan,
                                const uint64_t* ct_dy_dx, const uint64_t* ct_x_dw, const uint64_t* ct_dy_dw,
                                const int64_t* dy0, const int64_t* x0, const int64_t* w,
                                uint64_t* ct_dx, int64_t* dx0, uint64_t* ct_dw, int64_t* dw_mask,
                                void* ws, uint64_t nonce, void* stream);

/* DO: the decryption that closes Alg. 1 and Alg. 2 (the DO's share of Y, dX
 * or of the weight-gradient cross terms is the decryption of what the MO
 * returns; BFV decryption of Sec. II.B).  Decrypt the n_out[op] output
 * ciphertexts of product `op` (m = round(t [c0 + c1 s]_q / q) mod t, exact
 * CRT) and gather the output slots (App. A's output positions) into share
 * (shaped like Y, dX or W).  ws: ws_dec_bytes.  EINVAL for a bad op, layer,
 * plan or pointer. */
pencil_status pencil_decrypt(pencil_ctx* ctx, const pencil_layer* layer, const pencil_plan* plan, int op,
                             const uint64_t* ct, int64_t* share, void* ws, void* stream);

/* DO, debug: pencil_decrypt plus a noise check.  Decryption is correct while
 * the noise of every coefficient stays below q / (2t) (Sec. II.B); the check
 * measures, at every output slot, the distance between t [c0 + c1 s]_q / q and
 * the nearest integer -- the noise as a fraction of q / t -- and returns
 * PENCIL_ENOISE when the largest reaches 1/4 (the product noise plus the flood,
 * at most 2^flood_bits, should stay near 1/8 with the default flood_bits; a
 * larger flood, or product noise close to the budget, makes decryption
 * unreliable).  noise_frac (host, may be NULL) receives the largest fraction.
 * Synchronous: waits for `stream`.  Calls on one context must not overlap (one
 * device word of the context holds the running maximum). */
pencil_status pencil_decrypt_checked(pencil_ctx* ctx, const pencil_layer* layer, const pencil_plan* plan, int op,
                                     const uint64_t* ct, int64_t* share, void* ws, double* noise_frac /* host */,
                                     void* stream);

/* Plaintext product over Z_t of two tensors with the layer's operator
 * (op FWD: a = X, b = W -> Y; DX: a = dY, b = W -> dX; DW: a = X, b = dY -> dW),
 * exact mod t.  These are the "local" terms of Alg. 2 that each party computes
 * on its own shares (<dY>_0 o <X>_0 for the MO, <dY>_1 o <X>_1 for the DO);
 * out is shaped like Y, dX or W. */
pencil_status pencil_zt_linear(pencil_ctx* ctx, const pencil_layer* layer, int op, const int64_t* a,
                               const int64_t* b, int64_t* out, void* stream);

/* Z_t linear combination, element-wise: out = base + sum_i coeffs[i] * terms[i]
 * (mod t) over `count` int64 entries in [0, t).  These are the masked operands
 * u~ = u - sum k_i u'_i, v~ = v - sum l_j v'_j and the share combinations of the
 * online phase of the preprocessed products (Sec. IV.C, Alg. 3).
 * terms: host array of n_terms device pointers (n_terms >= 0; any number, the
 * library chains launches of 64 terms); coeffs: host array of n_terms signed
 * integers, taken mod t; base: device pointer or NULL (zero); out: device, may
 * alias base but no term.  Enqueued on `stream`. */
pencil_status pencil_zt_combine(pencil_ctx* ctx, int64_t count, int n_terms, const int64_t* const* terms,
                                const int64_t* coeffs, const int64_t* base, int64_t* out, void* stream);

/* The two-level sum of Alg. 3's online phase: out = base + sum_{i,j} ci[i] cj[j]
 * terms[i * n_j + j] (mod t), i < n_i, j < n_j (the parties' preprocessed
 * shares <u'_i o v'_j> weighted by the public coefficients k_i l_j).  ci, cj:
 * host arrays of signed integers, taken mod t; the products ci[i] cj[j] mod t
 * are formed here.  Otherwise as pencil_zt_combine. */
pencil_status pencil_zt_combine_outer(pencil_ctx* ctx, int64_t count, int n_i, int n_j, const int64_t* const* terms,
                                      const int64_t* ci, const int64_t* cj, const int64_t* base, int64_t* out,
                                      void* stream);

/* Fixed-point encoding (Sec. II.C) of values already scaled by 2^f and carried
 * in float64 (integers, |x| < 2^53): out[i] = round(x[i]) mod t (nearest, ties
 * to even), int64 in [0, t).  pencil_zt_decode is the inverse view: the
 * centred representative of v[i] in (-t/2, t/2) as float64.  Device arrays of
 * count entries; enqueued on `stream`. */
pencil_status pencil_zt_encode(pencil_ctx* ctx, int64_t count, const double* x, int64_t* out, void* stream);
pencil_status pencil_zt_decode(pencil_ctx* ctx, int64_t count, const int64_t* v, double* out, void* stream);

/* Additive secret sharing over Z_t (Sec. II.C): s0 uniform, s1 = v - s0 mod
 * t.  s0[i] is the 128-bit integer formed by words 2i and 2i+1 of the Philox
 * stream (nonce, object, purpose 49) of the context's seed, reduced mod t.
 * Use a distinct (nonce, object) per tensor.  v, s0, s1: device int64, count
 * entries, v in [0, t); s0 and s1 must not alias each other (either may alias
 * v).  Enqueued on `stream`. */
pencil_status pencil_zt_share(pencil_ctx* ctx, int64_t count, const int64_t* v, uint64_t nonce, uint64_t object,
                              int64_t* s0, int64_t* s1, void* stream);

/* Bias-gradient share (Sec. III.B.2): db[o] = sum of dy over the batch and,
 * for a convolution, over the output rows and columns, mod t.  Each party runs
 * it on its own share of dY; the DO perturbs its result (pencil_dp_noise) and
 * sends it to the MO.  dy: device, int64 in [0, t), the layer's dY layout
 * (batch, c_out[, h_out, w_out]); db: device, c_out entries.  EUNSUPPORTED if
 * batch * h_out * w_out > 2^(64 - bitlen(t)) (2^23 for the default t).
 * Enqueued on `stream`. */
pencil_status pencil_bias_grad(pencil_ctx* ctx, const pencil_layer* layer, const int64_t* dy, int64_t* db,
                               void* stream);

/* The DO's differential-privacy perturbation (Sec. III.B.2: DPSGD noise
 * N(0, sigma^2 C^2 / B) on its share of the weight gradient after Alg. 2's
 * decryption, and on its bias-gradient share): x[i] = x[i] + floor(sd * z_i)
 * mod t, in place, for count int64 entries in [0, t).  sd is the standard
 * deviation in fixed-point units (sigma C / sqrt(B) * 2^scale; scale 2f for
 * dW, f for db), 0 <= sd <= 2^52.  z_i are standard normals from Box-Muller on
 * the context's Philox stream (nonce, object): entries 2i and 2i+1 share
 * stream words 2i (radius) and 2i+1 (angle); the logarithm, sine and cosine are
 * fixed sequences of IEEE double operations, so the draws are reproducible.
 * Use a distinct (nonce, object) per tensor.  Enqueued on `stream`. */
pencil_status pencil_dp_noise(pencil_ctx* ctx, int64_t count, double sd, uint64_t nonce, uint64_t object,
                              int64_t* x, void* stream);

/* Strided layers.  A stride-s correlation equals a stride-1 correlation over
 * the space-to-depth image (Conv2d: s x s phases; Conv1d: s phases of the
 * length): channel c * s_y s_x + a s_x + e of X' holds Xpad[c, s_y y + a,
 * s_x x + e] and the same channel of W' holds W[c, s_y i + a, s_x j + e] (zero
 * past the kernel).  pencil_stride_map writes that equivalent layer
 * (c_in s_y s_x channels, ceil(k / s) kernel, pad 0, h_out + k' - 1 by
 * w_out + k' - 1 inputs; host only, ctx-free).  Both parties relayout their
 * own shares (the maps are linear), run Alg. 1 / Alg. 2 on the equivalent
 * layer, and map the gradients back; Y is the same tensor in both.
 * pencil_stride_relayout: which 0 = X -> X', 1 = W -> W', 2 = dX' -> dX (the
 * adjoint of 0: padding dropped), 3 = dW' -> dW (taps past the kernel dropped).
 * in, out: device int64, distinct, shaped as the strided layer's tensor and
 * its equivalent's.  Enqueued on `stream`. */
pencil_status pencil_stride_map(const pencil_layer* strided, pencil_layer* equiv /* host */);
pencil_status pencil_stride_relayout(pencil_ctx* ctx, const pencil_layer* strided, int which, const int64_t* in,
                                     int64_t* out, void* stream);

/* Autotuner: time, on this GPU with synthetic inputs, the choices that leave
 * the decrypted results unchanged, and keep the fastest -- the NTT's residues
 * per thread (16 or 32, per context; timed on the layer's three products),
 * each product's partition among the caller's tile and the planner's best-
 * ranked ones (App. A leaves the split of large operands open; the choice is
 * written into the plan's tiles), and each product's multiply-accumulate
 * schedule among all nine (written into plan->sched).  A partition fixes the
 * ciphertext layout: tune before the DO encrypts with the plan, and give both
 * parties the tuned plan.  Output ciphertexts and shares under one plan are
 * bit-identical for every schedule and NTT width.  cache_path (may be NULL) is
 * a text file of earlier choices keyed by GPU, ring degree, limbs, layer shape
 * and product; hits are applied without measuring, new choices are appended.
 * Synchronous; allocates and frees its own scratch buffers.  Tune a context
 * before creating steps on it. */
pencil_status pencil_autotune(pencil_ctx* ctx, const pencil_layer* layer, pencil_plan* plan /* host, in/out */,
                              const char* cache_path);

/* Negacyclic NTT of `count` polynomials laid out [count][L][N] (limb l of each
 * polynomial mod q_l), in place.  The transform domain is this library's
 * internal order: entry i of the forward transform holds the evaluation at
 * psi^(2 rev(i) + 1), rev = bit reversal of log2 N bits (Sec. V). */
pencil_status pencil_ntt_forward(pencil_ctx* ctx, uint64_t* polys, int64_t count, void* stream);
pencil_status pencil_ntt_inverse(pencil_ctx* ctx, uint64_t* polys, int64_t count, void* stream);

/* ------------------------------------------------------------------------
 * Batched step: every product of several layers (the forward product, the
 * input-gradient product and the weight-gradient cross terms of each) runs as
 * a handful of phase launches -- all forward NTTs, all multiply-accumulates,
 * all inverse NTTs, all floods -- whatever the layers' shapes, and can be
 * replayed as one captured HIP graph.  Layer i's products use nonce + 2i
 * (forward) and nonce + 2i + 1 (backward), so a step equals the per-layer calls
 * made with those nonces, bit for bit. */
typedef struct pencil_step pencil_step;

/* Device buffers of one layer in a step: the same arguments as
 * pencil_linear_fwd / pencil_linear_bwd (unused ones may be NULL). */
typedef struct {
    const uint64_t *ct_x1, *ct_dy_dx, *ct_x_dw, *ct_dy_dw;
    const int64_t *x0, *dy0, *w, *bias;
    uint64_t *ct_y, *ct_dx, *ct_dw;
    int64_t *y0, *dx0, *dw_mask;
} pencil_step_io;

/* n layers, layer i on context ctxs[i] with plan plans[i] (host arrays);
 * ops: bit 0 forward, bit 1 input gradient, bit 2 weight gradient. */
pencil_status pencil_step_create(pencil_ctx* const* ctxs, const pencil_layer* layers, const pencil_plan* plans,
                                 int n, uint32_t ops, pencil_step** out);
pencil_status pencil_step_destroy(pencil_step* step);
const char* pencil_step_last_error(const pencil_step* step);
/* Device workspace the step needs (every product's staging at once). */
pencil_status pencil_step_workspace(const pencil_step* step, uint64_t* bytes /* host */);
/* Fix the buffers (io: n host entries) and the workspace; builds the segment
 * tables on the device.  Synchronous. */
pencil_status pencil_step_bind(pencil_step* step, const pencil_step_io* io, void* ws);
/* Run the bound step on `stream` with base nonce `nonce`. */
pencil_status pencil_step_run(pencil_step* step, uint64_t nonce, void* stream);
/* Capture one run into a HIP graph whose first node advances the device-side
 * nonce by 2n, so consecutive replays use fresh nonces. */
pencil_status pencil_step_graph_capture(pencil_step* step);
/* The next replay uses base nonce `nonce`. */
pencil_status pencil_step_set_nonce(pencil_step* step, uint64_t nonce, void* stream);
pencil_status pencil_step_graph_launch(pencil_step* step, void* stream);

/* Worst-case noise of one product's output before decryption (Sec. II.B:
 * decryption is correct while it stays below q / (2t) ~ Delta / 2), from the
 * parameters and the partition alone (host only, no GPU): every input
 * coefficient's fresh noise is at most 42 N + 23 (CBD errors of magnitude
 * <= 21 times ternary u and s, plus the roundings of round(q m / t)); a
 * product sums `terms` contraction tiles of plaintext polynomials with at most
 * `nnz` nonzero coefficients of magnitude at most 2^(plaintext_bits - 1)
 * (centred; 41 for uniform shares of Z_t, about 13 for fixed-point weights
 * with f = 12); re-randomisation adds 42 N + 21 and the flood at most
 * 2^flood_bits.  All values are log2.  Returns PENCIL_ENOISE when
 * product + flood reaches Delta / 2 (decryption may fail), PENCIL_OK
 * otherwise; smudge_bits = flood_bits - product_bits is how far the flood
 * exceeds the product noise it hides. */
typedef struct {
    double product_bits, flood_bits, budget_bits, margin_bits, smudge_bits;
} pencil_noise;
pencil_status pencil_noise_bound(const pencil_params* params, const pencil_layer* layer, const pencil_plan* plan,
                                 int op, uint32_t plaintext_bits, pencil_noise* out /* host */);

/* Measurement aid for the integer roofline: the rate, per second over the
 * whole current GPU, of one 32-bit multiply instruction form -- kind 0
 * v_mad_u64_u32 (the multiply-accumulate's), 1 v_mul_lo_u32, 2 v_mul_hi_u32
 * (both in the NTT's Shoup products) -- from 8 waves per SIMD each running 8
 * independent chains.  Synchronous; allocates and frees a small buffer. */
pencil_status pencil_probe_mul32(int kind, double* per_s /* host */);

/* Kernel timing: while enabled, every kernel this context launches is bracketed
 * by HIP events recorded on its launch stream.  enable() clears the totals.
 * read() waits for the recorded events and fills up to `max` entries (host
 * memory): kernel name, launches and summed milliseconds. */
typedef struct {
    char name[24];
    uint64_t launches;
    double total_ms;
} pencil_kernel_stat;

pencil_status pencil_profile_enable(pencil_ctx* ctx, int enable);
pencil_status pencil_profile_read(pencil_ctx* ctx, pencil_kernel_stat* out /* host */, int max, int* count);

#ifdef __cplusplus
}
#endif

#endif /* PENCIL_H */
