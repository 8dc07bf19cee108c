/*
 * fenc.h -- C ABI of the MI355X (gfx950) FEnc^2 hot path.
 *
 * FEnc^2 (arXiv 2606.16359) evaluates CNN layers on CKKS ciphertexts whose
 * slots hold a 4-D tensor in the Conv-aware (fragment) Encoding: the padded
 * M x M feature maps are cut into an m x m grid of S x S blocks and all
 * elements with the same intra-block position (u, v) share ciphertexts
 * (Conv-aware Encoding, Alg. fragment-packing).  The server side consists of
 * homomorphic convolution (inner rotations for spatial aggregation, outer
 * rotations for channel aggregation; Motivation section, eq.
 * multi-channel-conv), FC layers by diagonal BSGS, polynomial activations,
 * average pooling / stride by discarding fragments, and Arch-aware Ct
 * Compression (rot-mask-add repacking).
 *
 * Conventions shared by every entry point
 *  - Return value: FENC_OK (0) or a negative fenc_status.  On error nothing is
 *    launched when the error is detected during argument validation;
 *    outputs are unspecified otherwise.  fenc_last_error() returns a
 *    thread-local message for the last failing call of the calling thread.
 *  - Ciphertext batches live in device memory owned by the caller, uint64
 *    residues in [0, q_i), layout [n_ct][2][level+1][N], limb i modulo the
 *    i-th ciphertext prime, each limb in NTT (evaluation) form stored in
 *    bit-reversed order.  fenc_ct_bytes() gives the size.
 *  - Sizing: calling an operation with out->data == NULL only fills out->lay
 *    (shape, level, scale, ciphertext count) and launches nothing.
 *  - Asynchrony: operations enqueue work on `stream` (a hipStream_t, NULL is
 *    the default stream) and return; keep buffers alive until the stream is
 *    synchronised.  Calls on one context are not thread-safe.
 *  - Operations allocate their workspace from a context-owned arena; it grows
 *    to the largest operation run so far (returning smaller free chunks to
 *    the device first, after a device-wide synchronisation) and keeps every
 *    chunk used during a stream capture.  The first call of an operation with
 *    a given shape builds and caches its plan (encoded plaintexts, index
 *    tables) and may allocate.  A repeated call with the same shapes and
 *    weights allocates nothing and can be captured into a hipGraph.
 *  - Secret material (Design Overview: the client holds the secret key, the
 *    server only evaluation keys): fenc_ctx_create makes a client context
 *    (secret key drawn from params.seed; it can also evaluate, generating
 *    missing switching keys on demand); fenc_ctx_create_server makes a server
 *    context that never holds a secret key: it evaluates with switching keys
 *    imported from a client (fenc_key_export_galois / fenc_key_import) and
 *    ciphertexts imported in coefficient form (fenc_ct_import); encryption,
 *    decryption and key generation there fail with FENC_ENOKEY.
 */
#ifndef FENC_H
#define FENC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FENC_OK = 0,
  FENC_EINVAL = -1,        /* bad argument, shape or plan mismatch */
  FENC_ENOMEM = -2,        /* device allocation failed */
  FENC_ENOKEY = -3,        /* strict key mode and a rotation key is missing */
  FENC_ELEVEL = -4,        /* not enough ciphertext levels left */
  FENC_ESCALE = -5,        /* scale mismatch */
  FENC_ELAYOUT = -6,       /* layout not accepted by the operation */
  FENC_EHIP = -7,          /* HIP runtime error */
  FENC_EUNSUPPORTED = -8   /* valid request outside what the library implements */
} fenc_status;

typedef struct fenc_ctx fenc_ctx;

/* RNS-CKKS parameters.  Primes: the n_q largest primes below 2^q_bits with
 * q = 1 mod 2N (descending), then the n_p next primes below 2^p_bits for the
 * special modulus P.  Hybrid key switching with dnum digits of
 * ceil(n_q/dnum) limbs; n_p must be >= the digit size and p_bits == q_bits
 * (q_bits <= 50).  log2_scale: Delta = 2^log2_scale.  seed keys the secret
 * and evaluation keys (SplitMix64 counter streams). */
typedef struct {
  uint32_t log_n, n_q, q_bits, n_p, p_bits, dnum;
  double log2_scale;
  uint64_t seed;
} fenc_params;

enum { FENC_LAYOUT_FRAGMENT = 0, FENC_LAYOUT_VECTOR = 1, FENC_LAYOUT_TOKENS = 2 };

/* Slot layout of an encrypted tensor [bs][c][h][w].
 * FRAGMENT (Alg. fragment-packing): M = next power of two >= max(h, w),
 *   block size S | M, m = M/S; bs_g images share a ciphertext,
 *   chan_per_ct = C' = (N/2)/(bs_g m^2) channel positions per ciphertext;
 *   element (b, ch, y, x) with (dil*y, dil*x) = (bi*S+u, bj*S+v) sits in
 *   ciphertext ((b/bs_g * n_cg + ch/C') * S + u) * S + v at slot
 *   ((ch%C' * m + bi) * m + bj) * bs_g + b%bs_g.  With replicate != 0 the
 *   c < C' channels are repeated in every group of c positions.
 * VECTOR (FC input/output): one ciphertext per batch group, feature f of the
 *   flattened [c][h][w] tensor at slot pos[f]*bs_g + b%bs_g with d = (N/2)/bs_g
 *   positions; pos is the context-owned map map_id (0: identity).
 * TOKENS (Discussions, extensibility to Transformers): bs tokens of c = E
 *   features (h = w = 1), each embedding split into S fragments: feature e
 *   goes to fragment e%S at position p = e/S; a fragment spans n_cg
 *   ciphertexts of d = (N/2)/bs_g positions; element (t, e) sits in
 *   ciphertext ((t/bs_g * S + e%S) * n_cg + p/d) at slot (p%d)*bs_g + t%bs_g.
 *   A ciphertext holds E/S features of S times more tokens than one holding
 *   whole embeddings. */
typedef struct {
  int32_t kind;
  int32_t bs, c, h, w;
  int32_t M, S, m;
  int32_t bs_g, chan_per_ct;
  int32_t n_bg, n_cg;
  int32_t replicate, dil;
  int32_t level;
  int32_t d, n_feat;
  double scale;
  uint64_t map_id;
} fenc_layout;

typedef struct {
  uint64_t* data;          /* device pointer, caller-owned */
  fenc_layout lay;
} fenc_ctbatch;

/* Operation counters, mirroring the paper's per-sample count table columns
 * (rotations, key switches, NTTs, ciphertexts, multiplications). */
typedef struct {
  int64_t rot_inner, rot_outer, rot_other;   /* rotations by role */
  int64_t keyswitch;                          /* rotations + relinearisations */
  int64_t modup, moddown;
  int64_t ntt_limbs, intt_limbs;              /* single-limb transforms */
  int64_t pmult, smult, rescale, relin;
  int64_t launches;                           /* kernel launches */
  int64_t cts_out;                            /* ciphertexts produced */
} fenc_counters;

enum { FENC_MODE_BATCHED = 0, FENC_MODE_PER_OP = 1 };

/* ---- context ------------------------------------------------------------
 * Creates a context (host tables only; device tables are built on first use
 * on the current HIP device).  Errors: EINVAL for unsupported parameters. */
int fenc_ctx_create(const fenc_params* p, fenc_ctx** out);
/* A server context: the same parameters and tables, no secret key. */
int fenc_ctx_create_server(const fenc_params* p, fenc_ctx** out);
void fenc_ctx_destroy(fenc_ctx* ctx);
/* n_q + n_p primes of the context (host array). */
int fenc_ctx_primes(const fenc_ctx* ctx, uint64_t* out);
/* Execution mode: BATCHED (default) launches every key switch, product and
 * rescale of a layer stage in one grid; PER_OP launches each homomorphic
 * operation of each ciphertext separately.  Results are identical. */
int fenc_set_mode(fenc_ctx* ctx, int mode);
/* Convolution plaintext form (Arch-aware Ct Compression, scale split): when
 * per-position weights are needed, the layer's weight diagonals are encoded as
 * full-scale plaintexts if those of one batch group (they repeat in every
 * group) fit `bytes` of device memory (default 1 GiB);
 * otherwise 0/1 position masks at scale Delta_m are combined with integer
 * weight codes at scale Delta_w, Delta_w * Delta_m = q_l * Delta / scale_in,
 * so one rescale follows either way.  The choice changes the ciphertext bits,
 * not the decrypted values beyond rounding. */
int fenc_set_plaintext_budget(fenc_ctx* ctx, int64_t bytes);
/* Key switching (hybrid, Background): where the key inner product finds each
 * digit's own limbs of the extended digits.  A stage whose extended digits
 * (all its ciphertexts) take at most `bytes` (default 1 GiB) has them
 * copied by ModUp and read with the rest, which is then still in cache; a
 * larger stage reads them from the input ciphertexts, saving the copy's
 * traffic.  0: never copied.  Residues do not change. */
int fenc_set_own_copy_limit(fenc_ctx* ctx, int64_t bytes);
/* Workspace limit (default 32 GiB, 0: none): an operation whose workspace
 * would exceed it runs over tiles of whole batch groups, one after the other,
 * each with the plan of the smaller batch.  Batch groups never share a
 * ciphertext, so tiles change neither results nor the arithmetic.  The limit
 * bounds the context's arena for batches of more than one group; a single
 * batch group is never split.  Errors: EINVAL for a negative limit. */
int fenc_set_workspace_limit(fenc_ctx* ctx, int64_t bytes);
/* Kernel profiling: every later launch of the named kernel (e.g. "kip",
 * "ntt_fwd_cols", "gmac") outside graph capture is bracketed by HIP events on
 * its stream; fenc_profile_result returns the summed event time, the number
 * of launches and their algorithmic HBM bytes (compulsory reads and writes).
 * NULL stops profiling and drops collected events. */
int fenc_profile_kernel(fenc_ctx* ctx, const char* name);
int fenc_profile_result(fenc_ctx* ctx, double* total_ms, int64_t* launches, double* bytes);
/* With the name "*" every kernel is profiled; this writes one line per kernel
 * ("name total_ms launches bytes modmuls\n": algorithmic HBM bytes and modular
 * products, 0 where not counted; a NUL-terminated host string of at most len
 * bytes, EINVAL when it does not fit).  Synchronises on the events. */
int fenc_profile_summary(fenc_ctx* ctx, char* buf, int64_t len);
int fenc_stats(const fenc_ctx* ctx, fenc_counters* out);
void fenc_stats_reset(fenc_ctx* ctx);
/* Device bytes held by the context (tables, keys, plans, workspace). */
int64_t fenc_device_bytes(const fenc_ctx* ctx);
const char* fenc_last_error(void);

/* ---- keys (Background, eq. rotation; hybrid key switching) --------------
 * Generates rotation keys for left rotations by rot_steps[i] slots and, if
 * relin != 0, the relinearisation key.  Keys are deterministic functions of
 * (seed, Galois element).  strict != 0 makes later operations fail with
 * FENC_ENOKEY instead of generating a missing key on demand. */
int fenc_keygen(fenc_ctx* ctx, const int32_t* rot_steps, uint32_t n_steps, int relin, int strict);
/* Host copy of a switching key in coefficient form [dnum'][2][n_q+n_p][N]
 * (shift = slot rotation, or INT32_MIN for the relinearisation key). */
int fenc_key_export(fenc_ctx* ctx, int32_t shift, uint64_t* out);
/* Galois elements of the switching keys the context holds (0: the
 * relinearisation key), at most cap written to galois; returns how many the
 * context holds (or a negative fenc_status). */
int fenc_key_list(const fenc_ctx* ctx, uint64_t* galois, int32_t cap);
/* fenc_key_export by Galois element g (0: relinearisation key). */
int fenc_key_export_galois(fenc_ctx* ctx, uint64_t g, uint64_t* out);
/* Adds the switching key of Galois element g (0: relinearisation), host
 * coefficient form [dnum'][2][n_q+n_p][N] as fenc_key_export writes it, to a
 * context (typically a server context).  Errors: EINVAL for an element that
 * is not an odd g < 2N other than 1, a key the context already holds, or a
 * residue not below its prime. */
int fenc_key_import(fenc_ctx* ctx, uint64_t g, const uint64_t* in);

/* ---- planning (Conv-aware Encoding: Alg. fragment-packing, eq. total-rot,
 * eq. opt, Theorem 1) --------------------------------------------------------
 * Layout for a fresh [bs][c][h][w] input whose next layer is a k x k
 * convolution to cout channels: block size S minimises eq. (total-rot) over
 * powers of two satisfying eq. (opt) (ties: smaller S); s_override > 0 forces
 * S.  Host only. */
int fenc_plan_layout(const fenc_ctx* ctx, uint32_t bs, uint32_t c, uint32_t h, uint32_t w,
                     uint32_t k_next, uint32_t cout_next, int32_t s_override, fenc_layout* out);
/* Block size per layer of a layer chain (the paper adapts S between layers
 * with HEAR-style rot-mask-add, Evaluation Methodology; eq. total-rot prices
 * one layer).  layers[i].kind: FENC_LAYER_CONV (cout, k, stride, pad, groups),
 * FENC_LAYER_POOL (2x2 average), FENC_LAYER_ACT (polynomial, no layout
 * change) or FENC_LAYER_COMPRESS (into the FC vector layout).  A dynamic
 * program over the layout after each layer chooses the input block size and,
 * before up to max_repacks convolutions whose input has at most 2^22
 * elements, a repack into a fragment layout of another block size
 * (fenc_compress with that target, one level each),
 * minimising key switches + MAC terms / 16: each convolution's exact key
 * switches and scalar MAC terms (as fenc_conv2d_keyswitches), each repack's
 * key switches (as fenc_compress_keyswitches), three rotations per
 * ciphertext for a pool at S = 1 (pools at S >= 2 sum fragments), one
 * relinearisation per ciphertext for an activation (two when its k field,
 * the degree, is 3) and the final compression.  The paper's objective is the
 * rotation count; the MAC term weight (a term moves about a ciphertext, a key
 * switch 10-20) keeps a block size whose replicated channels multiply the
 * scalar MACs from winning on rotations alone.  Ties: fewer repacks, then
 * smaller block sizes.  block_size[i] (n_layers entries, caller-owned): the
 * block size layer i runs at; block_size[0] is the input's encoding when
 * layer 0 is a convolution, and a convolution whose entry differs from the
 * block size its input arrives in is preceded by that repack.  keyswitches,
 * mac_terms (each may be NULL): the chosen chain's totals.  Host only.
 * Errors: EINVAL for a bad argument or layer kind, EUNSUPPORTED when no
 * block size admits some layer. */
enum { FENC_LAYER_CONV = 0, FENC_LAYER_POOL = 1, FENC_LAYER_ACT = 2, FENC_LAYER_COMPRESS = 3 };
typedef struct {
  int32_t kind, cout, k, stride, pad, groups;
} fenc_layer;
int fenc_plan_network(const fenc_ctx* ctx, uint32_t bs, uint32_t c, uint32_t h, uint32_t w,
                      const fenc_layer* layers, uint32_t n_layers, int32_t max_repacks, int32_t* block_size,
                      int64_t* keyswitches, int64_t* mac_terms);
/* Key switches fenc_conv2d performs on input layout `in` (inner: distinct
 * hoisted rotated copies; outer: one per output ciphertext and nonzero
 * diagonal; Conv-aware Encoding, eq. inner / eq. outer-rot give their
 * worst cases) and its scalar MAC terms in the mask-basis form (mac_terms,
 * may be NULL), and the key switches of fenc_compress from `in` to `target`
 * (NULL: the library's vector target), without building anything.  Host
 * only. */
int fenc_conv2d_keyswitches(const fenc_ctx* ctx, const fenc_layout* in, uint32_t cout, uint32_t k,
                            uint32_t stride, uint32_t pad, uint32_t groups, int64_t* inner, int64_t* outer,
                            int64_t* mac_terms);
int fenc_compress_keyswitches(const fenc_ctx* ctx, const fenc_layout* in, const fenc_layout* target,
                              int64_t* keyswitches);
/* TOKENS layout of n tokens with E features split into S fragments (S <= E),
 * at the top level and scale Delta.  group > 0 fixes the tokens per
 * ciphertext (a power of two; a linear layer's output keeps its input's);
 * 0 takes the most that fit the largest fragment's next power of two of
 * positions.  Host only.  Errors: EINVAL for a bad shape or grouping. */
int fenc_plan_tokens(const fenc_ctx* ctx, uint32_t n, uint32_t E, uint32_t S, uint32_t group, fenc_layout* out);
int fenc_layout_n_ct(const fenc_layout* lay);
int64_t fenc_ct_bytes(const fenc_ctx* ctx, const fenc_layout* lay);
/* First (ciphertext, slot) of element (b, ch, y, x).  Host only. */
int fenc_layout_slot(const fenc_ctx* ctx, const fenc_layout* lay, int b, int ch, int y, int x,
                     int32_t* ct, int32_t* slot);
/* Feature -> position map of a VECTOR layout (n_feat entries). */
int fenc_layout_map(const fenc_ctx* ctx, const fenc_layout* lay, int32_t* pos);

/* ---- client side (problem statement: the client encodes and encrypts by the
 * index-slot mapping and decrypts the result) ------------------------------
 * Encodes x[bs][c][h][w] (host) into integer plaintexts pt[n_ct][level+1][N]
 * (host, coefficient form): round(Delta * tau^{-1}(slots)), canonical
 * embedding, half away from zero. */
int fenc_encode_fragment(fenc_ctx* ctx, const double* x, const fenc_layout* lay, uint64_t* pt);
/* Encodes one slot vector z[N/2] at `scale` into pt[level+1][N]. */
int fenc_encode_slots(fenc_ctx* ctx, const double* z, int32_t level, double scale, uint64_t* pt);
/* Secret-key encryption of host plaintexts pt[n_ct][level+1][N] (coefficient
 * form) into out->data (device); ciphertext t draws its randomness from
 * (enc_seed, t).  out->lay is copied from lay. */
int fenc_encrypt(fenc_ctx* ctx, const uint64_t* pt, const fenc_layout* lay, uint64_t enc_seed,
                 fenc_ctbatch* out, void* stream);
/* Decrypts and decodes into x[bs][c][h][w] (host).  Synchronises the stream. */
int fenc_decrypt(fenc_ctx* ctx, const fenc_ctbatch* in, double* x, void* stream);
/* m = c0 + c1 s for every ciphertext and limb, coefficient form, host
 * [n_ct][level+1][N].  Synchronises the stream. */
int fenc_decrypt_raw(fenc_ctx* ctx, const fenc_ctbatch* in, uint64_t* m, void* stream);

/* ---- ciphertext transfer --------------------------------------------------
 * Host coefficient form [n_ct][2][level+1][N] <-> device NTT form.  Both
 * synchronise the stream. */
int fenc_ct_export(fenc_ctx* ctx, const fenc_ctbatch* in, uint64_t* host, void* stream);
int fenc_ct_import(fenc_ctx* ctx, const uint64_t* host, fenc_ctbatch* out, void* stream);

/* ---- server side: the hot path ---------------------------------------------
 * Convolution (eq. multi-channel-conv) on a FRAGMENT layout with dil == 1:
 * w[cout][c/groups][k][k] (host, float64, cross-correlation), stride | S,
 * zero padding pad, groups | c and | cout.  Hoisted inner rotations (one
 * ModUp per input ciphertext), masked scalar multiply-accumulate, diagonal
 * outer rotations summed with one ModDown per output ciphertext, one rescale.
 * bias: NULL or cout host doubles added to every valid output slot of their
 * channel, encoded at the output scale after the rescale (no level).
 * s_out == 0: output in the convolution's own layout (same m, bs_g, C'; S and
 *   M divided by the stride; channels at positions 0.. of each ciphertext).
 * s_out > 0: output written straight into the Alg. fragment-packing layout of
 *   the output tensor with block size s_out (M from the output's size,
 *   channels repeated in every group of positions when cout divides C'): the
 *   Arch-aware Ct Compression repack fused with the convolution.  Its 0/1
 *   masks multiply the convolution's own plaintexts (weights at Delta_w and
 *   masks at Delta_m, Delta_w Delta_m = q_l Delta / scale_in) and its shifts
 *   merge with the outer rotations, so it adds no product and no level; a
 *   change of block size moves pixel rows by many shifts and costs rotations.
 * Output level - 1, scale exactly Delta.  Errors: EINVAL (shapes, negative
 * s_out, non-finite bias), EUNSUPPORTED (stride not dividing S), ELAYOUT
 * (s_out not a power of two dividing the output's padded side), ELEVEL. */
int fenc_conv2d(fenc_ctx* ctx, const fenc_ctbatch* in, const double* w, const double* bias, uint32_t cout,
                uint32_t k, uint32_t stride, uint32_t pad, uint32_t groups, int32_t s_out, fenc_ctbatch* out,
                void* stream);
/* 2x2 average pooling, stride 2 (Evaluation methodology, implementation):
 * S >= 2 sums the four fragments of each block (no rotation); S == 1 sums
 * three hoisted rotations and doubles dil.  The factor 1/4 is carried in the
 * scale (x4); no level is consumed. */
int fenc_avgpool2(fenc_ctx* ctx, const fenc_ctbatch* in, fenc_ctbatch* out, void* stream);
/* Polynomial activation p(x) = coeffs[0] + coeffs[1] x + ... + coeffs[degree] x^degree,
 * degree <= 3 (Evaluation Methodology: ReLU replaced by a low-degree polynomial;
 * coeffs is a host array of degree+1 doubles).  Leading zero coefficients lower
 * the degree.  All terms of one rescale share one scale reached by integer
 * codes, and the leading coefficient is carried by that scale, so the output
 * scale is within a small factor of Delta (exact value in out->lay.scale):
 *   degree <= 2: one tensor product (x*x times an integer) with c1 x + c0
 *                added, relinearised and rescaled together (one level);
 *   degree 3:    x^2 as above, times u = c3 x + c2 with c1 x + c0 added,
 *                relinearised and rescaled together (two levels).
 * "Together": (d0, d1) P + KIP(d2) divided by P q_l in one ModDown whose fast
 * base conversion takes the special primes and q_l at once (Background:
 * hybrid key switching and Rescale, taken as one step). 
 * out->data may equal in->data: the output then overwrites the input (every
 * batch group's input is read before its output is written, and outputs are
 * no larger than inputs), which saves one activation-sized buffer.
 * Errors: EUNSUPPORTED for degree > 3, ELEVEL without the levels, EINVAL for
 * non-finite coefficients, ESCALE when a code exceeds 2^120. */
int fenc_poly_act(fenc_ctx* ctx, const fenc_ctbatch* in, const double* coeffs, uint32_t degree,
                  fenc_ctbatch* out, void* stream);
/* Arch-aware Ct Compression (rot-mask-add) of a batch into a target layout
 * of the same tensor: FRAGMENT (the Alg. fragment-packing layout of any block
 * size, e.g. from fenc_plan_layout with s_override, or the dense repeated-
 * channel layout) or VECTOR (an FC input; map_id 0 or a map the library
 * returned); target == NULL: one VECTOR ciphertext per batch group with each
 * source ciphertext's valid positions placed at the first free offset.  The
 * target's level and scale are ignored.  Each source ciphertext is rotated
 * once per shift it needs (one ModUp per source), the rotated copies are
 * masked to the slots that move and summed per target (one ModDown per
 * target); the masks are encoded at q_l Delta / scale_in and one rescale
 * restores Delta, so the standalone repack costs one level (fused with a
 * convolution it costs none: fenc_conv2d's s_out).  Errors: ELAYOUT for a
 * target of another tensor or an invalid one, EUNSUPPORTED when the default
 * vector does not fit one ciphertext, ELEVEL. */
int fenc_compress(fenc_ctx* ctx, const fenc_ctbatch* in, const fenc_layout* target,
                  fenc_ctbatch* out, void* stream);
/* Fully connected layer y = W x + bias, w[dout][n_feat] (host), bias NULL or
 * dout host doubles, on a VECTOR layout: diagonal method with baby-step
 * giant-step (hoisted baby steps, giant steps summed with one ModDown), one
 * rescale, the bias added at the output scale; output features at positions
 * 0..dout-1.
 * On a TOKENS layout (Discussions, extensibility to Transformers) it is the
 * linear layer of every token: the output is the TOKENS layout of dout
 * features with the input's S and bs_g; each (input ct, output ct) pair of a
 * token group is a d x d block taken by the same diagonal method, the baby
 * steps hoisted once per input ct and shared by every output ct, each output
 * ct summing all its inputs before one giant-step sum.  Only diagonals with a
 * nonzero weight are multiplied. */
int fenc_fc(fenc_ctx* ctx, const fenc_ctbatch* in, const double* w, const double* bias, uint32_t dout,
            fenc_ctbatch* out, void* stream);

/* ---- building blocks exposed for testing --------------------------------
 * Hoisted rotations of every ciphertext of `in` by shifts[0..n) (left, in
 * slots); out holds n_ct * n ciphertexts, ct-major. */
int fenc_rotate(fenc_ctx* ctx, const fenc_ctbatch* in, const int32_t* shifts, uint32_t n,
                fenc_ctbatch* out, void* stream);
/* out = z0 + sum_i Rot(z_i, shifts[i]) with one ModDown; zs holds n
 * ciphertexts, z0 may be NULL. */
int fenc_rotate_sum(fenc_ctx* ctx, const fenc_ctbatch* z0, const fenc_ctbatch* zs,
                    const int32_t* shifts, uint32_t n, fenc_ctbatch* out, void* stream);
int fenc_rescale(fenc_ctx* ctx, const fenc_ctbatch* in, fenc_ctbatch* out, void* stream);
/* Rescale that allocates nothing, for callers that cannot allocate device
 * memory (code under hipGraph capture, serving loops, harnesses that forbid
 * hipMalloc).  Same operation and residues as fenc_rescale; its workspace
 * ([n_ct][2][N] words for the last limb and [n_ct][2][level][N] for its lift
 * to the other limbs, every word written before it is read, nothing needs
 * clearing) lives in the library's static device array of 64 MiB instead of
 * the context's arena: at most 64 MiB / ((1 + level) * 16 * N) ciphertexts
 * per call (6 at N = 2^15 and level 19, 2 at N = 2^16 and level 23).
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other streams, other threads, other contexts) race and must be
 * serialised by the caller.  The output is the caller's.  Errors: EINVAL
 * when the batch needs more scratch than the array holds, when the context
 * has no device tables on the current device yet or none for this level (any
 * earlier fenc_rescale at this level builds them), ELEVEL at level 0. */
int fenc_rescale_noalloc(fenc_ctx* ctx, const fenc_ctbatch* in, fenc_ctbatch* out, void* stream);
/* Forward (inverse != 0: inverse) NTT of rows[n][N] (host) modulo prime index
 * prime[i] of row i, through the device kernels. */
int fenc_ntt_rows(fenc_ctx* ctx, uint64_t* rows, const int32_t* prime, uint32_t n, int inverse);
/* Sampler and codec hooks (host only). */
/* Hoisting schedule of convolutions and S = 1 average pooling (Motivation,
 * inner rotations; the paper leaves the placement of ModDown open).  Mode 1
 * (default): the hoisted rotated copies stay in the extended basis Q_l U P
 * as (KIP_0 + P sigma(c0), KIP_1), the linear combination (scalar weights,
 * masks or diagonals encoded over Q_l U P) is taken there, unrotated inputs
 * enter as P x, and each combined ciphertext is moved down once.  Mode 0:
 * every rotated copy is moved down.  The two modes round differently, so the
 * residues differ; each matches the oracle's schedule of the same number.
 * Mode 2: each layer's plan takes the schedule whose modelled HBM traffic is
 * smaller (schedule 0 pays a ModDown per rotated copy over nl limbs; schedule
 * 1 combines over nl + K limbs, lifts the unrotated inputs and pays a ModDown
 * per combined ciphertext); the choice is a function of the layer's shape
 * and weights' sparsity pattern, kept in its cached plan, the same on every
 * device.  Errors: EINVAL for other modes. */
int fenc_set_hoisting(fenc_ctx* ctx, int mode);
/* The schedule (0 or 1) the most recent fenc_conv2d, fenc_avgpool2 or
 * fenc_compress on this context ran with (0 where the layer has no rotated
 * copies), -1 before any; with mode 2 this is how a caller learns, and can
 * reproduce elsewhere, the schedule a layer's plan chose. */
int fenc_last_hoisting(const fenc_ctx* ctx);
/* Outer rotations of a convolution by baby-step giant-step (Motivation, HE
 * multi-channel convolution, eq. multi-channel-conv, which assumes BSGS).
 * The C' diagonals z_r of an output are rotated by r s (s = m^2 BS_g slots)
 * and summed.  With baby step n1, diagonal r = i + n1 j is formed from copies
 * rotated by i s more (extra hoisted rotations of the same inputs, shared by
 * every output) and from plaintexts encoded rotated by i s, summed into the
 * giant-step accumulator j, and y = sum_j Rot(Z_j, n1 j s): n2 - 1 = ceil(C'/n1)
 * - 1 rotations per output instead of C' - 1, against up to n1 - 1 more per
 * input copy.  n1 >= 1 fixes the baby step (1, the default: the plain form;
 * larger values are capped at C'); 0 chooses, per layer, the power of two up
 * to C' with the fewest key switches (ties: the smaller), kept in the cached
 * plan.  A convolution fused with a repack (s_out > 0) uses the plain form.
 * The baby step changes the residues; the oracle takes the same parameter.
 * fenc_last_baby_step: the baby step of the most recent fenc_conv2d, -1
 * before any.  Errors: EINVAL for n1 < 0. */
int fenc_set_baby_step(fenc_ctx* ctx, int n1);
int fenc_last_baby_step(const fenc_ctx* ctx);
/* NTT pass shapes, 8 ints: for [forward columns, forward rows, inverse rows,
 * inverse columns] the radix bits of a register round (3: radix 8, 4: radix
 * 16) and the log2 of the columns (column pass) or chunks (row pass) a block
 * stages, -1 for the default.  The shapes change speed, never results.  The
 * first device use times the candidates on the current GPU and keeps the
 * fastest (not on the CPU emulator, not during stream capture); setting a
 * shape turns that off.  Errors: EINVAL for radix bits other than 3/4 or a
 * tile beyond the pass or above 64 KiB of LDS. */
int fenc_ntt_config(fenc_ctx* ctx, int32_t* out);
int fenc_set_ntt_config(fenc_ctx* ctx, const int32_t* cfg);
uint64_t fenc_sample_word(uint64_t seed, uint64_t tag, uint64_t i);
int fenc_sample_gauss(uint64_t seed, uint64_t tag, uint64_t i);
int fenc_encode_int(int32_t log_n, const double* z, double scale, int64_t* m);

#ifdef __cplusplus
}
#endif
#endif /* FENC_H */
