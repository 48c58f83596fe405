/*
 * ckr.h -- C ABI of the MI355X (gfx950) library for encrypted ranking,
 * order statistics and sorting under RNS-CKKS (arXiv 2412.15126).
 *
 * The paper's problem statement fixes the user-level calls: an encrypted
 * vector v of N reals goes in; out come its fractional ranking (Algorithm
 * Rank, section 3.1), a one-hot mask of its minimum with the minimum's value
 * (Algorithm Order Statistic, section 3.2, with the Tie-Correction Offset of
 * section 4), or its sorted form (Algorithm Sorting, section 3.3).  The
 * comparison function is the f/g composite of section 2.2,
 *   Cmp(x, y) = (f^{d_f}(g^{d_g}(x - y)) + 1) / 2.
 *
 * Conventions for every call:
 *  - Handles returned to the caller are caller-owned; release each with the
 *    matching *_free.  Host arrays are borrowed for the duration of the call.
 *  - Device memory belongs to the context.  It comes from hipMalloc unless the
 *    caller installs an allocator (ckr_context_set_allocator).
 *  - No exception or abort crosses this boundary.  Every call returns a
 *    ckr_status; the message of the last failure on the calling thread is
 *    available from ckr_last_error().
 *  - Work is issued on the context's stream (the null stream unless set).
 *    Calls that return host data (decrypt, export) synchronise that stream.
 *  - Results are deterministic: equal seeds give equal ciphertexts, bit for
 *    bit, whether a query runs alone or inside a batch.
 *  - A ciphertext at level l holds 2 polynomials x (l+1) RNS limbs x n
 *    coefficients.  Exported form: uint64 words [poly][limb][coeff], each a
 *    canonical residue in [0, q_limb), in the coefficient domain.
 */
#ifndef CKR_H
#define CKR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CKR_OK = 0,
    CKR_E_INVALID = -1, /* bad argument, null handle, residue >= q on import   */
    CKR_E_RANGE = -2,   /* N not a power of two in [2, 2^15], or N^2 > n/2      */
    CKR_E_DEPTH = -3,   /* ciphertext has too few levels for the circuit       */
    CKR_E_NOMEM = -4,   /* device allocation failed or HBM budget exceeded     */
    CKR_E_DEVICE = -5,  /* HIP runtime error                                   */
    CKR_E_BUSY = -6     /* ticket not finished within the timeout              */
} ckr_status;

typedef struct ckr_context ckr_context;
typedef struct ckr_keys ckr_keys;
typedef struct ckr_ct ckr_ct;

/* Parameter set.  Ring degree n = 2^log_n (10..17).  The ciphertext modulus
 * chain is q_0..q_{n_q-1}: q_0 is the largest prime below 2^q0_bits, the
 * others are rescaling primes chosen level by level, from the top, as the
 * unused prime nearest to the running scale (top scale 2^log_scale).  n_p
 * special primes (largest primes below 2^p_bits) serve hybrid key switching
 * with dnum digits.  Every prime is 1 mod 2n and below 2^50. */
typedef struct {
    uint32_t log_n;
    uint32_t n_q;
    uint32_t q0_bits;
    uint32_t log_scale;
    uint32_t n_p;
    uint32_t p_bits;
    uint32_t dnum;
} ckr_params;

/* Comparator (section 2.2), one of:
 *  - the f/g composite: g applied d_g times, then f applied d_f times
 *    (cheb = minimax = 0, d_g + d_f >= 1); each application consumes 3 levels;
 *  - the Chebyshev interpolant of the comparison function of Eq. (1) on
 *    [-1, 1] at the 2^(cheb-1) Chebyshev nodes (degree 2^(cheb-1) - 1),
 *    evaluated by Paterson-Stockmeyer in the Chebyshev basis in cheb levels
 *    (d_g = d_f = minimax = 0, 2 <= cheb <= 16).  The paper's experiments use
 *    this form for rank and minimum at N <= 256, up to degree 2^11 (cheb = 12);
 *  - the first `minimax` stages (1..5) of the minimax composite that section
 *    2.2 names as the alternative to f and g (d_g = d_f = cheb = 0): stage 0
 *    is the odd degree-7 polynomial closest to sign(x) in the maximum norm on
 *    [2^-8.5, 1], each later stage the one closest to 1 on the interval the
 *    previous stage maps that onto; 3 levels per stage.  Four stages rank
 *    N = 128 values at a 2^-10 gap exactly, where the four-fold f/g split
 *    g^3 f does not.
 * Any other combination is rejected with CKR_E_INVALID. */
typedef struct {
    uint8_t d_g;
    uint8_t d_f;
    uint8_t cheb;
    uint8_t minimax;
} ckr_sign;

/* Create a context on HIP device `hip_device`.  hbm_budget bounds the bytes
 * the context may hold on the device (0 = no bound); beyond it allocations
 * fail with CKR_E_NOMEM.  Derives the prime chain and uploads the transform
 * tables. */
ckr_status ckr_context_create(const ckr_params *params, int hip_device, size_t hbm_budget, ckr_context **out);
void ckr_context_free(ckr_context *ctx);

/* Issue all work on `hip_stream` (a hipStream_t, e.g. torch's current stream). */
ckr_status ckr_context_set_stream(ckr_context *ctx, void *hip_stream);

/* Route device allocations through alloc/free (e.g. PyTorch's caching
 * allocator).  Must be called before any key or ciphertext exists. */
ckr_status ckr_context_set_allocator(ckr_context *ctx, void *(*alloc)(size_t bytes, void *user),
                                     void (*free_fn)(void *ptr, void *user), void *user);

/* Moduli (n_q + n_p values: q chain then special primes) and per-level scales
 * (n_q values).  Either pointer may be NULL. */
ckr_status ckr_context_info(const ckr_context *ctx, uint64_t *moduli, double *scales);

/* Host-only: derive the modulus chain of `params` without a device.  moduli
 * receives n_q + n_p values, scales n_q values (either may be NULL). */
ckr_status ckr_params_derive(const ckr_params *params, uint64_t *moduli, double *scales);

/* Host-only: encode real slot values z[0..count) (other slots 0) at `scale`
 * into the n = 2^log_n signed coefficients m_j = round((2 scale / n) *
 * Re sum_k z_k zeta^{-j 5^k}), zeta = exp(i pi / n), rounding half away from
 * zero.  CKR_E_RANGE if a coefficient exceeds 2^62. */
ckr_status ckr_encode(uint32_t log_n, const double *z, uint32_t count, double scale, int64_t *m);

/* Host-only: `count` samples of the ChaCha20 stream keyed by `seed` with
 * nonce (purpose, id): kind 0 ternary, 1 centred binomial (eta = 21),
 * 2 uniform in [0, q). */
ckr_status ckr_sample(const uint8_t seed[32], uint32_t purpose, uint64_t id, int kind, uint64_t q, size_t count,
                      int64_t *out);

/* Device bytes currently held by the context and its high-water mark. */
ckr_status ckr_context_memory(const ckr_context *ctx, size_t *in_use, size_t *high_water);

/* Key generation from a 32-byte seed (ChaCha20 streams, RFC 8439).  Makes the
 * secret key (kept in host memory), the public key, the relinearisation key
 * and the rotation keys the circuits need for every N in Ns[0..nN).  Keys
 * cover limbs q_0..q_max_level plus the special primes and stay resident on
 * the device.  `what` selects circuits: bit 0 rank, bit 1 argmin, bit 2 sort
 * (their rotation sets differ; bits 1 and 2 add the conjugation key).  An N
 * that is not a power of two gets the keys of the next power of two, the
 * layout its padded rank uses. */
ckr_status ckr_keygen(ckr_context *ctx, const uint8_t seed[32], uint32_t max_level, const uint32_t *Ns, size_t nN,
                      uint32_t what, ckr_keys **out);
void ckr_keys_free(ckr_keys *keys);

/* Rotation keys for explicit slot shifts (k > 0: left rotation new[j] = old[j+k];
 * k < 0: right rotation), added to `keys`. */
ckr_status ckr_keys_add_rotations(ckr_context *ctx, ckr_keys *keys, const int64_t *shifts, size_t count);

/* Encrypt v[0..N) into slots [0, N) (others 0) at `level` with the public key;
 * randomness from a 32-byte seed. */
ckr_status ckr_encrypt(ckr_context *ctx, const ckr_keys *keys, const double *v, uint32_t N, uint32_t level,
                       const uint8_t seed[32], ckr_ct **out);

/* Decrypt and decode slots [0, count) (real parts) into out. */
ckr_status ckr_decrypt(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *ct, double *out, uint32_t count);

/* Fractional ranking (Algorithm Rank): out slots [0,N) hold rank(v_j).
 * tie_correct != 0 adds the tie-correction offset (section 4), so the output
 * is a permutation of 1..N.  N need not be a power of two (section 3.1): the
 * vector is then zero-padded to the next power of two Np (slots [N, Np) of v
 * must be zero, as ckr_encrypt leaves them) and the comparison matrix is
 * masked to its N x N block, one more level.  Keys: those of ckr_keygen for
 * N (generated for Np).  The output sits at level(v) - ckr_rank_depth_n(N).
 * Errors: CKR_E_RANGE (N < 2 or Np^2 > n/2), CKR_E_DEPTH, CKR_E_INVALID. */
ckr_status ckr_rank(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *v, uint32_t N, ckr_sign cmp, int tie_correct,
                    ckr_ct **out);

/* Levels consumed by ckr_rank / ckr_argmin / ckr_sort / ckr_order_stat for
 * the given comparators. */
uint32_t ckr_rank_depth(ckr_sign cmp, int tie_correct);
uint32_t ckr_rank_depth_n(uint32_t N, ckr_sign cmp, int tie_correct);
uint32_t ckr_argmin_depth(ckr_sign cmp, ckr_sign ind);
uint32_t ckr_sort_depth(ckr_sign cmp, ckr_sign ind);
uint32_t ckr_sort_col_depth(ckr_sign cmp, ckr_sign ind);
uint32_t ckr_order_stat_depth(uint32_t N, uint32_t k, ckr_sign cmp, ckr_sign ind, int tie_correct);

/* Minimum with tie-correction (Algorithm Order Statistic with k = 1):
 * onehot slots [0,N) hold 1 at the lowest index among the minima, 0
 * elsewhere; value slot 0 holds the minimum.  `ind` is the composition of the
 * one-sided indicator Cmp(1.5, k). */
ckr_status ckr_argmin(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *v, uint32_t N, ckr_sign cmp, ckr_sign ind,
                      ckr_ct **onehot, ckr_ct **value);

/* Sorting (Algorithm Sorting), distinct inputs: out slots [0,N) hold v in
 * increasing order. */
ckr_status ckr_sort(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *v, uint32_t N, ckr_sign cmp, ckr_sign ind,
                    ckr_ct **out);

/* Column-form sorting (section 3.3, the variant without the final
 * transposition): the comparator's operands are swapped and the ranks are
 * summed by SumC into column 0, the sort then runs with rows and columns
 * exchanged and ReplC(TransR(v)) from the rank as the value matrix, and
 * SumR leaves the sorted vector in slots [0,N).  One level
 * (ckr_sort_col_depth = ckr_sort_depth - 1) and log N rotations fewer than
 * ckr_sort; no TransC rotation keys needed (ckr_keygen's argmin set).
 * Distinct inputs; errors as ckr_sort. */
ckr_status ckr_sort_col(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *v, uint32_t N, ckr_sign cmp,
                        ckr_sign ind, ckr_ct **out);

/* Order statistic k (Algorithm Order Statistic, section 3.2): onehot slots
 * [0,N) hold 1 at the k-th smallest element and 0 elsewhere; value slot 0
 * holds that element (k = 1 the minimum, k = N the maximum).  tie_correct != 0
 * adds the tie-correction offset (section 4): equal values then take
 * consecutive orders, lowest index first, so argmax lands on the highest
 * index among the maxima; without it the values must be distinct.  `ind` is
 * the indicator's composition: one-sided for k = 1 and k = N, the window
 * Cmp(x, -1/2) (1 - Cmp(x, 1/2)) otherwise.  onehot sits at level(v) - depth
 * + 1, value at level(v) - depth (ckr_order_stat_depth).  Errors: CKR_E_RANGE
 * (N), CKR_E_INVALID (k outside [1, N], empty composition), CKR_E_DEPTH. */
ckr_status ckr_order_stat(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *v, uint32_t N, uint32_t k,
                          ckr_sign cmp, ckr_sign ind, int tie_correct, ckr_ct **onehot, ckr_ct **value);

/* Order statistic k without tie-correction, with the value by division
 * (section 3.2): the mask O (onehot, slots [0,N)) marks every element of
 * fractional rank k -- several when equal values share that rank, none when
 * no element has it -- and value slot 0 holds SumC(O v) / SumC(O), computed
 * with `iters` (2..24) Goldschmidt steps on the count normalised by
 * 2/(N + 1) (relative error (1 - x)^(2^iters), x = 2 count / (N + 1)).  With
 * no element of rank k the value is 0 up to noise times 2^iters.  The
 * `count` inputs (single ciphertexts at one level, borrowed) run as one
 * batch; onehot[i] / value[i] (caller-owned) receive input i's results, the
 * value at level(v) - ckr_order_stat_div_depth.  Errors: as ckr_order_stat,
 * CKR_E_INVALID for iters outside [2, 24] or inputs at different levels. */
ckr_status ckr_order_stat_div(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *const *v, size_t count, uint32_t N,
                              uint32_t k, ckr_sign cmp, ckr_sign ind, uint32_t iters, ckr_ct **onehot,
                              ckr_ct **value);
uint32_t ckr_order_stat_div_depth(uint32_t N, uint32_t k, ckr_sign cmp, ckr_sign ind, uint32_t iters);

/* Order statistics over a window of ranks [a, b] (Algorithm Order Statistic,
 * section 3.2, with its median remark of section 4): onehot slots [0,N) hold 1
 * at the elements whose rank lies in [a, b] and 0 elsewhere; value slot 0
 * holds the mean of the order statistics a..b (SumC(O v) / (b - a + 1)).  The
 * median of an even N is a = N/2, b = N/2 + 1, of an odd N a = b = (N + 1)/2;
 * a = b = k gives ckr_order_stat's result bit for bit.  With tie_correct != 0
 * equal values take consecutive ranks, lowest index first, and N need not be
 * a power of two (zero-padded to the next one, section 3.1; the keys must be
 * made for that N); without it N is a power of two and the values distinct.
 * The indicator `ind` is one-sided for a = 1 (Cmp(b + 1/2, k_j)) and b = N
 * (Cmp(k_j, a - 1/2)), the window Cmp(k_j, a - 1/2) (1 - Cmp(k_j, b + 1/2))
 * otherwise, each argument over N.  The `count` inputs (single ciphertexts at
 * one level, borrowed) run as one batch (graph-captured after the first call
 * of a shape); onehot[i] / value[i] (caller-owned) receive input i's results,
 * onehot at level(v) - depth + 1, value at level(v) - depth
 * (ckr_order_range_depth).  Errors: CKR_E_RANGE (N), CKR_E_INVALID (not
 * 1 <= a <= b <= N, the window [1, N], a padded N without tie-correction,
 * empty composition, inputs not single ciphertexts of one level),
 * CKR_E_DEPTH. */
ckr_status ckr_order_range(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *const *v, size_t count, uint32_t N,
                           uint32_t a, uint32_t b, ckr_sign cmp, ckr_sign ind, int tie_correct, ckr_ct **onehot,
                           ckr_ct **value);
uint32_t ckr_order_range_depth(uint32_t N, uint32_t a, uint32_t b, ckr_sign cmp, ckr_sign ind, int tie_correct);

/* Multi-ciphertext ranking (section 5, Algorithm Multi-Ciphertext Ranking),
 * for vectors with N^2 > n/2: v is split into L blocks of b values (b a power
 * of two with b^2 <= n/2), block i holding v[i*b .. (i+1)*b) in slots [0,b)
 * of blocks[i], all blocks single ciphertexts at one level.  out (L entries,
 * caller-owned) receives in out[i] the fractional ranks of block i's elements
 * among all L*b values, slots [0,b), at level(blocks) - ckr_rank_multi_depth.
 * Comparisons run for block pairs j >= i only (Equation (3) gives the rest),
 * in batched comparator passes.  Keys need the rotations of ckr_keygen's
 * sort set for N = b.  Errors: CKR_E_RANGE (b), CKR_E_INVALID (L = 0, mixed
 * levels), CKR_E_DEPTH. */
ckr_status ckr_rank_multi(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *const *blocks, uint32_t L, uint32_t b,
                          ckr_sign cmp, ckr_ct **out);
uint32_t ckr_rank_multi_depth(ckr_sign cmp);

/* Multi-ciphertext sorting (section 5, Algorithm Multi-Ciphertext Sorting) of
 * L blocks of b distinct values laid out as for ckr_rank_multi.  out (L
 * entries, caller-owned) receives in out[i] the i-th block of the sorted vector
 * (the values of ranks i*b+1 .. (i+1)*b) in slots [0,b), at level(blocks) -
 * ckr_sort_multi_depth.  All L^2 indicators Ind_0(ReplR(R_j) - ranks of block
 * i) run in one batched comparator pass.  Keys: the sort set for N = b.
 * Errors: as ckr_rank_multi. */
ckr_status ckr_sort_multi(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *const *blocks, uint32_t L, uint32_t b,
                          ckr_sign cmp, ckr_sign ind, ckr_ct **out);
uint32_t ckr_sort_multi_depth(ckr_sign cmp, ckr_sign ind);

/* One query of a mixed batch.  kind: 1 rank (tie_correct selects the
 * tie-corrected rank), 2 argmin (the tie-corrected minimum; k and tie_correct
 * ignored), 3 sort, 4 order statistic k, 5 column-form sort.  v: a single
 * ciphertext, borrowed. */
typedef struct {
    int kind;
    uint32_t N;
    uint32_t k;
    int tie_correct;
    ckr_sign cmp, ind;
    const ckr_ct *v;
} ckr_query;

/* Run `count` independent queries of any kinds, sizes and levels as one unit
 * (batched execution across queries; the paper's own parallelism, sections 5
 * and 6.1, runs one query's independent comparisons on CPU threads): queries with the
 * same circuit and level form a group whose kernel launches cover all of its
 * members.  With graphs enabled (the default) the first call for a given mix
 * runs eagerly, the second captures every group into one hipGraph owned by
 * `keys`, and later calls with the same mix replay it as a single launch.
 * out (2 * count entries, caller-owned results) receives at out[2i] query i's
 * rank, sorted vector or one-hot and at out[2i+1] its value (order
 * statistics) or NULL.  Results equal single calls bit for bit.  Errors: as
 * the single calls; no output is produced on error. */
ckr_status ckr_run_mixed(ckr_context *ctx, const ckr_keys *keys, const ckr_query *q, size_t count, ckr_ct **out);

/* Batched execution: `count` ciphertexts of equal N and level run through one
 * circuit together -- every kernel launch covers all of them.  kind: 1 rank,
 * 2 argmin (outputs out[2i] one-hot, out[2i+1] value), 3 sort, 5 column-form
 * sort (out[i]).
 * With graphs enabled (the default) the first call for a shape (kind, N,
 * level, count, comparators) runs eagerly, the second captures the circuit
 * into a hipGraph owned by `keys`, later calls replay it.  Outputs equal
 * `count` single calls, bit for bit. */
ckr_status ckr_run_batch(ckr_context *ctx, const ckr_keys *keys, int kind, uint32_t N, ckr_sign cmp, ckr_sign ind,
                         const ckr_ct *const *v, size_t count, ckr_ct **out);
ckr_status ckr_rank_batch(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *const *v, size_t count, uint32_t N,
                          ckr_sign cmp, ckr_ct **out);
/* Enable (default) or disable hipGraph capture of batched circuits. */
ckr_status ckr_context_set_graphs(ckr_context *ctx, int enable);

/* Serving (continuous batching).  A server runs two worker slots per context
 * it routes to, each issuing work on a stream of its own.  A free slot takes
 * the oldest pending request of its context plus up to max_batch pending
 * requests of the same circuit, N and level, admits them against hbm_budget
 * (bytes of circuit working set in flight; 0 = unbounded; each route's
 * per-query working set is measured on its first batch, which runs alone on
 * its context), runs them as one batched circuit (graph-captured per slot
 * after the first call of a shape) and completes their tickets.  A request
 * that arrives while a batch of its context runs starts in the other slot as
 * soon as admission allows, so batches of one context, and of different
 * contexts, overlap on the device.  While a server runs, a block freed on one
 * stream of a context is reused on that stream only, until the host has
 * waited for it.  A request whose working set alone exceeds the budget fails
 * with CKR_E_NOMEM.  Results are the same bits as single calls.  The
 * ciphertext passed to submit must stay alive until its ticket completes.
 * API calls on a context are serialised with its workers' launches by a
 * per-context lock; waits run outside it. */
typedef struct ckr_server ckr_server;
ckr_status ckr_server_create(size_t hbm_budget, uint32_t max_batch, ckr_server **out);
/* kind 1 rank, 2 argmin, 3 sort; all routes are added before the first submit */
ckr_status ckr_server_add_route(ckr_server *srv, int kind, uint32_t N, ckr_context *ctx, const ckr_keys *keys,
                                ckr_sign cmp, ckr_sign ind);
ckr_status ckr_server_submit(ckr_server *srv, int kind, uint32_t N, const ckr_ct *v, uint64_t *ticket);
/* timeout_ms < 0 waits forever; CKR_E_BUSY on timeout.  outs receives 1
 * (rank, sort) or 2 (argmin) ciphertexts; latency_ms (3 values, may be NULL):
 * submit-to-done, submit-to-start, batch size. */
ckr_status ckr_server_wait(ckr_server *srv, uint64_t ticket, int timeout_ms, ckr_ct **outs, size_t n_outs,
                           double *latency_ms);
/* stats (5 values): completed requests, batches run, high-water bytes in
 * flight, pending requests, most batches of one context in flight at once */
ckr_status ckr_server_stats(ckr_server *srv, double *stats);
void ckr_server_free(ckr_server *srv);

/* Ciphertext access.  export: words = 2*(level+1)*n uint64 (layout above). */
uint32_t ckr_ct_level(const ckr_ct *ct);
double ckr_ct_scale(const ckr_ct *ct);
ckr_status ckr_ct_export(ckr_context *ctx, const ckr_ct *ct, uint64_t *coeff_limbs, size_t words);
/* import: rejects any residue >= its modulus (CKR_E_INVALID). */
ckr_status ckr_ct_import(ckr_context *ctx, const uint64_t *coeff_limbs, size_t words, uint32_t level, ckr_ct **out);
void ckr_ct_free(ckr_ct *ct);

/* Homomorphic operations on single ciphertexts (the building blocks the
 * circuits use; exposed for testing and custom circuits). */
ckr_status ckr_op_rotate(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *a, int64_t k, ckr_ct **out);
/* Allocation-free rotation, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Computes ckr_op_rotate(a, k) bit for bit into `out`, an existing
 * single ciphertext at a's level (caller-owned, e.g. from ckr_ct_import or a
 * previous call; it must not be a).  The key switch's temporaries live in a
 * file-scope device array of 128 MiB that every GPU the library runs on holds
 * until the process ends; no device memory is allocated or freed and nothing
 * is drawn from the context pool (ckr_context_memory does not move).  The
 * base-conversion tables of every level up to the keys' max_level are made by
 * ckr_keygen.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (other threads, other contexts or streams of the same
 * device) race; calls on one context are serialised by its lock and its
 * stream.  Errors: CKR_E_NOMEM when one key switch at a's ring and level
 * needs more than 128 MiB ((l+1) + beta E + 2E + 2(l+1) limbs of 8n bytes,
 * E = l + 1 + n_p; e.g. n = 2^16 up to level 21 with 7 special primes and
 * dnum = 3), CKR_E_INVALID (out not at a's level, out == a, handles of
 * another context, missing rotation key), CKR_E_DEPTH (a above the keys'
 * level). */
ckr_status ckr_op_rotate_into(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *a, int64_t k, ckr_ct *out);
ckr_status ckr_op_mul(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *a, const ckr_ct *b, ckr_ct **out);
/* sum_{i < deg1} coeffs[i] T_i(a) for a Chebyshev series of deg1 = 2^B terms
 * (1 <= B <= 15), the evaluation behind the Chebyshev comparator (section
 * 2.2): Paterson-Stockmeyer in the Chebyshev basis with 2^ceil(B/2) baby
 * steps, brought to one level and combined with integer constants (one
 * rescale, then + c_0) for every leaf of the division by the giant steps
 * T_{2^ceil(B/2) 2^r}.  The slots of a must lie in [-1, 1].  Consumes B + 1
 * levels (CKR_E_DEPTH if a has fewer); coeffs is borrowed for the call; a
 * length that is not a power of two is CKR_E_INVALID. */
ckr_status ckr_op_cheb_eval(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *a, const double *coeffs,
                            uint32_t deg1, ckr_ct **out);
/* Cmp(d) of section 2.2 on a ciphertext of differences d = x - y (slots in
 * [-1, 1]): the comparator `cmp` alone, (p(d) + 1)/2 for the f/g or minimax
 * composite p, or the Chebyshev interpolant.  Consumes the comparator's levels
 * (CKR_E_DEPTH if a has fewer); CKR_E_INVALID for an invalid comparator. */
ckr_status ckr_op_cmp_sign(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *a, ckr_sign cmp, ckr_ct **out);
ckr_status ckr_op_add(ckr_context *ctx, const ckr_ct *a, const ckr_ct *b, ckr_ct **out);
ckr_status ckr_op_sub(ckr_context *ctx, const ckr_ct *a, const ckr_ct *b, ckr_ct **out);
ckr_status ckr_op_rescale(ckr_context *ctx, const ckr_ct *a, ckr_ct **out);
/* c * a brought to level `target` (drop to target+1 limbs, multiply by
 * round(c * D_target * q_{target+1} / D_level), rescale). */
ckr_status ckr_op_cmul_to(ckr_context *ctx, const ckr_ct *a, double c, uint32_t target, ckr_ct **out);
ckr_status ckr_op_add_const(ckr_context *ctx, const ckr_ct *a, double c, ckr_ct **out);
/* slot-wise product with the plaintext z[0..count) (others 0), then rescale */
ckr_status ckr_op_mul_plain(ckr_context *ctx, const ckr_ct *a, const double *z, uint32_t count, ckr_ct **out);

/* Raw negacyclic NTT on device buffers: `limbs` limbs of n words at `data`
 * (device pointer), limb t reduced modulo modulus index first_mod + t.
 * inverse != 0 runs the inverse transform.  Forward output order is the
 * library's internal evaluation order; inverse(forward(x)) == x. */
ckr_status ckr_ntt_device(ckr_context *ctx, uint64_t *data, uint32_t limbs, uint32_t first_mod, int inverse);

/* Kernel timing.  While enabled, every kernel launch of the evaluator is
 * bracketed by HIP events on the context stream and charged to a category
 * (0 ntt_fwd_col, 1 ntt_fwd_row, 2 ntt_inv_row, 3 ntt_inv_col, 4 bconv, 5 ntt_row_ip
 * (forward row pass fused with the key-switch inner product),
 * 6 tensor, 7 automorph, 8 elementwise, 9 copy) together with its
 * algorithmic byte count (every operand read once, every result written
 * once).  read returns the launches, summed milliseconds and summed bytes of
 * one category since the last reset; it synchronises the stream. */
ckr_status ckr_set_profiling(ckr_context *ctx, int enable);
ckr_status ckr_profile_reset(ckr_context *ctx);
ckr_status ckr_profile_read(ckr_context *ctx, int category, uint64_t *launches, double *total_ms, double *bytes);
const char *ckr_profile_name(int category);

/* NTT autotuner: times each compiled tile variant (elements per thread x
 * columns per workgroup) of every (direction, pass) on `limbs` limbs (one launch
 * over polynomials of the whole q chain, then the rest), `iters`
 * repetitions, and keeps the fastest for this context.  ms, if not NULL,
 * receives the 2 x 2 x 5 average milliseconds [inverse][pass][variant].
 * Every variant computes the same transform bit for bit. */
ckr_status ckr_autotune(ckr_context *ctx, uint32_t limbs, uint32_t iters, float *ms);
/* Autotuner of the key switch's fused forward row pass + inner product: times
 * every tile variant on a synthetic key switch at the top level with `batch`
 * ciphertexts sharing the key (all-zero operands; device memory of about
 * batch * (dnum + 2) * (L + 1 + K) limbs is taken from the context pool for
 * the run), `iters` repetitions, and keeps the fastest.  ms, if not NULL,
 * receives 8 average milliseconds [variant].  Every variant computes the same
 * result bit for bit.  Errors: CKR_E_INVALID for batch 0 or above 4096. */
ckr_status ckr_autotune_row_ip(ckr_context *ctx, uint32_t batch, uint32_t iters, float *ms);
/* Run transforms of more than `limbs` limbs in chunks of whole polynomials
 * (0 = never), so each chunk's second pass reads data still in the
 * last-level cache.  Results do not depend on the chunking. */
ckr_status ckr_set_ntt_chunk(ckr_context *ctx, uint32_t limbs);
/* Force one tile variant (0..4) for a (direction, pass). */
ckr_status ckr_ntt_variant(ckr_context *ctx, int inverse, int pass, int variant);
/* Force one tile variant (0..7) of the key switch's fused forward row pass +
 * inner product (rows of 2^8 points; other ring sizes have one tile). */
ckr_status ckr_row_ip_variant(ckr_context *ctx, int variant);
/* The five calls above change the kernels later work runs.  A batched
 * circuit captured into a hipGraph before such a change is captured again on
 * its next run, so replays always use the current tiles and chunking. */

/* Wait for all work issued on the context stream. */
ckr_status ckr_synchronize(ckr_context *ctx);

const char *ckr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
