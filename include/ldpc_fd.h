/*
 * ldpc_fd.h -- C ABI of libldpcfd.so, a gfx950 (MI355X) decoder for non-binary
 * LDPC codes over GF(2^m), built for column weight 2, using the Log-Fourier
 * sum-product (LF-SP) algorithm of K. Kasai and K. Sakaniwa, "Fourier Domain
 * Decoding Algorithm of Non-Binary LDPC codes for Parallel Implementation",
 * IEICE Trans. Fundamentals 93(11), 2010 (arXiv:1008.4370).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Symbols: x in GF(2^m) is the m-bit vector (x_1..x_m) of its coefficients in
 *   the basis 1, alpha, ..., alpha^(m-1) (Sec. 2); as an integer, x_i is bit
 *   (i-1).  alpha is the class of the polynomial "x" modulo the primitive
 *   polynomial prim_poly.
 * Code: H is M x N over GF(2^m), given in compressed-row form (row_ptr, col,
 *   val).  Edge e is the e-th nonzero of H in row-major order; all per-edge
 *   arrays use this check-major order.  Columns have weight 1..16 and rows
 *   2..16.  The fused decoder, the decoding pool, symbol-prior decoding and
 *   the decode-time posteriors take codes whose every column has weight 2
 *   (the (2,k) codes the method is built for, Sec. 1 and Sec. 4); the PLAIN
 *   and LOGSP decoders and the round and imported-state posterior entry
 *   points also take other column weights (the extension to irregular codes
 *   noted in Sec. 2), and return E_UNSUPPORTED otherwise.
 * Channel: llr[f][v][i] = ln Pr(b=0|y)/Pr(b=1|y) for bit i (0-based, the
 *   coefficient of alpha^i) of symbol v of frame f, FP32, device memory,
 *   layout [frames][N][m] contiguous.  The symbol prior is the product of the
 *   bit posteriors (INITIALIZATION, Sec. 2.1 / Sec. 3.2).
 * Messages (the decoder state): Lambda_cv(z) = Gamma(P_cv(z)) of Sec. 3.2 for
 *   every edge, in the variable node's coordinates z (no label map applied),
 *   stored as one float per entry whose sign bit is the GF(2) sign and whose
 *   magnitude is -log2|P_cv(z)| in [0, 100] (base 2 instead of the paper's
 *   natural log; a positive rescaling).  Layout [frames][E][2^m] contiguous.
 *   With 16-bit storage (LDPC_FD_FP16, LDPC_FD_BF16) the FUSED decoder keeps
 *   each message as q times its pmf instead, q p_cv(x) = sum_z P_cv(z)
 *   (-1)^(x.z) clamped at zero (in [0, q]), rounded to the storage type: a
 *   16-bit float keeps every probability to a relative 2^-11 (FP16) or 2^-8
 *   (BF16), where a 16-bit signed-log Fourier word would carry P(z) only to
 *   an absolute ~1e-4.  Entry points that import or export a state always use
 *   the FP32 signed-log layout above.
 * Errors: every function returns LDPC_FD_OK (0) or a negative code; no
 *   exception crosses the ABI.  ldpc_fd_last_error() gives a message for the
 *   last failure on the calling thread.
 * Streams: `stream` is a hipStream_t passed as void* (NULL = default stream).
 *   Device-side work is enqueued on it; results are valid once it is
 *   synchronised.  A code object may be used concurrently on different streams,
 *   each call with its own workspace.
 */
#ifndef LDPC_FD_H
#define LDPC_FD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ldpc_fd_code_s *ldpc_fd_code;

enum {
  LDPC_FD_OK = 0,
  LDPC_FD_E_INVALID = -1,     /* bad argument or malformed H */
  LDPC_FD_E_UNSUPPORTED = -2, /* m outside 2..8, weight above 16, a mode the code cannot use */
  LDPC_FD_E_NOMEM = -3,       /* allocation failed or workspace too small */
  LDPC_FD_E_HIP = -4          /* a HIP runtime call failed */
};

/* Storage type of the message state (arithmetic is FP32 in every case).
 * LDPC_FD_LOG8 (LOGSP mode only): one byte per message entry, the code
 * k = 0..255 of the log2 probability -k, rounded to nearest and saturating
 * (the 8-bit form of the quantisation argument of Sec. 1 and Sec. 2.2; the
 * same values as FP32 storage with QUANT_BITS = 8 and QUANT_STEP = 4096). */
enum { LDPC_FD_FP32 = 0, LDPC_FD_FP16 = 1, LDPC_FD_BF16 = 2, LDPC_FD_LOG8 = 3 };

/* Decoder variants (PLAIN and FUSED: identical results up to rounding order):
 *  PLAIN: one kernel per node type per round, flooding schedule of Sec. 2
 *         (check-to-variable, variable-to-check, tentative decision), all frames
 *         processed until the host sees every frame stopped.  For codes with
 *         other column weights j the variable node forms the j-fold
 *         log-convolution of Sec. 3.2 through the convolution theorem (each
 *         message to the probability domain by Gamma^-1 and a Hadamard
 *         transform, products, back by a Hadamard transform and Gamma), over
 *         the list of still-active frames.
 *  FUSED: one pass per round over the checks; each pass recomputes the
 *         variable-to-check messages from the stored check-to-variable state,
 *         forms the tentative decision of the previous round, compacts the list
 *         of still-active frames on the device and runs in chunks of rounds.
 *  LOGSP: the conventional log-domain sum-product decoder of Sec. 2.2, the
 *         comparison point of Table 1: messages are log2 pmfs (FP32, maximum
 *         normalised to 0, floored at -200), the check node forms each outgoing
 *         message as the XOR convolution of the other k-1 incoming ones in the
 *         log domain (forward/backward partial convolutions, 3(k-2) pairwise
 *         convolutions of q^2 log-sum-exp terms), the variable node adds log
 *         vectors; flooding schedule and stopping rule as PLAIN.  Same outputs
 *         as the Log-Fourier modes up to rounding; FP32 or LOG8 storage; the
 *         PRECISE and DECISION_MFMA tuning keys do not apply.
 *  FSP:   the linear-domain Fourier SP of Sec. 3.1 (the algorithm the
 *         Log-Fourier SP is derived from): messages are P(z) itself (FP32,
 *         normalised to P(0) = 1), the check node multiplies the other k-1
 *         label-mapped messages component-wise, the variable node forms the
 *         j-fold convolution through the convolution theorem as PLAIN does for
 *         irregular codes; any column weight, FP32 only.  With the tuning key
 *         QUANT_BITS the PLAIN, FSP and LOGSP decoders store their messages on a b-bit
 *         grid (the quantisation comparison that motivates the paper, Sec. 1
 *         and Sec. 2.2). */
enum { LDPC_FD_MODE_PLAIN = 0, LDPC_FD_MODE_FUSED = 1, LDPC_FD_MODE_LOGSP = 2, LDPC_FD_MODE_FSP = 3 };

/* status[f] bits */
#define LDPC_FD_STATUS_CONVERGED 1u /* stopped on a passed codeword test */
#define LDPC_FD_STATUS_MISMATCH 2u  /* Fourier and direct syndromes differed at some round */

/* Create a code object (Sec. 2: the code {x : Hx = 0}).
 * M, N: H is M x N.  m: field GF(2^m), 2 <= m <= 8.
 * row_ptr[M+1], col[E], val[E]: host arrays, copied; E = row_ptr[M].
 *   val[e] in 1..2^m-1 is h_cv in the integer representation above.
 * prim_poly: primitive polynomial with bit m set (0 selects the default:
 *   x^2+x+1, x^3+x+1, x^4+x+1, x^5+x^2+1, x^6+x+1, x^7+x^3+1,
 *   x^8+x^4+x^3+x^2+1).
 * out: receives the handle; owns device tables until ldpc_fd_destroy_code.
 * Errors: E_INVALID (bad CSR, label 0 or >= 2^m, duplicate (c,v), row weight
 *   < 2, a column of weight 0, non-primitive prim_poly), E_UNSUPPORTED (m
 *   outside 2..8, row or column weight > 16), E_HIP / E_NOMEM on device
 *   allocation. */
int32_t ldpc_fd_create_code(int32_t M, int32_t N, int32_t m, const int32_t *row_ptr,
                            const int32_t *col, const uint16_t *val, uint32_t prim_poly,
                            ldpc_fd_code *out);

/* Release a code object and its device tables (NULL is a no-op). */
int32_t ldpc_fd_destroy_code(ldpc_fd_code code);

/* Shape of a code object; any output pointer may be NULL. */
int32_t ldpc_fd_code_info(ldpc_fd_code code, int32_t *M, int32_t *N, int32_t *m, int32_t *E,
                          int32_t *kmax);

/* Bytes of caller-owned device workspace that ldpc_fd_decode needs for
 * `frames` frames at storage precision `prec` in decoder variant `mode`.
 * Errors: E_INVALID (unknown prec or mode), E_UNSUPPORTED (a storage type the
 * mode does not have: PLAIN and FSP take FP32 only, LOGSP FP32 or LOG8,
 * FUSED FP32, FP16 or BF16). */
int32_t ldpc_fd_workspace_bytes(ldpc_fd_code code, int32_t frames, int32_t prec, int32_t mode,
                                int64_t *bytes);

/* Decode a batch of frames (Sec. 3.2, the Log-Fourier SP algorithm, with the
 * stopping rule of Sec. 2: stop at the first round whose tentative decision
 * passes the codeword test, FAIL when the round count reaches max_iter).
 *
 * frames >= 0; llr: device [frames][N][m] FP32 (see above); max_iter >= 1.
 * Outputs (device, caller-owned, written for every frame):
 *   hard[frames][N]  uint8: bitwise-MAP tentative symbols of the stopping round,
 *                    read from the signs of the Fourier-domain posterior at
 *                    alpha^(i-1) (Sec. 3.1 Eq. (5), Sec. 3.2);
 *   synd[frames][M]  uint8: direct syndrome H * hard (integer-exact);
 *   iters[frames]    int32: round l at which the frame stopped, 1..max_iter;
 *   status[frames]   uint32: LDPC_FD_STATUS_* bits.
 * A frame stops when both its Fourier-domain syndrome (Sec. 3.1/3.2) and its
 * direct syndrome are zero.
 * workspace: device memory of at least ldpc_fd_workspace_bytes(...) bytes,
 *   caller-owned, not retained after the call returns.
 * The call is stream-ordered; it synchronises with the stream internally only
 * to read the count of active frames between chunks of rounds.
 * Errors: E_INVALID (null pointers with frames > 0, max_iter < 1, unknown
 *   prec/mode), E_NOMEM (workspace too small), E_HIP. */
int32_t ldpc_fd_decode(ldpc_fd_code code, int32_t frames, const float *llr, int32_t max_iter,
                       int32_t prec, int32_t mode, uint8_t *hard, uint8_t *synd,
                       int32_t *iters, uint32_t *status, void *workspace,
                       int64_t workspace_bytes, void *stream);

/* Decode from symbol priors instead of BPSK LLRs (Sec. 2.1: the channel input
 * is Pr(X_v = x | Y_v = y_v) for every symbol, any memoryless channel).
 * prior: device float [frames][N][2^m], entry x of row (f, v) proportional to
 * Pr(X_v = x | y) (nonnegative, not all zero; rows need not be normalised).
 * The variable node convolves with the prior through two Hadamard transforms
 * (Y = WHT(p0 . WHT(X))) instead of the m butterflies of the BPSK form; FUSED
 * mode and FP32 storage only (the workspace of ldpc_fd_workspace_bytes(...,
 * FP32, FUSED)); the PRECISE and DECISION_MFMA tuning keys do not apply.
 * Outputs, stopping rule and errors as ldpc_fd_decode; E_UNSUPPORTED for
 * prec != FP32.  The
 * posterior and symbol entry points below take BPSK LLRs and do not apply to
 * such decodes. */
int32_t ldpc_fd_decode_prior(ldpc_fd_code code, int32_t frames, const float *prior, int32_t max_iter,
                             int32_t prec, uint8_t *hard, uint8_t *synd, int32_t *iters, uint32_t *status,
                             void *workspace, int64_t workspace_bytes, void *stream);

/* One flooding round from an imported state, for message-level parity checks
 * (Sec. 3.2 VARIABLE TO CHECK, TENTATIVE DECISION, then CHECK TO VARIABLE):
 *   from c2v_in = Lambda_cv^(l) (FP32 message layout above; NULL means round 0,
 *   i.e. the variable-to-check messages are the initial messages Lambda_v^(0)),
 *   writes v2c_out = Lambda_vc^(l) (normalised so that Lambda_vc(0) = (0,0);
 *   required in PLAIN mode, must be NULL in FUSED mode, which never stores
 *   variable-to-check messages), c2v_out = Lambda_cv^(l+1), and, when c2v_in is
 *   not NULL, the
 *   tentative decision of round l: hard[frames][N], fsynd[frames][M] (Fourier
 *   syndrome words, bit i = syndrome bit i+1 of the check) and synd[frames][M]
 *   (direct syndrome of hard).  All arrays are device memory in the FP32 message
 *   layout.  mode selects which kernels compute it (PLAIN or FUSED; LOGSP
 *   instead takes and writes log2 pmfs [frames][E][2^m] with maximum 0 in
 *   c2v_in, v2c_out and c2v_out, v2c_out required).  prec
 *   selects the storage type the FUSED pass reads and writes: with 16-bit
 *   storage the imported state is converted to the stored words first (q
 *   times the pmf, transformed in FP64, clamped at zero, rounded) and the
 *   stored result converted back to FP32 signed-log words normalised to
 *   P(0) = 1, so the difference to an FP32 round is the one-round storage
 *   error (PLAIN: FP32 only).  The call allocates temporary device memory and
 *   synchronises.
 * Errors: E_INVALID, E_UNSUPPORTED (PLAIN or LOGSP with prec != FP32; LDPC_FD_LOG8,
 * which whole LOGSP decodes take), E_HIP. */
int32_t ldpc_fd_round(ldpc_fd_code code, int32_t frames, const float *llr, const float *c2v_in,
                      float *v2c_out, float *c2v_out, uint8_t *hard, uint8_t *fsynd,
                      uint8_t *synd, int32_t mode, int32_t prec, void *stream);

/* ldpc_fd_round for callers that cannot allocate device memory: code recorded
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, kernels and results as ldpc_fd_round; the
 * temporaries come from a static device array of LDPC_FD_ROUND_SCRATCH_BYTES
 * (64 MiB) that the library holds on every GPU it runs on until the process
 * ends, so the call allocates and frees nothing and does not synchronise: the
 * work is enqueued on `stream` and the outputs are valid once the stream has
 * passed it.  Every call on one GPU uses that GPU's same array (the library
 * re-initialises whatever must start at zero on every call), so calls that
 * overlap on one GPU, on different streams or threads, race and must be
 * ordered by the caller.  The scratch need grows with frames, E, 2^m and, for
 * 16-bit storage, with the staging of the state (GF(64) N=1000: ~26 KB per
 * frame with FP32 storage, ~540 KB with FP16/BF16).
 * Errors: as ldpc_fd_round, plus E_NOMEM when the round needs more scratch
 * than the array holds (nothing is enqueued then). */
#define LDPC_FD_ROUND_SCRATCH_BYTES (64ll * 1024 * 1024)
int32_t ldpc_fd_round_noalloc(ldpc_fd_code code, int32_t frames, const float *llr, const float *c2v_in,
                              float *v2c_out, float *c2v_out, uint8_t *hard, uint8_t *fsynd,
                              uint8_t *synd, int32_t mode, int32_t prec, void *stream);

/* ---- Decode with an argument struct and flags ---------------------------------
 * The same decode as ldpc_fd_decode (Sec. 3.2 with the stopping rule of Sec. 2)
 * with its arguments in one struct and these flags:
 *   LDPC_FD_FLAG_NO_EARLY_STOP: every frame runs max_iter rounds whatever its
 *     syndromes; iters = max_iter, hard/synd are the last round's, and the
 *     converged status bit reports whether that last decision passed the
 *     codeword test (the mismatch bit still accumulates over all rounds).
 *   LDPC_FD_FLAG_VALIDATION (FUSED only): also write posterior[frames][N][2^m]
 *     (device double), the FP64 posterior of every frame at its stopping
 *     round (as ldpc_fd_decode_posterior).
 *   LDPC_FD_FLAG_ASYNC (FUSED and PLAIN with column weight 2 only): the call
 *     enqueues every round on the stream and returns without synchronising
 *     with it (no read of the active-frame count): max_iter + 1 passes are
 *     enqueued, the passes after the last frame has stopped find no active
 *     frame, and the few-frames variant is not used.  Results are the same.
 * Without ASYNC the call synchronises with the stream to read the count of
 * active frames between chunks of rounds (as ldpc_fd_decode).
 * Errors: as ldpc_fd_decode; E_INVALID for unknown flag bits or VALIDATION
 *   without a posterior buffer; E_UNSUPPORTED for VALIDATION outside FUSED
 *   mode or ASYNC with the LOGSP, FSP or irregular PLAIN decoders. */
#define LDPC_FD_FLAG_NO_EARLY_STOP 1u
#define LDPC_FD_FLAG_VALIDATION 2u
#define LDPC_FD_FLAG_ASYNC 4u
typedef struct {
  int32_t frames, max_iter, prec, mode;
  uint32_t flags;
  const float *llr;        /* device [frames][N][m] */
  uint8_t *hard;           /* device [frames][N] */
  uint8_t *synd;           /* device [frames][M] */
  int32_t *iters;          /* device [frames] */
  uint32_t *status;        /* device [frames] */
  double *posterior;       /* device [frames][N][2^m] or NULL (VALIDATION only) */
  void *workspace;         /* device, ldpc_fd_workspace_bytes(frames, prec, mode) */
  int64_t workspace_bytes;
} ldpc_fd_decode_args;
int32_t ldpc_fd_decode_ex(ldpc_fd_code code, const ldpc_fd_decode_args *args, void *stream);

/* `rounds` flooding rounds from an imported state (several ldpc_fd_round
 * steps in one call): on entry c2v_inout holds Lambda_cv^(l) in the FP32
 * message layout (ignored when from_channel != 0: the rounds then start at
 * round 0 from the channel prior), on return Lambda_cv^(l + rounds).  hard,
 * fsynd and synd receive the tentative decision of the last round that formed
 * one (round l + rounds - 1; none when from_channel and rounds == 1, then they
 * may be NULL).  No stopping rule is applied.  mode and prec as
 * ldpc_fd_round (16-bit storage: each round's state is rounded to the stored
 * word).  The call allocates temporary device memory and synchronises.
 * Errors: as ldpc_fd_round; E_INVALID for rounds outside 1..100000. */
int32_t ldpc_fd_run_rounds(ldpc_fd_code code, int32_t frames, const float *llr, int32_t rounds,
                           int32_t from_channel, float *c2v_inout, uint8_t *hard, uint8_t *fsynd,
                           uint8_t *synd, int32_t mode, int32_t prec, void *stream);

/* ---- Validation mode: FP64 symbol posteriors ----------------------------------
 * The a-posteriori pmf of every symbol, p_v(x) proportional to the channel pmf
 * times the pmfs of the two check-to-variable messages of v (Sec. 2.1,
 * tentative decision; Sec. 3.2 evaluates the same product as a 3-fold
 * log-convolution).  Each stored message word is widened to P(z) in FP64, taken
 * back to the probability domain by an FP64 Hadamard transform, multiplied with
 * the FP64 channel pmf from llr, clamped at zero and normalised in FP64.
 * posterior: device double[frames][N][2^m], caller-owned, written in full. */

/* From an imported state: c2v = Lambda_cv in the FP32 message layout above
 * (device [frames][E][2^m], e.g. ldpc_fd_round's c2v_out).
 * Errors: E_INVALID (NULL code or buffers with frames > 0, frames < 0), E_HIP. */
int32_t ldpc_fd_posterior(ldpc_fd_code code, int32_t frames, const float *llr, const float *c2v,
                          double *posterior, void *stream);

/* After an ldpc_fd_decode in FUSED mode with the same code, frames, llr, prec
 * and workspace (not reused in between): the posterior of each frame at the
 * round it stopped at (iters[f], the decode's device output), read from the
 * message buffer that holds that round's check-to-variable messages.
 * Errors: E_INVALID (NULL arguments with frames > 0, unknown prec, workspace
 *   smaller than the fused decode's), E_UNSUPPORTED (a code with column weights
 *   other than 2, or LDPC_FD_LOG8, neither of which a FUSED decode takes; a
 *   workspace whose last decode retired in batches, tuning key BATCH_RETIRE),
 *   E_HIP. */
int32_t ldpc_fd_decode_posterior(ldpc_fd_code code, int32_t frames, const float *llr, int32_t prec,
                                 const int32_t *iters, const void *workspace, int64_t workspace_bytes,
                                 double *posterior, void *stream);

/* Soft output and symbol-MAP decisions after an ldpc_fd_decode in FUSED mode
 * (same conditions as ldpc_fd_decode_posterior): symmap[frames][N] (device
 * uint8) receives argmax_x p_v(x) at each frame's stopping round (the
 * symbol-MAP decision, Sec. 3.1 Eq. (3), through the inverse transform of
 * Eq. (4); ties go to the smaller symbol), and posterior (device
 * float[frames][N][2^m], may be NULL) the normalised pmf, formed in FP64 as
 * above and rounded to FP32.  symmap can differ from the decode's bitwise-MAP
 * hard decisions where the posterior is not concentrated.
 * Errors: as ldpc_fd_decode_posterior. */
int32_t ldpc_fd_decode_symbols(ldpc_fd_code code, int32_t frames, const float *llr, int32_t prec,
                               const int32_t *iters, const void *workspace, int64_t workspace_bytes,
                               uint8_t *symmap, float *posterior, void *stream);

/* ---- Decoding pool: continuous batching over several codes -------------------
 * A pool owns, for each of its codes, `slots[k]` frame slots in device memory
 * (message state, decisions and per-frame round counter; ldpc_fd_pool_slot_bytes
 * gives the bytes per slot, for admission against an HBM budget).  Frames are
 * admitted into free slots at any time and decoded by passes that cover every
 * active frame of every code; frames at different rounds share a pass, so
 * newly admitted frames join the ones in flight.  A frame stops exactly as in
 * ldpc_fd_decode (same kernels and per-frame arithmetic, so its results do not
 * depend on what else is in the pool); stopped frames are harvested and their
 * slots freed.  All pool calls are ordered on the pool's stream; the pool is
 * not thread-safe.  The codes must outlive the pool. */
typedef struct ldpc_fd_pool_s *ldpc_fd_pool;

/* Device bytes one frame slot of `code` occupies at storage precision prec. */
int32_t ldpc_fd_pool_slot_bytes(ldpc_fd_code code, int32_t prec, int64_t *bytes);

/* Create a pool over codes[0..ncodes) (1..16) with slots[k] frame slots for
 * code k, message storage prec, operating on `stream` (hipStream_t as void*).
 * Errors: E_INVALID, E_NOMEM (device or pinned-host allocation), E_HIP. */
int32_t ldpc_fd_pool_create(const ldpc_fd_code *codes, int32_t ncodes, const int32_t *slots, int32_t prec,
                            void *stream, ldpc_fd_pool *out);

/* A pool whose slot counts come from an HBM budget: each code gets an equal
 * share of hbm_budget bytes, divided by its ldpc_fd_pool_slot_bytes at prec
 * (at least one slot, at most 2^22; ldpc_fd_pool_free_slots reports the
 * counts).  Errors: as ldpc_fd_pool_create; E_NOMEM when a code's share holds
 * no slot. */
int32_t ldpc_fd_pool_create_budget(const ldpc_fd_code *codes, int32_t ncodes, int64_t hbm_budget, int32_t prec,
                                   void *stream, ldpc_fd_pool *out);

/* The slot counts ldpc_fd_pool_create_budget gives for these arguments, into
 * slots[0..ncodes) (host memory), without allocating (for sizing work to a
 * pool before creating it).  Errors: E_INVALID; E_NOMEM when a code's share
 * holds no slot. */
int32_t ldpc_fd_pool_budget_slots(const ldpc_fd_code *codes, int32_t ncodes, int64_t hbm_budget, int32_t prec,
                                  int32_t *slots);

/* Synchronise the pool's stream and free all its resources (NULL: no-op). */
int32_t ldpc_fd_pool_destroy(ldpc_fd_pool pool);

/* Number of free slots of code `code` (host-side bookkeeping, no device call). */
int32_t ldpc_fd_pool_free_slots(ldpc_fd_pool pool, int32_t code, int32_t *n);

/* Admit up to n frames of code `code`: llr is device memory [n][N][m] FP32 that
 * must stay valid until the pool's stream has passed this call; tags (host,
 * may be NULL) are returned by harvest.  Frames beyond the free slots are not
 * admitted; *admitted receives the number taken (from the front of llr).
 * max_iter >= 1 is the frames' round limit.  Errors: E_INVALID, E_HIP. */
int32_t ldpc_fd_pool_submit(ldpc_fd_pool pool, int32_t code, const float *llr, int32_t n,
                            const uint64_t *tags, int32_t max_iter, int32_t *admitted);

/* Enqueue `passes` (1..1000) passes over the active frames of every code: one
 * replay of a captured graph whose per-code branches run concurrently.  Each
 * code's kernel forms follow a bound on its active frames: the smaller of its
 * admitted-but-unharvested frames and its last active count read by
 * ldpc_fd_pool_active plus the frames admitted since.  A code whose bound is
 * at most its tail threshold (LDPC_FD_TUNE_TAIL_FRAMES) runs the few-frames
 * form in this step (syndromes and retirement in one launch while the bound
 * is at most 128), and a code whose bound is zero is left out of the step;
 * steps are captured once per (passes, forms per code, schedule) with the
 * codes' tuning at that time.  Asynchronous.  Errors: E_INVALID,
 * E_UNSUPPORTED, E_HIP. */
int32_t ldpc_fd_pool_step(ldpc_fd_pool pool, int32_t passes);

/* How a step's per-code branches are ordered.  schedule 0 (default): every
 * code's passes run on its own stream, all concurrently.  schedule 1
 * (staggered): the code with the most work per pass (its bound on active
 * frames times the bytes of one of its frame-rounds) starts once every other
 * code has run `lead` (0..1000) passes of the step; the rest overlaps.  With a
 * code that fills the GPU alone, concurrency only adds interference, while
 * the other codes' last passes (a few frames, latency-bound) still overlap
 * with it.  Results do not depend on the schedule.  Errors: E_INVALID. */
int32_t ldpc_fd_pool_set_schedule(ldpc_fd_pool pool, int32_t schedule, int32_t lead);

/* Collect up to cap stopped frames of code `code` (synchronises the pool's
 * stream): tags[cap], iters[cap], status[cap] (LDPC_FD_STATUS_* bits) and
 * hard[cap][N] (host arrays; any may be NULL).  Their slots become free.
 * *n receives the number returned.  Errors: E_INVALID, E_HIP. */
int32_t ldpc_fd_pool_harvest(ldpc_fd_pool pool, int32_t code, int32_t cap, uint64_t *tags, int32_t *iters,
                             uint32_t *status, uint8_t *hard, int32_t *n);

/* Number of frames of code `code` still being decoded (synchronises); later
 * steps choose the code's kernel forms from it (see ldpc_fd_pool_step). */
int32_t ldpc_fd_pool_active(ldpc_fd_pool pool, int32_t code, int32_t *n);

/* Tuning of a code object's kernels (results are identical for every setting
 * except LDPC_FD_TUNE_PRECISE and LDPC_FD_TUNE_DECISION_MFMA; only speed changes).  Set by the autotuner, read back for its cache.
 *   LDPC_FD_TUNE_LANE_ENTRIES: entries of a frame's 2^m-vector held per lane
 *     (4, 8 or 16; 16 needs m >= 4 and rows of weight <= 8).  Fewer entries
 *     per lane means more lanes per frame, fewer registers and more waves.
 *   LDPC_FD_TUNE_GRID_BLOCKS: workgroups of the grid-stride fused pass (>= 8).
 *   LDPC_FD_TUNE_CHUNK: rounds between host reads of the active-frame count.
 *   LDPC_FD_TUNE_GRAPHS: 1 (default) = the FUSED decoder captures a chunk of
 *     rounds into a HIP graph once per (frames, buffers, settings) and replays
 *     it; 0 = launch every kernel from the host.  While kernel timing is
 *     enabled (ldpc_fd_profile_enable) kernels are launched from the host.
 *   LDPC_FD_TUNE_TAIL_ENTRIES, LDPC_FD_TUNE_TAIL_FRAMES: a chunk of rounds
 *     that starts with at most TAIL_FRAMES active frames (default 128) runs
 *     the variant with TAIL_ENTRIES entries per lane (default 4): with few
 *     frames left a pass is bound by one check's latency, which more lanes
 *     per frame shorten.  TAIL_FRAMES = 0 keeps one variant throughout.
 *   LDPC_FD_TUNE_TAIL_SPLIT: 1 (default) = those chunks run the edge-parallel
 *     pass, one wavefront per edge of a check (identical results); 0 = the
 *     check-serial pass with the tail variant.
 *   LDPC_FD_TUNE_PRECISE: the FUSED pass's variable node (prior convolution
 *     and normalisation, Sec. 3.2 VARIABLE TO CHECK).  2 (default) = FP32
 *     through the convolution theorem (Eq. (6)): the message's pmf (a Hadamard
 *     transform of P, its negative rounding residue set to zero) times the
 *     channel pmf formed from the bit probabilities at full relative
 *     precision, transformed back; 0 = FP32 with the prior convolution as m
 *     butterflies with tanh(L/2) factors (cheaper, but it loses the small
 *     differences from certainty that decide messages where the channel and
 *     the check messages disagree: GF(64) N=1000 at 2.5 dB, FER 3.2e-3 vs
 *     1.0e-3); 1 = the butterflies in FP64 from the stored words, with 1 - |P|
 *     and 1 - |tanh(L/2)| carried at FP32 relative precision.  16-bit
 *     storage (pmf words) is built for the default form only: with PRECISE
 *     0 or 1 and FP16/BF16, decode, round and pool creation return
 *     E_UNSUPPORTED.
 *     Unlike the other keys this one changes results.  A pool uses the
 *     setting its codes had when it was created.
 *   LDPC_FD_TUNE_DECISION_MFMA (with PRECISE = 0 only): 1 = the three Hadamard transforms of the
 *     tentative decision run as FP16 MFMAs with FP32 accumulation (each FP32
 *     operand split into two FP16 terms, ~22 bits), in the variants with 4
 *     lanes per frame (2^m = 16, 32, 64; elsewhere, and with PRECISE, the FP32
 *     VALU transforms are used).  Decisions can differ from the VALU form only
 *     where a posterior value at a read point is within rounding of zero.
 *   LDPC_FD_TUNE_QUANT_BITS: b in 3..16 = the PLAIN, FSP and LOGSP decoders (decode
 *     and round) replace every message they store by the nearest word of a
 *     b-bit format, emulating b-bit message memory (the arrays stay FP32; the
 *     bandwidth is not reduced); 0 (default) = off.  PLAIN (Log-Fourier words):
 *     sign bit plus a (b-1)-bit magnitude -log2|P| on the grid k * step,
 *     k = 0 .. 2^(b-1) - 1 (nearest, saturating).  FSP (linear P in [-1, 1]):
 *     b-bit two's complement fixed point with step 2^-(b-1).  LOGSP (log2
 *     pmfs <= 0): b-bit unsigned -k * step, k = 0 .. 2^b - 1.  FUSED ignores
 *     it, and so does LOGSP with LDPC_FD_LOG8 storage (already 8-bit).
 *     Changes results by design.
 *   LDPC_FD_TUNE_QUANT_STEP: the PLAIN and LOGSP step in units of 2^-12
 *     (1..65536; default 256, i.e. 1/16).
 *   LDPC_FD_TUNE_TAIL_CHUNK: FUSED passes per captured graph (host read of the
 *     active count between graphs) for chunks that start with at most
 *     TAIL_FRAMES active frames; 0 (default) = CHUNK; 1..1000.  Results are
 *     identical for every value.
 *   LDPC_FD_TUNE_BATCH_RETIRE: 1 = such a chunk of at most 32 edge-parallel
 *     passes over at most 128 frames keeps every pass's decisions and checks
 *     them all after the chunk (two launches: the syndromes of every pass and
 *     frame in parallel, then the stopping rule and compaction; each frame
 *     still stops at its first codeword round, with that round's hard, synd,
 *     iters and status; the history buffers take 4096 (N + E + M + 4) bytes of
 *     the workspace, none when that exceeds 64 MiB, and then nothing batches);
 *     0 (default) = syndromes and retirement after every pass.  The decode's
 *     outputs are identical, but a frame that stopped inside a batched chunk
 *     has its message state overwritten by the chunk's later passes, so
 *     ldpc_fd_decode_posterior and ldpc_fd_decode_symbols return
 *     E_UNSUPPORTED for a workspace whose last decode batched; a decode with
 *     LDPC_FD_FLAG_VALIDATION never batches.
 *   LDPC_FD_TUNE_FIRST_CHUNK: FUSED passes before the first host read of the
 *     active count (the first captured graph); 0 (default) = CHUNK; 1..1000.
 *     With a long first chunk and a short CHUNK the decoder reads the count
 *     often only once most frames have stopped, and reaches the tail form
 *     sooner.  Results are identical for every value.
 * The edge-parallel pass of a tail chunk covers 32 frames when the chunk
 * starts with at most 32 active, 128 when with at most 128, else TAIL_FRAMES
 * (and at most the batch).
 * Errors: E_INVALID (unknown key or value), E_UNSUPPORTED (no such variant). */
enum { LDPC_FD_TUNE_LANE_ENTRIES = 0, LDPC_FD_TUNE_GRID_BLOCKS = 1, LDPC_FD_TUNE_CHUNK = 2,
       LDPC_FD_TUNE_GRAPHS = 3, LDPC_FD_TUNE_TAIL_ENTRIES = 4, LDPC_FD_TUNE_TAIL_FRAMES = 5,
       LDPC_FD_TUNE_PRECISE = 6, LDPC_FD_TUNE_DECISION_MFMA = 7, LDPC_FD_TUNE_TAIL_SPLIT = 8,
       LDPC_FD_TUNE_QUANT_BITS = 9, LDPC_FD_TUNE_QUANT_STEP = 10, LDPC_FD_TUNE_TAIL_CHUNK = 11,
       LDPC_FD_TUNE_BATCH_RETIRE = 12, LDPC_FD_TUNE_FIRST_CHUNK = 13 };
int32_t ldpc_fd_set_tuning(ldpc_fd_code code, int32_t key, int32_t value);
int32_t ldpc_fd_get_tuning(ldpc_fd_code code, int32_t key, int32_t *value);

/* Kernel timing for measurement (calling thread only).  While enabled,
 * ldpc_fd_decode records a pair of HIP events on its stream around every launch
 * of the per-round kernels: LDPC_FD_K_FUSED (the fused pass), LDPC_FD_K_CHECK
 * and LDPC_FD_K_VAR (the PLAIN check-node and variable-node kernels).
 * ldpc_fd_profile_read waits for the recorded events, returns the summed
 * duration in milliseconds and the number of launches of `kernel`, and clears
 * that kernel's record.  Errors: E_INVALID (unknown kernel), E_HIP. */
enum { LDPC_FD_K_FUSED = 0, LDPC_FD_K_CHECK = 1, LDPC_FD_K_VAR = 2 };
int32_t ldpc_fd_profile_enable(int32_t on);
int32_t ldpc_fd_profile_read(int32_t kernel, double *ms, int64_t *launches);

/* Message of the last failure on the calling thread ("" if none). */
const char *ldpc_fd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LDPC_FD_H */
