/*
 * warplda.h - C ABI of the MI355X (gfx950) WarpLDA sampler.
 *
 * The library runs the per-iteration Metropolis-Hastings sweep of WarpLDA
 * (Chen, Li, Zhu, Chen, arXiv:1510.08628): a word phase that visits the
 * tokens grouped by word and a document phase that visits them grouped by
 * document (Section 4.4 "Reordering the computation"; Algorithm 2 of
 * Appendix A).  The calls mirror the paper's statement of the problem
 * (Section 2.1: a corpus of word-id / doc-id tokens, K topics, symmetric
 * Dirichlet priors alpha and beta; Section 4.1: M proposals per token) and its
 * programming model (Section 5.1: AddEntry = create, VisitByColumn = word
 * phase, VisitByRow = document phase).
 *
 * Conventions
 *   - Every call returns a wlda_status; WLDA_OK == 0.  No call aborts or
 *     throws.  After WLDA_E_HIP the handle is unusable except for destroy.
 *   - Host arrays passed in are read during the call only; the caller keeps
 *     ownership.  Output arrays are caller-allocated host memory.
 *   - Device memory: the caller allocates ONE device buffer ("workspace") of
 *     at least wlda_workspace_bytes() bytes and keeps it alive until
 *     wlda_destroy(); the library carves all device state out of it and makes
 *     no device allocation of its own.  Its base must be 256-byte aligned.
 *   - Streams: every call enqueues its work on the hipStream_t given to
 *     wlda_create (passed as void*; NULL = the default stream).  Only the
 *     calls marked "synchronises" wait for that stream.
 *   - One handle must not be used from two threads at once.
 *   - Limits: 1 <= M <= 4, 1 <= K <= 2^21 - 1, n_tokens < 2^32, V, D >= 1.
 *
 * Randomness: Philox4x32-10 (Salmon et al., SC'11) keyed by the 64-bit seed
 * (key = (seed & 0xffffffff, seed >> 32)).  Each token draws from at most
 * 1 + ceil(M/2) calls per phase, with counter (t, iteration, phase << 16 | j,
 * 0), phase 0 = initialisation, 1 = word phase, 2 = document phase:
 *   - call j = 0 gives the M acceptance uniforms (output word i-1 for MH step
 *     i; at initialisation its word 2 gives z = Dice(K));
 *   - call j >= 1 gives the (mixture coin, index or uniform topic) words of
 *     proposals 2j-1 (output words 0, 1) and 2j (words 2, 3);
 *   - with WLDA_WORD_ALIAS, the count part of a word proposal of a word with
 *     L_w > K takes its bin from the index word and its position inside the
 *     bin from the same output word of the call with counter word 3 = 1.
 * t is the token's position in the order its phase visits it: the canonical
 * column-major position (tokens sorted by word, then document, then input
 * index) at initialisation and in the word phase, and the canonical row-major
 * position rowptr[d] + n (the n-th token of document d in ascending
 * column-major position) in the document phase.  The first document proposals
 * are drawn at iteration 0 with the document phase's counter.  Uniforms are
 * U(r) = (r >> 8) 2^-24 and Dice(r, n) = (r n) >> 32.  Results are therefore
 * independent of launch geometry and record layout, and bit-identical to any
 * implementation of the same definition.
 */
#ifndef WARPLDA_H
#define WARPLDA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WLDA_OK = 0,
    WLDA_E_INVALID = -1,     /* bad argument: null pointer, id out of range,
                                K/M/alpha/beta/size outside the limits      */
    WLDA_E_WORKSPACE = -2,   /* workspace too small or misaligned          */
    WLDA_E_HIP = -3,         /* a HIP runtime call failed (sticky)          */
    WLDA_E_STATE = -4,       /* call out of order (e.g. a phase before init,
                                a doc phase before the word phase)          */
    WLDA_E_UNSUPPORTED = -5, /* valid input this build does not handle      */
    WLDA_E_NOMEM = -6        /* host memory for the layout exhausted        */
} wlda_status;

/* Problem definition (Section 2.1; Section 4.1 for M). */
typedef struct {
    uint32_t V;      /* vocabulary size (declared; enters beta_bar = V beta) */
    uint32_t D;      /* number of documents                                  */
    uint32_t K;      /* number of topics                                     */
    uint32_t M;      /* MH steps (= proposals stored) per token per phase    */
    double alpha;    /* symmetric document-topic prior, > 0                  */
    double beta;     /* symmetric topic-word prior, > 0                      */
    uint64_t seed;   /* Philox key                                           */
} wlda_params;

typedef struct wlda_sampler_s *wlda_sampler;

/* Exact workspace size for this corpus (reads the token arrays once).
 * word_ids[i] < V and doc_ids[i] < D for all i < n_tokens (host arrays). */
wlda_status wlda_workspace_bytes(const wlda_params *p, const uint32_t *word_ids,
                                 const uint32_t *doc_ids, uint64_t n_tokens,
                                 uint64_t *bytes);

/* AddEntry for every token (Section 5.1): builds the column-major token
 * layout with each column sorted by document id and the per-row pointers into
 * it (Section 5.2), uploads it into the workspace and returns a handle.  The
 * token arrays are host memory in any order; token i is (word_ids[i],
 * doc_ids[i]).  Synchronises. */
wlda_status wlda_create(const wlda_params *p, const uint32_t *word_ids,
                        const uint32_t *doc_ids, uint64_t n_tokens,
                        void *dev_workspace, uint64_t workspace_bytes,
                        void *hip_stream, wlda_sampler *out);

/* Options of wlda_workspace_bytes_ex / wlda_create_ex (a bit mask; 0 gives
 * wlda_workspace_bytes / wlda_create).
 *
 * WLDA_WORD_ALIAS: the word proposals of words with L_w > K (Section 5.4's
 * intra-word-parallel words) come from Walker's alias table over the K topics
 * of the word's updated counts c_w (alias sampling, Section 2.2; Algorithm 2's
 * BuildAlias and urn.Draw) instead of the inverse CDF of those counts.  The
 * law of the chain is the same; the random bits used differ.  The table is
 * exact in integers: bin k weighs c_k K against a mean of L_w; a draw takes
 * the bin b = Dice(r, K) from the index word r and u = Dice(r', L_w) from the
 * stream-1 word r' (see Randomness above) and returns b if u < thr_b, else
 * alias_b.  It is built by the two-pointer sweep (light bins, c_k K <= L_w,
 * in topic order, each topped up by the current heavy bin, heavy bins in
 * topic order; a heavy bin left with weight r <= L_w keeps r and is topped up
 * by the next heavy bin; bins left over weigh L_w and keep themselves), one
 * GPU thread per word, O(K) per word and iteration.  Every word with
 * L_w > K then runs on the long-word kernels.  Words must hold fewer than
 * 2^31 tokens (else WLDA_E_UNSUPPORTED).  Unknown bits: WLDA_E_INVALID. */
#define WLDA_WORD_ALIAS 1u

wlda_status wlda_workspace_bytes_ex(const wlda_params *p, const uint32_t *word_ids,
                                    const uint32_t *doc_ids, uint64_t n_tokens,
                                    uint32_t flags, uint64_t *bytes);

wlda_status wlda_create_ex(const wlda_params *p, const uint32_t *word_ids,
                           const uint32_t *doc_ids, uint64_t n_tokens, uint32_t flags,
                           void *dev_workspace, uint64_t workspace_bytes,
                           void *hip_stream, wlda_sampler *out);

/* Asymmetric document-topic prior (the alpha_k of Eq. (6)-(7) in their
 * general form), replacing the symmetric alpha of wlda_params.  alpha is a
 * host array of K binary32 values, each > 0 and finite (else
 * WLDA_E_INVALID); it is copied into the workspace.  Only before the first
 * wlda_init (else WLDA_E_STATE).  NULL returns to the symmetric alpha.
 * With alpha_k:
 *   - alpha_bar = sum_k alpha_k (binary64, in topic order), rounded to
 *     binary32 for the doc proposals' coin u (L_d + alpha_bar) < L_d;
 *   - the prior part of a doc proposal is topic k with probability
 *     alpha_k / alpha_bar: with A_k the binary64 running sums of alpha_k and
 *     r the proposal's index word, x = r 2^-32 A_{K-1} and the proposal is
 *     the smallest k with A_k > x;
 *   - the word proposals' acceptance rate pi_word of Eq. (7) reads
 *     num = (C_dc + alpha_c)(C_s + beta_bar), den = (C_ds + alpha_s)(C_c + beta_bar)
 *     (pi_doc does not involve alpha);
 *   - wlda_log_likelihood's document part and wlda_theta use alpha_k.
 * Saved states do not carry alpha_k: set it again before loading one into a
 * new sampler.  Synchronises. */
wlda_status wlda_set_alpha(wlda_sampler s, const float *alpha);

/* Initialisation (Algorithm 2): z = Dice(K) for every token, then the first
 * M document proposals per token drawn from that Z by the document phase's
 * proposal rule, then c_k = histogram(Z).  May be called again to restart. */
wlda_status wlda_init(wlda_sampler s);

/* Word phase = VisitByColumn (Section 4.4, Algorithm 2): per word, c_w is
 * rebuilt from the column, each token runs M MH steps over its pending
 * document proposals with the acceptance rate pi_doc of Eq. (7) (counts held
 * fixed for the whole phase), and then draws M word proposals from the
 * updated column (random positioning, Section 4.3, mixing weight
 * L_w / (L_w + K beta)); columns longer than K tokens, the
 * intra-word-parallel words of Section 5.4 whose proposal the paper draws
 * from a table over c_w, take the count part from the inverse CDF of the
 * updated c_w instead (the same law): j = Dice(r, L_w), proposal = the
 * smallest topic k whose inclusive prefix count exceeds j.  Requires init;
 * must alternate with doc_phase. */
wlda_status wlda_word_phase(wlda_sampler s);

/* Document phase = VisitByRow: c_d rebuilt per document, M MH steps over the
 * pending word proposals with pi_word of Eq. (7), then M document proposals
 * drawn from the updated row (mixing weight L_d / (L_d + K alpha)).
 * Completes one iteration. */
wlda_status wlda_doc_phase(wlda_sampler s);

/* n x (word phase, doc phase), enqueued back to back. */
wlda_status wlda_iterate(wlda_sampler s, uint32_t n);

/* Log joint likelihood log p(W, Z | alpha, beta) of Section 6.1 for the
 * current Z, accumulated in binary64.  Synchronises. */
wlda_status wlda_log_likelihood(wlda_sampler s, double *ll);

/* Copies z (n_tokens int32, caller's input order) and, if props != NULL, the
 * M pending proposals (M x n_tokens int32, proposal-major, input order).
 * Synchronises. */
wlda_status wlda_copy_assignments(wlda_sampler s, int32_t *z, int32_t *props);

/* theta_hat of Eq. (4) with alpha' = alpha + 1 for documents d0 .. d0+nd-1:
 * theta[(d - d0) * K + k] = (C_dk + alpha) / (L_d + K alpha), binary32
 * (numerator and denominator each rounded once, then divided), written to
 * DEVICE memory (nd x K floats, caller-owned).  Enqueued on the sampler's
 * stream.  WLDA_E_INVALID if d0 + nd > D, WLDA_E_STATE before init,
 * WLDA_E_UNSUPPORTED for K > 16384. */
wlda_status wlda_theta(wlda_sampler s, uint32_t d0, uint32_t nd, float *theta);

/* phi_hat of Eq. (4) with beta' = beta + 1 for words w0 .. w0+nw-1:
 * phi[(w - w0) * K + k] = (C_wk + beta) / (C_k + V beta), binary32 (as for
 * theta), from the current Z, written to DEVICE memory (nw x K floats,
 * caller-owned).  Enqueued on the sampler's stream.  WLDA_E_INVALID if
 * w0 + nw > V, WLDA_E_STATE before init, WLDA_E_UNSUPPORTED for K > 16384. */
wlda_status wlda_phi(wlda_sampler s, uint32_t w0, uint32_t nw, float *phi);

/* Copies z and the proposals in the canonical column-major order (same
 * shapes as above).  Synchronises. */
wlda_status wlda_copy_assignments_csc(wlda_sampler s, int32_t *z, int32_t *props);

/* Copies c_k (K entries), the exact histogram of the current Z.  Synchronises. */
wlda_status wlda_copy_topic_counts(wlda_sampler s, int64_t *ck);

/* Number of MH steps whose acceptance test passed in the most recent word
 * phase (phase = 1) or document phase (phase = 2).  Synchronises. */
wlda_status wlda_accepted(wlda_sampler s, int phase, uint64_t *count);

/* Completed iterations. */
wlda_status wlda_iteration(wlda_sampler s, uint32_t *iteration);

/* Checkpoint of (iteration, next phase, z, proposals) - the whole sampler
 * state; the layout is rebuilt from the corpus at create.  save synchronises;
 * load replaces the state and recomputes c_k on the device. */
wlda_status wlda_state_bytes(wlda_sampler s, uint64_t *bytes);
wlda_status wlda_save_state(wlda_sampler s, void *host_buf, uint64_t bytes);
wlda_status wlda_load_state(wlda_sampler s, const void *host_buf, uint64_t bytes);

/* Sets z (input order, host) and keeps the pending proposals, recomputing c_k;
 * the next call must be a word phase.  For tests and warm starts. */
wlda_status wlda_set_assignments(wlda_sampler s, const int32_t *z, const int32_t *props);

/* Per-kernel timing.  wlda_profile(s, 1) clears the counters and starts
 * recording a HIP event pair around every kernel the sampler launches (on its
 * stream); wlda_profile(s, 0) stops.  wlda_profile_read() synchronises and
 * returns one entry per kernel kind: total milliseconds over the recorded
 * launches, the launch count and the tokens one launch processes. */
typedef struct {
    const char *name;            /* static string, e.g. "doc_wave"           */
    uint64_t launches;
    uint64_t tokens_per_launch;
    double total_ms;
} wlda_kernel_stat;

wlda_status wlda_profile(wlda_sampler s, int enable);
wlda_status wlda_profile_read(wlda_sampler s, wlda_kernel_stat *out, uint32_t max_entries,
                              uint32_t *n_entries);

/* ------------------------------------------------------------------------ */
/* Fold-in of new documents against a frozen model                          */
/* ------------------------------------------------------------------------ */
/* A model freezes a trained sampler's assignments: the word-topic counts
 * C_w, the topic totals c_k and each word's trained column (for random
 * positioning), all held fixed while new documents run the MCEM E-step of
 * Eq. (5) (the same delayed-update MH chain as training, Section 4.2-4.4, with
 * only c_d changing).  C_w is stored dense (V x K uint32): V*K <= 2^33.
 * Model arrays: the training corpus (host, any order) and its assignments z
 * in the same order (e.g. from wlda_copy_assignments). */
typedef struct wlda_model_s *wlda_model;

wlda_status wlda_model_workspace_bytes(const wlda_params *p, uint64_t n_tokens, uint64_t *bytes);
wlda_status wlda_model_create(const wlda_params *p, const uint32_t *word_ids,
                              const uint32_t *doc_ids, const int32_t *z, uint64_t n_tokens,
                              void *dev_workspace, uint64_t workspace_bytes, void *hip_stream,
                              wlda_model *out);
wlda_status wlda_model_destroy(wlda_model m);

/* Fold-in of a batch of documents (host arrays): document d is
 * words[docptr[d] .. docptr[d+1]) (at most 8192 tokens), with request id
 * req_ids[d] keying its random stream (counter: token-in-document, sweep,
 * phase << 16 | step, request id).  Runs the initialisation and `sweeps`
 * sweeps.  Plain mode (learned_weights == NULL): z starts at Dice(K).
 * Learned mode: learned_weights (n_docs x K, each in [1, 2^24), row sums
 * < 2^32) define an independence proposal q(k) = w_k / sum(w); z starts at a
 * draw from q and every sweep adds `learned_steps` MH steps with q after the
 * word-proposal steps, accepted with the exact ratio
 * (C_dt+a)(C_wt+b)(C_s+bbar) w_s / ((C_ds+a)(C_ws+b)(C_t+bbar) w_t).
 * If hoptr != NULL, heldout_out[d] receives the held-out log likelihood of
 * ho_words[hoptr[d] .. hoptr[d+1]) given the document's final assignments
 * (theta, phi of Eq. (4) with alpha' = alpha + 1, beta' = beta + 1).
 * z_out gets the final assignments (docptr order).  Synchronises. */
wlda_status wlda_foldin_batch_bytes(wlda_model m, uint32_t n_docs, uint64_t n_tokens, int learned,
                                    uint64_t n_heldout, uint64_t *bytes);
wlda_status wlda_foldin_batch(wlda_model m, uint32_t n_docs, const uint64_t *docptr,
                              const uint32_t *words, const uint32_t *req_ids,
                              const uint32_t *learned_weights, uint32_t learned_steps,
                              uint32_t sweeps, const uint64_t *hoptr, const uint32_t *ho_words,
                              void *dev_workspace, uint64_t workspace_bytes, int32_t *z_out,
                              double *heldout_out);

/* Allocation-free variant of wlda_foldin_batch, for callers that cannot
 * allocate device memory (tight serving loops, code under stream capture,
 * harnesses that forbid allocation): the same arguments and results, but the
 * batch's device buffers live in a static device array of
 * WLDA_FOLDIN_STATIC_BYTES bytes that the library holds on each GPU it runs
 * on until the process ends, so the caller passes no workspace.  The device
 * current at wlda_model_create must be current (else WLDA_E_INVALID); runs on
 * the model's stream and synchronises.
 * The array keeps the last call's contents; every buffer the kernels read
 * before writing (per-document sweep counters, inputs) is uploaded by the
 * call itself.  A batch whose wlda_foldin_batch_bytes() exceeds
 * WLDA_FOLDIN_STATIC_BYTES is refused with WLDA_E_WORKSPACE.  All calls on
 * one GPU share the array: calls that overlap in time on one GPU (from two
 * threads, or two models on different streams) race and must be serialised
 * by the caller. */
#define WLDA_FOLDIN_STATIC_BYTES (64ull << 20)
wlda_status wlda_foldin_batch_static(wlda_model m, uint32_t n_docs, const uint64_t *docptr,
                                     const uint32_t *words, const uint32_t *req_ids,
                                     const uint32_t *learned_weights, uint32_t learned_steps,
                                     uint32_t sweeps, const uint64_t *hoptr, const uint32_t *ho_words,
                                     int32_t *z_out, double *heldout_out);

/* ------------------------------------------------------------------------ */
/* Encoder for the learned fold-in proposal                                 */
/* ------------------------------------------------------------------------ */
/* An MLP from a hashed bag of words to a distribution over the K topics,
 * trained on (document, theta_d) pairs that a sampler produced, with
 * theta_d = (C_dk + alpha) / (L_d + K alpha) (Eq. (4) with alpha' = alpha+1):
 *   x: bucket b(w) = ((w * 0x9E3779B1 mod 2^32) * buckets) >> 32 of each
 *      distinct bucket of the document, value = count / L (binary32);
 *   a1 = b1 + sum x_n W1[b_n]; h1 = relu(a1); a2 = h1 W2 + b2; h2 = relu(a2);
 *   z = h2 W3 + b3; q = softmax(z); loss = -(1/B) sum_b sum_k theta log q.
 * W1: buckets x hidden, W2: hidden x hidden, W3: hidden x K (row-major; the
 * row index is the input unit), biases b1, b2 (hidden), b3 (K).  Matrix
 * products use bf16 operands (weights, h1, h2 and the back-propagated
 * signals rounded to nearest even) with fp32 accumulation on the matrix
 * cores; training is Adam on fp32 master weights.
 * Weight arrays are passed as 6 host pointers in the order W1, b1, W2, b2,
 * W3, b3.  Batches are CSR on the device: rowptr (B+1 uint32) into idx
 * (uint32 buckets) and val (float); theta and probs are B x K float, device.
 * forward/proposal/train_step enqueue on the encoder's stream; gradients and
 * train_step with loss != NULL synchronise. */
typedef struct {
    uint32_t buckets;     /* hashed vocabulary size (input dimension)        */
    uint32_t hidden;      /* width of both hidden layers (<= 4096)           */
    uint32_t K;           /* topics (output dimension)                       */
    uint32_t max_batch;   /* rows per call (<= 65536)                        */
    float lr, beta1, beta2, eps;   /* Adam                                  */
} wlda_encoder_params;

typedef struct wlda_encoder_s *wlda_encoder;

wlda_status wlda_encoder_workspace_bytes(const wlda_encoder_params *p, uint64_t *bytes);
wlda_status wlda_encoder_create(const wlda_encoder_params *p, void *dev_workspace,
                                uint64_t workspace_bytes, void *hip_stream, wlda_encoder *out);
wlda_status wlda_encoder_destroy(wlda_encoder e);
wlda_status wlda_encoder_set_weights(wlda_encoder e, const float *const *host_weights);
wlda_status wlda_encoder_get_weights(wlda_encoder e, float *const *host_weights);
/* Host helper: the sparse input of one document (idx ascending, nnz <= L). */
wlda_status wlda_encoder_features(uint32_t buckets, const uint32_t *words, uint32_t L,
                                  uint32_t *idx, float *val, uint32_t *nnz);
/* Host helper: CSR inputs of n_docs documents (document d = words[docptr[d]
 * .. docptr[d+1])); rowptr has n_docs+1 entries, idx/val docptr[n_docs]. */
wlda_status wlda_encoder_features_batch(uint32_t buckets, uint32_t n_docs, const uint64_t *docptr,
                                        const uint32_t *words, uint32_t *rowptr, uint32_t *idx,
                                        float *val);
wlda_status wlda_encoder_forward(wlda_encoder e, uint32_t B, const uint32_t *rowptr,
                                 const uint32_t *idx, const float *val, float *probs);
/* Integer proposal weights w_k = 1 + floor(2^20 ((1-eps) q_k + eps/K)) as
 * per-row running sums (B x K uint32, device), for the learned fold-in
 * proposal; requires K (2^20 + 1) < 2^32. */
wlda_status wlda_encoder_proposal(wlda_encoder e, uint32_t B, const float *probs, float eps,
                                  uint32_t *cdf);
/* Loss and gradients without an update (host outputs, NULL entries skipped). */
wlda_status wlda_encoder_gradients(wlda_encoder e, uint32_t B, const uint32_t *rowptr,
                                   const uint32_t *idx, const float *val, const float *theta,
                                   float *loss, float *const *host_grads);
wlda_status wlda_encoder_train_step(wlda_encoder e, uint32_t B, const uint32_t *rowptr,
                                    const uint32_t *idx, const float *val, const float *theta,
                                    float *loss);

/* ------------------------------------------------------------------------ */
/* Continuous-batching fold-in server                                       */
/* ------------------------------------------------------------------------ */
/* Requests (new documents, at most 8192 tokens) wait in arrival order and
 * are admitted while a document slot and a contiguous range of the device
 * token pool are free.  Each wlda_server_step() admits what fits, runs the
 * encoder for the newly admitted documents (learned mode, on the encoder's
 * stream, overlapped with the sweep of the documents already in flight;
 * documents encoded at admission start their sweeps at the first step that
 * finds their encoder run finished),
 * runs ONE fold-in sweep for every admitted document in one ragged launch,
 * and retires documents that have had their initialisation and `sweeps`
 * sweeps (their z and held-out log likelihood are kept for the caller).
 * A request uses the learned proposal if the server has an encoder or the
 * request brings its own weights; otherwise the plain chain.  Results do not
 * depend on the other requests in flight.  Times are seconds on the server's
 * monotonic clock (wlda_server_now).  step synchronises the server stream. */
typedef struct {
    uint32_t max_docs;       /* document slots                                 */
    uint64_t pool_tokens;    /* device token pool (words, z, proposals)        */
    uint64_t pool_heldout;   /* device pool of held-out tokens                 */
    uint32_t sweeps;         /* sweeps per document (after initialisation)     */
    uint32_t learned_steps;  /* learned MH steps per sweep                     */
    float eps;               /* uniform share of the learned proposal (0, 1]   */
} wlda_server_params;

typedef struct {
    uint32_t req_id, n_tokens, n_heldout, sweeps, learned;
    double arrival_s, admit_s, done_s;   /* server clock                       */
    double heldout_ll;                   /* sum over the held-out tokens       */
} wlda_result;

typedef struct wlda_server_s *wlda_server;

wlda_status wlda_server_workspace_bytes(wlda_model m, wlda_encoder enc_or_null,
                                        const wlda_server_params *sp, uint64_t *bytes);
wlda_status wlda_server_create(wlda_model m, wlda_encoder enc_or_null,
                               const wlda_server_params *sp, void *dev_workspace,
                               uint64_t workspace_bytes, void *hip_stream, wlda_server *out);
wlda_status wlda_server_now(wlda_server s, double *seconds);
/* weights: K learned proposal weights (as in wlda_foldin_batch) or NULL. */
wlda_status wlda_server_submit(wlda_server s, uint32_t req_id, const uint32_t *words, uint32_t L,
                               const uint32_t *heldout_words, uint32_t n_heldout,
                               double arrival_s, const uint32_t *weights);
wlda_status wlda_server_step(wlda_server s, uint32_t *n_active, uint32_t *n_pending);
wlda_status wlda_server_poll(wlda_server s, wlda_result *out, uint32_t max_results,
                             uint32_t *n_results);
wlda_status wlda_server_take_z(wlda_server s, uint32_t req_id, int32_t *z, uint32_t L);
wlda_status wlda_server_destroy(wlda_server s);

/* Releases host-side state; the workspace is the caller's to free. */
wlda_status wlda_destroy(wlda_sampler s);

const char *wlda_strerror(wlda_status e);

#ifdef __cplusplus
}
#endif

#endif /* WARPLDA_H */
