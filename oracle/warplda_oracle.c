/*
 * warplda_oracle.c - plain single-threaded CPU oracle for the WarpLDA sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP library; both sides are written
 * separately from the paper (Chen, Li, Zhu, Chen, "WarpLDA: a Cache Efficient
 * O(1) Algorithm for Latent Dirichlet Allocation", arXiv:1510.08628).
 *
 * What it computes (paper Section 4, Algorithm 2 of Appendix A):
 *   - the token layout: the sparse matrix Y stored column-major, every column
 *     sorted by document id, plus per-row pointers into it (Section 5.2);
 *   - initialisation z ~ Dice(K) (Algorithm 2) and a first draw of the
 *     document proposals from that Z (the word phase consumes doc proposals
 *     "from the last iteration", which the listing never initialises);
 *   - the word phase (VisitByColumn): c_w rebuilt from the column, M MH steps
 *     on the pending doc proposals with the doc-proposal acceptance rate of
 *     Eq. (7), then M new word proposals drawn from the updated column;
 *   - the doc phase (VisitByRow): c_d rebuilt from the row, M MH steps on the
 *     pending word proposals with the word-proposal acceptance rate of
 *     Eq. (7), then M new doc proposals drawn from the updated row;
 *   - c_k, the exact histogram of Z at the start of every phase (Section 4.4,
 *     "M-step": counts computed on the fly from Z);
 *   - the log joint likelihood of Section 6.1, in double precision;
 *   - optionally an asymmetric document-topic prior alpha_k (the general
 *     form of Eq. (6)-(7)): doc proposals q_doc(k) ~ C_dk + alpha_k, the
 *     word-proposal acceptance rate with alpha_c, alpha_s, the LL and theta
 *     with alpha_k (oracle_set_alpha);
 *   - fold-in of new documents against frozen word-topic counts (MCEM E-step
 *     of Eq. (5) with C_w and c_k held fixed), used by the serving path.
 *
 * Readings of points the paper leaves open (each listed in the design notes):
 *   - the MH chain state starts at z and moves on acceptance (Algorithm 1);
 *     Algorithm 2's "s <- z^(i-1)" is read as the current state;
 *   - Algorithm 2's "C_s + beta_bar V" is read as C_s + beta_bar (Eq. 7);
 *   - counts include the token's own assignment (Eq. 5 has no "not dn");
 *   - proposals are drawn from the counts *after* this phase's updates;
 *   - both proposals use random positioning (Section 4.3) over the canonical
 *     row/column order, except that words with L_w > K (Section 5.4's
 *     intra-word-parallel words, whose proposal the paper draws from a table
 *     over c_w) take the inverse CDF of the updated c_w;
 *     the word-proposal mixing weight is L_w / (L_w + K beta) (the prior
 *     mass of C_wk + beta over K topics);
 *   - optionally (oracle_set_word_alias) those words draw from Walker's alias
 *     table over the updated c_w instead (Algorithm 2's BuildAlias and
 *     urn.Draw), built exactly in integers by oracle_alias_table: the same
 *     law, other random bits; the bin comes from the index word and the
 *     position inside it from a second word (stream 1 of the same call);
 *   - all acceptance and coin arithmetic is IEEE binary32 with the exact
 *     expressions below, no fused multiply-add, strict "<";
 *   - randomness is Philox4x32-10 (Salmon et al., SC'11) with the counter
 *     layout of rng_call(): per (token, iteration, phase), call 0 gives the
 *     M acceptance uniforms and calls 1..ceil(M/2) the (coin, index) words
 *     of two proposals each (accept_words, draw_words);
 *     the token index is the token's position in the order its phase visits
 *     it: the canonical column-major (CSC) position at initialisation and in
 *     the word phase, the canonical row-major (CSR) position, rowptr[d] + n,
 *     in the doc phase.  Neither depends on how an implementation stores Y.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fno-fast-math -shared -fPIC
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (Salmon et al., SC'11):     */
/* ten rounds of two 32x32->64 multiplies with the Weyl key schedule.       */
/* ------------------------------------------------------------------------ */
#define PHILOX_MUL_A 0xD2511F53u
#define PHILOX_MUL_B 0xCD9E8D57u
#define PHILOX_WEYL_A 0x9E3779B9u
#define PHILOX_WEYL_B 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t key_in[2], const uint32_t ctr_in[4],
                          uint32_t out[4])
{
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t pa = (uint64_t)PHILOX_MUL_A * x0;
        uint64_t pb = (uint64_t)PHILOX_MUL_B * x2;
        uint32_t n0 = (uint32_t)(pb >> 32) ^ x1 ^ k0;
        uint32_t n1 = (uint32_t)pb;
        uint32_t n2 = (uint32_t)(pa >> 32) ^ x3 ^ k1;
        uint32_t n3 = (uint32_t)pa;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
        k0 += PHILOX_WEYL_A;
        k1 += PHILOX_WEYL_B;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

enum { PH_INIT = 0, PH_WORD = 1, PH_DOC = 2, PH_FOLD_DOC = 3, PH_FOLD_WORD = 4,
       PH_FROZEN = 7 };

/* One RNG call.  Counter = (token, iteration, phase<<16 | step, stream). */
static void rng_call(uint64_t seed, uint32_t token, uint32_t iter,
                     uint32_t phase, uint32_t step, uint32_t stream,
                     uint32_t r[4])
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t ctr[4] = { token, iter, (phase << 16) | step, stream };
    oracle_philox4x32_10(key, ctr, r);
}

/* The random words of one token in one phase: call 0 holds the M
 * acceptance uniforms (word i-1 for step i, M <= 4); call j >= 1 holds the
 * mixture coin and the index/topic word of proposals 2j-1 (words 0, 1) and
 * 2j (words 2, 3).  draw_words() returns those of proposal i. */
static void accept_words(uint64_t seed, uint32_t token, uint32_t iter,
                         uint32_t phase, uint32_t r[4])
{
    rng_call(seed, token, iter, phase, 0, 0, r);
}

static void draw_words(uint64_t seed, uint32_t token, uint32_t iter,
                       uint32_t phase, uint32_t i, uint32_t *coin_word,
                       uint32_t *index_word)
{
    uint32_t r[4];
    rng_call(seed, token, iter, phase, (i + 1) / 2, 0, r);
    *coin_word = r[2 * ((i - 1) % 2)];
    *index_word = r[2 * ((i - 1) % 2) + 1];
}

/* Uniform in [0,1) on the 2^-24 grid. */
static float unif24(uint32_t r) { return (float)(r >> 8) * 0x1p-24f; }

/* Dice(n): a draw from {0, ..., n-1} by multiply-shift. */
static uint32_t dice(uint32_t r, uint32_t n)
{
    return (uint32_t)(((uint64_t)r * (uint64_t)n) >> 32);
}

/* MH acceptance test for Eq. (7).  cnt_* are the row counts (c_w in the word
 * phase, c_d in the doc phase) of the candidate c and the current state s,
 * prior is beta (word phase) or alpha (doc phase); ck_* are the global topic
 * counts.  Accept iff u * den < num, i.e. with probability min(1, num/den). */
static int mh_accept2(float u, int64_t cnt_c, int64_t cnt_s, float prior_c, float prior_s,
                      int64_t ck_s, int64_t ck_c, float beta_bar)
{
    float num = ((float)cnt_c + prior_c) * ((float)ck_s + beta_bar);
    float den = ((float)cnt_s + prior_s) * ((float)ck_c + beta_bar);
    return u * den < num;
}

static int mh_accept(float u, int64_t cnt_c, int64_t cnt_s, float prior,
                     int64_t ck_s, int64_t ck_c, float beta_bar)
{
    return mh_accept2(u, cnt_c, cnt_s, prior, prior, ck_s, ck_c, beta_bar);
}

/* Mixture coin of Section 2.2 / Section 4.3: pick the count part (random
 * positioning) with probability L / (L + prior_mass). */
static int take_count_part(float u, uint64_t L, float prior_mass)
{
    return u * ((float)L + prior_mass) < (float)L;
}

/* Smallest topic k with cum[k] > j, cum an inclusive prefix count over
 * topics 0..K-1 and j < cum[K-1] (binary search). */
static int32_t cdf_topic(const int64_t *cum, uint32_t K, uint32_t j)
{
    uint32_t lo = 0, hi = K - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi) / 2;
        if (cum[mid] > (int64_t)j) hi = mid;
        else lo = mid + 1;
    }
    return (int32_t)lo;
}

/* Walker's alias table (alias sampling, Section 2.2; Algorithm 2 builds one
 * over C_w) for the counts c[0..K-1] of a column of L = sum c tokens, in
 * integers.  Bin b carries the scaled weight x_b = c_b K, so the bins' mean
 * weight is exactly L.  A draw picks a bin b uniformly and u uniformly from
 * [0, L) and returns b if u < thr[b], else alias[b]; topic k is then returned
 * with probability (thr_k + sum over bins b with alias_b = k of L - thr_b) /
 * (K L) = c_k / L.
 * Construction, a deterministic two-pointer sweep (the sequential "sweeping"
 * construction of Huebschle-Schneider and Sanders, Parallel Weighted Random
 * Sampling, ESA 2019): bins with x <= L ("light") are taken in topic order,
 * bins with x > L ("heavy") in topic order.  The current heavy bin h, with
 * remaining weight r, fills the next light bin i (thr_i = x_i, alias_i = h,
 * r -= L - x_i) while r > L; once r <= L, h itself becomes a bin with
 * thr_h = r and alias_h = the next heavy bin, whose remaining weight is its
 * x minus the L - r it gives away.  When the heavy bins run out every bin
 * left has x = L exactly (the weights sum to K L), and keeps itself.
 * Returns 0, or -1 if the counts do not sum to L or L >= 2^31 (the device
 * table keeps a flag in bit 31 of the threshold word). */
static int alias_light(const int64_t *c, uint32_t K, uint64_t L, uint32_t b)
{
    return (uint64_t)c[b] * K <= L;
}

int oracle_alias_table(const int64_t *c, uint32_t K, uint64_t L, uint32_t *thr, uint32_t *alias)
{
    uint64_t sum = 0;
    for (uint32_t k = 0; k < K; ++k) {
        if (c[k] < 0) return -1;
        sum += (uint64_t)c[k];
    }
    if (K == 0 || sum != L || L == 0 || L >= (1ull << 31)) return -1;
    uint32_t i = 0, h = 0;
    while (i < K && !alias_light(c, K, L, i)) ++i;
    while (h < K && alias_light(c, K, L, h)) ++h;
    if (h < K) {
        uint64_t r = (uint64_t)c[h] * K;
        for (;;) {
            if (r > L) {
                if (i >= K) return -1;             /* cannot happen: sum c = L */
                uint64_t x = (uint64_t)c[i] * K;
                thr[i] = (uint32_t)x;
                alias[i] = h;
                r -= L - x;
                do ++i; while (i < K && !alias_light(c, K, L, i));
            } else {
                uint32_t hn = h + 1;
                while (hn < K && alias_light(c, K, L, hn)) ++hn;
                thr[h] = (uint32_t)r;
                alias[h] = hn < K ? hn : h;
                if (hn >= K) break;
                r = (uint64_t)c[hn] * K - (L - r);
                h = hn;
            }
        }
    }
    for (; i < K; ++i) {
        if (!alias_light(c, K, L, i)) continue;
        if ((uint64_t)c[i] * K != L) return -1;    /* cannot happen: sum c = L */
        thr[i] = (uint32_t)L;
        alias[i] = i;
    }
    return 0;
}

/* The second word of an alias draw: proposal i's position inside its bin,
 * from the index-word slot of the same call on stream 1. */
static uint32_t alias_u_word(uint64_t seed, uint32_t token, uint32_t iter,
                             uint32_t phase, uint32_t i)
{
    uint32_t r[4];
    rng_call(seed, token, iter, phase, (i + 1) / 2, 1, r);
    return r[2 * ((i - 1) % 2) + 1];
}

/* ------------------------------------------------------------------------ */
/* Sampler state                                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t V, D, K, M;
    double alpha, beta;
    uint64_t seed;
    uint64_t T;
    /* layout (Section 5.2): column-major token order, rows by pointer */
    uint64_t *colptr;   /* V+1 */
    uint64_t *rowptr;   /* D+1 */
    uint32_t *row;      /* T: CSC positions of each row, ascending */
    uint32_t *inv;      /* T: input index -> CSC position */
    uint32_t *word_of;  /* T: word of each CSC position */
    uint32_t *doc_of;   /* T: doc of each CSC position */
    /* per-token data y = (z, z^(1..M)) in CSC order */
    int32_t *z;         /* T */
    int32_t *prop;      /* M*T, proposal i (0-based) of token t at i*T + t */
    int64_t *ck;        /* K: histogram of Z */
    uint32_t iter;      /* completed iterations */
    int next_phase;     /* 0 = not initialised, PH_WORD or PH_DOC */
    uint64_t accepted_word, accepted_doc;   /* last phase of each kind */
    int visit_reversed; /* visit rows/columns in reverse order (tests) */
    /* binary32 constants */
    float a, b, alpha_bar, beta_k, beta_bar;
    /* asymmetric alpha (NULL: symmetric): alpha_k as binary32, and its
     * running sums in topic order, binary64 */
    float *alpha_k;
    double *alpha_cum;
    /* test harness: added to the token index of the Philox counter in the
     * word phase (CSC) and the doc phase (CSR), so that a corpus holding one
     * column or one row of a larger corpus draws that corpus's numbers */
    uint32_t t_off_csc, t_off_csr;
    /* word proposals of columns with L_w > K from an alias table (1) or the
     * inverse CDF (0) of the updated c_w */
    int word_alias;
    uint32_t *alias_thr, *alias_tab;   /* K each, scratch of the alias draw */
} oracle_t;

typedef struct {
    uint32_t V, D, K, M;
    double alpha, beta;
    uint64_t seed;
} oracle_params;

static void set_constants(oracle_t *o)
{
    o->a = (float)o->alpha;
    o->b = (float)o->beta;
    o->alpha_bar = (float)o->K * o->a;   /* alpha_bar = K alpha */
    o->beta_k = (float)o->K * o->b;      /* prior mass of C_wk + beta */
    o->beta_bar = (float)o->V * o->b;    /* beta_bar = V beta */
}

/* alpha of topic k (Eq. 6-7): alpha_k, or the symmetric alpha. */
static float alpha_of(const oracle_t *o, int32_t k)
{
    return o->alpha_k ? o->alpha_k[k] : o->a;
}

/* The prior part of a doc proposal: topic k with probability alpha_k /
 * alpha_bar.  Symmetric alpha: Dice(K).  Asymmetric: x = r 2^-32 A_{K-1} in
 * binary64, with A_k the running sums of alpha_k in topic order, and the
 * smallest k with A_k > x (x < A_{K-1} always). */
static int32_t prior_topic(const oracle_t *o, uint32_t r)
{
    if (!o->alpha_k) return (int32_t)dice(r, o->K);
    double x = (double)r * 0x1p-32 * o->alpha_cum[o->K - 1];
    uint32_t lo = 0, hi = o->K - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi) / 2;
        if (o->alpha_cum[mid] > x) hi = mid;
        else lo = mid + 1;
    }
    return (int32_t)lo;
}

/* Layout of Section 5.2: Y in CSC form with every column sorted by row id,
 * ties kept in input order (stable), and P_CSR pointing into it.  Built as a
 * stable counting sort by document followed by a stable counting sort by
 * word, which orders tokens by (word, doc, input index). */
static int build_layout(oracle_t *o, const uint32_t *word_ids,
                        const uint32_t *doc_ids)
{
    uint64_t T = o->T;
    uint32_t *by_doc = malloc(T * sizeof(uint32_t) + 1);
    uint64_t *cnt = calloc((size_t)(o->D > o->V ? o->D : o->V) + 1, sizeof(uint64_t));
    if (!by_doc || !cnt) { free(by_doc); free(cnt); return -1; }
    /* pass 1: stable sort of input indices by doc id */
    for (uint64_t i = 0; i < T; ++i) cnt[doc_ids[i] + 1]++;
    for (uint32_t d = 0; d < o->D; ++d) cnt[d + 1] += cnt[d];
    for (uint64_t i = 0; i < T; ++i) by_doc[cnt[doc_ids[i]]++] = (uint32_t)i;
    /* pass 2: stable sort of that sequence by word id */
    memset(o->colptr, 0, (o->V + 1) * sizeof(uint64_t));
    for (uint64_t i = 0; i < T; ++i) o->colptr[word_ids[i] + 1]++;
    for (uint32_t w = 0; w < o->V; ++w) o->colptr[w + 1] += o->colptr[w];
    memcpy(cnt, o->colptr, o->V * sizeof(uint64_t));
    for (uint64_t j = 0; j < T; ++j) {
        uint32_t i = by_doc[j];
        uint64_t t = cnt[word_ids[i]]++;
        o->inv[i] = (uint32_t)t;
        o->word_of[t] = word_ids[i];
        o->doc_of[t] = doc_ids[i];
    }
    /* rows: CSC positions of each document, ascending */
    memset(o->rowptr, 0, (o->D + 1) * sizeof(uint64_t));
    for (uint64_t t = 0; t < T; ++t) o->rowptr[o->doc_of[t] + 1]++;
    for (uint32_t d = 0; d < o->D; ++d) o->rowptr[d + 1] += o->rowptr[d];
    memcpy(cnt, o->rowptr, o->D * sizeof(uint64_t));
    for (uint64_t t = 0; t < T; ++t) o->row[cnt[o->doc_of[t]]++] = (uint32_t)t;
    free(by_doc);
    free(cnt);
    return 0;
}

void oracle_destroy(oracle_t *o)
{
    if (!o) return;
    free(o->colptr); free(o->rowptr); free(o->row); free(o->inv);
    free(o->word_of); free(o->doc_of); free(o->z); free(o->prop); free(o->ck);
    free(o->alpha_k); free(o->alpha_cum);
    free(o->alias_thr); free(o->alias_tab);
    free(o);
}

/* Word proposals of columns with L_w > K from Walker's alias table over the
 * updated c_w (on != 0) or from its inverse CDF (0, the default).  Any time
 * between phases.  Returns 0, or -1 when out of memory. */
int oracle_set_word_alias(oracle_t *o, int on)
{
    if (on && !o->alias_thr) {
        o->alias_thr = malloc(o->K * sizeof(uint32_t));
        o->alias_tab = malloc(o->K * sizeof(uint32_t));
        if (!o->alias_thr || !o->alias_tab) {
            free(o->alias_thr); free(o->alias_tab);
            o->alias_thr = o->alias_tab = NULL;
            return -1;
        }
    }
    o->word_alias = on != 0;
    return 0;
}

/* Returns NULL on invalid input or allocation failure. */
oracle_t *oracle_create(const oracle_params *p, const uint32_t *word_ids,
                        const uint32_t *doc_ids, uint64_t n_tokens)
{
    if (!p || p->K == 0 || p->M == 0 || p->M > 4 || p->V == 0 ||
        p->D == 0 || !(p->alpha > 0) || !(p->beta > 0) ||
        n_tokens >= ((uint64_t)1 << 32))
        return NULL;
    if (n_tokens > 0 && (!word_ids || !doc_ids)) return NULL;
    for (uint64_t i = 0; i < n_tokens; ++i)
        if (word_ids[i] >= p->V || doc_ids[i] >= p->D) return NULL;
    oracle_t *o = calloc(1, sizeof(oracle_t));
    if (!o) return NULL;
    o->V = p->V; o->D = p->D; o->K = p->K; o->M = p->M;
    o->alpha = p->alpha; o->beta = p->beta; o->seed = p->seed;
    o->T = n_tokens;
    set_constants(o);
    size_t T = (size_t)n_tokens;
    o->colptr = malloc((o->V + 1) * sizeof(uint64_t));
    o->rowptr = malloc((o->D + 1) * sizeof(uint64_t));
    o->row = malloc(T * sizeof(uint32_t) + 1);
    o->inv = malloc(T * sizeof(uint32_t) + 1);
    o->word_of = malloc(T * sizeof(uint32_t) + 1);
    o->doc_of = malloc(T * sizeof(uint32_t) + 1);
    o->z = malloc(T * sizeof(int32_t) + 1);
    o->prop = malloc((size_t)o->M * T * sizeof(int32_t) + 1);
    o->ck = calloc(o->K, sizeof(int64_t));
    if (!o->colptr || !o->rowptr || !o->row || !o->inv || !o->word_of ||
        !o->doc_of || !o->z || !o->prop || !o->ck ||
        build_layout(o, word_ids, doc_ids) != 0) {
        oracle_destroy(o);
        return NULL;
    }
    return o;
}

static void recount_ck(oracle_t *o)
{
    memset(o->ck, 0, o->K * sizeof(int64_t));
    for (uint64_t t = 0; t < o->T; ++t) o->ck[o->z[t]]++;
}

/* Draw M doc proposals for every token of row d from the current row
 * (random positioning with mixing weight L_d / (L_d + alpha_bar), Section 4.3
 * and Algorithm 2's document phase). */
static void draw_doc_proposals(oracle_t *o, uint32_t d, uint32_t iter)
{
    uint64_t beg = o->rowptr[d], L = o->rowptr[d + 1] - beg;
    for (uint64_t n = 0; n < L; ++n) {
        uint32_t t = o->row[beg + n];
        for (uint32_t i = 1; i <= o->M; ++i) {
            uint32_t cw_, iw;
            draw_words(o->seed, o->t_off_csr + (uint32_t)(beg + n), iter, PH_DOC, i, &cw_, &iw);
            int32_t prop;
            if (take_count_part(unif24(cw_), L, o->alpha_bar))
                prop = o->z[o->row[beg + dice(iw, (uint32_t)L)]];
            else
                prop = prior_topic(o, iw);
            o->prop[(uint64_t)(i - 1) * o->T + t] = prop;
        }
    }
}

/* Initialisation: z = Dice(K) for every token (Algorithm 2), then the first
 * doc proposals from that Z, then c_k = histogram(Z). */
int oracle_init(oracle_t *o)
{
    for (uint64_t t = 0; t < o->T; ++t) {
        uint32_t r[4];
        rng_call(o->seed, (uint32_t)t, 0, PH_INIT, 0, 0, r);
        o->z[t] = (int32_t)dice(r[2], o->K);
    }
    for (uint32_t d = 0; d < o->D; ++d) draw_doc_proposals(o, d, 0);
    recount_ck(o);
    o->iter = 0;
    o->next_phase = PH_WORD;
    o->accepted_word = o->accepted_doc = 0;
    return 0;
}

/* Asymmetric document-topic prior: alpha[k] > 0 (finite, binary32) for every
 * topic, or NULL to return to the symmetric alpha.  Only before oracle_init.
 * alpha_bar becomes the binary64 sum of the alpha_k, rounded to binary32. */
int oracle_set_alpha(oracle_t *o, const float *alpha)
{
    if (o->next_phase != 0) return -4;
    free(o->alpha_k); free(o->alpha_cum);
    o->alpha_k = NULL; o->alpha_cum = NULL;
    set_constants(o);
    if (!alpha) return 0;
    for (uint32_t k = 0; k < o->K; ++k)
        if (!(alpha[k] > 0.0f) || !isfinite(alpha[k])) return -1;
    o->alpha_k = malloc(o->K * sizeof(float));
    o->alpha_cum = malloc(o->K * sizeof(double));
    if (!o->alpha_k || !o->alpha_cum) {
        free(o->alpha_k); free(o->alpha_cum);
        o->alpha_k = NULL; o->alpha_cum = NULL;
        return -1;
    }
    double run = 0.0;
    for (uint32_t k = 0; k < o->K; ++k) {
        o->alpha_k[k] = alpha[k];
        run += (double)alpha[k];
        o->alpha_cum[k] = run;
    }
    o->alpha_bar = (float)run;
    return 0;
}

/* Test harness for corpora too large for the whole oracle: a corpus that is
 * one column (or one row) of a larger one, set to that corpus's state, runs
 * one phase exactly as the larger corpus would for that column (row).
 * oracle_set_token_offsets: the column's (row's) first canonical position in
 * the larger corpus; oracle_set_phase_state: the larger corpus's c_k at the
 * start of the phase, the phase to run next and the completed iterations
 * (after oracle_init and oracle_set_csc_state). */
void oracle_set_token_offsets(oracle_t *o, uint32_t csc_off, uint32_t csr_off)
{
    o->t_off_csc = csc_off;
    o->t_off_csr = csr_off;
}

int oracle_set_phase_state(oracle_t *o, const int64_t *ck, int next_phase, uint32_t iter)
{
    if (o->next_phase == 0 || (next_phase != PH_WORD && next_phase != PH_DOC)) return -4;
    memcpy(o->ck, ck, o->K * sizeof(int64_t));
    o->next_phase = next_phase;
    o->iter = iter;
    return 0;
}

/* f_c of Section 5.1 for one column w: c_w from the column's assignments at
 * the start of the phase, M MH steps per token on its doc proposals with the
 * counts frozen (delayed update, Section 4.2), commit of the whole column,
 * then M word proposals per token drawn from the updated column.  Adds the
 * column's new assignments to ck_next (if given) and the passed acceptance
 * tests to *accepted.  cw and znew are scratch (K and T entries). */
static void word_column(oracle_t *o, uint32_t w, uint32_t iter, int64_t *ck_next,
                        uint64_t *accepted, int64_t *cw, int32_t *znew)
{
    uint64_t beg = o->colptr[w], L = o->colptr[w + 1] - beg;
    if (L == 0) return;
    /* cw is all zero on entry and is returned all zero */
    for (uint64_t n = 0; n < L; ++n) cw[o->z[beg + n]]++;
    for (uint64_t n = 0; n < L; ++n) {
        uint32_t t = (uint32_t)(beg + n);
        int32_t s = o->z[t];
        uint32_t ra[4];
        accept_words(o->seed, o->t_off_csc + t, iter, PH_WORD, ra);
        for (uint32_t i = 1; i <= o->M; ++i) {
            int32_t c = o->prop[(uint64_t)(i - 1) * o->T + t];
            if (mh_accept(unif24(ra[i - 1]), cw[c], cw[s], o->b, o->ck[s],
                          o->ck[c], o->beta_bar)) {
                s = c;
                (*accepted)++;
            }
        }
        znew[t] = s;
    }
    for (uint64_t n = 0; n < L; ++n) cw[o->z[beg + n]] = 0;
    for (uint64_t n = 0; n < L; ++n) o->z[beg + n] = znew[beg + n];
    /* Words with L_w > K are the intra-word-parallel words of Section 5.4,
     * whose word proposal the paper draws from a table built over the
     * column's counts c_w rather than from a token position.  For them the
     * count part is the inverse CDF of the updated c_w: j = Dice(r, L_w), and
     * the proposal is the smallest topic k whose inclusive prefix count C(k)
     * exceeds j.  Each token's topic occupies one unit of [0, L_w), so the
     * law is that of random positioning. */
    int by_cdf = L > o->K;
    int by_alias = by_cdf && o->word_alias;
    if (by_cdf) {
        for (uint64_t n = 0; n < L; ++n) cw[o->z[beg + n]]++;
        if (by_alias) {
            if (oracle_alias_table(cw, o->K, L, o->alias_thr, o->alias_tab) != 0) abort();
        } else {
            for (uint32_t k = 1; k < o->K; ++k) cw[k] += cw[k - 1];
        }
    }
    for (uint64_t n = 0; n < L; ++n) {
        uint32_t t = (uint32_t)(beg + n);
        for (uint32_t i = 1; i <= o->M; ++i) {
            uint32_t cw_, iw;
            draw_words(o->seed, o->t_off_csc + t, iter, PH_WORD, i, &cw_, &iw);
            int32_t prop;
            if (take_count_part(unif24(cw_), L, o->beta_k)) {
                if (by_alias) {
                    /* urn.Draw: a bin, then a position inside it */
                    uint32_t b = dice(iw, o->K);
                    uint32_t u = dice(alias_u_word(o->seed, o->t_off_csc + t, iter, PH_WORD, i),
                                      (uint32_t)L);
                    prop = (int32_t)(u < o->alias_thr[b] ? b : o->alias_tab[b]);
                } else {
                    uint32_t j = dice(iw, (uint32_t)L);
                    prop = by_cdf ? cdf_topic(cw, o->K, j) : o->z[beg + j];
                }
            } else {
                prop = (int32_t)dice(iw, o->K);
            }
            o->prop[(uint64_t)(i - 1) * o->T + t] = prop;
        }
        if (ck_next) ck_next[o->z[t]]++;
    }
    if (by_cdf) memset(cw, 0, o->K * sizeof(int64_t));
}

/* Word phase, VisitByColumn with f_c (Section 4.4, Algorithm 2). */
int oracle_word_phase(oracle_t *o)
{
    if (o->next_phase != PH_WORD) return -4;
    uint32_t iter = o->iter + 1;
    int64_t *cw = calloc(o->K, sizeof(int64_t));
    int64_t *ck_next = calloc(o->K, sizeof(int64_t));
    int32_t *znew = malloc(o->T * sizeof(int32_t) + 1);
    if (!cw || !ck_next || !znew) { free(cw); free(ck_next); free(znew); return -1; }
    uint64_t accepted = 0;
    for (uint32_t v = 0; v < o->V; ++v) {
        uint32_t w = o->visit_reversed ? o->V - 1 - v : v;
        word_column(o, w, iter, ck_next, &accepted, cw, znew);
    }
    memcpy(o->ck, ck_next, o->K * sizeof(int64_t));
    free(cw); free(ck_next); free(znew);
    o->accepted_word = accepted;
    o->next_phase = PH_DOC;
    return 0;
}

/* f_r of Section 5.1 for one row d: c_d from the row, M MH steps per token
 * on its word proposals, commit of the row, M doc proposals per token drawn
 * from the updated row. */
static void doc_row(oracle_t *o, uint32_t d, uint32_t iter, int64_t *ck_next,
                    uint64_t *accepted, int64_t *cd, int32_t *znew)
{
    uint64_t beg = o->rowptr[d], L = o->rowptr[d + 1] - beg;
    if (L == 0) return;
    /* cd is all zero on entry and is returned all zero */
    for (uint64_t n = 0; n < L; ++n) cd[o->z[o->row[beg + n]]]++;
    for (uint64_t n = 0; n < L; ++n) {
        uint32_t t = o->row[beg + n];
        int32_t s = o->z[t];
        uint32_t ra[4];
        accept_words(o->seed, o->t_off_csr + (uint32_t)(beg + n), iter, PH_DOC, ra);
        for (uint32_t i = 1; i <= o->M; ++i) {
            int32_t c = o->prop[(uint64_t)(i - 1) * o->T + t];
            if (mh_accept2(unif24(ra[i - 1]), cd[c], cd[s], alpha_of(o, c), alpha_of(o, s),
                           o->ck[s], o->ck[c], o->beta_bar)) {
                s = c;
                (*accepted)++;
            }
        }
        znew[t] = s;
    }
    for (uint64_t n = 0; n < L; ++n) cd[o->z[o->row[beg + n]]] = 0;
    for (uint64_t n = 0; n < L; ++n) {
        uint32_t t = o->row[beg + n];
        o->z[t] = znew[t];
    }
    draw_doc_proposals(o, d, iter);
    if (ck_next)
        for (uint64_t n = 0; n < L; ++n) ck_next[o->z[o->row[beg + n]]]++;
}

/* Document phase, VisitByRow with f_r (Section 4.4, Algorithm 2). */
int oracle_doc_phase(oracle_t *o)
{
    if (o->next_phase != PH_DOC) return -4;
    uint32_t iter = o->iter + 1;
    int64_t *cd = calloc(o->K, sizeof(int64_t));
    int64_t *ck_next = calloc(o->K, sizeof(int64_t));
    int32_t *znew = malloc(o->T * sizeof(int32_t) + 1);
    if (!cd || !ck_next || !znew) { free(cd); free(ck_next); free(znew); return -1; }
    uint64_t accepted = 0;
    for (uint32_t e = 0; e < o->D; ++e) {
        uint32_t d = o->visit_reversed ? o->D - 1 - e : e;
        doc_row(o, d, iter, ck_next, &accepted, cd, znew);
    }
    memcpy(o->ck, ck_next, o->K * sizeof(int64_t));
    free(cd); free(ck_next); free(znew);
    o->accepted_doc = accepted;
    o->iter = iter;
    o->next_phase = PH_WORD;
    return 0;
}

int oracle_iterate(oracle_t *o, uint32_t n)
{
    for (uint32_t k = 0; k < n; ++k) {
        int rc = oracle_word_phase(o);
        if (rc) return rc;
        rc = oracle_doc_phase(o);
        if (rc) return rc;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Log joint likelihood log p(W, Z | alpha, beta) of Section 6.1, binary64. */
/* ------------------------------------------------------------------------ */
double oracle_log_joint(uint64_t T, uint32_t V, uint32_t D, uint32_t K,
                        double alpha, double beta, const uint32_t *word_ids,
                        const uint32_t *doc_ids, const int32_t *z)
{
    double alpha_bar = K * alpha, beta_bar = V * beta;
    int64_t *cdk = calloc((size_t)D * K, sizeof(int64_t));
    int64_t *cwk = calloc((size_t)V * K, sizeof(int64_t));
    int64_t *ck = calloc(K, sizeof(int64_t));
    int64_t *Ld = calloc(D, sizeof(int64_t));
    if (!cdk || !cwk || !ck || !Ld) {
        free(cdk); free(cwk); free(ck); free(Ld);
        return NAN;
    }
    for (uint64_t i = 0; i < T; ++i) {
        cdk[(size_t)doc_ids[i] * K + z[i]]++;
        cwk[(size_t)word_ids[i] * K + z[i]]++;
        ck[z[i]]++;
        Ld[doc_ids[i]]++;
    }
    double ll = 0.0;
    /* document part: prod_d Gamma(abar)/Gamma(abar+L_d) prod_k Gamma(a+C_dk)/Gamma(a) */
    for (uint32_t d = 0; d < D; ++d) {
        if (Ld[d] == 0) continue;
        ll += lgamma(alpha_bar) - lgamma(alpha_bar + (double)Ld[d]);
        for (uint32_t k = 0; k < K; ++k) {
            int64_t c = cdk[(size_t)d * K + k];
            if (c) ll += lgamma(alpha + (double)c) - lgamma(alpha);
        }
    }
    /* word part: prod_k Gamma(bbar)/Gamma(bbar+C_k) prod_w Gamma(b+C_kw)/Gamma(b) */
    for (uint32_t k = 0; k < K; ++k) {
        if (ck[k]) ll += lgamma(beta_bar) - lgamma(beta_bar + (double)ck[k]);
    }
    for (uint32_t w = 0; w < V; ++w)
        for (uint32_t k = 0; k < K; ++k) {
            int64_t c = cwk[(size_t)w * K + k];
            if (c) ll += lgamma(beta + (double)c) - lgamma(beta);
        }
    free(cdk); free(cwk); free(ck); free(Ld);
    return ll;
}

/* LL of the sampler's current Z (same formula, counts from the layout). */
double oracle_log_likelihood(const oracle_t *o)
{
    double alpha_bar = o->alpha_k ? o->alpha_cum[o->K - 1] : o->K * o->alpha;
    double beta_bar = o->V * o->beta;
    int64_t *cnt = calloc(o->K, sizeof(int64_t));
    if (!cnt) return NAN;
    double ll = 0.0;
    for (uint32_t d = 0; d < o->D; ++d) {
        uint64_t beg = o->rowptr[d], L = o->rowptr[d + 1] - beg;
        if (L == 0) continue;
        for (uint64_t n = 0; n < L; ++n) cnt[o->z[o->row[beg + n]]]++;
        ll += lgamma(alpha_bar) - lgamma(alpha_bar + (double)L);
        /* each distinct topic of the row once: add, then clear */
        for (uint64_t n = 0; n < L; ++n) {
            int32_t k = o->z[o->row[beg + n]];
            double ak = o->alpha_k ? (double)o->alpha_k[k] : o->alpha;
            if (cnt[k]) ll += lgamma(ak + (double)cnt[k]) - lgamma(ak);
            cnt[k] = 0;
        }
    }
    for (uint32_t w = 0; w < o->V; ++w) {
        uint64_t beg = o->colptr[w], L = o->colptr[w + 1] - beg;
        if (L == 0) continue;
        for (uint64_t n = 0; n < L; ++n) cnt[o->z[beg + n]]++;
        for (uint64_t n = 0; n < L; ++n) {
            int32_t k = o->z[beg + n];
            if (cnt[k]) ll += lgamma(o->beta + (double)cnt[k]) - lgamma(o->beta);
            cnt[k] = 0;
        }
    }
    memset(cnt, 0, o->K * sizeof(int64_t));
    for (uint64_t t = 0; t < o->T; ++t) cnt[o->z[t]]++;
    for (uint32_t k = 0; k < o->K; ++k)
        if (cnt[k]) ll += lgamma(beta_bar) - lgamma(beta_bar + (double)cnt[k]);
    free(cnt);
    return ll;
}

/* ------------------------------------------------------------------------ */
/* Accessors                                                                */
/* ------------------------------------------------------------------------ */
uint64_t oracle_num_tokens(const oracle_t *o) { return o->T; }
uint32_t oracle_iteration(const oracle_t *o) { return o->iter; }
uint64_t oracle_accepted(const oracle_t *o, int phase)
{
    return phase == PH_WORD ? o->accepted_word : o->accepted_doc;
}
void oracle_set_visit_reversed(oracle_t *o, int rev) { o->visit_reversed = rev; }

/* z (and the M proposals, proposal-major) in input order. */
void oracle_copy_assignments(const oracle_t *o, int32_t *z_input,
                             int32_t *props_input)
{
    for (uint64_t i = 0; i < o->T; ++i) {
        uint32_t t = o->inv[i];
        if (z_input) z_input[i] = o->z[t];
        if (props_input)
            for (uint32_t m = 0; m < o->M; ++m)
                props_input[(uint64_t)m * o->T + i] = o->prop[(uint64_t)m * o->T + t];
    }
}

/* z and proposals in CSC (column-major) order. */
void oracle_copy_csc(const oracle_t *o, int32_t *z_csc, int32_t *props_csc)
{
    if (z_csc) memcpy(z_csc, o->z, o->T * sizeof(int32_t));
    if (props_csc) memcpy(props_csc, o->prop, (size_t)o->M * o->T * sizeof(int32_t));
}

void oracle_copy_layout(const oracle_t *o, uint64_t *colptr, uint64_t *rowptr,
                        uint32_t *row, uint32_t *inv)
{
    if (colptr) memcpy(colptr, o->colptr, (o->V + 1) * sizeof(uint64_t));
    if (rowptr) memcpy(rowptr, o->rowptr, (o->D + 1) * sizeof(uint64_t));
    if (row) memcpy(row, o->row, o->T * sizeof(uint32_t));
    if (inv) memcpy(inv, o->inv, o->T * sizeof(uint32_t));
}

void oracle_copy_topic_counts(const oracle_t *o, int64_t *ck)
{
    memcpy(ck, o->ck, o->K * sizeof(int64_t));
}

/* Checkpoint: (iteration, next phase, z, proposals, ck) in CSC order. */
uint64_t oracle_state_bytes(const oracle_t *o)
{
    return 16 + (uint64_t)(1 + o->M) * o->T * 4 + (uint64_t)o->K * 8;
}

int oracle_save_state(const oracle_t *o, void *buf, uint64_t bytes)
{
    if (bytes < oracle_state_bytes(o)) return -1;
    uint8_t *p = buf;
    uint64_t hdr[2] = { o->iter, (uint64_t)o->next_phase };
    memcpy(p, hdr, 16); p += 16;
    memcpy(p, o->z, o->T * 4); p += o->T * 4;
    memcpy(p, o->prop, (size_t)o->M * o->T * 4); p += (size_t)o->M * o->T * 4;
    memcpy(p, o->ck, (size_t)o->K * 8);
    return 0;
}

int oracle_load_state(oracle_t *o, const void *buf, uint64_t bytes)
{
    if (bytes < oracle_state_bytes(o)) return -1;
    const uint8_t *p = buf;
    uint64_t hdr[2];
    memcpy(hdr, p, 16); p += 16;
    o->iter = (uint32_t)hdr[0];
    o->next_phase = (int)hdr[1];
    memcpy(o->z, p, o->T * 4); p += o->T * 4;
    memcpy(o->prop, p, (size_t)o->M * o->T * 4); p += (size_t)o->M * o->T * 4;
    memcpy(o->ck, p, (size_t)o->K * 8);
    return 0;
}

/* Overwrite z (CSC order) and recompute c_k; proposals are left unchanged.
 * Used by the tests to start the sampler from a chosen state. */
void oracle_set_csc_state(oracle_t *o, const int32_t *z_csc,
                          const int32_t *props_csc)
{
    memcpy(o->z, z_csc, o->T * sizeof(int32_t));
    if (props_csc) memcpy(o->prop, props_csc, (size_t)o->M * o->T * sizeof(int32_t));
    recount_ck(o);
}

/* ------------------------------------------------------------------------ */
/* Point estimates of Eq. (4) from the current Z, binary64:                 */
/*   theta_dk = (C_dk + alpha_k) / (L_d + alpha_bar)                        */
/*   phi_wk   = (C_wk + beta)  / (C_k + V beta)                             */
/* (the M-step of Section 4.2 with alpha' = alpha + 1, beta' = beta + 1).    */
/* theta: nd x K for documents d0 .. d0+nd-1; phi: nw x K for words         */
/* w0 .. w0+nw-1, row-major.                                                */
/* ------------------------------------------------------------------------ */
int oracle_theta(const oracle_t *o, uint32_t d0, uint32_t nd, double *out)
{
    if ((uint64_t)d0 + nd > o->D) return -1;
    for (uint32_t e = 0; e < nd; ++e) {
        uint32_t d = d0 + e;
        uint64_t beg = o->rowptr[d], L = o->rowptr[d + 1] - beg;
        double *row = out + (size_t)e * o->K;
        for (uint32_t k = 0; k < o->K; ++k) row[k] = 0.0;
        for (uint64_t n = 0; n < L; ++n) row[o->z[o->row[beg + n]]] += 1.0;
        double den = (double)L + (o->alpha_k ? o->alpha_cum[o->K - 1] : (double)o->K * o->alpha);
        for (uint32_t k = 0; k < o->K; ++k)
            row[k] = (row[k] + (o->alpha_k ? (double)o->alpha_k[k] : o->alpha)) / den;
    }
    return 0;
}

int oracle_phi(const oracle_t *o, uint32_t w0, uint32_t nw, double *out)
{
    if ((uint64_t)w0 + nw > o->V) return -1;
    double beta_bar = (double)o->V * o->beta;
    for (uint32_t e = 0; e < nw; ++e) {
        uint32_t w = w0 + e;
        uint64_t beg = o->colptr[w], L = o->colptr[w + 1] - beg;
        double *row = out + (size_t)e * o->K;
        for (uint32_t k = 0; k < o->K; ++k) row[k] = 0.0;
        for (uint64_t n = 0; n < L; ++n) row[o->z[beg + n]] += 1.0;
        for (uint32_t k = 0; k < o->K; ++k)
            row[k] = (row[k] + o->beta) / ((double)o->ck[k] + beta_bar);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Instant-update variant (quality study of Section 6.3, not the sampler).  */
/* The counts C_d, C_w and C_k change as soon as a token moves, as in       */
/* LightLDA's collapsed Gibbs-MH, instead of once per phase.  Tokens are    */
/* visited document by document in canonical row order.  For each token:   */
/* its own assignment is taken out of the counts ("not dn", Eq. (1)); M     */
/* steps with the document proposal q_doc ~ C_dk + alpha (random            */
/* positioning over the document's other tokens, coin                       */
/* (L_d - 1) / (L_d - 1 + K alpha)) judged with the word-side ratio of      */
/* Eq. (7); M steps with the word proposal q_word ~ C_wk + beta (the        */
/* column's other tokens, coin (L_w - 1) / (L_w - 1 + K beta)) judged with  */
/* the document-side ratio; the assignment is put back.  Each step leaves   */
/* p(z_dn = k | rest) ~ (C_dk+alpha)(C_wk+beta)/(C_k+V beta) invariant, so  */
/* the scan targets the collapsed posterior p(Z | W) of Eq. (1), which the  */
/* delayed-update sampler does not do exactly.  Binary32 decisions as in    */
/* mh_accept(); random words: counter (t, iteration, PH_INSTANT << 16 |     */
/* step, 0) with t the canonical CSR position and step 1..2M (doc steps     */
/* first); words 0, 1, 2 = acceptance uniform, coin, index/topic.           */
/* c_k, the acceptance count (reported as the doc phase's) and the          */
/* iteration count are kept; pending proposals are left untouched.         */
/* ------------------------------------------------------------------------ */
enum { PH_INSTANT = 10 };

/* The other tokens of a row (or column) in order, skipping position `self`:
 * index u in [0, L-1) -> position u or u+1. */
static uint64_t skip_self(uint64_t u, uint64_t self) { return u < self ? u : u + 1; }

int oracle_instant_iterate(oracle_t *o, uint32_t n_iter)
{
    if (o->next_phase != PH_WORD) return -4;
    int64_t *cd = calloc(o->K, sizeof(int64_t));
    int64_t *cwk = calloc((size_t)o->V * o->K, sizeof(int64_t));
    uint64_t *pos_in_col = malloc(o->T * sizeof(uint64_t) + 1);
    if (!cd || !cwk || !pos_in_col) { free(cd); free(cwk); free(pos_in_col); return -1; }
    for (uint32_t w = 0; w < o->V; ++w)
        for (uint64_t t = o->colptr[w]; t < o->colptr[w + 1]; ++t) {
            cwk[(size_t)w * o->K + o->z[t]]++;
            pos_in_col[t] = t - o->colptr[w];
        }
    recount_ck(o);
    for (uint32_t it = 0; it < n_iter; ++it) {
        uint32_t iter = o->iter + 1;
        uint64_t accepted = 0;
        for (uint32_t d = 0; d < o->D; ++d) {
            uint64_t beg = o->rowptr[d], Ld = o->rowptr[d + 1] - beg;
            if (Ld == 0) continue;
            for (uint64_t n = 0; n < Ld; ++n) cd[o->z[o->row[beg + n]]]++;
            for (uint64_t n = 0; n < Ld; ++n) {
                uint32_t t = o->row[beg + n];
                uint32_t w = o->word_of[t];
                int64_t *cw = cwk + (size_t)w * o->K;
                uint64_t cbeg = o->colptr[w], Lw = o->colptr[w + 1] - cbeg;
                int32_t s = o->z[t];
                cd[s]--; cw[s]--; o->ck[s]--;           /* not dn */
                for (uint32_t step = 1; step <= 2 * o->M; ++step) {
                    uint32_t r[4];
                    rng_call(o->seed, (uint32_t)(beg + n), iter, PH_INSTANT, step, 0, r);
                    int32_t c;
                    if (step <= o->M) {   /* doc proposal, word-side ratio */
                        c = Ld > 1 && take_count_part(unif24(r[1]), Ld - 1, o->alpha_bar)
                                ? o->z[o->row[beg + skip_self(dice(r[2], (uint32_t)(Ld - 1)), n)]]
                                : prior_topic(o, r[2]);
                        if (mh_accept(unif24(r[0]), cw[c], cw[s], o->b, o->ck[s], o->ck[c],
                                      o->beta_bar)) {
                            s = c;
                            accepted++;
                        }
                    } else {              /* word proposal, doc-side ratio */
                        c = Lw > 1 && take_count_part(unif24(r[1]), Lw - 1, o->beta_k)
                                ? o->z[cbeg + skip_self(dice(r[2], (uint32_t)(Lw - 1)),
                                                        pos_in_col[t])]
                                : (int32_t)dice(r[2], o->K);
                        if (mh_accept2(unif24(r[0]), cd[c], cd[s], alpha_of(o, c), alpha_of(o, s),
                                       o->ck[s], o->ck[c], o->beta_bar)) {
                            s = c;
                            accepted++;
                        }
                    }
                }
                o->z[t] = s;
                cd[s]++; cw[s]++; o->ck[s]++;
            }
            for (uint64_t n = 0; n < Ld; ++n) cd[o->z[o->row[beg + n]]] = 0;
        }
        o->iter = iter;
        o->accepted_word = 0;
        o->accepted_doc = accepted;
    }
    free(cd); free(cwk); free(pos_in_col);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Frozen-count chain of one token (test harness for Eq. (5)-(7)).          */
/* With Z held fixed, the state x of token t is moved by M steps of the doc */
/* proposal (drawn by random positioning over row d) and/or M steps of the  */
/* word proposal (random positioning over column w), each accepted with the */
/* rate of Eq. (7).  Both kernels leave q(k) of Eq. (5) invariant; hist     */
/* receives the state after every round.  mode: 1 doc, 2 word, 3 both.      */
/* ------------------------------------------------------------------------ */
int oracle_frozen_chain(const oracle_t *o, uint32_t t, uint32_t rounds,
                        int mode, uint64_t *hist)
{
    if (t >= o->T) return -1;
    uint32_t w = o->word_of[t], d = o->doc_of[t];
    uint64_t cbeg = o->colptr[w], Lw = o->colptr[w + 1] - cbeg;
    uint64_t rbeg = o->rowptr[d], Ld = o->rowptr[d + 1] - rbeg;
    int64_t *cw = calloc(o->K, sizeof(int64_t));
    int64_t *cd = calloc(o->K, sizeof(int64_t));
    if (!cw || !cd) { free(cw); free(cd); return -1; }
    for (uint64_t n = 0; n < Lw; ++n) cw[o->z[cbeg + n]]++;
    for (uint64_t n = 0; n < Ld; ++n) cd[o->z[o->row[rbeg + n]]]++;
    memset(hist, 0, o->K * sizeof(uint64_t));
    int32_t x = o->z[t];
    for (uint32_t rd = 0; rd < rounds; ++rd) {
        for (uint32_t i = 1; i <= o->M; ++i) {
            uint32_t r[4];
            if (mode & 1) {   /* doc proposal, judged with c_w (Eq. 7 top) */
                rng_call(o->seed, rd, i, PH_FROZEN, 1, t, r);
                int32_t c = take_count_part(unif24(r[1]), Ld, o->alpha_bar)
                                ? o->z[o->row[rbeg + dice(r[2], (uint32_t)Ld)]]
                                : prior_topic(o, r[2]);
                if (mh_accept(unif24(r[0]), cw[c], cw[x], o->b, o->ck[x],
                              o->ck[c], o->beta_bar))
                    x = c;
            }
            if (mode & 2) {   /* word proposal, judged with c_d (Eq. 7 bottom) */
                rng_call(o->seed, rd, i, PH_FROZEN, 2, t, r);
                int32_t c = take_count_part(unif24(r[1]), Lw, o->beta_k)
                                ? o->z[cbeg + dice(r[2], (uint32_t)Lw)]
                                : (int32_t)dice(r[2], o->K);
                if (mh_accept2(unif24(r[0]), cd[c], cd[x], alpha_of(o, c), alpha_of(o, x),
                               o->ck[x], o->ck[c], o->beta_bar))
                    x = c;
            }
        }
        hist[x]++;
    }
    free(cw); free(cd);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Fold-in of new documents (MCEM E-step of Eq. (5) with the word-topic     */
/* counts C_w and the topic totals c_k held at a trained model's values).   */
/* Each new document runs its own delayed-update chain, sweep by sweep:     */
/*   word step - its pending doc proposals are judged with pi_doc of Eq. (7)*/
/*               using the frozen C_w and c_k; M word proposals are drawn   */
/*               by random positioning over the trained column of the word  */
/*               (mixing weight L_w / (L_w + K beta));                      */
/*   doc step  - c_d is rebuilt from the document, the word proposals are   */
/*               judged with pi_word, then (learned mode) LS further steps  */
/*               with an independence proposal q given as integer weights,  */
/*               and M doc proposals are drawn from the updated document.   */
/* Randomness: counter (token-in-doc, sweep, phase << 16 | step, request).  */
/* Learned weights: q(k) = w_k / sum(w); a draw takes u = Dice(sum(w)) and  */
/* the first k whose running sum exceeds u.  The learned MH ratio is        */
/* (C_dt+a)(C_wt+b)(C_s+bbar) w_s / ((C_ds+a)(C_ws+b)(C_t+bbar) w_t),       */
/* multiplied left to right in binary32.                                    */
/* ------------------------------------------------------------------------ */
enum { PH_F_INIT = 5, PH_F_WORD = 6, PH_F_DOC = 8, PH_F_LEARN = 9 };

typedef struct {
    uint32_t V, K, M;
    double alpha, beta;
    uint64_t seed;
    const uint64_t *colptr;   /* V+1: trained columns */
    const int32_t *z_csc;     /* trained assignments, canonical column order */
    const int64_t *ck;        /* K: topic totals of the trained Z */
} oracle_model;

static uint32_t learned_draw(const uint32_t *w, uint32_t K, uint64_t total, uint32_t r)
{
    uint64_t u = ((uint64_t)r * total) >> 32, run = 0;
    for (uint32_t k = 0; k < K; ++k) {
        run += w[k];
        if (run > u) return k;
    }
    return K - 1;
}

/* One document.  z (L) in/out state, pd (M x L) pending doc proposals.
 * first_sweep == 0 initialises (z from Dice(K) or from q, then the first doc
 * proposals) and continues with sweeps 1..last_sweep. */
static int fold_doc(const oracle_model *m, uint32_t req, const uint32_t *words, uint32_t L,
                    uint32_t first_sweep, uint32_t last_sweep, const uint32_t *qw,
                    uint32_t learned_steps, int32_t *z, int32_t *pd)
{
    const uint32_t K = m->K, M = m->M;
    const float a = (float)m->alpha, b = (float)m->beta;
    const float alpha_bar = (float)K * a, beta_k = (float)K * b, beta_bar = (float)m->V * b;
    uint64_t qtot = 0;
    if (qw) for (uint32_t k = 0; k < K; ++k) qtot += qw[k];
    int64_t *cw_c = NULL;
    int64_t *cd = calloc(K, sizeof(int64_t));
    int32_t *pw = malloc((size_t)M * L * sizeof(int32_t) + 1);
    if (!cd || !pw) { free(cd); free(pw); return -1; }
    uint32_t r[4];
    if (first_sweep == 0) {
        for (uint32_t n = 0; n < L; ++n) {
            rng_call(m->seed, n, 0, PH_F_INIT, 0, req, r);
            z[n] = qw ? (int32_t)learned_draw(qw, K, qtot, r[2]) : (int32_t)dice(r[2], K);
        }
        for (uint32_t n = 0; n < L; ++n)
            for (uint32_t i = 1; i <= M; ++i) {
                rng_call(m->seed, n, 0, PH_F_DOC, i, req, r);
                pd[(size_t)(i - 1) * L + n] = take_count_part(unif24(r[1]), L, alpha_bar)
                                                  ? z[dice(r[2], L)] : (int32_t)dice(r[2], K);
            }
        first_sweep = 1;
    }
    (void)cw_c;
    for (uint32_t s = first_sweep; s <= last_sweep; ++s) {
        /* word step: frozen C_w, c_k */
        for (uint32_t n = 0; n < L; ++n) {
            uint32_t w = words[n];
            uint64_t cb = m->colptr[w], Lw = m->colptr[w + 1] - cb;
            int32_t x = z[n];
            for (uint32_t i = 1; i <= M; ++i) {
                rng_call(m->seed, n, s, PH_F_WORD, i, req, r);
                int32_t c = pd[(size_t)(i - 1) * L + n];
                int64_t cwc = 0, cwx = 0;
                for (uint64_t j = 0; j < Lw; ++j) {
                    cwc += m->z_csc[cb + j] == c;
                    cwx += m->z_csc[cb + j] == x;
                }
                if (mh_accept(unif24(r[0]), cwc, cwx, b, m->ck[x], m->ck[c], beta_bar)) x = c;
                pw[(size_t)(i - 1) * L + n] =
                    Lw && take_count_part(unif24(r[1]), Lw, beta_k)
                        ? m->z_csc[cb + dice(r[2], (uint32_t)Lw)] : (int32_t)dice(r[2], K);
            }
            z[n] = x;
        }
        /* doc step: c_d rebuilt, word proposals, learned steps, doc proposals */
        memset(cd, 0, K * sizeof(int64_t));
        for (uint32_t n = 0; n < L; ++n) cd[z[n]]++;
        int32_t *znew = malloc((size_t)L * sizeof(int32_t) + 1);
        if (!znew) { free(cd); free(pw); return -1; }
        for (uint32_t n = 0; n < L; ++n) {
            int32_t x = z[n];
            for (uint32_t i = 1; i <= M; ++i) {
                rng_call(m->seed, n, s, PH_F_DOC, i, req, r);
                int32_t c = pw[(size_t)(i - 1) * L + n];
                if (mh_accept(unif24(r[0]), cd[c], cd[x], a, m->ck[x], m->ck[c], beta_bar)) x = c;
            }
            if (qw) {
                uint32_t w = words[n];
                uint64_t cb = m->colptr[w], Lw = m->colptr[w + 1] - cb;
                for (uint32_t j = 1; j <= learned_steps; ++j) {
                    rng_call(m->seed, n, s, PH_F_LEARN, j, req, r);
                    int32_t t = (int32_t)learned_draw(qw, K, qtot, r[2]);
                    int64_t cwt = 0, cwx = 0;
                    for (uint64_t q = 0; q < Lw; ++q) {
                        cwt += m->z_csc[cb + q] == t;
                        cwx += m->z_csc[cb + q] == x;
                    }
                    float num = ((float)cd[t] + a) * ((float)cwt + b) * ((float)m->ck[x] + beta_bar) *
                                (float)qw[x];
                    float den = ((float)cd[x] + a) * ((float)cwx + b) * ((float)m->ck[t] + beta_bar) *
                                (float)qw[t];
                    if (unif24(r[0]) * den < num) x = t;
                }
            }
            znew[n] = x;
        }
        memcpy(z, znew, (size_t)L * sizeof(int32_t));
        free(znew);
        for (uint32_t n = 0; n < L; ++n)
            for (uint32_t i = 1; i <= M; ++i) {
                rng_call(m->seed, n, s, PH_F_DOC, i, req, r);
                pd[(size_t)(i - 1) * L + n] = take_count_part(unif24(r[1]), L, alpha_bar)
                                                  ? z[dice(r[2], L)] : (int32_t)dice(r[2], K);
            }
    }
    free(cd);
    free(pw);
    return 0;
}

/* Fold-in of a batch.  docptr (n_docs+1) indexes words, z and pd (pd is
 * M x total, proposal-major with stride `total`, sliced per document as
 * M x L_d contiguous runs at M*docptr[d]).  qw: n_docs x K weights or NULL. */
int oracle_foldin(uint32_t V, uint32_t K, uint32_t M, double alpha, double beta, uint64_t seed,
                  const uint64_t *colptr, const int32_t *z_csc, const int64_t *ck,
                  uint32_t n_docs, const uint64_t *docptr, const uint32_t *words,
                  const uint32_t *req_ids, uint32_t first_sweep, uint32_t last_sweep,
                  const uint32_t *qw, uint32_t learned_steps, int32_t *z, int32_t *pd)
{
    oracle_model m = { V, K, M, alpha, beta, seed, colptr, z_csc, ck };
    for (uint32_t d = 0; d < n_docs; ++d) {
        uint64_t beg = docptr[d];
        uint32_t L = (uint32_t)(docptr[d + 1] - beg);
        if (L == 0) continue;
        int rc = fold_doc(&m, req_ids[d], words + beg, L, first_sweep, last_sweep,
                          qw ? qw + (size_t)d * K : NULL, learned_steps, z + beg,
                          pd + (size_t)M * beg);
        if (rc) return rc;
    }
    return 0;
}

/* Held-out log likelihood by document completion: for each document, theta
 * from its folded-in assignments (Eq. (4) with alpha' = alpha + 1), phi from
 * the trained counts (beta' = beta + 1), and sum over its held-out tokens of
 * log sum_k theta_dk phi_wk.  Returns the total (binary64). */
double oracle_heldout_ll(uint32_t V, uint32_t K, double alpha, double beta,
                         const uint64_t *colptr, const int32_t *z_csc, const int64_t *ck,
                         uint32_t n_docs, const uint64_t *docptr, const int32_t *z,
                         const uint64_t *hoptr, const uint32_t *ho_words)
{
    double *theta = malloc(K * sizeof(double));
    int64_t *cw = malloc(K * sizeof(int64_t));
    if (!theta || !cw) { free(theta); free(cw); return NAN; }
    double total = 0;
    for (uint32_t d = 0; d < n_docs; ++d) {
        uint64_t beg = docptr[d], L = docptr[d + 1] - beg;
        for (uint32_t k = 0; k < K; ++k) theta[k] = alpha;
        for (uint64_t n = 0; n < L; ++n) theta[z[beg + n]] += 1.0;
        for (uint32_t k = 0; k < K; ++k) theta[k] /= (double)L + K * alpha;
        for (uint64_t h = hoptr[d]; h < hoptr[d + 1]; ++h) {
            uint32_t w = ho_words[h];
            memset(cw, 0, K * sizeof(int64_t));
            for (uint64_t j = colptr[w]; j < colptr[w + 1]; ++j) cw[z_csc[j]]++;
            double p = 0;
            for (uint32_t k = 0; k < K; ++k)
                p += theta[k] * ((double)cw[k] + beta) / ((double)ck[k] + V * beta);
            total += log(p);
        }
    }
    free(theta); free(cw);
    return total;
}
