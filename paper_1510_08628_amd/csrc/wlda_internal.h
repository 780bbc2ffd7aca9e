// Internal interface between the host runtime (wlda_host.cpp) and the gfx950
// kernels (wlda_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wlda {

enum Phase : uint32_t { PH_INIT = 0, PH_WORD = 1, PH_DOC = 2 };

// One packed record per token: field 0 is z, field i (1..M) the i-th pending
// proposal.  When K fits, the 1 + M fields share one 32-bit word, floor(32 /
// (1 + M)) bits each (K <= 65536 for M = 1, 1024 for M = 2, 256 for M = 3,
// 64 for M = 4); else, for K <= 65536, 16-bit fields two to a 32-bit word
// (8 bytes for M = 2 or 3, 12 bytes for M = 4); otherwise topics take 21
// bits, three to a 64-bit word (one word for M <= 2, two for M <= 5).
// Kernels name the format by RF: -b for a 32-bit record of b-bit fields,
// 100 + n for n 32-bit words of 16-bit fields, 1 or 2 for 64-bit words.
constexpr uint32_t FIELD_BITS = 21;
constexpr uint32_t FIELD_MASK = (1u << FIELD_BITS) - 1;
constexpr uint32_t MAX_K = FIELD_MASK;   // topics are < 2^21 - 1

inline uint32_t rec32_bits(uint32_t M) { return 32 / (1 + M); }
inline bool rec32_fits(uint32_t M, uint32_t K) { return M <= 4 && K <= (1u << rec32_bits(M)); }
inline int record_format(uint32_t M, uint32_t K) {
    if (rec32_fits(M, K)) return -(int)rec32_bits(M);
    if (K <= 65536 && M >= 2 && M <= 5) return 100 + (int)((M + 2) / 2);
    return (int)((M + 1 + 2) / 3);
}
inline uint32_t record_bytes(uint32_t M, uint32_t K) {
    const int rf = record_format(M, K);
    return rf < 0 ? 4u : rf >= 100 ? 4u * (uint32_t)(rf - 100) : 8u * (uint32_t)rf;
}

// Segment = one column (word phase) or one row (doc phase).  The n-th token
// of segment s has the canonical position segptr[s] + n of its phase (CSC in
// the word phase, CSR in the doc phase; the RNG counter uses it) and its
// record at recs[idx[segptr[s] + n]] (idx = colidx or rowidx: the record
// layout is blocked by documents, see the host runtime).  A list also holds
// each segment's span, so a kernel reaches its tokens' record positions in
// one dependent load fewer.
struct SegList {
    const uint32_t *ids = nullptr;   // segment ids, ascending
    uint32_t n = 0;
    const uint32_t *xcd_cut = nullptr;   // 9 list offsets: XCD x owns [cut[x], cut[x+1])
    const uint2 *span = nullptr;     // per listed segment: segptr[id], segptr[id + 1]
};

// Segments longer than one workgroup's share ("long") are cut into chunks of
// LONG_CHUNK tokens; every long segment is owned by one XCD (greedy balance by
// tokens) and its chunks are listed contiguously in that XCD's share.
struct LongList {
    const uint32_t *ids = nullptr;     // long segment ids, ascending
    const uint32_t *prefix = nullptr;  // n+1 offsets of each segment in the compact z array
    uint32_t n = 0;
    uint32_t total = 0;                // prefix[n]
    const uint32_t *chunk_seg = nullptr;    // per chunk: index j into ids
    const uint32_t *chunk_start = nullptr;  // per chunk: first token within the segment
    uint32_t n_chunks = 0;
    uint32_t chunk = 0;                // tokens per chunk (long_chunk(K))
    const uint32_t *chunk_cut = nullptr;    // 9 chunk-list offsets, one share per XCD
    // Per-segment counts in global memory: segment j owns the words
    // tables[tab_off[j] ..); tab_cap[j] == 0 means dense (K counts), otherwise
    // an open-addressed table of tab_cap[j] (power of two) slots laid out as
    // tab_cap keys (topic + 1, 0 = empty) followed by tab_cap counts.  All-zero
    // words are an empty table.
    uint32_t *tables = nullptr;
    const uint64_t *tab_off = nullptr;
    const uint32_t *tab_cap = nullptr;
    uint64_t table_words = 0;
    void *zc = nullptr;                // total compact topics (u16 if K <= 65535, else u32)
    // Dense counts of the updated z of every word past the inverse-CDF
    // threshold (word_cdf; same offsets as `tables`, which are dense for
    // those words since 2L > K), turned into inclusive
    // prefix counts for the inverse-CDF word proposals; zeroed before use.
    // With the alias-table proposals they become the table's thresholds
    // (ALIAS_DONE | threshold) and `tables` its alias topics.
    uint32_t *tables_new = nullptr;
};

struct Tuning {
    // wave kernel (and the 16- and 32-lane groups): TPT_WAVE tokens per lane,
    // half as many for M > 2, whose counts and records take twice the registers
    static constexpr int TPT_WAVE = 8;
    // block kernels (one 256-thread workgroup per segment): the narrow one
    // keeps TPT_BLOCK tokens per thread in registers (high occupancy), the
    // wide one twice as many; M > 2 halves both (two-word records)
    static constexpr int TPT_BLOCK = 8;
    static constexpr int TPT_WIDE = 16;
    static constexpr uint32_t WIDE_MAX = 256 * TPT_WIDE;     // longest segment below the long path
    // segment kernels: LDS bytes per workgroup within which the c_k
    // histogram and c_k + beta_bar are staged: the CU's LDS over the
    // workgroups per CU a bin runs at, at most SEG_LDS_BUDGET
    static constexpr uint32_t LDS_PER_CU = 160 * 1024;
    static constexpr uint32_t SEG_LDS_BUDGET = 80 * 1024;
    // beyond the budget: c_k histogram / c_k + beta_bar in LDS up to these K
    static constexpr uint32_t CK_LDS_MAX = 4096;
    static constexpr uint32_t CKB_LDS_MAX = 16384;
    // long kernels: c_k + beta_bar (MH pass) and the c_k histogram (draw pass)
    // in LDS; they run few workgroups per CU anyway, where the segment kernels
    // would lose half their occupancy to a K-word histogram
    static constexpr uint32_t LONG_CK_LDS_MAX = 16384;
    // tokens per long-path chunk: LONG_CHUNK when the chunk histogram is a
    // dense LDS array (K <= LDS_DENSE_MAX), else LONG_CHUNK_HASHED so that the
    // LDS hash table (2 * LONG_CHUNK_HASHED slots) always has free slots
    static constexpr uint32_t LONG_CHUNK = 8192;
    static constexpr uint32_t LONG_CHUNK_HASHED = 4096;
    static constexpr uint32_t LDS_DENSE_MAX = 16384;         // dense LDS counts up to this K
    static constexpr uint32_t CDF_LDS_MAX = 16384;           // long-word prefix counts in LDS
    // the inverse CDF of a long word starts from a guide table built in LDS
    // for every chunk up to this K (a binary search of the LDS prefix counts
    // up to CDF_LDS_MAX, a guide built once per word in global memory above)
    static constexpr uint32_t GUIDE_K_MAX = 4096;
};

struct PhaseArgs {
    uint64_t *recs = nullptr;
    const uint32_t *segptr = nullptr;
    const uint32_t *idx = nullptr;     // record position of each canonical position
    uint32_t K = 0, iter = 0, seed_lo = 0, seed_hi = 0;
    const uint32_t *ck = nullptr;      // c_k at the start of the phase
    uint32_t *ck_next = nullptr;       // histogram of the phase's new Z
    float prior = 0.f;                 // beta (word phase) or alpha (doc phase)
    float mass = 0.f;                  // K beta or alpha_bar
    // doc phase with an asymmetric alpha (else null): alpha_k as binary32 and
    // its running sums in binary64 (K entries each)
    const float *alpha_k = nullptr;
    const double *alpha_cum = nullptr;
    float beta_bar = 0.f;              // V beta
    unsigned long long *accepted = nullptr;
    uint32_t draw_only = 0;            // initial proposal draw (no MH)
    uint32_t word_alias = 0;           // word phase: alias-table proposals for L > K
    uint32_t max_blocks = 2048;        // grid bound of the segment kernels (launch shape only)
    uint32_t seg_lds_budget = Tuning::SEG_LDS_BUDGET;   // LDS bytes per segment workgroup (launch shape only)
    int rf = 1;                        // record format (see record_format)
};


// Word proposals (count part): columns longer than K tokens (the words
// Section 5.4 processes with intra-word parallelism and samples from a table
// over c_w) take the inverse CDF of their updated counts, or with
// WLDA_WORD_ALIAS Walker's alias table over them, all others a token of the
// updated column (random positioning); all three sample the same law.
__host__ __device__ inline bool word_cdf(uint32_t L, uint32_t K) { return L > K; }

inline uint32_t long_chunk(uint32_t K) {
    return K <= Tuning::LDS_DENSE_MAX ? Tuning::LONG_CHUNK : Tuning::LONG_CHUNK_HASHED;
}

// Segment bins below the long path, by length: sub-wavefront groups of 16
// and 32 lanes (several short segments per wavefront), the wave kernel, and
// the narrow and the wide block kernel.
enum Bin : int { BIN_G16 = 0, BIN_G32 = 1, BIN_WAVE = 2, BIN_BLOCK = 3, BIN_WIDE = 4, NBINS = 5 };

// Lanes that own one segment in a bin.
inline uint32_t bin_group(int bin) {
    return bin == BIN_G16 ? 16u : bin == BIN_G32 ? 32u : bin == BIN_WAVE ? 64u : 256u;
}

inline uint32_t bin_tpt(int bin, uint32_t M) {
    if (bin <= BIN_WAVE) return M <= 2 ? (uint32_t)Tuning::TPT_WAVE : (uint32_t)Tuning::TPT_WAVE / 2;
    const int t = bin == BIN_BLOCK ? Tuning::TPT_BLOCK : Tuning::TPT_WIDE;
    return M <= 2 ? (uint32_t)t : (uint32_t)t / 2;
}

inline uint32_t bin_max_tokens(int bin, uint32_t M) { return bin_group(bin) * bin_tpt(bin, M); }

// ---- launchers (all enqueue on `st`, return hipError_t of the launch) ----
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, uint64_t n, hipStream_t st);
hipError_t launch_init_z(uint64_t *recs, const uint32_t *colidx, uint32_t T, uint32_t M, uint32_t K,
                         uint32_t seed_lo, uint32_t seed_hi, hipStream_t st);
// bin = BIN_WAVE, BIN_BLOCK or BIN_WIDE
hipError_t launch_segments(const PhaseArgs &a, uint32_t phase, uint32_t M, const SegList &l,
                           int bin, hipStream_t st);
// Records ev[0..3] (if non-null) before the histogram, MH and draw kernels and
// after the draw kernel, so that the host can time each of them.
hipError_t launch_long_segments(const PhaseArgs &a, uint32_t phase, uint32_t M,
                                const LongList &l, hipStream_t st, hipEvent_t *ev = nullptr);
hipError_t launch_histogram_z(const uint64_t *recs, uint32_t T, uint32_t M, uint32_t K,
                              uint32_t *ck, hipStream_t st);
// LL: adds the document, word and topic parts into *out (binary64).
// Per segment: sum over nonzero counts c of lgamma(prior + c) - lgamma(prior)
// (prior = alpha_k[topic] when alpha_k is given: asymmetric alpha), plus
// lgamma(prior_total) - lgamma(prior_total + L) when length_term != 0.
// LL parts over the segments of a list (at most block_max tokens each) and
// over the long segments (through their global tables, which are left zeroed).
hipError_t launch_ll_list(const uint64_t *recs, uint32_t M, const uint32_t *segptr,
                          const uint32_t *idx, const uint32_t *ids, uint32_t n, uint32_t K,
                          double prior, double prior_total, int length_term, double *out,
                          hipStream_t st, const float *alpha_k = nullptr);
// (takes alpha_k from a)
hipError_t launch_ll_long(const PhaseArgs &a, uint32_t phase, uint32_t M, const LongList &l,
                          double prior, double prior_total, int length_term, double *out,
                          hipStream_t st);
hipError_t launch_theta(const uint64_t *recs, uint32_t M, const uint32_t *rowptr, const uint32_t *rowidx,
                        uint32_t d0, uint32_t nd, uint32_t K, float alpha, const float *alpha_k,
                        float alpha_bar, float *out, hipStream_t st);
hipError_t launch_phi(const uint64_t *recs, uint32_t M, const uint32_t *colptr, const uint32_t *colidx,
                      const uint32_t *ck, uint32_t w0, uint32_t nw, uint32_t K, float beta, float beta_bar,
                      float *out, hipStream_t st);
hipError_t launch_ll_topics(const uint32_t *ck, uint32_t K, double beta_bar, double *out,
                            hipStream_t st);

// The phase kernels of one M, each M compiled in a translation unit of its own
// (wlda_kernels_m.hip); the launchers above dispatch to them.
template <int M>
hipError_t seg_launch(const PhaseArgs &a, uint32_t phase, const SegList &l, int bin, hipStream_t st);
template <int M>
hipError_t long_launch(const PhaseArgs &a, uint32_t phase, const LongList &l, hipStream_t st, hipEvent_t *ev);
template <int M>
hipError_t long_hist_launch(const PhaseArgs &a, uint32_t phase, const LongList &l, hipStream_t st);
#define WLDA_DECLARE_M(M)                                                                                 \
    template <>                                                                                           \
    hipError_t seg_launch<M>(const PhaseArgs &, uint32_t, const SegList &, int, hipStream_t);             \
    template <>                                                                                           \
    hipError_t long_launch<M>(const PhaseArgs &, uint32_t, const LongList &, hipStream_t, hipEvent_t *);  \
    template <>                                                                                           \
    hipError_t long_hist_launch<M>(const PhaseArgs &, uint32_t, const LongList &, hipStream_t);
WLDA_DECLARE_M(1)
WLDA_DECLARE_M(2)
WLDA_DECLARE_M(3)
WLDA_DECLARE_M(4)
#undef WLDA_DECLARE_M

}  // namespace wlda
