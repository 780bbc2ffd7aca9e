// Host runtime of the WarpLDA sampler: input validation, the canonical token
// orders and the blocked record layout (Section 5.2), segment binning by
// length, workspace carving and the phase schedule (Section 4.4, Algorithm 2).
// Implements include/warplda.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/warplda.h"
#include "wlda_internal.h"

using namespace wlda;

namespace {

constexpr uint64_t ALIGN = 256;
// records per document block: 1 MiB stays resident in an XCD's 4 MiB L2 while
// that XCD's document window (about 1k rows in flight) gathers from it
constexpr uint64_t DOC_BLOCK_KIB = 1024;
inline uint64_t align_up(uint64_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Segment ids of one bin, in ascending order, cut into eight XCD shares.
struct BinList {
    std::vector<uint32_t> ids;
    uint32_t cut[9] = {};
    uint32_t *d_ids = nullptr, *d_cut = nullptr;   // device copies
    uint2 *d_span = nullptr;                       // [segptr[id], segptr[id + 1]) per listed id
};

struct PhasePlan {
    BinList bins[NBINS];
    std::vector<uint32_t> long_ids, long_prefix;
    std::vector<uint32_t> chunk_seg, chunk_start, tab_cap;
    std::vector<uint64_t> tab_off;          // n+1 word offsets of the per-segment tables
    uint32_t chunk_cut[9] = {};
    uint32_t chunk = 0;                     // tokens per long-path chunk
    // device copies (inside the workspace)
    uint32_t *d_long_ids = nullptr, *d_long_prefix = nullptr,
             *d_tables = nullptr, *d_chunk_seg = nullptr, *d_chunk_start = nullptr,
             *d_chunk_cut = nullptr, *d_tab_cap = nullptr;
    uint64_t *d_tab_off = nullptr;
    void *d_zc = nullptr;
};

// Split a length-sorted-by-id list into 8 contiguous shares of ~equal tokens
// (one per XCD).
void xcd_cuts(const std::vector<uint32_t> &ids, const std::vector<uint64_t> &len, uint32_t cut[9]) {
    uint64_t total = 0;
    for (uint32_t s : ids) total += len[s];
    uint64_t run = 0;
    uint32_t x = 1;
    cut[0] = 0;
    for (uint32_t i = 0; i < ids.size() && x < 8; ++i) {
        run += len[ids[i]];
        while (x < 8 && run * 8 >= total * x) cut[x++] = i + 1;
    }
    while (x < 8) cut[x++] = (uint32_t)ids.size();
    cut[8] = (uint32_t)ids.size();
}

uint32_t pow2_ge(uint64_t x) {
    uint64_t c = 1;
    while (c < x) c <<= 1;
    return (uint32_t)c;
}

// The smallest bin used.  The 16- and 32-lane groups keep their counts in
// open-addressed tables of at most 2 * 128 or 2 * 256 slots, so they pay only
// where the wave kernel hashes too (K > its 1024-slot bound); with smaller K
// short segments go to the wave kernel's dense tables.  WLDA_FIRST_BIN
// overrides (a launch-shape switch: the chain does not depend on it).
int first_bin(uint32_t K) {
    if (const char *env = std::getenv("WLDA_FIRST_BIN")) {
        const int b = std::atoi(env);
        return b < 0 ? 0 : (b >= NBINS ? NBINS - 1 : b);
    }
    return K > 2 * bin_max_tokens(BIN_WAVE, 1) ? (int)BIN_G16 : (int)BIN_WAVE;
}

// Each segment goes to the first bin that holds its length (16- and 32-lane
// groups, wave, block, wide), else to the long path.  With long_above_k every
// segment longer than K goes to the long path (the word plan of the
// alias-table word proposal, whose tables only the long path builds).
void build_plan(const std::vector<uint64_t> &len, uint32_t M, uint32_t K, PhasePlan &pl,
                bool long_above_k = false) {
    for (BinList &b : pl.bins) b.ids.clear();
    pl.long_ids.clear();
    pl.long_prefix.assign(1, 0);
    const int bin0 = first_bin(K);
    for (uint32_t s = 0; s < len.size(); ++s) {
        const uint64_t L = len[s];
        if (L == 0) continue;
        int bin = long_above_k && L > K ? NBINS : bin0;
        while (bin < NBINS && L > bin_max_tokens(bin, M)) ++bin;
        if (bin < NBINS) {
            pl.bins[bin].ids.push_back(s);
        } else {
            pl.long_ids.push_back(s);
            pl.long_prefix.push_back((uint32_t)(pl.long_prefix.back() + L));
        }
    }
    for (BinList &b : pl.bins) xcd_cuts(b.ids, len, b.cut);
    // Long segments whose compact z fits comfortably in one XCD's L2 go whole
    // to one XCD: longest first, each to the XCD with the fewest tokens so far
    // (the greedy balanced partition of the paper's Section 5.3, over the
    // eight XCDs).  Larger ("huge") segments are dealt chunk by chunk to all
    // XCDs: their random-positioning reads miss L2 anyway, and one XCD alone
    // would be the straggler.
    const size_t n = pl.long_ids.size();
    const uint64_t huge_tokens = 1u << 20;
    const uint32_t chunk = long_chunk(K);
    std::vector<uint32_t> order, owner(n, 8);
    uint64_t load[8] = {};
    std::vector<std::vector<std::pair<uint32_t, uint32_t>>> chunks(8);
    uint32_t rr = 0;
    for (uint32_t j = 0; j < n; ++j) {
        const uint64_t L = len[pl.long_ids[j]];
        if (L < huge_tokens) {
            order.push_back(j);
            continue;
        }
        for (uint64_t n0 = 0; n0 < L; n0 += chunk, rr = (rr + 1) & 7) {
            chunks[rr].push_back({j, (uint32_t)n0});
            load[rr] += std::min<uint64_t>(chunk, L - n0);
        }
    }
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
        return len[pl.long_ids[x]] > len[pl.long_ids[y]];
    });
    for (uint32_t j : order) {
        int best = 0;
        for (int x = 1; x < 8; ++x)
            if (load[x] < load[best]) best = x;
        owner[j] = best;
        load[best] += len[pl.long_ids[j]];
    }
    pl.chunk_seg.clear();
    pl.chunk_start.clear();
    for (int x = 0; x < 8; ++x) {
        pl.chunk_cut[x] = (uint32_t)pl.chunk_seg.size();
        for (auto &c : chunks[x]) {
            pl.chunk_seg.push_back(c.first);
            pl.chunk_start.push_back(c.second);
        }
        for (uint32_t j = 0; j < n; ++j) {
            if (owner[j] != (uint32_t)x) continue;
            const uint64_t L = len[pl.long_ids[j]];
            for (uint64_t n0 = 0; n0 < L; n0 += chunk) {
                pl.chunk_seg.push_back(j);
                pl.chunk_start.push_back((uint32_t)n0);
            }
        }
    }
    pl.chunk_cut[8] = (uint32_t)pl.chunk_seg.size();
    pl.chunk = chunk;
    // global count tables of the long segments: dense K counts when K is
    // small or the table would reach K slots, else open addressing with the
    // smallest power of two >= 2L slots (Section 5.4's hash tables)
    pl.tab_off.assign(1, 0);
    pl.tab_cap.clear();
    for (uint32_t j = 0; j < n; ++j) {
        const uint64_t L = len[pl.long_ids[j]];
        uint32_t cap = 0;
        if (K > Tuning::LDS_DENSE_MAX) {
            const uint32_t c = pow2_ge(std::min<uint64_t>(K, 2 * L));
            if (c < K) cap = c;
        }
        pl.tab_cap.push_back(cap);
        pl.tab_off.push_back(pl.tab_off.back() + (cap ? 2ull * cap : (uint64_t)K));
    }
}

// ---- record layout ---------------------------------------------------------
// Y is stored once (Section 5.2), blocked by documents (plain CSC order is
// the alternative): documents, in the doc phase's visiting order (each bin's
// list, XCD share by XCD share), are cut into blocks of about `block_tokens`
// tokens; a block never spans two bins or two XCD shares, and a long row is a
// block of its own.  Inside a block the tokens are ordered by (word rank,
// document, input index), the word rank being the word phase's visiting order
// (bins and shares again).  So a doc-phase window gathers inside one or two
// blocks that fit its XCD's L2, and one XCD's words occupy one contiguous run
// of every block.  mem[t] receives the record position of CSC token t.
void build_layout(const PhasePlan &wp, const PhasePlan &dp, const std::vector<uint64_t> &ld,
                  const std::vector<uint32_t> &colptr, const std::vector<uint32_t> &doc_csc,
                  uint64_t block_tokens, std::vector<uint32_t> &mem) {
    std::vector<uint32_t> block_of(ld.size(), 0);
    std::vector<uint64_t> start;   // block sizes, then running record offsets
    auto cut = [&](const std::vector<uint32_t> &ids, uint32_t b, uint32_t e, bool own) {
        uint64_t run = block_tokens;
        for (uint32_t i = b; i < e; ++i) {
            const uint32_t d = ids[i];
            if (own || run >= block_tokens) {
                start.push_back(0);
                run = 0;
            }
            block_of[d] = (uint32_t)start.size() - 1;
            start.back() += ld[d];
            run += ld[d];
        }
    };
    for (const BinList &b : dp.bins)
        for (int x = 0; x < 8; ++x) cut(b.ids, b.cut[x], b.cut[x + 1], false);
    cut(dp.long_ids, 0, (uint32_t)dp.long_ids.size(), true);
    uint64_t off = 0;
    for (uint64_t &v : start) {
        const uint64_t n = v;
        v = off;
        off += n;
    }
    std::vector<uint32_t> words;
    for (const BinList &b : wp.bins) words.insert(words.end(), b.ids.begin(), b.ids.end());
    std::vector<char> seen(wp.long_ids.size(), 0);
    for (uint32_t j : wp.chunk_seg)
        if (!seen[j]) {
            seen[j] = 1;
            words.push_back(wp.long_ids[j]);
        }
    for (uint32_t w : words)
        for (uint32_t t = colptr[w]; t < colptr[w + 1]; ++t) mem[t] = (uint32_t)start[block_of[doc_csc[t]]]++;
}

inline uint64_t zc_bytes(const PhasePlan &pl, uint32_t K) {
    return (uint64_t)pl.long_prefix.back() * (K <= 65535 ? 2 : 4) + 4;
}

struct Sizes {
    uint64_t recs, colptr, rowptr, colidx, rowidx, ck, alpha, misc;
    uint64_t plan_word, plan_doc;
    uint64_t total;
};

uint64_t plan_bytes(const PhasePlan &pl, uint32_t K) {
    uint64_t b = 0;
    for (const BinList &bl : pl.bins) b += align_up(4ull * bl.ids.size() + 4) + align_up(9 * 4) + align_up(8ull * bl.ids.size() + 8);
    return b + align_up(4ull * pl.long_ids.size() + 4) + align_up(4ull * pl.long_prefix.size()) +
           align_up(8ull * pl.tab_off.back() + 4) + align_up(8ull * pl.tab_off.size()) +
           align_up(4ull * pl.tab_cap.size() + 4) + 2 * align_up(4ull * pl.chunk_seg.size() + 4) +
           align_up(9 * 4) + align_up(zc_bytes(pl, K));
}

Sizes compute_sizes(const wlda_params &p, uint64_t T, const PhasePlan &w, const PhasePlan &d) {
    Sizes s;
    s.recs = align_up(T * (uint64_t)record_bytes(p.M, p.K) + 16);
    s.colptr = align_up(4ull * (p.V + 1));
    s.rowptr = align_up(4ull * (p.D + 1));
    s.colidx = align_up(4ull * T + 4);
    s.rowidx = align_up(4ull * T + 4);
    s.ck = 2 * align_up(4ull * p.K);
    s.alpha = align_up(4ull * p.K) + align_up(8ull * p.K);   // asymmetric alpha and its running sums
    s.misc = ALIGN;
    s.plan_word = plan_bytes(w, p.K);
    s.plan_doc = plan_bytes(d, p.K);
    s.total = s.recs + s.colptr + s.rowptr + s.colidx + s.rowidx + s.ck + s.alpha + s.misc + s.plan_word +
              s.plan_doc;
    return s;
}

wlda_status validate(const wlda_params *p, const uint32_t *word_ids, const uint32_t *doc_ids,
                     uint64_t T) {
    if (!p) return WLDA_E_INVALID;
    if (p->K < 1 || p->K > MAX_K || p->M < 1 || p->M > 4 || p->V < 1 || p->D < 1)
        return WLDA_E_INVALID;
    if (!(p->alpha > 0) || !(p->beta > 0)) return WLDA_E_INVALID;
    if (T >= (1ull << 32)) return WLDA_E_INVALID;
    if (T > 0 && (!word_ids || !doc_ids)) return WLDA_E_INVALID;
    for (uint64_t i = 0; i < T; ++i)
        if (word_ids[i] >= p->V || doc_ids[i] >= p->D) return WLDA_E_INVALID;
    return WLDA_OK;
}

void lengths(const wlda_params &p, const uint32_t *word_ids, const uint32_t *doc_ids, uint64_t T,
             std::vector<uint64_t> &lw, std::vector<uint64_t> &ld) {
    lw.assign(p.V, 0);
    ld.assign(p.D, 0);
    for (uint64_t i = 0; i < T; ++i) {
        lw[word_ids[i]]++;
        ld[doc_ids[i]]++;
    }
}

// Profiling slots: the bins of each phase, then its three long-path kernels.
enum Slot {
    S_WORD_BIN = 0, S_WORD_LONG_HIST = NBINS, S_WORD_LONG_MH, S_WORD_LONG_DRAW,
    S_DOC_BIN, S_DOC_LONG_HIST = S_DOC_BIN + NBINS, S_DOC_LONG_MH, S_DOC_LONG_DRAW, KSLOTS
};
const char *const SLOT_NAMES[KSLOTS] = {
    "word_g16", "word_g32", "word_wave", "word_block", "word_wide", "word_long_hist", "word_long_mh",
    "word_long_draw", "doc_g16", "doc_g32", "doc_wave", "doc_block", "doc_wide", "doc_long_hist",
    "doc_long_mh", "doc_long_draw"};
static_assert(NBINS == 5 && KSLOTS == 16, "slot names follow the bins");

uint64_t list_tokens(const std::vector<uint32_t> &ids, const std::vector<uint64_t> &len) {
    uint64_t t = 0;
    for (uint32_t s : ids) t += len[s];
    return t;
}

}  // namespace

struct wlda_sampler_s {
    wlda_params p{};
    uint64_t T = 0;
    hipStream_t st = nullptr;
    int nw = 8;                          // bytes per record
    uint64_t *recs = nullptr;
    uint32_t *colptr = nullptr, *rowptr = nullptr;
    uint32_t *colidx = nullptr, *rowidx = nullptr;   // canonical position -> record
    uint32_t *ck[2] = {nullptr, nullptr};
    int cur = 0;
    unsigned long long *acc = nullptr;   // [0] word phase, [1] doc phase
    double *ll = nullptr;
    PhasePlan word, doc;
    std::vector<uint32_t> inv;           // input index -> record position
    std::vector<uint32_t> mem;           // canonical CSC position -> record position
    bool blocked = false;                // records blocked by documents (else CSC order)
    uint32_t iter = 0;
    int next_phase = 0;                  // 0: not initialised, 1: word, 2: doc
    bool broken = false;
    float a = 0, b = 0, alpha_bar = 0, beta_k = 0, beta_bar = 0;
    // asymmetric alpha (wlda_set_alpha): alpha_k and its binary64 running
    // sums on the device, and their total
    bool asym = false;
    bool word_alias = false;             // WLDA_WORD_ALIAS
    float *d_alpha = nullptr;
    double *d_alpha_cum = nullptr;
    double alpha_total = 0;
    // profiling: event pairs per kernel kind
    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pairs[KSLOTS];
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    uint64_t slot_tokens[KSLOTS] = {};
    // launch-shape bounds (grid size of the segment kernels), per phase and
    // bin: [word g16, g32, wave, block, wide, doc g16, g32, wave, block, wide];
    // set from the CU count at create, overridable with WLDA_SEG_BLOCKS (ten
    // comma-separated values)
    uint32_t seg_blocks[2 * NBINS] = {768, 768, 768, 1024, 768, 768, 768, 512, 768, 512};
    // grid bound of the long-segment kernels [word, doc]; WLDA_LONG_BLOCKS="a,b"
    uint32_t long_blocks[2] = {4096, 2048};
    // LDS bytes per segment workgroup within which c_k is staged: the CU's
    // LDS shared by the workgroups per CU the bin runs at (seg_blocks / CUs);
    // WLDA_SEG_LDS_KIB sets one budget for all bins
    uint32_t cus = 256;
    uint32_t seg_lds_budget = 0;
};

namespace {

wlda_status hip_ok(wlda_sampler s, hipError_t e) {
    if (e == hipSuccess) return WLDA_OK;
    if (e == hipErrorNotSupported) return WLDA_E_UNSUPPORTED;
    if (s) s->broken = true;
    return WLDA_E_HIP;
}

#define WLDA_TRY(s, expr)                                   \
    do {                                                    \
        wlda_status _st = hip_ok((s), (expr));              \
        if (_st != WLDA_OK) return _st;                     \
    } while (0)

uint8_t *carve(uint8_t *&cur, uint64_t bytes) {
    uint8_t *p = cur;
    cur += align_up(bytes);
    return p;
}

hipError_t upload(void *dst, const void *src, uint64_t bytes, hipStream_t st) {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
}

hipError_t place_plan(PhasePlan &pl, const std::vector<uint32_t> &segptr, uint8_t *&cur, uint32_t K, hipStream_t st) {
    for (BinList &b : pl.bins) {
        b.d_ids = (uint32_t *)carve(cur, 4ull * b.ids.size() + 4);
        b.d_cut = (uint32_t *)carve(cur, 9 * 4);
        b.d_span = (uint2 *)carve(cur, 8ull * b.ids.size() + 8);
    }
    pl.d_long_ids = (uint32_t *)carve(cur, 4ull * pl.long_ids.size() + 4);
    pl.d_long_prefix = (uint32_t *)carve(cur, 4ull * pl.long_prefix.size());
    pl.d_tables = (uint32_t *)carve(cur, 8ull * pl.tab_off.back() + 4);   // old | updated counts
    pl.d_tab_off = (uint64_t *)carve(cur, 8ull * pl.tab_off.size());
    pl.d_tab_cap = (uint32_t *)carve(cur, 4ull * pl.tab_cap.size() + 4);
    pl.d_chunk_seg = (uint32_t *)carve(cur, 4ull * pl.chunk_seg.size() + 4);
    pl.d_chunk_start = (uint32_t *)carve(cur, 4ull * pl.chunk_seg.size() + 4);
    pl.d_chunk_cut = (uint32_t *)carve(cur, 9 * 4);
    pl.d_zc = carve(cur, zc_bytes(pl, K));
    hipError_t e;
    if ((e = upload(pl.d_chunk_seg, pl.chunk_seg.data(), 4ull * pl.chunk_seg.size(), st))) return e;
    if ((e = upload(pl.d_chunk_start, pl.chunk_start.data(), 4ull * pl.chunk_start.size(), st))) return e;
    if ((e = upload(pl.d_chunk_cut, pl.chunk_cut, 9 * 4, st))) return e;
    if ((e = upload(pl.d_tab_off, pl.tab_off.data(), 8ull * pl.tab_off.size(), st))) return e;
    if ((e = upload(pl.d_tab_cap, pl.tab_cap.data(), 4ull * pl.tab_cap.size(), st))) return e;
    for (BinList &b : pl.bins) {
        if ((e = upload(b.d_ids, b.ids.data(), 4ull * b.ids.size(), st))) return e;
        if ((e = upload(b.d_cut, b.cut, 9 * 4, st))) return e;
        std::vector<uint2> span(b.ids.size());
        for (size_t i = 0; i < b.ids.size(); ++i) span[i] = make_uint2(segptr[b.ids[i]], segptr[b.ids[i] + 1]);
        if ((e = upload(b.d_span, span.data(), 8ull * span.size(), st))) return e;
        // the copy is enqueued; keep the host buffer alive until it is done
        if ((e = hipStreamSynchronize(st))) return e;
    }
    if ((e = upload(pl.d_long_ids, pl.long_ids.data(), 4ull * pl.long_ids.size(), st))) return e;
    if ((e = upload(pl.d_long_prefix, pl.long_prefix.data(), 4ull * pl.long_prefix.size(), st)))
        return e;
    (void)K;
    return launch_fill_u32(pl.d_tables, 0, 2 * pl.tab_off.back(), st);
}

hipError_t take_event(wlda_sampler s, hipEvent_t *e) {
    if (s->ev_used == s->ev_pool.size()) {
        hipEvent_t ne;
        hipError_t err = hipEventCreate(&ne);
        if (err != hipSuccess) return err;
        s->ev_pool.push_back(ne);
    }
    *e = s->ev_pool[s->ev_used++];
    return hipSuccess;
}

// Records an event pair around `launch` when profiling is on.
template <typename F>
hipError_t timed(wlda_sampler s, int slot, F &&launch) {
    if (!s->prof) return launch();
    hipEvent_t a, b;
    hipError_t e;
    if ((e = take_event(s, &a)) || (e = take_event(s, &b))) return e;
    if ((e = hipEventRecord(a, s->st))) return e;
    if ((e = launch())) return e;
    if ((e = hipEventRecord(b, s->st))) return e;
    s->ev_pairs[slot].push_back({a, b});
    return hipSuccess;
}

LongList long_list(const PhasePlan &pl) {
    LongList ll;
    ll.ids = pl.d_long_ids;
    ll.prefix = pl.d_long_prefix;
    ll.n = (uint32_t)pl.long_ids.size();
    ll.total = pl.long_prefix.back();
    ll.tables = pl.d_tables;
    ll.chunk_seg = pl.d_chunk_seg;
    ll.chunk_start = pl.d_chunk_start;
    ll.n_chunks = (uint32_t)pl.chunk_seg.size();
    ll.chunk_cut = pl.d_chunk_cut;
    ll.zc = pl.d_zc;
    ll.tab_off = pl.d_tab_off;
    ll.tab_cap = pl.d_tab_cap;
    ll.table_words = pl.tab_off.back();
    ll.chunk = pl.chunk;
    ll.tables_new = pl.d_tables + pl.tab_off.back();
    return ll;
}

// One phase: every segment of the phase's plan, c_k of the new Z into the
// other buffer, then swap.
wlda_status run_phase(wlda_sampler s, uint32_t phase, uint32_t iter, bool draw_only) {
    PhasePlan &pl = phase == PH_WORD ? s->word : s->doc;
    PhaseArgs a;
    a.recs = s->recs;
    a.rf = record_format(s->p.M, s->p.K);
    a.segptr = phase == PH_WORD ? s->colptr : s->rowptr;
    a.idx = phase == PH_WORD ? s->colidx : s->rowidx;
    a.K = s->p.K;
    a.iter = iter;
    a.seed_lo = (uint32_t)s->p.seed;
    a.seed_hi = (uint32_t)(s->p.seed >> 32);
    a.ck = s->ck[s->cur];
    a.ck_next = s->ck[1 - s->cur];
    a.prior = phase == PH_WORD ? s->b : s->a;
    a.mass = phase == PH_WORD ? s->beta_k : s->alpha_bar;
    if (phase == PH_DOC && s->asym) {
        a.alpha_k = s->d_alpha;
        a.alpha_cum = s->d_alpha_cum;
    }
    a.beta_bar = s->beta_bar;
    a.accepted = s->acc + (phase == PH_WORD ? 0 : 1);
    a.draw_only = draw_only ? 1 : 0;
    a.word_alias = phase == PH_WORD && s->word_alias ? 1 : 0;
    WLDA_TRY(s, launch_fill_u32(a.ck_next, 0, s->p.K, s->st));
    WLDA_TRY(s, launch_fill_u32((uint32_t *)a.accepted, 0, 2, s->st));
    const int kb = phase == PH_WORD ? 0 : NBINS;
    LongList ll = long_list(pl);
    const int base = phase == PH_WORD ? S_WORD_BIN : S_DOC_BIN;
    const bool prof = s->prof && !draw_only;
    for (int bin = 0; bin < NBINS; ++bin) {
        const BinList &b = pl.bins[bin];
        const SegList l{b.d_ids, (uint32_t)b.ids.size(), b.d_cut, b.d_span};
        a.max_blocks = s->seg_blocks[kb + bin];
        if (s->seg_lds_budget) {
            a.seg_lds_budget = s->seg_lds_budget;
        } else {
            const uint32_t per_cu = std::max(1u, a.max_blocks / s->cus);
            a.seg_lds_budget = std::min(Tuning::LDS_PER_CU / per_cu, Tuning::SEG_LDS_BUDGET);
        }
        auto launch = [&] {
            return launch_segments(a, phase, s->p.M, l, bin, s->st);
        };
        if (prof)
            WLDA_TRY(s, timed(s, base + bin, launch));
        else
            WLDA_TRY(s, launch());
    }
    a.max_blocks = s->long_blocks[phase == PH_WORD ? 0 : 1];
    if (prof) {
        if (ll.n) {
            hipEvent_t ev[4];
            for (int i = 0; i < 4; ++i) WLDA_TRY(s, take_event(s, &ev[i]));
            WLDA_TRY(s, launch_long_segments(a, phase, s->p.M, ll, s->st, ev));
            for (int i = 0; i < 3; ++i) s->ev_pairs[base + NBINS + i].push_back({ev[i], ev[i + 1]});
        }
    } else {
        WLDA_TRY(s, launch_long_segments(a, phase, s->p.M, ll, s->st));
    }
    s->cur = 1 - s->cur;
    return WLDA_OK;
}

// Host copies of the records: T records of record_bytes(M, K) bytes, as
// 64-bit words (the 32-bit formats use half words).
struct HostRecs {
    std::vector<uint64_t> w;
    int rf = 1;
    uint32_t get(uint64_t i, int f) const {
        if (rf < 0) {
            const uint32_t b = (uint32_t)(-rf);
            const uint32_t r = reinterpret_cast<const uint32_t *>(w.data())[i];
            return (r >> (b * f)) & ((1u << b) - 1u);
        }
        if (rf >= 100) {
            const uint32_t r = reinterpret_cast<const uint32_t *>(w.data())[i * (rf - 100) + f / 2];
            return (r >> (16 * (f % 2))) & 0xFFFFu;
        }
        const uint64_t *rec = &w[i * rf];
        return (uint32_t)(rec[f / 3] >> (FIELD_BITS * (f % 3))) & FIELD_MASK;
    }
    void set(uint64_t i, int f, uint32_t v) {
        if (rf < 0) {
            const uint32_t b = (uint32_t)(-rf), sh = b * f;
            uint32_t &r = reinterpret_cast<uint32_t *>(w.data())[i];
            r = (r & ~(((1u << b) - 1u) << sh)) | (v << sh);
            return;
        }
        if (rf >= 100) {
            uint32_t &r = reinterpret_cast<uint32_t *>(w.data())[i * (rf - 100) + f / 2];
            const uint32_t sh = 16 * (f % 2);
            r = (r & ~(0xFFFFu << sh)) | (v << sh);
            return;
        }
        uint64_t *rec = &w[i * rf];
        const int sh = FIELD_BITS * (f % 3);
        rec[f / 3] = (rec[f / 3] & ~((uint64_t)FIELD_MASK << sh)) | ((uint64_t)v << sh);
    }
};

uint64_t record_array_bytes(wlda_sampler s) { return s->T * (uint64_t)record_bytes(s->p.M, s->p.K); }

void host_records(wlda_sampler s, HostRecs &h) {
    h.rf = record_format(s->p.M, s->p.K);
    h.w.assign(record_array_bytes(s) / 8 + 1, 0);
}

wlda_status download_records(wlda_sampler s, HostRecs &h) {
    host_records(s, h);
    if (s->T) WLDA_TRY(s, hipMemcpyAsync(h.w.data(), s->recs, record_array_bytes(s), hipMemcpyDeviceToHost, s->st));
    WLDA_TRY(s, hipStreamSynchronize(s->st));
    return WLDA_OK;
}

wlda_status upload_records_and_recount(wlda_sampler s, const HostRecs &h) {
    if (s->T) WLDA_TRY(s, hipMemcpyAsync(s->recs, h.w.data(), record_array_bytes(s), hipMemcpyHostToDevice, s->st));
    WLDA_TRY(s, launch_fill_u32(s->ck[s->cur], 0, s->p.K, s->st));
    WLDA_TRY(s, launch_histogram_z(s->recs, (uint32_t)s->T, s->p.M, s->p.K, s->ck[s->cur], s->st));
    WLDA_TRY(s, hipStreamSynchronize(s->st));
    return WLDA_OK;
}

}  // namespace

extern "C" {

const char *wlda_strerror(wlda_status e) {
    switch (e) {
        case WLDA_OK: return "ok";
        case WLDA_E_INVALID: return "invalid argument";
        case WLDA_E_WORKSPACE: return "workspace too small or misaligned";
        case WLDA_E_HIP: return "HIP runtime error";
        case WLDA_E_STATE: return "call out of order";
        case WLDA_E_UNSUPPORTED: return "unsupported by this build";
        case WLDA_E_NOMEM: return "host memory exhausted";
    }
    return "unknown status";
}

// Flags of the _ex calls: known bits, and the words an alias table can hold
// (bit 31 of its threshold word marks a finished bin).
wlda_status check_flags(uint32_t flags, const std::vector<uint64_t> &lw) {
    if (flags & ~(uint32_t)WLDA_WORD_ALIAS) return WLDA_E_INVALID;
    if (flags & WLDA_WORD_ALIAS)
        for (uint64_t L : lw)
            if (L >= (1ull << 31)) return WLDA_E_UNSUPPORTED;
    return WLDA_OK;
}

static wlda_status workspace_bytes_impl(const wlda_params *p, const uint32_t *word_ids,
                                        const uint32_t *doc_ids, uint64_t n_tokens, uint32_t flags,
                                        uint64_t *bytes) {
    if (!bytes) return WLDA_E_INVALID;
    wlda_status v = validate(p, word_ids, doc_ids, n_tokens);
    if (v != WLDA_OK) return v;
    std::vector<uint64_t> lw, ld;
    lengths(*p, word_ids, doc_ids, n_tokens, lw, ld);
    if ((v = check_flags(flags, lw)) != WLDA_OK) return v;
    PhasePlan w, d;
    build_plan(lw, p->M, p->K, w, (flags & WLDA_WORD_ALIAS) != 0);
    build_plan(ld, p->M, p->K, d);
    *bytes = compute_sizes(*p, n_tokens, w, d).total;
    return WLDA_OK;
}

wlda_status wlda_workspace_bytes_ex(const wlda_params *p, const uint32_t *word_ids,
                                    const uint32_t *doc_ids, uint64_t n_tokens, uint32_t flags,
                                    uint64_t *bytes) {
    try {
        return workspace_bytes_impl(p, word_ids, doc_ids, n_tokens, flags, bytes);
    } catch (const std::bad_alloc &) {
        return WLDA_E_NOMEM;
    }
}

wlda_status wlda_workspace_bytes(const wlda_params *p, const uint32_t *word_ids,
                                 const uint32_t *doc_ids, uint64_t n_tokens, uint64_t *bytes) {
    return wlda_workspace_bytes_ex(p, word_ids, doc_ids, n_tokens, 0, bytes);
}

wlda_status wlda_create(const wlda_params *p, const uint32_t *word_ids, const uint32_t *doc_ids,
                        uint64_t T, void *dev_workspace, uint64_t workspace_bytes,
                        void *hip_stream, wlda_sampler *out) {
    return wlda_create_ex(p, word_ids, doc_ids, T, 0, dev_workspace, workspace_bytes, hip_stream, out);
}

wlda_status wlda_create_ex(const wlda_params *p, const uint32_t *word_ids, const uint32_t *doc_ids,
                           uint64_t T, uint32_t flags, void *dev_workspace, uint64_t workspace_bytes,
                           void *hip_stream, wlda_sampler *out) {
    if (!out) return WLDA_E_INVALID;
    *out = nullptr;
    wlda_status v = validate(p, word_ids, doc_ids, T);
    if (v != WLDA_OK) return v;
    if (flags & ~(uint32_t)WLDA_WORD_ALIAS) return WLDA_E_INVALID;
    if (!dev_workspace || ((uintptr_t)dev_workspace % ALIGN) != 0) return WLDA_E_WORKSPACE;
    wlda_sampler s = new (std::nothrow) wlda_sampler_s();
    if (!s) return WLDA_E_NOMEM;
    s->p = *p;
    s->T = T;
    s->st = (hipStream_t)hip_stream;
    s->nw = (int)record_bytes(p->M, p->K);   // bytes per record
    s->a = (float)p->alpha;
    s->b = (float)p->beta;
    s->alpha_bar = (float)p->K * s->a;
    s->beta_k = (float)p->K * s->b;
    s->beta_bar = (float)p->V * s->b;
    {
        // Workgroups per CU of each segment kernel, measured at C1: the doc
        // phase gathers and scatters inside L2-resident blocks, and more rows
        // in flight than about two (rows <= 512) or three (longer rows)
        // workgroups per CU make the L2 write dirty lines back before they
        // fill (4 per CU costs the row kernel 20%); the word phase's column
        // kernels peak at 2-3.  The long-segment kernels stream chunks and
        // want many more.  Multiples of the CU count keep every CU of an XCD
        // equally loaded.  The doc phase's 16- and 32-lane groups (used where
        // K > 1024) run at three per CU, which their LDS allows with the
        // 16-bit c_k histogram; for M > 2 the sub-workgroup bins hold half as
        // many tokens per lane, and the 16-lane groups and the workgroup bin
        // run at four, the wave kernel at three (measured on the PubMed-shaped
        // corpus, K = 1e4).
        static const uint32_t per_cu[2 * NBINS] = {3, 3, 3, 4, 3, 3, 3, 2, 3, 2};
        static const uint32_t long_per_cu[2] = {16, 8};
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) {
            s->cus = (uint32_t)cus;
            for (int i = 0; i < 2 * NBINS; ++i) {
                uint32_t pc = per_cu[i];
                if (p->M > 2 && (i == NBINS + BIN_G16 || i == NBINS + BIN_BLOCK)) pc = 4;
                if (p->M > 2 && i == NBINS + BIN_WAVE) pc = 3;
                s->seg_blocks[i] = pc * (uint32_t)cus;
            }
            for (int i = 0; i < 2; ++i) s->long_blocks[i] = long_per_cu[i] * (uint32_t)cus;
        }
    }
    if (const char *env = std::getenv("WLDA_LONG_BLOCKS")) {
        unsigned v[2];
        if (std::sscanf(env, "%u,%u", &v[0], &v[1]) == 2)
            for (int i = 0; i < 2; ++i) s->long_blocks[i] = v[i] < 8 ? 8 : (v[i] > 65536 ? 65536 : v[i]);
    }
    if (const char *env = std::getenv("WLDA_SEG_LDS_KIB")) {
        const int v = std::atoi(env);
        if (v >= 1 && v <= 160) s->seg_lds_budget = (uint32_t)v * 1024u;
    }
    if (const char *env = std::getenv("WLDA_SEG_BLOCKS")) {
        unsigned v[2 * NBINS];
        if (std::sscanf(env, "%u,%u,%u,%u,%u,%u,%u,%u,%u,%u", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6],
                        &v[7], &v[8], &v[9]) == 2 * NBINS)
            for (int i = 0; i < 2 * NBINS; ++i) s->seg_blocks[i] = v[i] < 8 ? 8 : (v[i] > 65536 ? 65536 : v[i]);
    }

    // ---- layout: stable order by (word, doc, input index) -------------------
    std::vector<uint64_t> lw, ld;
    std::vector<uint32_t> colptr, rowptr;
    try {
        lengths(*p, word_ids, doc_ids, T, lw, ld);
        if ((v = check_flags(flags, lw)) != WLDA_OK) {
            delete s;
            return v;
        }
        s->word_alias = (flags & WLDA_WORD_ALIAS) != 0;
        build_plan(lw, p->M, p->K, s->word, s->word_alias);
        build_plan(ld, p->M, p->K, s->doc);
        colptr.resize(p->V + 1);
        rowptr.resize(p->D + 1);
    } catch (const std::bad_alloc &) {
        delete s;
        return WLDA_E_NOMEM;
    }
    for (int bin = 0; bin < NBINS; ++bin) {
        s->slot_tokens[S_WORD_BIN + bin] = list_tokens(s->word.bins[bin].ids, lw);
        s->slot_tokens[S_DOC_BIN + bin] = list_tokens(s->doc.bins[bin].ids, ld);
    }
    s->slot_tokens[S_WORD_LONG_HIST] = s->slot_tokens[S_WORD_LONG_MH] =
        s->slot_tokens[S_WORD_LONG_DRAW] = s->word.long_prefix.back();
    s->slot_tokens[S_DOC_LONG_HIST] = s->slot_tokens[S_DOC_LONG_MH] =
        s->slot_tokens[S_DOC_LONG_DRAW] = s->doc.long_prefix.back();
    const Sizes sz = compute_sizes(*p, T, s->word, s->doc);
    if (workspace_bytes < sz.total) {
        delete s;
        return WLDA_E_WORKSPACE;
    }
    colptr[0] = rowptr[0] = 0;
    for (uint32_t w = 0; w < p->V; ++w) colptr[w + 1] = colptr[w] + (uint32_t)lw[w];
    for (uint32_t d = 0; d < p->D; ++d) rowptr[d + 1] = rowptr[d] + (uint32_t)ld[d];
    // canonical CSC position t of input token i: stable order by (word, doc,
    // input index); canonical CSR position: rows in ascending CSC position
    std::vector<uint32_t> rowidx;
    try {
        std::vector<uint32_t> doc_csc(T);
        {
            std::vector<uint32_t> by_doc(T), cursor(rowptr.begin(), rowptr.end() - 1);
            for (uint64_t i = 0; i < T; ++i) by_doc[cursor[doc_ids[i]]++] = (uint32_t)i;
            s->inv.resize(T);
            std::vector<uint32_t> wc(colptr.begin(), colptr.end() - 1);
            for (uint64_t j = 0; j < T; ++j) {
                const uint32_t i = by_doc[j];
                const uint32_t t = wc[word_ids[i]]++;
                s->inv[i] = t;
                doc_csc[t] = doc_ids[i];
            }
        }
        // record layout: blocked by documents, blocks of DOC_BLOCK_KIB of
        // records (WLDA_DOC_BLOCK_KIB overrides; 0 selects plain CSC order,
        // where colidx is the identity)
        s->mem.resize(T);
        uint64_t block_kib = DOC_BLOCK_KIB;
        if (const char *env = std::getenv("WLDA_DOC_BLOCK_KIB")) block_kib = std::strtoull(env, nullptr, 10);
        s->blocked = block_kib >= 16 && block_kib <= (1ull << 20);
        if (s->blocked) {
            build_layout(s->word, s->doc, ld, colptr, doc_csc, (block_kib << 10) / (uint64_t)s->nw, s->mem);
            for (uint64_t i = 0; i < T; ++i) s->inv[i] = s->mem[s->inv[i]];
        } else {
            for (uint64_t t = 0; t < T; ++t) s->mem[t] = (uint32_t)t;
        }
        rowidx.resize(T);
        std::vector<uint32_t> cursor(rowptr.begin(), rowptr.end() - 1);
        for (uint64_t t = 0; t < T; ++t) rowidx[cursor[doc_csc[t]]++] = s->mem[t];
    } catch (const std::bad_alloc &) {
        delete s;
        return WLDA_E_NOMEM;
    }

    // ---- workspace ----------------------------------------------------------
    uint8_t *cur = (uint8_t *)dev_workspace;
    s->recs = (uint64_t *)carve(cur, T * (uint64_t)s->nw + 16);
    s->colptr = (uint32_t *)carve(cur, 4ull * (p->V + 1));
    s->rowptr = (uint32_t *)carve(cur, 4ull * (p->D + 1));
    s->colidx = (uint32_t *)carve(cur, 4ull * T + 4);
    s->rowidx = (uint32_t *)carve(cur, 4ull * T + 4);
    s->ck[0] = (uint32_t *)carve(cur, 4ull * p->K);
    s->ck[1] = (uint32_t *)carve(cur, 4ull * p->K);
    s->d_alpha = (float *)carve(cur, 4ull * p->K);
    s->d_alpha_cum = (double *)carve(cur, 8ull * p->K);
    uint8_t *misc = carve(cur, ALIGN);
    s->acc = (unsigned long long *)misc;
    s->ll = (double *)(misc + 16);
    wlda_status st = WLDA_OK;
    hipError_t e = hipSuccess;
    if (!e) e = upload(s->colptr, colptr.data(), 4ull * (p->V + 1), s->st);
    if (!e) e = upload(s->rowptr, rowptr.data(), 4ull * (p->D + 1), s->st);
    if (!e && s->blocked) e = upload(s->colidx, s->mem.data(), 4ull * T, s->st);
    if (!s->blocked) s->colidx = nullptr;   // identity: kernels use the CSC position
    if (!e) e = upload(s->rowidx, rowidx.data(), 4ull * T, s->st);
    if (!e) e = place_plan(s->word, colptr, cur, p->K, s->st);
    if (!e) e = place_plan(s->doc, rowptr, cur, p->K, s->st);
    if (!e) e = launch_fill_u32(s->ck[0], 0, 2ull * align_up(4ull * p->K) / 4, s->st);
    if (!e) e = hipStreamSynchronize(s->st);
    if (e) {
        st = hip_ok(s, e);
        delete s;
        return st;
    }
    *out = s;
    return WLDA_OK;
}

wlda_status wlda_set_alpha(wlda_sampler s, const float *alpha) {
    if (!s) return WLDA_E_INVALID;
    if (s->broken) return WLDA_E_HIP;
    if (s->next_phase != 0) return WLDA_E_STATE;
    const uint32_t K = s->p.K;
    if (!alpha) {
        s->asym = false;
        s->alpha_bar = (float)K * s->a;
        return WLDA_OK;
    }
    std::vector<double> cum;
    try {
        cum.resize(K);
    } catch (const std::bad_alloc &) {
        return WLDA_E_NOMEM;
    }
    double run = 0.0;
    for (uint32_t k = 0; k < K; ++k) {
        if (!(alpha[k] > 0.0f) || !std::isfinite(alpha[k])) return WLDA_E_INVALID;
        run += (double)alpha[k];
        cum[k] = run;
    }
    WLDA_TRY(s, upload(s->d_alpha, alpha, 4ull * K, s->st));
    WLDA_TRY(s, upload(s->d_alpha_cum, cum.data(), 8ull * K, s->st));
    WLDA_TRY(s, hipStreamSynchronize(s->st));
    s->asym = true;
    s->alpha_total = run;
    s->alpha_bar = (float)run;
    return WLDA_OK;
}

wlda_status wlda_init(wlda_sampler s) {
    if (!s) return WLDA_E_INVALID;
    if (s->broken) return WLDA_E_HIP;
    WLDA_TRY(s, launch_init_z(s->recs, s->colidx, (uint32_t)s->T, s->p.M, s->p.K, (uint32_t)s->p.seed,
                              (uint32_t)(s->p.seed >> 32), s->st));
    // first doc proposals from the initial Z; c_k of Z lands in the other buffer
    wlda_status st = run_phase(s, PH_DOC, 0, true);
    if (st != WLDA_OK) return st;
    s->iter = 0;
    s->next_phase = PH_WORD;
    return WLDA_OK;
}

wlda_status wlda_word_phase(wlda_sampler s) {
    if (!s) return WLDA_E_INVALID;
    if (s->broken) return WLDA_E_HIP;
    if (s->next_phase != PH_WORD) return WLDA_E_STATE;
    wlda_status st = run_phase(s, PH_WORD, s->iter + 1, false);
    if (st != WLDA_OK) return st;
    s->next_phase = PH_DOC;
    return WLDA_OK;
}

wlda_status wlda_doc_phase(wlda_sampler s) {
    if (!s) return WLDA_E_INVALID;
    if (s->broken) return WLDA_E_HIP;
    if (s->next_phase != PH_DOC) return WLDA_E_STATE;
    wlda_status st = run_phase(s, PH_DOC, s->iter + 1, false);
    if (st != WLDA_OK) return st;
    s->iter += 1;
    s->next_phase = PH_WORD;
    return WLDA_OK;
}

wlda_status wlda_iterate(wlda_sampler s, uint32_t n) {
    for (uint32_t k = 0; k < n; ++k) {
        wlda_status st = wlda_word_phase(s);
        if (st != WLDA_OK) return st;
        st = wlda_doc_phase(s);
        if (st != WLDA_OK) return st;
    }
    return WLDA_OK;
}

wlda_status wlda_log_likelihood(wlda_sampler s, double *ll) {
    if (!s || !ll) return WLDA_E_INVALID;
    if (s->broken) return WLDA_E_HIP;
    if (s->next_phase == 0) return WLDA_E_STATE;
    const uint32_t K = s->p.K;
    WLDA_TRY(s, launch_fill_u32((uint32_t *)s->ll, 0, 2, s->st));
    for (int ph = PH_WORD; ph <= PH_DOC; ++ph) {
        const PhasePlan &pl = ph == PH_WORD ? s->word : s->doc;
        const uint32_t *segptr = ph == PH_WORD ? s->colptr : s->rowptr;
        const uint32_t *idx = ph == PH_WORD ? s->colidx : s->rowidx;
        const double prior = ph == PH_WORD ? s->p.beta : s->p.alpha;
        const bool asym = ph == PH_DOC && s->asym;
        const double total = ph == PH_WORD ? 0.0 : (asym ? s->alpha_total : (double)K * s->p.alpha);
        const int lt = ph == PH_DOC;
        for (const BinList &b : pl.bins)
            WLDA_TRY(s, launch_ll_list(s->recs, s->p.M, segptr, idx, b.d_ids, (uint32_t)b.ids.size(), K,
                                       prior, total, lt, s->ll, s->st, asym ? s->d_alpha : nullptr));
        PhaseArgs a;
        a.recs = s->recs;
        a.rf = record_format(s->p.M, s->p.K);
        a.segptr = segptr;
        a.idx = idx;
        a.K = K;
        a.alpha_k = asym ? s->d_alpha : nullptr;
        WLDA_TRY(s, launch_ll_long(a, ph, s->p.M, long_list(pl), prior, total, lt, s->ll, s->st));
    }
    WLDA_TRY(s, launch_ll_topics(s->ck[s->cur], K, (double)s->p.V * s->p.beta, s->ll, s->st));
    WLDA_TRY(s, hipMemcpyAsync(ll, s->ll, sizeof(double), hipMemcpyDeviceToHost, s->st));
    WLDA_TRY(s, hipStreamSynchronize(s->st));
    return WLDA_OK;
}

wlda_status wlda_theta(wlda_sampler s, uint32_t d0, uint32_t nd, float *theta) {
    if (!s || !theta || (uint64_t)d0 + nd > s->p.D) return WLDA_E_INVALID;
    if (s->broken) return WLDA_E_HIP;
    if (s->next_phase == 0) return WLDA_E_STATE;
    WLDA_TRY(s, launch_theta(s->recs, s->p.M, s->rowptr, s->rowidx, d0, nd, s->p.K, s->a,
                             s->asym ? s->d_alpha : nullptr, s->alpha_bar, theta,
                             s->st));
    return WLDA_OK;
}

wlda_status wlda_phi(wlda_sampler s, uint32_t w0, uint32_t nw, float *phi) {
    if (!s || !phi || (uint64_t)w0 + nw > s->p.V) return WLDA_E_INVALID;
    if (s->broken) return WLDA_E_HIP;
    if (s->next_phase == 0) return WLDA_E_STATE;
    WLDA_TRY(s, launch_phi(s->recs, s->p.M, s->colptr, s->colidx, s->ck[s->cur], w0, nw, s->p.K, s->b,
                           s->beta_bar, phi, s->st));
    return WLDA_OK;
}

static wlda_status copy_out(wlda_sampler s, int32_t *z, int32_t *props, bool input_order) {
    if (!s || !z) return WLDA_E_INVALID;
    if (s->broken) return WLDA_E_HIP;
    HostRecs h;
    wlda_status st = download_records(s, h);
    if (st != WLDA_OK) return st;
    const uint64_t T = s->T;
    for (uint64_t i = 0; i < T; ++i) {
        const uint64_t t = input_order ? s->inv[i] : s->mem[i];
        z[i] = (int32_t)h.get(t, 0);
        if (props)
            for (uint32_t m = 1; m <= s->p.M; ++m) props[(m - 1) * T + i] = (int32_t)h.get(t, m);
    }
    return WLDA_OK;
}

wlda_status wlda_copy_assignments(wlda_sampler s, int32_t *z, int32_t *props) {
    return copy_out(s, z, props, true);
}

wlda_status wlda_copy_assignments_csc(wlda_sampler s, int32_t *z, int32_t *props) {
    return copy_out(s, z, props, false);
}

wlda_status wlda_copy_topic_counts(wlda_sampler s, int64_t *ck) {
    if (!s || !ck) return WLDA_E_INVALID;
    if (s->broken) return WLDA_E_HIP;
    std::vector<uint32_t> h(s->p.K);
    WLDA_TRY(s, hipMemcpyAsync(h.data(), s->ck[s->cur], 4ull * s->p.K, hipMemcpyDeviceToHost, s->st));
    WLDA_TRY(s, hipStreamSynchronize(s->st));
    for (uint32_t k = 0; k < s->p.K; ++k) ck[k] = h[k];
    return WLDA_OK;
}

wlda_status wlda_accepted(wlda_sampler s, int phase, uint64_t *count) {
    if (!s || !count || (phase != 1 && phase != 2)) return WLDA_E_INVALID;
    if (s->broken) return WLDA_E_HIP;
    unsigned long long h = 0;
    WLDA_TRY(s, hipMemcpyAsync(&h, s->acc + (phase - 1), 8, hipMemcpyDeviceToHost, s->st));
    WLDA_TRY(s, hipStreamSynchronize(s->st));
    *count = h;
    return WLDA_OK;
}

wlda_status wlda_iteration(wlda_sampler s, uint32_t *iteration) {
    if (!s || !iteration) return WLDA_E_INVALID;
    *iteration = s->iter;
    return WLDA_OK;
}

wlda_status wlda_state_bytes(wlda_sampler s, uint64_t *bytes) {
    if (!s || !bytes) return WLDA_E_INVALID;
    *bytes = 16 + 4ull * (1 + s->p.M) * s->T;
    return WLDA_OK;
}

wlda_status wlda_save_state(wlda_sampler s, void *host_buf, uint64_t bytes) {
    uint64_t need = 0;
    wlda_state_bytes(s, &need);
    if (!s || !host_buf || bytes < need) return WLDA_E_INVALID;
    if (s->next_phase == 0) return WLDA_E_STATE;
    uint8_t *p = (uint8_t *)host_buf;
    const uint64_t hdr[2] = {s->iter, (uint64_t)s->next_phase};
    std::memcpy(p, hdr, 16);
    int32_t *z = (int32_t *)(p + 16);
    return copy_out(s, z, z + s->T, false);
}

wlda_status wlda_load_state(wlda_sampler s, const void *host_buf, uint64_t bytes) {
    uint64_t need = 0;
    wlda_state_bytes(s, &need);
    if (!s || !host_buf || bytes < need) return WLDA_E_INVALID;
    if (s->broken) return WLDA_E_HIP;
    const uint8_t *p = (const uint8_t *)host_buf;
    uint64_t hdr[2];
    std::memcpy(hdr, p, 16);
    if (hdr[1] != PH_WORD && hdr[1] != PH_DOC) return WLDA_E_INVALID;
    const int32_t *z = (const int32_t *)(p + 16);
    const int32_t *props = z + s->T;
    const uint64_t T = s->T;
    HostRecs h;
    host_records(s, h);
    for (uint64_t t = 0; t < T; ++t) {
        const uint64_t r = s->mem[t];
        if ((uint32_t)z[t] >= s->p.K) return WLDA_E_INVALID;
        h.set(r, 0, (uint32_t)z[t]);
        for (uint32_t m = 1; m <= s->p.M; ++m) {
            const uint32_t v = (uint32_t)props[(m - 1) * T + t];
            if (v >= s->p.K) return WLDA_E_INVALID;
            h.set(r, m, v);
        }
    }
    wlda_status st = upload_records_and_recount(s, h);
    if (st != WLDA_OK) return st;
    s->iter = (uint32_t)hdr[0];
    s->next_phase = (int)hdr[1];
    return WLDA_OK;
}

wlda_status wlda_set_assignments(wlda_sampler s, const int32_t *z, const int32_t *props) {
    if (!s || !z) return WLDA_E_INVALID;
    if (s->broken) return WLDA_E_HIP;
    if (!props && s->next_phase == 0) return WLDA_E_STATE;
    HostRecs h;
    wlda_status st = download_records(s, h);
    if (st != WLDA_OK) return st;
    const uint64_t T = s->T;
    for (uint64_t i = 0; i < T; ++i) {
        const uint64_t t = s->inv[i];
        if ((uint32_t)z[i] >= s->p.K) return WLDA_E_INVALID;
        h.set(t, 0, (uint32_t)z[i]);
        if (props)
            for (uint32_t m = 1; m <= s->p.M; ++m) {
                const uint32_t v = (uint32_t)props[(m - 1) * T + i];
                if (v >= s->p.K) return WLDA_E_INVALID;
                h.set(t, m, v);
            }
    }
    st = upload_records_and_recount(s, h);
    if (st != WLDA_OK) return st;
    s->next_phase = PH_WORD;
    return WLDA_OK;
}

wlda_status wlda_profile(wlda_sampler s, int enable) {
    if (!s) return WLDA_E_INVALID;
    if (s->broken) return WLDA_E_HIP;
    if (enable) {
        WLDA_TRY(s, hipStreamSynchronize(s->st));
        for (auto &v : s->ev_pairs) v.clear();
        s->ev_used = 0;
    }
    s->prof = enable != 0;
    return WLDA_OK;
}

wlda_status wlda_profile_read(wlda_sampler s, wlda_kernel_stat *out, uint32_t max_entries,
                              uint32_t *n_entries) {
    if (!s || !n_entries || (!out && max_entries)) return WLDA_E_INVALID;
    if (s->broken) return WLDA_E_HIP;
    WLDA_TRY(s, hipStreamSynchronize(s->st));
    uint32_t n = 0;
    for (int k = 0; k < KSLOTS; ++k) {
        if (n >= max_entries) break;
        double tot = 0;
        for (auto &pr : s->ev_pairs[k]) {
            float ms = 0;
            WLDA_TRY(s, hipEventElapsedTime(&ms, pr.first, pr.second));
            tot += ms;
        }
        out[n].name = SLOT_NAMES[k];
        out[n].launches = s->ev_pairs[k].size();
        out[n].tokens_per_launch = s->slot_tokens[k];
        out[n].total_ms = tot;
        ++n;
    }
    *n_entries = n;
    return WLDA_OK;
}

wlda_status wlda_destroy(wlda_sampler s) {
    if (!s) return WLDA_E_INVALID;
    if (!s->broken) (void)hipStreamSynchronize(s->st);
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    delete s;
    return WLDA_OK;
}

}  // extern "C"
