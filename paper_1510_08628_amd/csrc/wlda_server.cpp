// Continuous-batching fold-in server.
//
// Requests (new documents) are queued on the host as they arrive and admitted
// in arrival order while a document slot and a contiguous range of the
// device token pool are free (memory admission).  Every step runs ONE
// fold-in sweep for every admitted document in a single ragged launch, so
// documents admitted at different times share the device; a document leaves
// (its slot and pool range are freed) once it has had its initialisation and
// `sweeps` sweeps.  In learned mode the encoder's forward pass for newly
// admitted documents runs on the encoder's own stream, overlapped with the
// sweep of the documents already in flight.  Requests at the head of the
// queue are encoded one step ahead, into one of two stage buffers, so that
// by their admission the proposal is usually ready and the step does not
// wait for the encoder; a request admitted before it was encoded is encoded
// at admission and joins the sweeps at the first step that finds its encoder
// run finished (an event query on the host), so the encoder overlaps the
// sweeps instead of holding up the documents in flight.  A document's result
// depends only on its words and request id (its random stream), not on the
// batch it shared or on when it was encoded.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <new>
#include <vector>

#include "../../include/warplda.h"
#include "wlda_fold.h"

using namespace wlda;
using wlda::wlda_encoder_get_k;

namespace {
constexpr uint64_t SALIGN = 256;
inline uint64_t sa(uint64_t x) { return (x + SALIGN - 1) / SALIGN * SALIGN; }

struct Pending {
    uint32_t req;
    std::vector<uint32_t> words, ho;
    std::vector<uint32_t> weights;   // caller-provided learned weights (K) or empty
    double arrival;
    int stage = -1;                  // encoded ahead into stage buffer 0/1, row stage_row
    uint32_t stage_row = 0;
};

struct Range {
    uint64_t off, len;
};

// First-fit allocator over [0, cap) with coalescing.
struct Pool {
    std::list<Range> free_;
    void reset(uint64_t cap) { free_.assign(1, Range{0, cap}); }
    bool alloc(uint64_t n, uint64_t *off) {
        if (n == 0) {
            *off = 0;
            return true;
        }
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->len >= n) {
                *off = it->off;
                it->off += n;
                it->len -= n;
                if (it->len == 0) free_.erase(it);
                return true;
            }
        return false;
    }
    void release(uint64_t off, uint64_t n) {
        if (n == 0) return;
        auto it = free_.begin();
        while (it != free_.end() && it->off < off) ++it;
        it = free_.insert(it, Range{off, n});
        auto nx = std::next(it);
        if (nx != free_.end() && it->off + it->len == nx->off) {
            it->len += nx->len;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->off + pv->len == it->off) {
                pv->len += it->len;
                free_.erase(it);
            }
        }
    }
};

struct Slot {
    bool busy = false;
    uint32_t req = 0, len = 0, n_ho = 0, sweep = 0;   // sweep = launches done
    uint64_t off = 0, ho_off = 0;
    double arrival = 0, admit = 0;
    bool learned = false;
};

}  // namespace

struct wlda_server_s {
    wlda_model model = nullptr;
    wlda_encoder enc = nullptr;
    wlda_server_params sp{};
    hipStream_t st = nullptr, enc_st = nullptr;
    // encoder runs for the documents admitted at a step (two events,
    // alternating); documents encoded at admission wait, out of the sweep
    // lists, until the host sees the latest such run finished (the encoder
    // stream runs in order, so that run finishing covers the earlier ones)
    hipEvent_t enc_ev[2] = {nullptr, nullptr};
    int enc_cur = 0;                 // the event this step records
    std::vector<uint32_t> deferred;  // documents encoded at admission, not yet sweeping
    hipEvent_t deferred_ev = nullptr;  // the encoder run they wait for
    uint32_t K = 0, M = 0, buckets = 0;
    // device
    uint32_t *d_slots = nullptr, *d_off = nullptr, *d_len = nullptr, *d_req = nullptr, *d_sweep = nullptr,
             *d_useq = nullptr, *d_hoff = nullptr, *d_hlen = nullptr;
    uint32_t *d_words = nullptr, *d_z = nullptr, *d_pd = nullptr, *d_pw = nullptr, *d_how = nullptr;
    uint32_t *d_qcdf = nullptr;
    double *d_out = nullptr;
    uint32_t *d_hchunk = nullptr;    // held-out blocks of the retiring documents (prefix sums)
    double *d_holog = nullptr;       // log p of every held-out token (held-out pool order)
    uint32_t *d_frow = nullptr, *d_fidx = nullptr;
    float *d_fval = nullptr, *d_probs = nullptr;
    uint32_t *d_cdf_stage = nullptr;
    // encode-ahead stages (two, used alternately)
    uint32_t *d_ah_cdf[2] = {nullptr, nullptr}, *d_ah_frow[2] = {nullptr, nullptr},
             *d_ah_fidx[2] = {nullptr, nullptr};
    float *d_ah_fval[2] = {nullptr, nullptr};
    hipEvent_t ah_done[2] = {nullptr, nullptr};
    hipEvent_t ah_copied = nullptr;   // the sweep stream has read the stages it admitted from
    bool ah_live[2] = {false, false};
    int ah_next = 0;
    std::vector<uint32_t> h_ah_rows[2], h_ah_idx[2];
    std::vector<float> h_ah_val[2];
    // host
    std::vector<Slot> slots;
    std::vector<uint32_t> h_off, h_len, h_req, h_sweep, h_useq, h_hoff, h_hlen;
    // the slot list last uploaded to d_slots (valid until the retire step
    // reuses d_slots), so that steady steps upload nothing
    std::vector<uint32_t> up_lists;
    bool lists_valid = false;
    Pool pool, ho_pool;
    std::deque<Pending> pending;
    std::vector<wlda_result> done;
    std::map<uint32_t, std::vector<int32_t>> done_z;
    std::chrono::steady_clock::time_point t0;
    bool broken = false;
};

namespace {

double now_s(const wlda_server_s *s) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

uint64_t server_bytes(const wlda_params &p, const wlda_server_params &sp, bool learned) {
    const uint64_t n = sp.max_docs, T = sp.pool_tokens, H = sp.pool_heldout;
    uint64_t b = 8 * sa(4 * n + 4) + sa(4 * T + 4) * (2 + 2ull * p.M) + sa(4 * H + 4) + sa(8 * n + 8) +
                 sa(4 * n * p.K + 4) + sa(4 * n + 8) + sa(8 * H + 8);
    if (learned)
        b += 3 * (sa(4 * n + 4) + sa(4 * T + 4) + sa(4 * T + 4)) + 4 * sa(4 * n * p.K);
    return b;
}

bool valid_sp(const wlda_server_params *sp) {
    return sp && sp->max_docs >= 1 && sp->pool_tokens >= 1 && sp->pool_tokens < (1ull << 32) &&
           sp->pool_heldout < (1ull << 32) && sp->sweeps >= 1 && sp->eps > 0 && sp->eps <= 1;
}

wlda_status fail(wlda_server s) {
    s->broken = true;
    return WLDA_E_HIP;
}

}  // namespace

extern "C" {

wlda_status wlda_server_workspace_bytes(wlda_model m, wlda_encoder enc, const wlda_server_params *sp,
                                        uint64_t *bytes) {
    if (!m || !valid_sp(sp) || !bytes) return WLDA_E_INVALID;
    *bytes = server_bytes(model_params(m), *sp, enc != nullptr);
    return WLDA_OK;
}

wlda_status wlda_server_create(wlda_model m, wlda_encoder enc, const wlda_server_params *sp, void *ws,
                               uint64_t ws_bytes, void *stream, wlda_server *out) {
    if (!m || !valid_sp(sp) || !out) return WLDA_E_INVALID;
    *out = nullptr;
    const wlda_params &p = model_params(m);
    if (enc && (wlda_encoder_get_k(enc) != p.K)) return WLDA_E_INVALID;
    if (!ws || ((uintptr_t)ws % SALIGN) || ws_bytes < server_bytes(p, *sp, enc != nullptr))
        return WLDA_E_WORKSPACE;
    wlda_server s = new (std::nothrow) wlda_server_s();
    if (!s) return WLDA_E_INVALID;
    s->model = m;
    s->enc = enc;
    s->sp = *sp;
    s->st = (hipStream_t)stream;
    s->K = p.K;
    s->M = p.M;
    const uint64_t n = sp->max_docs, T = sp->pool_tokens, H = sp->pool_heldout;
    uint8_t *c = (uint8_t *)ws;
    auto take = [&](uint64_t b) { uint8_t *q = c; c += sa(b); return q; };
    s->d_slots = (uint32_t *)take(4 * n + 4);
    s->d_off = (uint32_t *)take(4 * n + 4);
    s->d_len = (uint32_t *)take(4 * n + 4);
    s->d_req = (uint32_t *)take(4 * n + 4);
    s->d_sweep = (uint32_t *)take(4 * n + 4);
    s->d_useq = (uint32_t *)take(4 * n + 4);
    s->d_hoff = (uint32_t *)take(4 * n + 4);
    s->d_hlen = (uint32_t *)take(4 * n + 4);
    s->d_words = (uint32_t *)take(4 * T + 4);
    s->d_z = (uint32_t *)take(4 * T + 4);
    s->d_pd = (uint32_t *)take(4 * T * p.M + 4);
    s->d_pw = (uint32_t *)take(4 * T * p.M + 4);
    s->d_how = (uint32_t *)take(4 * H + 4);
    s->d_out = (double *)take(8 * n + 8);
    s->d_qcdf = (uint32_t *)take(4 * n * p.K + 4);
    s->d_hchunk = (uint32_t *)take(4 * n + 8);
    s->d_holog = (double *)take(8 * H + 8);
    if (enc) {
        s->d_frow = (uint32_t *)take(4 * n + 4);
        s->d_fidx = (uint32_t *)take(4 * T + 4);
        s->d_fval = (float *)take(4 * T + 4);
        s->d_probs = (float *)take(4 * n * p.K);
        s->d_cdf_stage = (uint32_t *)take(4 * n * p.K);
        for (int x = 0; x < 2; ++x) {
            s->d_ah_frow[x] = (uint32_t *)take(4 * n + 4);
            s->d_ah_fidx[x] = (uint32_t *)take(4 * T + 4);
            s->d_ah_fval[x] = (float *)take(4 * T + 4);
            s->d_ah_cdf[x] = (uint32_t *)take(4 * n * p.K);
        }
        s->enc_st = (hipStream_t)wlda_encoder_get_stream(enc);
        s->buckets = wlda_encoder_get_buckets(enc);
        if (hipEventCreateWithFlags(&s->enc_ev[0], hipEventDisableTiming) ||
            hipEventCreateWithFlags(&s->enc_ev[1], hipEventDisableTiming) ||
            hipEventCreateWithFlags(&s->ah_done[0], hipEventDisableTiming) ||
            hipEventCreateWithFlags(&s->ah_done[1], hipEventDisableTiming) ||
            hipEventCreateWithFlags(&s->ah_copied, hipEventDisableTiming)) {
            for (hipEvent_t ev : {s->enc_ev[0], s->enc_ev[1], s->ah_done[0], s->ah_done[1], s->ah_copied})
                if (ev) (void)hipEventDestroy(ev);
            delete s;
            return WLDA_E_HIP;
        }
    }
    s->slots.resize(n);
    s->h_off.assign(n, 0);
    s->h_len.assign(n, 0);
    s->h_req.assign(n, 0);
    s->h_sweep.assign(n, 0);
    s->h_useq.assign(n, 0);
    s->h_hoff.assign(n, 0);
    s->h_hlen.assign(n, 0);
    s->pool.reset(T);
    s->ho_pool.reset(H);
    s->t0 = std::chrono::steady_clock::now();
    *out = s;
    return WLDA_OK;
}

wlda_status wlda_server_now(wlda_server s, double *t) {
    if (!s || !t) return WLDA_E_INVALID;
    *t = now_s(s);
    return WLDA_OK;
}

wlda_status wlda_server_submit(wlda_server s, uint32_t req_id, const uint32_t *words, uint32_t L,
                               const uint32_t *ho_words, uint32_t n_ho, double arrival_s,
                               const uint32_t *weights) {
    if (!s || L == 0 || !words || L > FOLD_MAX_TOKENS || L > s->sp.pool_tokens ||
        (n_ho && !ho_words) || n_ho > s->sp.pool_heldout)
        return WLDA_E_INVALID;
    const wlda_params &p = model_params(s->model);
    Pending q;
    q.req = req_id;
    q.words.assign(words, words + L);
    for (uint32_t w : q.words)
        if (w >= p.V) return WLDA_E_INVALID;
    if (n_ho) q.ho.assign(ho_words, ho_words + n_ho);
    for (uint32_t w : q.ho)
        if (w >= p.V) return WLDA_E_INVALID;
    if (weights) {
        q.weights.resize(s->K);
        uint64_t run = 0;
        for (uint32_t k = 0; k < s->K; ++k) {
            const uint32_t v = weights[k];
            if (v == 0 || v >= (1u << 24)) return WLDA_E_INVALID;
            run += v;
            q.weights[k] = (uint32_t)run;
        }
        if (run >= (1ull << 32)) return WLDA_E_INVALID;
    }
    q.arrival = arrival_s;
    s->pending.push_back(std::move(q));
    return WLDA_OK;
}

wlda_status wlda_server_step(wlda_server s, uint32_t *n_active, uint32_t *n_pending) {
    if (!s) return WLDA_E_INVALID;
    if (s->broken) return WLDA_E_HIP;
    const wlda_params &p = model_params(s->model);
    const uint32_t K = s->K, M = s->M;
    hipError_t e = hipSuccess;
    auto up = [&](void *dst, const void *src, uint64_t bytes, hipStream_t st) {
        if (!e && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
    };
    // ---- admission (arrival order; stop at the first request that does not fit)
    std::vector<uint32_t> fresh, fresh_enc;
    struct Ahead {
        uint32_t slot, stage, row;
    };
    std::vector<Ahead> ahead;               // admitted with a proposal encoded ahead
    std::vector<Pending> admitted;          // host copies stay alive until the sync below
    std::vector<uint32_t> f_rows(1, 0), f_idx;
    std::vector<float> f_val;
    const double t_admit = now_s(s);
    while (!s->pending.empty()) {
        Pending &q = s->pending.front();
        if (s->enc && q.weights.empty() && fresh_enc.size() >= wlda_encoder_get_max_batch(s->enc)) break;
        uint32_t si = 0;
        while (si < s->slots.size() && s->slots[si].busy) ++si;
        if (si == s->slots.size()) break;
        uint64_t off = 0, hoff = 0;
        if (!s->pool.alloc(q.words.size(), &off)) break;
        if (!s->ho_pool.alloc(q.ho.size(), &hoff)) {
            s->pool.release(off, q.words.size());
            break;
        }
        Slot &sl = s->slots[si];
        sl.busy = true;
        sl.req = q.req;
        sl.len = (uint32_t)q.words.size();
        sl.n_ho = (uint32_t)q.ho.size();
        sl.off = off;
        sl.ho_off = hoff;
        sl.sweep = 0;
        sl.arrival = q.arrival;
        sl.admit = t_admit;
        sl.learned = !q.weights.empty() || s->enc != nullptr;
        s->h_off[si] = (uint32_t)off;
        s->h_len[si] = sl.len;
        s->h_req[si] = sl.req;
        s->h_sweep[si] = 0;
        s->h_useq[si] = sl.learned ? 1u : 0u;
        s->h_hoff[si] = (uint32_t)hoff;
        s->h_hlen[si] = sl.n_ho;
        if (q.weights.empty() && s->enc && q.stage >= 0) {
            ahead.push_back({si, (uint32_t)q.stage, q.stage_row});
        } else if (q.weights.empty() && s->enc) {
            // encoder input of this document (hashed bag of words)
            const size_t base = f_idx.size();
            f_idx.resize(base + sl.len);
            f_val.resize(base + sl.len);
            uint32_t nnz = 0;
            wlda_encoder_features(s->buckets, q.words.data(), sl.len, f_idx.data() + base,
                                  f_val.data() + base, &nnz);
            f_idx.resize(base + nnz);
            f_val.resize(base + nnz);
            f_rows.push_back((uint32_t)f_idx.size());
            fresh_enc.push_back(si);
        }
        fresh.push_back(si);
        admitted.push_back(std::move(q));
        s->pending.pop_front();
    }
    // proposals encoded ahead: wait for their stage on the sweep stream, copy
    bool waited[2] = {false, false};
    for (const Ahead &ah : ahead) {
        if (!e && !waited[ah.stage]) {
            e = hipStreamWaitEvent(s->st, s->ah_done[ah.stage], 0);
            waited[ah.stage] = true;
        }
        if (!e)
            e = hipMemcpyAsync(s->d_qcdf + (size_t)ah.slot * K, s->d_ah_cdf[ah.stage] + (size_t)ah.row * K, 4ull * K,
                               hipMemcpyDeviceToDevice, s->st);
    }
    // a stage is rewritten below (encode-ahead, encoder stream) only after the
    // sweep stream has copied out the rows admitted from it
    const bool ah_read = !ahead.empty();
    if (!e && ah_read) e = hipEventRecord(s->ah_copied, s->st);
    for (size_t a = 0; a < admitted.size(); ++a) {
        const uint32_t si = fresh[a];
        const Slot &sl = s->slots[si];
        up(s->d_words + sl.off, admitted[a].words.data(), 4ull * sl.len, s->st);
        if (sl.n_ho) up(s->d_how + sl.ho_off, admitted[a].ho.data(), 4ull * sl.n_ho, s->st);
        if (!admitted[a].weights.empty())
            up(s->d_qcdf + (size_t)si * K, admitted[a].weights.data(), 4ull * K, s->st);
    }
    // per-slot tables for the launch
    // Documents encoded at admission start their sweeps at the next step: the
    // encoder then overlaps this step's sweep instead of holding up the new
    // documents of the step (their launch waits for it on the device).
    bool deferred_ready = false;
    if (!e && !s->deferred.empty()) {
        const hipError_t q = hipEventQuery(s->deferred_ev);
        if (q == hipSuccess)
            deferred_ready = true;
        else if (q != hipErrorNotReady)
            e = q;
    }
    std::vector<char> enc_now(s->slots.size(), 0);
    for (uint32_t si : fresh_enc) enc_now[si] = 1;
    if (!deferred_ready)
        for (uint32_t si : s->deferred) enc_now[si] = 1;
    std::vector<uint32_t> old_list, new_list;
    for (uint32_t si = 0; si < s->slots.size(); ++si)
        if (s->slots[si].busy && !enc_now[si]) (s->slots[si].sweep == 0 ? new_list : old_list).push_back(si);
    const uint64_t n = s->slots.size();
    // per-slot descriptors change only where documents were admitted: upload
    // the range of this step's admissions (a pageable copy costs several
    // microseconds of host time, most of a step's)
    if (!fresh.empty()) {
        const uint32_t lo = *std::min_element(fresh.begin(), fresh.end());
        const uint32_t hi = *std::max_element(fresh.begin(), fresh.end()) + 1;
        const uint64_t nb = 4ull * (hi - lo);
        up(s->d_off + lo, s->h_off.data() + lo, nb, s->st);
        up(s->d_len + lo, s->h_len.data() + lo, nb, s->st);
        up(s->d_req + lo, s->h_req.data() + lo, nb, s->st);
        up(s->d_useq + lo, s->h_useq.data() + lo, nb, s->st);
        up(s->d_hoff + lo, s->h_hoff.data() + lo, nb, s->st);
        up(s->d_hlen + lo, s->h_hlen.data() + lo, nb, s->st);
        // the device advances the sweep counters of active slots: only the
        // admitted ones are reset
        for (uint32_t si : fresh) up(s->d_sweep + si, &s->h_sweep[si], 4, s->st);
    }
    std::vector<uint32_t> lists(old_list);
    lists.insert(lists.end(), new_list.begin(), new_list.end());
    if (!s->lists_valid || lists != s->up_lists) {
        up(s->d_slots, lists.data(), 4ull * lists.size(), s->st);
        s->up_lists = lists;
        s->lists_valid = true;
    }
    // ---- encoder forward for newly admitted documents, on the encoder's
    // stream, overlapped with the sweep of the documents already in flight
    if (!e && !fresh_enc.empty()) {
        const uint32_t B = (uint32_t)fresh_enc.size();
        up(s->d_frow, f_rows.data(), 4ull * (B + 1), s->enc_st);
        up(s->d_fidx, f_idx.data(), 4ull * f_idx.size(), s->enc_st);
        up(s->d_fval, f_val.data(), 4ull * f_val.size(), s->enc_st);
        if (!e && (wlda_encoder_forward(s->enc, B, s->d_frow, s->d_fidx, s->d_fval, s->d_probs) != WLDA_OK ||
                   wlda_encoder_proposal(s->enc, B, s->d_probs, s->sp.eps, s->d_cdf_stage) != WLDA_OK))
            e = hipErrorLaunchFailure;
        for (uint32_t r = 0; r < B && !e; ++r)
            e = hipMemcpyAsync(s->d_qcdf + (size_t)fresh_enc[r] * K, s->d_cdf_stage + (size_t)r * K, 4ull * K,
                               hipMemcpyDeviceToDevice, s->enc_st);
        if (!e) e = hipEventRecord(s->enc_ev[s->enc_cur], s->enc_st);
    }
    // ---- encode ahead: the head of the queue, into the next stage buffer
    if (!e && s->enc) {
        const int x = s->ah_next;
        if (s->ah_live[x]) {        // its requests not admitted by now are encoded again later
            e = hipEventSynchronize(s->ah_done[x]);
            for (Pending &q : s->pending)
                if (q.stage == x) q.stage = -1;
            s->ah_live[x] = false;
        }
        const uint32_t bmax = std::min<uint32_t>(wlda_encoder_get_max_batch(s->enc), (uint32_t)s->slots.size());
        std::vector<uint32_t> &rows = s->h_ah_rows[x], &idx = s->h_ah_idx[x];
        std::vector<float> &val = s->h_ah_val[x];
        rows.assign(1, 0);
        idx.clear();
        val.clear();
        std::vector<Pending *> picked;
        for (Pending &q : s->pending) {
            if (picked.size() >= bmax) break;
            if (!q.weights.empty() || q.stage >= 0) continue;
            if (idx.size() + q.words.size() > s->sp.pool_tokens) break;
            const size_t base = idx.size();
            idx.resize(base + q.words.size());
            val.resize(base + q.words.size());
            uint32_t nnz = 0;
            wlda_encoder_features(s->buckets, q.words.data(), (uint32_t)q.words.size(), idx.data() + base,
                                  val.data() + base, &nnz);
            idx.resize(base + nnz);
            val.resize(base + nnz);
            rows.push_back((uint32_t)idx.size());
            picked.push_back(&q);
        }
        if (!e && !picked.empty()) {
            const uint32_t B = (uint32_t)picked.size();
            if (ah_read) e = hipStreamWaitEvent(s->enc_st, s->ah_copied, 0);
            up(s->d_ah_frow[x], rows.data(), 4ull * (B + 1), s->enc_st);
            up(s->d_ah_fidx[x], idx.data(), 4ull * idx.size(), s->enc_st);
            up(s->d_ah_fval[x], val.data(), 4ull * val.size(), s->enc_st);
            if (!e && (wlda_encoder_forward(s->enc, B, s->d_ah_frow[x], s->d_ah_fidx[x], s->d_ah_fval[x],
                                            s->d_probs) != WLDA_OK ||
                       wlda_encoder_proposal(s->enc, B, s->d_probs, s->sp.eps, s->d_ah_cdf[x]) != WLDA_OK))
                e = hipErrorLaunchFailure;
            if (!e) e = hipEventRecord(s->ah_done[x], s->enc_st);
            if (!e) {
                for (uint32_t r = 0; r < B; ++r) {
                    picked[r]->stage = x;
                    picked[r]->stage_row = r;
                }
                s->ah_live[x] = true;
                s->ah_next = 1 - x;
            }
        }
    }
    if (e) return fail(s);
    // ---- one sweep for every admitted document
    FoldBatch b{};
    b.slots = s->d_slots;
    b.off = s->d_off;
    b.len = s->d_len;
    b.req = s->d_req;
    b.sweep = s->d_sweep;
    b.words = s->d_words;
    b.z = s->d_z;
    b.pd = s->d_pd;
    b.pw = s->d_pw;
    b.cap = (uint32_t)s->sp.pool_tokens;
    b.qcdf = s->d_qcdf;
    b.use_q = s->d_useq;
    b.learned_steps = s->sp.learned_steps;
    b.max_sweep = 0xFFFFFFFFu;
    const FoldModel &fm = model_internal(s->model);
    b.n = (uint32_t)old_list.size();
    if (!e) e = fold_launch(fm, b, s->st);
    if (!e && !new_list.empty()) {
        FoldBatch bn = b;
        bn.slots = s->d_slots + old_list.size();
        bn.n = (uint32_t)new_list.size();
        if (!e) e = fold_launch(fm, bn, s->st);
    }
    for (uint32_t si : old_list) s->slots[si].sweep++;
    for (uint32_t si : new_list) s->slots[si].sweep++;
    if (deferred_ready) s->deferred.clear();
    if (!fresh_enc.empty()) {
        s->deferred.insert(s->deferred.end(), fresh_enc.begin(), fresh_enc.end());
        s->deferred_ev = s->enc_ev[s->enc_cur];
        s->enc_cur = 1 - s->enc_cur;
    }
    // ---- retire documents that have had init + `sweeps` sweeps
    std::vector<uint32_t> retire;
    for (uint32_t si : lists)
        if (s->slots[si].sweep >= s->sp.sweeps + 1) retire.push_back(si);
    std::vector<std::vector<uint32_t>> zs(retire.size());
    std::vector<double> ho(n, 0.0);
    if (!e && !retire.empty()) {
        FoldBatch br = b;
        up(s->d_slots, retire.data(), 4ull * retire.size(), s->st);
        s->lists_valid = false;
        br.n = (uint32_t)retire.size();
        std::vector<uint32_t> hchunk(retire.size() + 1, 0);
        for (size_t r = 0; r < retire.size(); ++r)
            hchunk[r + 1] = hchunk[r] + heldout_chunks(s->slots[retire[r]].n_ho);
        up(s->d_hchunk, hchunk.data(), 4ull * hchunk.size(), s->st);
        if (!e)
            e = fold_heldout(fm, br, s->d_hoff, s->d_hlen, s->d_how, s->d_hchunk, hchunk.back(), s->d_holog,
                             p.alpha, p.beta, s->d_out, s->st);
        for (size_t r = 0; r < retire.size() && !e; ++r) {
            const Slot &sl = s->slots[retire[r]];
            zs[r].resize(sl.len);
            e = hipMemcpyAsync(zs[r].data(), s->d_z + sl.off, 4ull * sl.len, hipMemcpyDeviceToHost, s->st);
        }
        if (!e) e = hipMemcpyAsync(ho.data(), s->d_out, 8 * n, hipMemcpyDeviceToHost, s->st);
    }
    if (!e) e = hipStreamSynchronize(s->st);
    if (e) return fail(s);
    const double t_done = now_s(s);
    for (size_t r = 0; r < retire.size(); ++r) {
        Slot &sl = s->slots[retire[r]];
        wlda_result res{};
        res.req_id = sl.req;
        res.n_tokens = sl.len;
        res.n_heldout = sl.n_ho;
        res.sweeps = s->sp.sweeps;
        res.arrival_s = sl.arrival;
        res.admit_s = sl.admit;
        res.done_s = t_done;
        res.heldout_ll = ho[retire[r]];
        res.learned = sl.learned ? 1 : 0;
        s->done.push_back(res);
        std::vector<int32_t> z(sl.len);
        for (uint32_t t = 0; t < sl.len; ++t) z[t] = (int32_t)zs[r][t];
        s->done_z[sl.req] = std::move(z);
        s->pool.release(sl.off, sl.len);
        s->ho_pool.release(sl.ho_off, sl.n_ho);
        sl.busy = false;
        s->h_len[retire[r]] = 0;
    }
    uint32_t act = 0;
    for (auto &sl : s->slots) act += sl.busy;
    if (n_active) *n_active = act;
    if (n_pending) *n_pending = (uint32_t)s->pending.size();
    (void)M;
    return WLDA_OK;
}

wlda_status wlda_server_poll(wlda_server s, wlda_result *out, uint32_t max, uint32_t *n) {
    if (!s || !n || (max && !out)) return WLDA_E_INVALID;
    const uint32_t k = (uint32_t)std::min<size_t>(max, s->done.size());
    for (uint32_t i = 0; i < k; ++i) out[i] = s->done[i];
    s->done.erase(s->done.begin(), s->done.begin() + k);
    *n = k;
    return WLDA_OK;
}

wlda_status wlda_server_take_z(wlda_server s, uint32_t req_id, int32_t *z, uint32_t L) {
    if (!s || !z) return WLDA_E_INVALID;
    auto it = s->done_z.find(req_id);
    if (it == s->done_z.end() || it->second.size() != L) return WLDA_E_INVALID;
    std::memcpy(z, it->second.data(), 4ull * L);
    s->done_z.erase(it);
    return WLDA_OK;
}

wlda_status wlda_server_destroy(wlda_server s) {
    if (!s) return WLDA_E_INVALID;
    if (!s->broken) (void)hipStreamSynchronize(s->st);
    for (hipEvent_t ev : s->enc_ev)
        if (ev) (void)hipEventDestroy(ev);
    if (s->ah_copied) (void)hipEventDestroy(s->ah_copied);
    for (hipEvent_t ev : s->ah_done)
        if (ev) (void)hipEventDestroy(ev);
    delete s;
    return WLDA_OK;
}

}  // extern "C"
