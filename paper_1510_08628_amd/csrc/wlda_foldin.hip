// Fold-in of new documents against a frozen model (gfx950).
//
// The E-step of the paper's MCEM algorithm (Eq. 5) run on new documents with
// the word-topic counts C_w and the topic totals c_k held at a trained
// model's values: per document, sweep by sweep,
//   word step - pending doc proposals judged with pi_doc of Eq. (7) against
//               the frozen C_w and c_k, then M word proposals by random
//               positioning over the word's trained column (Section 4.3);
//   doc step  - c_d rebuilt from the document (delayed update), the word
//               proposals judged with pi_word, then (learned mode) further MH
//               steps with an independence proposal given as integer weights,
//               then M doc proposals drawn from the updated document.
// One workgroup per document of a ragged batch; each document carries its
// own sweep counter and request id, so its result does not depend on which
// other documents share the launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/warplda.h"
#include "wlda_device.h"
#include "wlda_fold.h"

namespace wlda {

enum FoldPhase : uint32_t { PH_F_INIT = 5, PH_F_WORD = 6, PH_F_DOC = 8, PH_F_LEARN = 9 };

__device__ __forceinline__ uint32_t cdf_draw(const uint32_t *cdf, uint32_t K, uint32_t r) {
    const uint32_t total = cdf[K - 1];
    const uint32_t u = (uint32_t)(((uint64_t)r * total) >> 32);
    uint32_t lo = 0, hi = K - 1;   // first k with cdf[k] > u
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (cdf[mid] > u)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

template <typename ZT>
__global__ __launch_bounds__(256) void fold_sweep_kernel(FoldModel m, FoldBatch b) {
    extern __shared__ uint32_t lds[];
    const uint32_t K = m.K, M = m.M;
    const uint32_t slot = b.slots[blockIdx.x];
    const uint32_t off = b.off[slot], L = b.len[slot], req = b.req[slot];
    const uint32_t s = b.sweep[slot];
    if (s > b.max_sweep || L == 0) return;
    uint32_t *zs = lds;                 // L
    uint32_t *cd = lds + FOLD_MAX_TOKENS;   // K
    uint32_t *qs = cd + K;              // K: the learned CDF staged in LDS (K <= FOLD_Q_LDS_MAX)
    const ZT *zc = reinterpret_cast<const ZT *>(m.zcsc);
    const uint32_t *qcdf =
        b.qcdf && (!b.use_q || b.use_q[slot]) ? b.qcdf + (size_t)slot * K : nullptr;
    const uint32_t cap = b.cap;
    const bool q_lds = qcdf && K <= FOLD_Q_LDS_MAX;
    if (q_lds) {
        for (uint32_t k = threadIdx.x; k < K; k += 256) qs[k] = qcdf[k];
        __syncthreads();
    }
    // The learned independence steps of one token (Alg. 1 with target Eq. 5
    // and proposal q): q read from LDS or global memory through a pointer of
    // known address space.
    auto learned = [&](const uint32_t *q, uint32_t n, uint32_t x) {
        const uint32_t w = b.words[off + n];
        const uint32_t *cw = m.cwk + (size_t)w * K;
        for (uint32_t j = 1; j <= b.learned_steps; ++j) {
            const uint4 R = philox(n, s, (PH_F_LEARN << 16) | j, req, m.seed_lo, m.seed_hi);
            const uint32_t t = cdf_draw(q, K, R.z);
            const float wx = (float)(q[x] - (x ? q[x - 1] : 0u));
            const float wt = (float)(q[t] - (t ? q[t - 1] : 0u));
            const float num = ((float)cd[t] + m.a) * ((float)cw[t] + m.b) * ((float)m.ck[x] + m.beta_bar) * wx;
            const float den = ((float)cd[x] + m.a) * ((float)cw[x] + m.b) * ((float)m.ck[t] + m.beta_bar) * wt;
            if (unif24(R.x) * den < num) x = t;
        }
        return x;
    };

    if (s == 0) {
        for (uint32_t n = threadIdx.x; n < L; n += 256) {
            const uint4 R = philox(n, 0, PH_F_INIT << 16, req, m.seed_lo, m.seed_hi);
            zs[n] = q_lds ? cdf_draw(qs, K, R.z) : qcdf ? cdf_draw(qcdf, K, R.z) : dice(R.z, K);
        }
        __syncthreads();
    } else {
        // word step: frozen C_w and c_k
        for (uint32_t n = threadIdx.x; n < L; n += 256) {
            const uint32_t w = b.words[off + n];
            const uint32_t cb = m.colptr[w], Lw = m.colptr[w + 1] - cb;
            const uint32_t *cw = m.cwk + (size_t)w * K;
            uint32_t x = b.z[off + n];
            for (uint32_t i = 1; i <= M; ++i) {
                const uint4 R = philox(n, s, (PH_F_WORD << 16) | i, req, m.seed_lo, m.seed_hi);
                const uint32_t c = b.pd[(size_t)(i - 1) * cap + off + n];
                if (mh_accept(unif24(R.x), cw[c], cw[x], m.b, m.ck[x], m.ck[c], m.beta_bar)) x = c;
                b.pw[(size_t)(i - 1) * cap + off + n] =
                    take_count_part(unif24(R.y), Lw, m.beta_k) ? (uint32_t)zc[cb + dice(R.z, Lw)] : dice(R.z, K);
            }
            zs[n] = x;
        }
        for (uint32_t k = threadIdx.x; k < K; k += 256) cd[k] = 0;
        __syncthreads();
        for (uint32_t n = threadIdx.x; n < L; n += 256) atomicAdd(&cd[zs[n]], 1u);
        __syncthreads();
        // doc step: word proposals, then learned steps, with c_d frozen (each
        // thread reads and rewrites only its own tokens of zs here)
        for (uint32_t n = threadIdx.x; n < L; n += 256) {
            uint32_t x = zs[n];
            for (uint32_t i = 1; i <= M; ++i) {
                const uint4 R = philox(n, s, (PH_F_DOC << 16) | i, req, m.seed_lo, m.seed_hi);
                const uint32_t c = b.pw[(size_t)(i - 1) * cap + off + n];
                if (mh_accept(unif24(R.x), cd[c], cd[x], m.a, m.ck[x], m.ck[c], m.beta_bar)) x = c;
            }
            if (q_lds)
                x = learned(qs, n, x);
            else if (qcdf)
                x = learned(qcdf, n, x);
            zs[n] = x;
        }
        __syncthreads();
    }
    // doc proposals from the updated document; publish z
    for (uint32_t n = threadIdx.x; n < L; n += 256) {
        for (uint32_t i = 1; i <= M; ++i) {
            const uint4 R = philox(n, s, (PH_F_DOC << 16) | i, req, m.seed_lo, m.seed_hi);
            b.pd[(size_t)(i - 1) * cap + off + n] =
                take_count_part(unif24(R.y), L, m.alpha_bar) ? zs[dice(R.z, L)] : dice(R.z, K);
        }
        b.z[off + n] = zs[n];
    }
    if (threadIdx.x == 0) b.sweep[slot] = s + 1;
}

// Held-out log likelihood by document completion (binary64): theta from the
// document's assignments, phi from the frozen counts (Eq. 4, alpha' = alpha+1,
// beta' = beta+1); out[d] = sum over held-out tokens of log sum_k theta phi.
// Two kernels: heldout_word_kernel takes blocks of HO_CHUNK held-out words of
// one document (hchunk: prefix sums of the documents' block counts) and
// writes log p(w | d) of each word to ho_log (indexed like ho_words);
// heldout_sum_kernel adds each document's words in a fixed order.  So a
// document's result does not depend on which others share the launch, and
// many blocks keep the row loads of C_w in flight at once.
// theta_k / (c_k + beta_bar) of the document is staged in LDS (binary64) up
// to this K; each held-out word then costs one dot product with its row of C_w.
constexpr uint32_t HELDOUT_LDS_MAX = 8192;
constexpr uint32_t HO_CHUNK = 16;

__global__ __launch_bounds__(256) void heldout_word_kernel(FoldModel m, FoldBatch b, const uint32_t *ho_off,
                                                           const uint32_t *ho_len, const uint32_t *ho_words,
                                                           const uint32_t *hchunk, double a, double beta,
                                                           double *ho_log) {
    extern __shared__ uint32_t cnt[];   // K counts, then (K <= HELDOUT_LDS_MAX) K doubles
    const uint32_t K = m.K;
    // the document of this block: the last i with hchunk[i] <= blockIdx.x
    uint32_t lo = 0, hi = b.n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (hchunk[mid] <= blockIdx.x)
            lo = mid;
        else
            hi = mid;
    }
    const uint32_t slot = b.slots[lo];
    const uint32_t h0 = (blockIdx.x - hchunk[lo]) * HO_CHUNK, h1 = min(ho_len[slot], h0 + HO_CHUNK);
    const uint32_t off = b.off[slot], L = b.len[slot];
    for (uint32_t k = threadIdx.x; k < K; k += 256) cnt[k] = 0;
    __syncthreads();
    for (uint32_t n = threadIdx.x; n < L; n += 256) atomicAdd(&cnt[b.z[off + n]], 1u);
    __syncthreads();
    const double denom_d = (double)L + K * a, bbar = m.V * beta;
    const bool staged = K <= HELDOUT_LDS_MAX;
    double *tk = reinterpret_cast<double *>(cnt + ((K + 1) & ~1u));   // 8-byte aligned
    if (staged) {
        for (uint32_t k = threadIdx.x; k < K; k += 256)
            tk[k] = ((double)cnt[k] + a) / denom_d / ((double)m.ck[k] + bbar);
        __syncthreads();
    }
    // one wavefront per held-out word: p_h = sum_k theta_k phi_k(w) (Eq. 4),
    // four row loads per lane in flight, then a wavefront-wide sum
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (uint32_t h = h0 + wave; h < h1; h += 4) {
        const uint32_t w = ho_words[ho_off[slot] + h];
        const uint32_t *cw = m.cwk + (size_t)w * K;
        double p[4] = {0, 0, 0, 0};
        uint32_t k = lane;
        if (staged) {
            for (; k + 192 < K; k += 256) {
                const uint32_t c0 = cw[k], c1 = cw[k + 64], c2 = cw[k + 128], c3 = cw[k + 192];
                p[0] += tk[k] * ((double)c0 + beta);
                p[1] += tk[k + 64] * ((double)c1 + beta);
                p[2] += tk[k + 128] * ((double)c2 + beta);
                p[3] += tk[k + 192] * ((double)c3 + beta);
            }
            for (; k < K; k += 64) p[0] += tk[k] * ((double)cw[k] + beta);
        } else {
            for (; k < K; k += 64)
                p[0] += ((double)cnt[k] + a) / denom_d * (((double)cw[k] + beta) / ((double)m.ck[k] + bbar));
        }
        double q = (p[0] + p[1]) + (p[2] + p[3]);
        for (int o = 32; o > 0; o >>= 1) q += __shfl_down(q, o, 64);
        if (lane == 0) ho_log[ho_off[slot] + h] = log(q);
    }
}

__global__ __launch_bounds__(256) void heldout_sum_kernel(FoldBatch b, const uint32_t *ho_off,
                                                          const uint32_t *ho_len, const double *ho_log,
                                                          double *out) {
    __shared__ double part[4];
    const uint32_t slot = b.slots[blockIdx.x];
    const double *x = ho_log + ho_off[slot];
    double t = 0;
    for (uint32_t h = threadIdx.x; h < ho_len[slot]; h += 256) t += x[h];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_down(t, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) out[slot] = (part[0] + part[1]) + (part[2] + part[3]);
}

// Frozen counts of a model: C_wk and c_k from the canonical assignments.
__global__ void model_counts_kernel(const uint32_t *colptr, uint32_t V, const uint32_t *z, uint32_t K,
                                    uint32_t *cwk, uint32_t *ck) {
    for (uint32_t w = blockIdx.x; w < V; w += gridDim.x)
        for (uint32_t t = colptr[w] + threadIdx.x; t < colptr[w + 1]; t += 256) {
            atomicAdd(&cwk[(size_t)w * K + z[t]], 1u);
            atomicAdd(&ck[z[t]], 1u);
        }
}

template <typename ZT>
__global__ void compact_kernel(const uint32_t *z, uint64_t T, ZT *out) {
    for (uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x; t < T; t += (uint64_t)gridDim.x * 256)
        out[t] = (ZT)z[t];
}

}  // namespace wlda

using namespace wlda;

// ============================================================================
// Host side
// ============================================================================
namespace {
constexpr uint64_t FALIGN = 256;
inline uint64_t fa(uint64_t x) { return (x + FALIGN - 1) / FALIGN * FALIGN; }
inline uint8_t *fcarve(uint8_t *&cur, uint64_t bytes) {
    uint8_t *p = cur;
    cur += fa(bytes);
    return p;
}
}  // namespace

struct wlda_model_s {
    FoldModel m{};
    wlda_params p{};
    hipStream_t st = nullptr;
    uint64_t T = 0;
    int dev = -1;             // device current at create (the workspace's)
};

namespace {

uint64_t model_bytes(const wlda_params &p, uint64_t T) {
    const uint64_t zc = p.K <= 65535 ? 2 : 4;
    return fa(4ull * (p.V + 1)) + fa(zc * T + 4) + fa(4ull * p.V * p.K) + fa(4ull * p.K) + fa(4ull * T + 4);
}

hipError_t launch_fold(const FoldModel &m, const FoldBatch &b, hipStream_t st) {
    if (b.n == 0) return hipSuccess;
    const size_t lds = 4ull * (FOLD_MAX_TOKENS + m.K + (b.qcdf && m.K <= FOLD_Q_LDS_MAX ? m.K : 0));
    if (m.zc16) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fold_sweep_kernel<uint16_t>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(fold_sweep_kernel<uint16_t>, dim3(b.n), dim3(256), lds, st, m, b);
    } else {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fold_sweep_kernel<uint32_t>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(fold_sweep_kernel<uint32_t>, dim3(b.n), dim3(256), lds, st, m, b);
    }
    return hipGetLastError();
}

hipError_t launch_heldout(const FoldModel &m, const FoldBatch &b, const uint32_t *ho_off,
                          const uint32_t *ho_len, const uint32_t *ho_words, const uint32_t *hchunk,
                          uint32_t n_chunks, double *ho_log, double alpha, double beta, double *out,
                          hipStream_t st) {
    if (b.n == 0) return hipSuccess;
    if (n_chunks) {
        const size_t lds = 4ull * ((m.K + 1) & ~1u) + (m.K <= HELDOUT_LDS_MAX ? 8ull * m.K : 0);
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(heldout_word_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(heldout_word_kernel, dim3(n_chunks), dim3(256), lds, st, m, b, ho_off, ho_len, ho_words,
                           hchunk, alpha, beta, ho_log);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(heldout_sum_kernel, dim3(b.n), dim3(256), 0, st, b, ho_off, ho_len, ho_log, out);
    return hipGetLastError();
}

}  // namespace

// exported for the server (wlda_server.hip)
namespace wlda {
const FoldModel &model_internal(wlda_model m) { return m->m; }
const wlda_params &model_params(wlda_model m) { return m->p; }
hipError_t fold_launch(const FoldModel &m, const FoldBatch &b, hipStream_t st) { return launch_fold(m, b, st); }
hipError_t fold_heldout(const FoldModel &m, const FoldBatch &b, const uint32_t *ho_off,
                        const uint32_t *ho_len, const uint32_t *ho_words, const uint32_t *hchunk,
                        uint32_t n_chunks, double *ho_log, double alpha, double beta, double *out,
                        hipStream_t st) {
    return launch_heldout(m, b, ho_off, ho_len, ho_words, hchunk, n_chunks, ho_log, alpha, beta, out, st);
}

uint32_t heldout_chunks(uint32_t n_heldout) { return (n_heldout + HO_CHUNK - 1) / HO_CHUNK; }
}  // namespace wlda

extern "C" {

wlda_status wlda_model_workspace_bytes(const wlda_params *p, uint64_t n_tokens, uint64_t *bytes) {
    if (!p || !bytes || p->K < 1 || p->K > MAX_K || p->V < 1 || p->M < 1 || p->M > 4 ||
        n_tokens >= (1ull << 32))
        return WLDA_E_INVALID;
    if ((uint64_t)p->V * p->K > (8ull << 30)) return WLDA_E_UNSUPPORTED;   // dense C_w limit
    *bytes = model_bytes(*p, n_tokens);
    return WLDA_OK;
}

wlda_status wlda_model_create(const wlda_params *p, const uint32_t *word_ids, const uint32_t *doc_ids,
                              const int32_t *z, uint64_t T, void *ws, uint64_t ws_bytes, void *stream,
                              wlda_model *out) {
    if (!out) return WLDA_E_INVALID;
    *out = nullptr;
    uint64_t need = 0;
    wlda_status st = wlda_model_workspace_bytes(p, T, &need);
    if (st != WLDA_OK) return st;
    if (!(p->alpha > 0) || !(p->beta > 0) || (T && (!word_ids || !doc_ids || !z)))
        return WLDA_E_INVALID;
    if (!ws || ((uintptr_t)ws % FALIGN) || ws_bytes < need) return WLDA_E_WORKSPACE;
    for (uint64_t i = 0; i < T; ++i)
        if (word_ids[i] >= p->V || doc_ids[i] >= p->D || (uint32_t)z[i] >= p->K) return WLDA_E_INVALID;
    wlda_model m = new (std::nothrow) wlda_model_s();
    if (!m) return WLDA_E_INVALID;
    m->p = *p;
    m->T = T;
    m->st = (hipStream_t)stream;
    if (hipGetDevice(&m->dev) != hipSuccess) {
        delete m;
        return WLDA_E_HIP;
    }
    // canonical column order: stable by (word, doc, input index)
    std::vector<uint32_t> colptr(p->V + 1, 0), dcnt(p->D + 1, 0);
    for (uint64_t i = 0; i < T; ++i) {
        colptr[word_ids[i] + 1]++;
        dcnt[doc_ids[i] + 1]++;
    }
    for (uint32_t w = 0; w < p->V; ++w) colptr[w + 1] += colptr[w];
    for (uint32_t d = 0; d < p->D; ++d) dcnt[d + 1] += dcnt[d];
    std::vector<uint32_t> by_doc(T), zc(T);
    for (uint64_t i = 0; i < T; ++i) by_doc[dcnt[doc_ids[i]]++] = (uint32_t)i;
    std::vector<uint32_t> cur(colptr.begin(), colptr.end() - 1);
    for (uint64_t j = 0; j < T; ++j) {
        const uint32_t i = by_doc[j];
        zc[cur[word_ids[i]]++] = (uint32_t)z[i];
    }
    uint8_t *c = (uint8_t *)ws;
    uint32_t *d_colptr = (uint32_t *)fcarve(c, 4ull * (p->V + 1));
    void *d_zc = fcarve(c, (p->K <= 65535 ? 2ull : 4ull) * T + 4);
    uint32_t *d_cwk = (uint32_t *)fcarve(c, 4ull * p->V * p->K);
    uint32_t *d_ck = (uint32_t *)fcarve(c, 4ull * p->K);
    uint32_t *d_z32 = (uint32_t *)fcarve(c, 4ull * T + 4);
    hipError_t e = hipSuccess;
    hipStream_t s = m->st;
    if (!e) e = hipMemcpyAsync(d_colptr, colptr.data(), 4ull * (p->V + 1), hipMemcpyHostToDevice, s);
    if (!e && T) e = hipMemcpyAsync(d_z32, zc.data(), 4ull * T, hipMemcpyHostToDevice, s);
    if (!e) e = launch_fill_u32(d_cwk, 0, (uint64_t)p->V * p->K, s);
    if (!e) e = launch_fill_u32(d_ck, 0, p->K, s);
    if (!e) {
        hipLaunchKernelGGL(model_counts_kernel, dim3(std::min<uint32_t>(p->V, 65535)), dim3(256), 0, s,
                           d_colptr, p->V, d_z32, p->K, d_cwk, d_ck);
        e = hipGetLastError();
    }
    if (!e && T) {
        const int g = (int)std::min<uint64_t>((T + 255) / 256, 8192);
        if (p->K <= 65535)
            hipLaunchKernelGGL(compact_kernel<uint16_t>, dim3(g), dim3(256), 0, s, d_z32, T, (uint16_t *)d_zc);
        else
            hipLaunchKernelGGL(compact_kernel<uint32_t>, dim3(g), dim3(256), 0, s, d_z32, T, (uint32_t *)d_zc);
        e = hipGetLastError();
    }
    if (!e) e = hipStreamSynchronize(s);
    if (e) {
        delete m;
        return WLDA_E_HIP;
    }
    FoldModel &fm = m->m;
    fm.colptr = d_colptr;
    fm.zcsc = d_zc;
    fm.cwk = d_cwk;
    fm.ck = d_ck;
    fm.V = p->V;
    fm.K = p->K;
    fm.M = p->M;
    fm.zc16 = p->K <= 65535;
    fm.a = (float)p->alpha;
    fm.b = (float)p->beta;
    fm.alpha_bar = (float)p->K * fm.a;
    fm.beta_k = (float)p->K * fm.b;
    fm.beta_bar = (float)p->V * fm.b;
    fm.seed_lo = (uint32_t)p->seed;
    fm.seed_hi = (uint32_t)(p->seed >> 32);
    *out = m;
    return WLDA_OK;
}

static uint64_t batch_bytes(const wlda_params &p, uint32_t n, uint64_t T, bool learned, uint64_t n_ho) {
    return 5 * fa(4ull * n + 4) + 2 * fa(4ull * n + 4) + fa(4ull * T + 4) * (2 + 2ull * p.M) +
           (learned ? fa(4ull * n * p.K) : 0) + fa(4ull * n_ho + 4) + fa(8ull * n + 8) + fa(4ull * n + 8) +
           fa(8ull * n_ho + 8);
}

wlda_status wlda_foldin_batch_bytes(wlda_model m, uint32_t n_docs, uint64_t n_tokens, int learned,
                                    uint64_t n_heldout, uint64_t *bytes) {
    if (!m || !bytes || n_tokens >= (1ull << 32)) return WLDA_E_INVALID;
    *bytes = batch_bytes(m->p, n_docs, n_tokens, learned != 0, n_heldout);
    return WLDA_OK;
}

wlda_status wlda_foldin_batch(wlda_model m, uint32_t n_docs, const uint64_t *docptr, const uint32_t *words,
                              const uint32_t *req_ids, const uint32_t *learned_weights,
                              uint32_t learned_steps, uint32_t sweeps, const uint64_t *hoptr,
                              const uint32_t *ho_words, void *ws, uint64_t ws_bytes, int32_t *z_out,
                              double *heldout_out) {
    if (!m || !docptr || !req_ids || !z_out || (n_docs && !words)) return WLDA_E_INVALID;
    const wlda_params &p = m->p;
    const uint32_t K = p.K, M = p.M;
    const uint64_t T = docptr[n_docs];
    if (T >= (1ull << 32)) return WLDA_E_INVALID;
    const uint64_t n_ho = hoptr ? hoptr[n_docs] : 0;
    if (ws_bytes < batch_bytes(p, n_docs, T, learned_weights != nullptr, n_ho) || !ws ||
        ((uintptr_t)ws % FALIGN))
        return WLDA_E_WORKSPACE;
    std::vector<uint32_t> slots(n_docs), off(n_docs), len(n_docs), sweep(n_docs, 0), ho_off(n_docs),
        ho_len(n_docs);
    for (uint32_t d = 0; d < n_docs; ++d) {
        if (docptr[d + 1] < docptr[d]) return WLDA_E_INVALID;
        slots[d] = d;
        off[d] = (uint32_t)docptr[d];
        len[d] = (uint32_t)(docptr[d + 1] - docptr[d]);
        if (len[d] > FOLD_MAX_TOKENS) return WLDA_E_UNSUPPORTED;
        if (hoptr) {
            ho_off[d] = (uint32_t)hoptr[d];
            ho_len[d] = (uint32_t)(hoptr[d + 1] - hoptr[d]);
        }
    }
    for (uint64_t t = 0; t < T; ++t)
        if (words[t] >= p.V) return WLDA_E_INVALID;
    for (uint64_t h = 0; h < n_ho; ++h)
        if (ho_words[h] >= p.V) return WLDA_E_INVALID;
    std::vector<uint32_t> cdf;
    if (learned_weights) {
        cdf.resize((size_t)n_docs * K);
        for (uint32_t d = 0; d < n_docs; ++d) {
            uint64_t run = 0;
            for (uint32_t k = 0; k < K; ++k) {
                run += learned_weights[(size_t)d * K + k];
                if (learned_weights[(size_t)d * K + k] == 0 || run >= (1ull << 32) ||
                    learned_weights[(size_t)d * K + k] >= (1u << 24))
                    return WLDA_E_INVALID;
                cdf[(size_t)d * K + k] = (uint32_t)run;
            }
        }
    }
    uint8_t *c = (uint8_t *)ws;
    uint32_t *d_slots = (uint32_t *)fcarve(c, 4ull * n_docs + 4);
    uint32_t *d_off = (uint32_t *)fcarve(c, 4ull * n_docs + 4);
    uint32_t *d_len = (uint32_t *)fcarve(c, 4ull * n_docs + 4);
    uint32_t *d_req = (uint32_t *)fcarve(c, 4ull * n_docs + 4);
    uint32_t *d_sweep = (uint32_t *)fcarve(c, 4ull * n_docs + 4);
    uint32_t *d_hoff = (uint32_t *)fcarve(c, 4ull * n_docs + 4);
    uint32_t *d_hlen = (uint32_t *)fcarve(c, 4ull * n_docs + 4);
    uint32_t *d_words = (uint32_t *)fcarve(c, 4ull * T + 4);
    uint32_t *d_z = (uint32_t *)fcarve(c, 4ull * T + 4);
    uint32_t *d_pd = (uint32_t *)fcarve(c, 4ull * T * M + 4);
    uint32_t *d_pw = (uint32_t *)fcarve(c, 4ull * T * M + 4);
    uint32_t *d_cdf = learned_weights ? (uint32_t *)fcarve(c, 4ull * n_docs * K) : nullptr;
    uint32_t *d_how = (uint32_t *)fcarve(c, 4ull * n_ho + 4);
    double *d_out = (double *)fcarve(c, 8ull * n_docs + 8);
    uint32_t *d_hchunk = (uint32_t *)fcarve(c, 4ull * n_docs + 8);
    double *d_holog = (double *)fcarve(c, 8ull * n_ho + 8);
    std::vector<uint32_t> hchunk(n_docs + 1, 0);
    for (uint32_t d = 0; d < n_docs; ++d) hchunk[d + 1] = hchunk[d] + heldout_chunks(ho_len[d]);
    hipStream_t st = m->st;
    hipError_t e = hipSuccess;
    auto up = [&](void *dst, const void *src, uint64_t bytes) {
        if (!e && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
    };
    up(d_slots, slots.data(), 4ull * n_docs);
    up(d_off, off.data(), 4ull * n_docs);
    up(d_len, len.data(), 4ull * n_docs);
    up(d_req, req_ids, 4ull * n_docs);
    up(d_sweep, sweep.data(), 4ull * n_docs);
    up(d_hoff, ho_off.data(), 4ull * n_docs);
    up(d_hlen, ho_len.data(), 4ull * n_docs);
    up(d_words, words, 4ull * T);
    if (learned_weights) up(d_cdf, cdf.data(), 4ull * n_docs * K);
    if (hoptr) up(d_hchunk, hchunk.data(), 4ull * (n_docs + 1));
    if (n_ho) up(d_how, ho_words, 4ull * n_ho);
    FoldBatch b{};
    b.n = n_docs;
    b.slots = d_slots;
    b.off = d_off;
    b.len = d_len;
    b.req = d_req;
    b.sweep = d_sweep;
    b.words = d_words;
    b.z = d_z;
    b.pd = d_pd;
    b.pw = d_pw;
    b.cap = (uint32_t)T;
    b.qcdf = d_cdf;
    b.learned_steps = learned_weights ? learned_steps : 0;
    b.max_sweep = 0xFFFFFFFFu;
    for (uint32_t s = 0; s <= sweeps && !e; ++s) e = launch_fold(m->m, b, st);
    if (!e && heldout_out && hoptr)
        e = launch_heldout(m->m, b, d_hoff, d_hlen, d_how, d_hchunk, hchunk[n_docs], d_holog, p.alpha, p.beta,
                           d_out, st);
    std::vector<uint32_t> zh(T);
    if (!e && T) e = hipMemcpyAsync(zh.data(), d_z, 4ull * T, hipMemcpyDeviceToHost, st);
    if (!e && heldout_out && hoptr)
        e = hipMemcpyAsync(heldout_out, d_out, 8ull * n_docs, hipMemcpyDeviceToHost, st);
    if (!e) e = hipStreamSynchronize(st);
    if (e) return WLDA_E_HIP;
    for (uint64_t t = 0; t < T; ++t) z_out[t] = (int32_t)zh[t];
    return WLDA_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free fold-in: the same batch, its device buffers carved out of a
// file-scope device array instead of a caller's workspace.  Each GPU the
// library runs on holds its own copy of the array (WLDA_FOLDIN_STATIC_BYTES)
// until the process ends; in host code the array's name is only a stand-in,
// so its device address is looked up once per device and kept.
// ---------------------------------------------------------------------------
}  // extern "C"

static __device__ __align__(256) uint8_t scratch[WLDA_FOLDIN_STATIC_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_dev[SCRATCH_MAX_DEVICES] = {};

// Device address of `scratch` on device dev, which must be current (looked up
// on the first call on each device).
hipError_t scratch_address(int dev, void **out) {
    hipError_t e;
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        scratch_dev[dev] = ptr;
    }
    *out = scratch_dev[dev];
    return hipSuccess;
}
}  // namespace

extern "C" {

wlda_status wlda_foldin_batch_static(wlda_model m, uint32_t n_docs, const uint64_t *docptr,
                                     const uint32_t *words, const uint32_t *req_ids,
                                     const uint32_t *learned_weights, uint32_t learned_steps,
                                     uint32_t sweeps, const uint64_t *hoptr, const uint32_t *ho_words,
                                     int32_t *z_out, double *heldout_out) {
    if (!m || !docptr || !req_ids || !z_out || (n_docs && !words)) return WLDA_E_INVALID;
    const uint64_t T = docptr[n_docs];
    if (T >= (1ull << 32)) return WLDA_E_INVALID;
    const uint64_t need = batch_bytes(m->p, n_docs, T, learned_weights != nullptr, hoptr ? hoptr[n_docs] : 0);
    if (need > WLDA_FOLDIN_STATIC_BYTES) return WLDA_E_WORKSPACE;
    // the array used must be the one on the model's device
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return WLDA_E_HIP;
    if (dev != m->dev) return WLDA_E_INVALID;
    void *ws = nullptr;
    if (scratch_address(dev, &ws) != hipSuccess) return WLDA_E_HIP;
    return wlda_foldin_batch(m, n_docs, docptr, words, req_ids, learned_weights, learned_steps, sweeps, hoptr,
                             ho_words, ws, WLDA_FOLDIN_STATIC_BYTES, z_out, heldout_out);
}

wlda_status wlda_model_destroy(wlda_model m) {
    if (!m) return WLDA_E_INVALID;
    (void)hipStreamSynchronize(m->st);
    delete m;
    return WLDA_OK;
}

}  // extern "C"
