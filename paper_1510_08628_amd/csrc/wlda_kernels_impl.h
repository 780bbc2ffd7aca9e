// gfx950 kernels of the WarpLDA sweep (device code shared by the translation
// units wlda_kernels.hip and wlda_kernels_m.hip).
//
// Paper: Chen, Li, Zhu, Chen, "WarpLDA: a Cache Efficient O(1) Algorithm for
// Latent Dirichlet Allocation" (arXiv:1510.08628).
//
// Data: one packed record per token (field 0 = z, fields 1..M = pending
// proposals), stored once (Section 5.2) and blocked by documents: blocks of
// consecutive rows of the doc phase's visiting order, column-major inside a
// block.  Both phases reach their segments through a pointer array into that
// copy of Y, the role P_CSR plays in Section 5.2: `colidx` (canonical CSC
// position -> record) in the word phase and `rowidx` (canonical CSR position
// -> record) in the document phase.  A document window then gathers inside
// blocks resident in its XCD's L2, and a column reads one run per block.
// With records in plain CSC order (the alternative) colidx is null and the
// word phase streams its columns.  The RNG counter of a token is its
// canonical position in the phase's order, independent of the layout.
//
// A "segment" is a column (word phase) or a row (document phase).  Segments
// are binned by length on the host:
//   * wave kernel   - one 64-lane wavefront per segment (<= 512 tokens);
//   * block kernel  - one 256-thread workgroup per segment (<= 4096 tokens);
//   * long path     - segments split over many workgroups (intra-word
//                     parallelism, Section 5.4): histogram -> MH -> draw.
// Per-segment counts (c_w or c_d) live in LDS, dense when K fits and otherwise
// in an open-addressed table with linear probing and an AND hash whose
// capacity is the power of two >= 2L (Section 5.4, "sparse vectors as hash
// tables").  c_k is an exact integer histogram of the phase's new Z, kept in
// LDS per workgroup and added to global memory once per workgroup.
//
// Arithmetic that decides the chain (must match any implementation of the
// same definition bit for bit; compiled without FP contraction):
//   accept  iff  U * den < num,
//     num = (cnt[c] + prior) * (ck[s] + beta_bar),
//     den = (cnt[s] + prior) * (ck[c] + beta_bar)            (Eq. 7)
//   count part iff U * (L + mass) < L, then the topic of a uniformly chosen
//   token of the (updated) segment, else a uniform topic       (Eq. 6, Sec. 4.3);
//   word-phase columns longer than K take the count part as the inverse CDF
//   of their updated counts at Dice(r, L) instead (same law; Section 5.4
//   draws these words' proposals from a table over c_w)
//   U(r) = (r >> 8) * 2^-24,  Dice(r, n) = (r * n) >> 32.
// Random words per (token, iteration, phase): Philox call 0 gives the M
// acceptance uniforms; call j >= 1 the (coin, index) words of proposals 2j-1
// and 2j.  The MH pass and the draw pass of the long path each compute only
// their own calls.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "wlda_device.h"
#include "wlda_internal.h"



namespace wlda {

// --------------------------------------------------------------------------
// Packed records
// --------------------------------------------------------------------------
// RF = -b: one 32-bit word of b-bit fields; RF = 100 + n: n 32-bit words of
// 16-bit fields, two to a word (n = 2: 8-byte, n = 3: 12-byte records);
// RF = 1 or 2: that many 64-bit words of 21-bit fields, three to a word.
template <int RF>
constexpr int rec_words() {
    return RF < 0 ? 1 : RF >= 100 ? RF - 100 : RF;
}

template <int RF>
struct Rec {
    static_assert(RF == 1 || RF == 2 || RF == 102 || RF == 103 || (RF < 0 && RF >= -16), "record format");
    using W = std::conditional_t<(RF < 0 || RF >= 100), uint32_t, uint64_t>;
    W w[rec_words<RF>()];
};

template <int RF>
__device__ __forceinline__ Rec<RF> rec_zero() {
    Rec<RF> r;
#pragma unroll
    for (int i = 0; i < rec_words<RF>(); ++i) r.w[i] = 0;
    return r;
}

template <int RF>
__device__ __forceinline__ Rec<RF> ld_rec(const uint64_t *recs, uint32_t pos) {
    Rec<RF> r;
    if constexpr (RF < 0) {
        r.w[0] = reinterpret_cast<const uint32_t *>(recs)[pos];
    } else if constexpr (RF == 102) {
        const uint2 v = reinterpret_cast<const uint2 *>(recs)[pos];
        r.w[0] = v.x;
        r.w[1] = v.y;
    } else if constexpr (RF == 103) {
        // 12-byte records: three consecutive dwords (one dwordx3 access)
        const uint32_t *p = reinterpret_cast<const uint32_t *>(recs) + (size_t)pos * 3;
        r.w[0] = p[0];
        r.w[1] = p[1];
        r.w[2] = p[2];
    } else if constexpr (RF == 1) {
        r.w[0] = recs[pos];
    } else {
        const uint4 v = reinterpret_cast<const uint4 *>(recs)[pos];
        r.w[0] = ((uint64_t)v.y << 32) | v.x;
        r.w[1] = ((uint64_t)v.w << 32) | v.z;
    }
    return r;
}

template <int RF>
__device__ __forceinline__ void st_rec(uint64_t *recs, uint32_t pos, const Rec<RF> &r) {
    if constexpr (RF < 0) {
        reinterpret_cast<uint32_t *>(recs)[pos] = r.w[0];
    } else if constexpr (RF == 102) {
        reinterpret_cast<uint2 *>(recs)[pos] = make_uint2(r.w[0], r.w[1]);
    } else if constexpr (RF == 103) {
        uint32_t *p = reinterpret_cast<uint32_t *>(recs) + (size_t)pos * 3;
        p[0] = r.w[0];
        p[1] = r.w[1];
        p[2] = r.w[2];
    } else if constexpr (RF == 1) {
        recs[pos] = r.w[0];
    } else {
        reinterpret_cast<uint4 *>(recs)[pos] =
            make_uint4((uint32_t)r.w[0], (uint32_t)(r.w[0] >> 32), (uint32_t)r.w[1],
                       (uint32_t)(r.w[1] >> 32));
    }
}

template <int RF>
__device__ __forceinline__ uint32_t fld(const Rec<RF> &r, int f) {
    if constexpr (RF < 0) {
        constexpr uint32_t B = (uint32_t)(-RF);
        return (r.w[0] >> (B * f)) & ((1u << B) - 1u);
    } else if constexpr (RF >= 100) {
        return (r.w[f >> 1] >> (16 * (f & 1))) & 0xFFFFu;
    } else {
        return (uint32_t)(r.w[f / 3] >> (FIELD_BITS * (f % 3))) & FIELD_MASK;
    }
}

template <int RF>
__device__ __forceinline__ void set_fld(Rec<RF> &r, int f, uint32_t v) {
    if constexpr (RF < 0) {
        constexpr uint32_t B = (uint32_t)(-RF);
        const uint32_t sh = B * f;
        r.w[0] = (r.w[0] & ~(((1u << B) - 1u) << sh)) | (v << sh);
    } else if constexpr (RF >= 100) {
        const uint32_t sh = 16 * (f & 1);
        r.w[f >> 1] = (r.w[f >> 1] & ~(0xFFFFu << sh)) | (v << sh);
    } else {
        const int sh = FIELD_BITS * (f % 3);
        r.w[f / 3] = (r.w[f / 3] & ~((uint64_t)FIELD_MASK << sh)) | ((uint64_t)v << sh);
    }
}



// Word w (0..3) of a Philox output.
__device__ __forceinline__ uint32_t word4(const uint4 &r, int w) {
    return w == 0 ? r.x : w == 1 ? r.y : w == 2 ? r.z : r.w;
}

// The random words of a token in a phase: call 0 (step field 0) holds the M
// acceptance uniforms, word i-1 for step i; call j >= 1 holds the mixture
// coin and the index/topic word of proposals 2j-1 (words 0, 1) and 2j
// (words 2, 3).

// --------------------------------------------------------------------------
// LDS count tables
// --------------------------------------------------------------------------
constexpr uint32_t EMPTY_KEY = 0xFFFFFFFFu;

__device__ __forceinline__ void tab_insert(uint32_t *key, uint32_t *cnt, uint32_t mask, bool dense,
                                           uint32_t k) {
    if (dense) {
        atomicAdd(&cnt[k], 1u);
        return;
    }
    uint32_t h = k & mask;
    while (true) {
        const uint32_t old = atomicCAS(&key[h], EMPTY_KEY, k);
        if (old == EMPTY_KEY || old == k) {
            atomicAdd(&cnt[h], 1u);
            return;
        }
        h = (h + 1) & mask;
    }
}

__device__ __forceinline__ uint32_t tab_get(const uint32_t *key, const uint32_t *cnt, uint32_t mask,
                                            bool dense, uint32_t k) {
    if (dense) return cnt[k];
    uint32_t h = k & mask;
    while (true) {
        const uint32_t kk = key[h];
        if (kk == k) return cnt[h];
        if (kk == EMPTY_KEY) return 0u;
        h = (h + 1) & mask;
    }
}

// Packed open-addressed counts for K <= 65535: one 32-bit word per slot,
// (topic + 1) in the high half and the count in the low half, 0 = empty, so a
// probe is one LDS access and the table half the size.  Counts stay below
// 2^16 (segments hold at most 4096 tokens).
constexpr uint32_t PACKED_MAX_K = 65535;

__device__ __forceinline__ void ptab_insert(uint32_t *tab, uint32_t mask, uint32_t k) {
    const uint32_t key = (k + 1) << 16;
    uint32_t h = k & mask;
    while (true) {
        const uint32_t old = atomicCAS(&tab[h], 0u, key | 1u);
        if (old == 0u) return;
        if ((old & 0xFFFF0000u) == key) {
            atomicAdd(&tab[h], 1u);
            return;
        }
        h = (h + 1) & mask;
    }
}

__device__ __forceinline__ uint32_t ptab_get(const uint32_t *tab, uint32_t mask, uint32_t k) {
    const uint32_t key = (k + 1) << 16;
    uint32_t h = k & mask;
    while (true) {
        const uint32_t v = tab[h];
        if ((v & 0xFFFF0000u) == key) return v & 0xFFFFu;
        if (v == 0u) return 0u;
        h = (h + 1) & mask;
    }
}

__device__ __forceinline__ uint32_t pow2_at_least(uint32_t x) {
    return x <= 1 ? 1u : 1u << (32 - __clz(x - 1));
}

template <int GROUP>
__device__ __forceinline__ void group_sync() {
    if constexpr (GROUP <= 64) {
        // one wavefront (or part of one): LDS operations of a wavefront
        // complete in order, so a compiler-level wavefront fence is all that
        // is needed.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Inclusive prefix sums of a[0..K) in place by the GROUP threads of a group
// (each thread a contiguous run of entries); ends with a group barrier.
template <int GROUP>
__device__ void group_inclusive_scan(uint32_t *a, uint32_t K, uint32_t lane) {
    constexpr int WS = GROUP < 64 ? GROUP : 64;   // lanes of one shuffle scan
    const uint32_t per = (K + GROUP - 1) / GROUP;
    const uint32_t k0 = min(K, lane * per), k1 = min(K, k0 + per);
    uint32_t sum = 0;
    for (uint32_t k = k0; k < k1; ++k) sum += a[k];
    uint32_t x = sum;
    const uint32_t wl = lane % WS;
#pragma unroll
    for (int off = 1; off < WS; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, WS);
        if (wl >= (uint32_t)off) x += y;
    }
    if constexpr (GROUP > 64) {
        __shared__ uint32_t wsum[GROUP / 64];
        if (wl == 63) wsum[lane >> 6] = x;
        __syncthreads();
        for (uint32_t w = 0; w < (lane >> 6); ++w) x += wsum[w];
        __syncthreads();
    }
    uint32_t run = x - sum;
    for (uint32_t k = k0; k < k1; ++k) {
        run += a[k];
        a[k] = run;
    }
    group_sync<GROUP>();
}

// Inverse CDF, N lookups at once: each j[d] (< cum[K-1]) is replaced by the
// smallest topic k with cum[k] > j[d], cum holding inclusive prefix counts
// over topics 0..K-1.  Over prefix counts in LDS, a branch-free binary search
// whose trip count depends on K only (the N loads of each step are in flight
// together), stepping 32-bit LDS pointers: one add, one LDS load, one compare
// and one select per lookup and step.
typedef __attribute__((address_space(3))) const uint32_t lds_cu32;
template <int N>
__device__ __forceinline__ void cdf_find_lds(const uint32_t *cum_generic, uint32_t K, uint32_t (&j)[N]) {
    lds_cu32 *cum = (lds_cu32 *)cum_generic;
    lds_cu32 *b[N];
#pragma unroll
    for (int d = 0; d < N; ++d) b[d] = cum;
    for (uint32_t n = K; n > 1;) {
        const uint32_t half = n >> 1;
#pragma unroll
        for (int d = 0; d < N; ++d) {
            lds_cu32 *p = b[d] + half;
            b[d] = *p <= j[d] ? p : b[d];
        }
        n -= half;
    }
#pragma unroll
    for (int d = 0; d < N; ++d) j[d] = (uint32_t)(b[d] - cum) + (*b[d] <= j[d] ? 1u : 0u);
}

// Through a guide table in LDS: guide[i] (i < nb) is
// the smallest topic k with cum[k] > i << gs, so the answer for j lies in
// [guide[j >> gs], guide[(j >> gs) + 1]] (the last bucket ends at K - 1) and a
// binary search of that range, a few topics wide, finds it.
constexpr uint32_t GUIDE_MAX = 4096;     // guide entries (16-bit topics)
template <int N>
__device__ __forceinline__ void cdf_find_guided(const uint32_t *cum_generic, const uint16_t *guide, uint32_t gs,
                                                uint32_t nb, uint32_t K, uint32_t (&j)[N]) {
    lds_cu32 *cum = (lds_cu32 *)cum_generic;
    uint32_t base[N], n[N];
#pragma unroll
    for (int d = 0; d < N; ++d) {
        const uint32_t i = j[d] >> gs;
        base[d] = guide[i];
        n[d] = (i + 1 < nb ? (uint32_t)guide[i + 1] : K - 1) - base[d] + 1;
    }
    for (;;) {
        bool open = false;
#pragma unroll
        for (int d = 0; d < N; ++d) {
            if (n[d] > 1) {
                const uint32_t half = n[d] >> 1;
                if (cum[base[d] + half - 1] <= j[d]) base[d] += half;
                n[d] -= half;
                open = true;
            }
        }
        if (!open) break;
    }
#pragma unroll
    for (int d = 0; d < N; ++d) j[d] = base[d];
}

// Guide buckets for a column of L tokens: 2^gs token indices each, the
// smallest gs that leaves at most nb_max buckets.
__device__ __forceinline__ uint32_t guide_shift(uint32_t L, uint32_t nb_max) {
    uint32_t gs = 0;
    while ((((uint64_t)L + (1u << gs) - 1) >> gs) > nb_max) ++gs;
    return gs;
}

// cdf_find_guided with the prefix counts and a guide of 32-bit topics in
// global memory (K beyond what LDS holds).
template <int N>
__device__ __forceinline__ void cdf_find_guided_g(const uint32_t *cum, const uint32_t *guide, uint32_t gs,
                                                  uint32_t nb, uint32_t K, uint32_t (&j)[N]) {
    uint32_t base[N], n[N];
#pragma unroll
    for (int d = 0; d < N; ++d) {
        const uint32_t i = j[d] >> gs;
        base[d] = guide[i];
        n[d] = (i + 1 < nb ? guide[i + 1] : K - 1) - base[d] + 1;
    }
    for (;;) {
        bool open = false;
#pragma unroll
        for (int d = 0; d < N; ++d) {
            if (n[d] > 1) {
                const uint32_t half = n[d] >> 1;
                if (cum[base[d] + half - 1] <= j[d]) base[d] += half;
                n[d] -= half;
                open = true;
            }
        }
        if (!open) break;
    }
#pragma unroll
    for (int d = 0; d < N; ++d) j[d] = base[d];
}

__device__ __forceinline__ void add_accepted(unsigned long long *dst, unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(dst, v);
}

// --------------------------------------------------------------------------
// Segment kernel: GROUP threads (16 or 32 lanes of a wavefront, a wavefront,
// or the workgroup) own one segment of at most GROUP*TPT tokens at a time; segments of an XCD's share of the
// list are taken in ascending order so that the rows visited at the same time
// are neighbours (their tokens share cache lines of each column, Section 5.2).
// --------------------------------------------------------------------------
// c_k histogram of 16-bit counters, two to a 32-bit LDS word (topic k in
// half k & 1 of word k >> 1).  A counter never reaches 2^16: the one add that
// takes it from 0x7FFF to 0x8000 (the atomic returns each old value exactly
// once) moves 0x8000 to the global count and takes it off the counter again;
// for the counter to wrap before that, the workgroup would have to add 2^15
// more tokens of that topic between two consecutive LDS operations of one
// wavefront.
__device__ __forceinline__ void ckh16_add(uint32_t *ckh, uint32_t k, uint32_t *ck_next) {
    const uint32_t sh = (k & 1u) << 4;
    const uint32_t old = atomicAdd(&ckh[k >> 1], 1u << sh);
    if (((old >> sh) & 0xFFFFu) == 0x7FFFu) {
        atomicSub(&ckh[k >> 1], 0x8000u << sh);
        atomicAdd(&ck_next[k], 0x8000u);
    }
}

template <int PHASE, int M, int NW, int GROUP, int TPT, bool CDF, bool CKG, bool PK, bool ASYM>
__global__ __launch_bounds__(256) void seg_kernel(PhaseArgs a, SegList l, uint32_t cap_max,
                                                  uint32_t dense_u, uint32_t ck_lds_u) {
    extern __shared__ uint32_t lds[];
    constexpr int GPB = 256 / GROUP;
    static_assert(TPT * (M + 1) <= 64, "one bit per lookup of a lane's tokens");
    static_assert(!ASYM || PHASE == PH_DOC, "alpha_k enters the doc phase only");
    // ck_lds_u: bit 0 = the c_k histogram of the new Z in LDS, bit 1 = c_k +
    // beta_bar staged in LDS (what fits the LDS budget; see run_seg)
    const bool dense = dense_u != 0, ckh_lds = (ck_lds_u & 1u) != 0, ckb_lds = (ck_lds_u & 2u) != 0;
    const bool h16 = (ck_lds_u & 4u) != 0;   // histogram of 16-bit counters, two per word
    const uint32_t g = threadIdx.x / GROUP, lane = threadIdx.x % GROUP;
    const uint32_t K = a.K;
    // LDS: [c_k + beta_bar as binary32 (ckb_lds)] [c_k histogram of the new
    // Z (ckh_lds)], then per group [count table | new z of the segment]
    const uint32_t h_words = h16 ? (K + 1) / 2 : K;
    const uint32_t ck_words = (ckb_lds ? K : 0) + (ckh_lds ? h_words : 0);
    // count table: dense K words, or cap_max packed words (PK), or cap_max
    // keys followed by cap_max counts
    const uint32_t tab_words = dense ? K : (PK ? cap_max : 2 * cap_max);
    float *ckb = reinterpret_cast<float *>(lds);
    uint32_t *ckh = lds + (ckb_lds ? K : 0);
    uint32_t *gbase = lds + ck_words + g * (tab_words + GROUP * TPT);
    uint32_t *tkey = gbase;
    uint32_t *tcnt = dense ? gbase : gbase + cap_max;
    uint32_t *zarr = gbase + tab_words;

    if (ckh_lds || ckb_lds)
        for (uint32_t i = threadIdx.x; i < K; i += 256) {
            if (ckh_lds && i < h_words) ckh[i] = 0;
            if (ckb_lds) ckb[i] = (float)a.ck[i] + a.beta_bar;
        }
    if (dense)
        for (uint32_t i = lane; i < K; i += GROUP) tcnt[i] = 0;
    __syncthreads();

    const uint32_t xcd = blockIdx.x & 7, nbx = gridDim.x >> 3, bj = blockIdx.x >> 3;
    const uint32_t lo = l.xcd_cut[xcd], hi = l.xcd_cut[xcd + 1];
    const uint32_t ngx = nbx * GPB;
    const float prior = a.prior, mass = a.mass, beta_bar = a.beta_bar;
    const uint32_t ph = (uint32_t)PHASE << 16;
    unsigned long long acc = 0;

    // Segment li's span and records.  All pointers first, then all records,
    // with no branch around any load (slots past the segment's end re-read its
    // last token), so each batch is in flight at once.
    auto fetch = [&](uint32_t lj, uint32_t &fbeg, uint32_t &fL, uint32_t(&fpos)[TPT], Rec<NW>(&frec)[TPT]) {
        const uint2 sp = l.span[lj];
        fbeg = sp.x;
        fL = sp.y - sp.x;
        if (a.idx) {
#pragma unroll
            for (int r = 0; r < TPT; ++r) fpos[r] = a.idx[fbeg + min(r * GROUP + lane, fL - 1)];
        } else {
#pragma unroll
            for (int r = 0; r < TPT; ++r) fpos[r] = fbeg + min(r * GROUP + lane, fL - 1);
        }
#pragma unroll
        for (int r = 0; r < TPT; ++r) frec[r] = ld_rec<NW>(a.recs, fpos[r]);
    };
    uint32_t li = lo + bj * GPB + g;
    uint32_t beg = 0, L = 1;
    uint32_t pos[TPT];
    Rec<NW> rec[TPT];
    if (li < hi) fetch(li, beg, L, pos, rec);
    for (; li < hi; li += ngx) {
        uint32_t znew[TPT];
        // word proposals of a column with L > K: inverse CDF of its updated
        // counts (the table is dense whenever L > K, since K < L <= GROUP * TPT)
        const bool by_cdf = CDF && PHASE == PH_WORD && !a.draw_only && dense && L > K;
        if (!a.draw_only) {
            uint32_t mask = 0;
            if (!dense) {
                const uint32_t cap = pow2_at_least(2 * L);
                mask = cap - 1;
                for (uint32_t i = lane; i < cap; i += GROUP) {
                    if constexpr (PK) {
                        tkey[i] = 0;
                    } else {
                        tkey[i] = EMPTY_KEY;
                        tcnt[i] = 0;
                    }
                }
                group_sync<GROUP>();
            }
            // c_k + beta_bar of every token's state and candidates, when c_k
            // is not staged in LDS: all loads of the segment issued at once
            // (every slot holds a valid record, so no load needs a guard)
            float gck[CKG ? TPT : 1][M + 1];
            if constexpr (CKG) {
#pragma unroll
                for (int r = 0; r < TPT; ++r)
#pragma unroll
                    for (int f = 0; f <= M; ++f) gck[r][f] = (float)a.ck[fld(rec[r], f)] + beta_bar;
            }
            // alpha of the same topics under an asymmetric alpha
            float gal[ASYM ? TPT : 1][M + 1];
            if constexpr (ASYM) {
#pragma unroll
                for (int r = 0; r < TPT; ++r)
#pragma unroll
                    for (int f = 0; f <= M; ++f) gal[r][f] = a.alpha_k[fld(rec[r], f)];
            }
#pragma unroll
            for (int r = 0; r < TPT; ++r)
                if (r * GROUP + lane < L) {
                    if constexpr (PK)
                        ptab_insert(tkey, mask, fld(rec[r], 0));
                    else
                        tab_insert(tkey, tcnt, mask, dense, fld(rec[r], 0));
                }
            group_sync<GROUP>();
            // The counts each token needs: its state s0 and its M candidates
            // (the chain's state is always one of them).  All first probes of
            // the segment's tokens are issued together; the rare lookups that
            // hit a slot of another topic finish with a probing loop.
            uint32_t cnt[TPT][M + 1];
            uint64_t pend = 0;   // bit r * (M + 1) + f: lookup still open
#pragma unroll
            for (int r = 0; r < TPT; ++r)
#pragma unroll
                for (int f = 0; f <= M; ++f) {
                    const uint32_t k = fld(rec[r], f);
                    if (dense) {
                        cnt[r][f] = tcnt[k];
                    } else if constexpr (PK) {
                        const uint32_t v = tkey[k & mask];
                        cnt[r][f] = (v & 0xFFFF0000u) == (k + 1) << 16 ? v & 0xFFFFu : 0u;
                        if (v != 0u && (v & 0xFFFF0000u) != (k + 1) << 16) pend |= 1ull << (r * (M + 1) + f);
                    } else {
                        const uint32_t kk = tkey[k & mask];
                        cnt[r][f] = 0;
                        if (kk == k) cnt[r][f] = tcnt[k & mask];
                        else if (kk != EMPTY_KEY) pend |= 1ull << (r * (M + 1) + f);
                    }
                }
            if (pend) {
#pragma unroll
                for (int r = 0; r < TPT; ++r)
#pragma unroll
                    for (int f = 0; f <= M; ++f)
                        if ((pend >> (r * (M + 1) + f)) & 1ull) {
                            const uint32_t k = fld(rec[r], f);
                            if constexpr (PK)
                                cnt[r][f] = ptab_get(tkey, mask, k);
                            else
                                cnt[r][f] = tab_get(tkey, tcnt, mask, false, k);
                        }
            }
#pragma unroll
            for (int r = 0; r < TPT; ++r) {
                if (r * GROUP + lane < L) {
                    uint32_t s = fld(rec[r], 0), cs = cnt[r][0];
                    float bs, as = prior;
                    if constexpr (CKG) bs = gck[r][0]; else bs = ckb[s];
                    if constexpr (ASYM) as = gal[r][0];
                    const uint4 RA = philox(beg + r * GROUP + lane, a.iter, ph, 0, a.seed_lo, a.seed_hi);
#pragma unroll
                    for (int i = 1; i <= M; ++i) {
                        const uint32_t c = fld(rec[r], i), cc = cnt[r][i];
                        const float u = unif24(word4(RA, i - 1));
                        float bc;
                        if constexpr (CKG) bc = gck[r][i]; else bc = ckb[c];
                        bool ok;
                        if constexpr (ASYM)
                            ok = mh_accept_b2(u, cc, cs, gal[r][i], as, bs, bc);
                        else
                            ok = mh_accept_b(u, cc, cs, prior, bs, bc);
                        if (ok) {
                            s = c;
                            cs = cc;
                            bs = bc;
                            if constexpr (ASYM) as = gal[r][i];
                            ++acc;
                        }
                    }
                    znew[r] = s;
                }
            }
            group_sync<GROUP>();
            if (dense) {
#pragma unroll
                for (int r = 0; r < TPT; ++r)
                    if (r * GROUP + lane < L) tcnt[fld(rec[r], 0)] = 0;
            }
            if constexpr (CDF) {
                if (by_cdf) {   // counts of the updated column, then prefix sums
                    group_sync<GROUP>();
#pragma unroll
                    for (int r = 0; r < TPT; ++r)
                        if (r * GROUP + lane < L) atomicAdd(&tcnt[znew[r]], 1u);
                    group_sync<GROUP>();
                    group_inclusive_scan<GROUP>(tcnt, K, lane);
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < TPT; ++r) znew[r] = fld(rec[r], 0);
        }
        // The segment's new z in LDS, in segment order for random positioning.
        // For a column with L > K the count part of a word proposal is the
        // inverse CDF of its updated counts at an index j < L, which is entry j
        // of the column's new topics sorted by topic: a counting sort through
        // the prefix sums writes them in that order (entries of one topic are
        // equal, so the order in which the atomics land does not matter), and
        // the draw reads one entry in both cases.
        bool sorted = false;
        if constexpr (CDF) sorted = by_cdf;
#pragma unroll
        for (int r = 0; r < TPT; ++r)
            if (r * GROUP + lane < L) {
                const uint32_t at = sorted ? atomicSub(&tcnt[znew[r]], 1u) - 1u : r * GROUP + lane;
                zarr[at] = znew[r];
            }
        group_sync<GROUP>();
        // Word phase: the next segment's loads go out before this one's stores
        // (loads and stores share one in-order counter, so loads issued after
        // the stores would wait for them).  Measured slower in the doc phase,
        // whose gathers and scatters compete for the same L2 lines.
        constexpr bool PREFETCH = PHASE == PH_WORD;
        uint32_t nbeg = 0, nL = 1;
        uint32_t npos[TPT];
        Rec<NW> nrec[TPT];
        if (PREFETCH && li + ngx < hi) fetch(li + ngx, nbeg, nL, npos, nrec);
        // Draws, DB tokens at a time: the count part is entry j of the
        // segment's new z array in LDS (see above).
        constexpr int DB = TPT < 4 ? TPT : 4;
#pragma unroll
        for (int r0 = 0; r0 < TPT; r0 += DB) {
            uint32_t pw[DB * M];
#pragma unroll
            for (int q = 0; q < DB; ++q) {
                const uint32_t n = (r0 + q) * GROUP + lane;
#pragma unroll
                for (int i = 0; i < M; ++i) pw[q * M + i] = 0;
                if (n < L) {
#pragma unroll
                    for (int j = 1; j <= (M + 1) / 2; ++j) {
                        const uint4 RB = philox(beg + n, a.iter, ph | j, 0, a.seed_lo, a.seed_hi);
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int i = 2 * j - 1 + h;
                            if (i > M) continue;
                            const uint32_t w = word4(RB, 2 * h + 1);
                            if (take_count_part(unif24(word4(RB, 2 * h)), L, mass))
                                pw[q * M + i - 1] = zarr[dice(w, L)];
                            else if constexpr (ASYM)
                                pw[q * M + i - 1] = alpha_prior_topic(a.alpha_cum, K, w);
                            else
                                pw[q * M + i - 1] = dice(w, K);
                        }
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < DB; ++q) {
                const int r = r0 + q;
                if (r * GROUP + lane < L) {
                    Rec<NW> out = rec_zero<NW>();
                    set_fld(out, 0, znew[r]);
#pragma unroll
                    for (int i = 1; i <= M; ++i) set_fld(out, i, pw[q * M + i - 1]);
                    st_rec<NW>(a.recs, pos[r], out);
                    if (!ckh_lds)
                        atomicAdd(&a.ck_next[znew[r]], 1u);
                    else if (h16)
                        ckh16_add(ckh, znew[r], a.ck_next);
                    else
                        atomicAdd(&ckh[znew[r]], 1u);
                }
            }
        }
        group_sync<GROUP>();
        if constexpr (CDF) {
            if (by_cdf) {       // what the sort left of the prefix sums: clear all of it
                for (uint32_t k = lane; k < K; k += GROUP) tcnt[k] = 0;
                group_sync<GROUP>();
            }
        }
        if constexpr (PREFETCH) {
            beg = nbeg;
            L = nL;
#pragma unroll
            for (int r = 0; r < TPT; ++r) {
                pos[r] = npos[r];
                rec[r] = nrec[r];
            }
        } else if (li + ngx < hi) {
            fetch(li + ngx, beg, L, pos, rec);
        }
    }
    add_accepted(a.accepted, acc);
    __syncthreads();
    if (ckh_lds && h16) {
        for (uint32_t w = threadIdx.x; w < h_words; w += 256) {
            const uint32_t v = ckh[w];
            if (v & 0xFFFFu) atomicAdd(&a.ck_next[2 * w], v & 0xFFFFu);
            if (v >> 16) atomicAdd(&a.ck_next[2 * w + 1], v >> 16);
        }
    } else if (ckh_lds) {
        for (uint32_t k = threadIdx.x; k < K; k += 256) {
            const uint32_t v = ckh[k];
            if (v) atomicAdd(&a.ck_next[k], v);
        }
    }
}

// --------------------------------------------------------------------------
// Long segments (intra-word parallelism, Section 5.4).  Three passes over the
// chunks of all long segments:
//   hist - c_w (or c_d) of each long segment from the phase-start Z, summed
//          into a global table per segment;
//   mh   - the table staged in LDS, M MH steps per token, the new z written
//          to a compact per-segment array only (records are left as they are);
//   draw - each token's z read back from the compact array in chunk order,
//          proposals by random positioning over that array (the segment's
//          updated assignments) or the inverse CDF of its counts, and the
//          whole record written, c_k accumulated.
// Each XCD owns whole segments, so a segment's compact array is read from
// that XCD's L2.
// --------------------------------------------------------------------------
// Global per-segment counts (dense or open-addressed, keys stored as topic+1).
__device__ __forceinline__ void gtab_add(const LongList &l, uint32_t j, uint32_t K, uint32_t k, uint32_t add) {
    uint32_t *base = l.tables + l.tab_off[j];
    const uint32_t cap = l.tab_cap[j];
    if (cap == 0) {
        atomicAdd(&base[k], add);
        return;
    }
    const uint32_t mask = cap - 1, key = k + 1;
    uint32_t h = k & mask;
    while (true) {
        const uint32_t old = atomicCAS(&base[h], 0u, key);
        if (old == 0u || old == key) {
            atomicAdd(&base[cap + h], add);
            return;
        }
        h = (h + 1) & mask;
    }
}

__device__ __forceinline__ uint32_t gtab_get(const uint32_t *base, uint32_t cap, uint32_t k) {
    if (cap == 0) return base[k];
    const uint32_t mask = cap - 1, key = k + 1;
    uint32_t h = k & mask;
    while (true) {
        const uint32_t kk = base[h];
        if (kk == key) return base[cap + h];
        if (kk == 0u) return 0u;
        h = (h + 1) & mask;
    }
}

// Tokens per thread whose loads are issued together in the long kernels.  The
// histogram and MH passes wait on their gathers and want many in flight; the
// draw pass is bound by its arithmetic (Philox, the CDF search), and a
// larger batch only costs it registers.
constexpr int HIST_BATCH = 16;
constexpr int MH_BATCH = 16;
constexpr int DRAW_BATCH = 4;

// Record positions of tokens nb, nb + 256, ... of a segment starting at
// canonical position beg, clamped to the chunk's last token n1 - 1 so that
// every load is in bounds and the batch issues without per-token branches.
template <int B>
__device__ __forceinline__ void load_positions(const uint32_t *idx, uint32_t beg, uint32_t nb, uint32_t n1,
                                               uint32_t (&pos)[B]) {
    if (idx) {
#pragma unroll
        for (int u = 0; u < B; ++u) pos[u] = idx[beg + min(nb + u * 256, n1 - 1)];
    } else {
#pragma unroll
        for (int u = 0; u < B; ++u) pos[u] = beg + min(nb + u * 256, n1 - 1);
    }
}

#define WLDA_FOR_CHUNKS(l)                                                        \
    const uint32_t xcd_ = blockIdx.x & 7, nbx_ = gridDim.x >> 3;                 \
    for (uint32_t ci = (l).chunk_cut[xcd_] + (blockIdx.x >> 3); ci < (l).chunk_cut[xcd_ + 1]; \
         ci += nbx_)

template <int PHASE, int M, int NW>
__global__ __launch_bounds__(256) void long_hist_kernel(PhaseArgs a, LongList l, uint32_t lds_dense) {
    extern __shared__ uint32_t hist[];
    const uint32_t K = a.K;
    // LDS: dense K counts, or an open-addressed table of 2 * LONG_CHUNK_HASHED
    // slots (chunks are LONG_CHUNK_HASHED tokens whenever the table is hashed)
    constexpr uint32_t HCAP = 2 * Tuning::LONG_CHUNK_HASHED;
    uint32_t *hkey = hist, *hcnt = hist + HCAP;
    WLDA_FOR_CHUNKS(l) {
        const uint32_t j = l.chunk_seg[ci], n0 = l.chunk_start[ci];
        const uint32_t s_id = l.ids[j];
        const uint32_t beg = a.segptr[s_id], L = a.segptr[s_id + 1] - beg;
        const uint32_t n1 = min(L, n0 + l.chunk);
        if (lds_dense) {
            for (uint32_t k = threadIdx.x; k < K; k += 256) hist[k] = 0;
        } else {
            for (uint32_t k = threadIdx.x; k < HCAP; k += 256) hkey[k] = EMPTY_KEY, hcnt[k] = 0;
        }
        __syncthreads();
        // HIST_BATCH tokens per thread in flight: all loads, then the inserts
        for (uint32_t nb = n0 + threadIdx.x; nb < n1; nb += 256 * HIST_BATCH) {
            uint32_t pos[HIST_BATCH], z[HIST_BATCH];
            load_positions<HIST_BATCH>(a.idx, beg, nb, n1, pos);
#pragma unroll
            for (int u = 0; u < HIST_BATCH; ++u) z[u] = fld(ld_rec<NW>(a.recs, pos[u]), 0);
#pragma unroll
            for (int u = 0; u < HIST_BATCH; ++u)
                if (nb + u * 256 < n1) tab_insert(hkey, lds_dense ? hist : hcnt, HCAP - 1, lds_dense != 0, z[u]);
        }
        __syncthreads();
        if (lds_dense) {
            for (uint32_t k = threadIdx.x; k < K; k += 256) {
                const uint32_t c = hist[k];
                if (c) gtab_add(l, j, K, k, c);
            }
        } else {
            for (uint32_t k = threadIdx.x; k < HCAP; k += 256) {
                const uint32_t c = hcnt[k];
                if (c) gtab_add(l, j, K, hkey[k], c);
            }
        }
        __syncthreads();
    }
}

template <int PHASE, int M, int NW, typename ZT>
__global__ __launch_bounds__(256) void long_mh_kernel(PhaseArgs a, LongList l, uint32_t lds_tab,
                                                      uint32_t ck_lds_u) {
    // LDS: [the segment's count table (lds_tab) | c_k + beta_bar (ck_lds)]
    extern __shared__ uint32_t tab[];
    const uint32_t K = a.K;
    const bool ck_lds = ck_lds_u != 0;
    float *ckb = reinterpret_cast<float *>(tab + (lds_tab ? K : 0));
    if (ck_lds) {
        for (uint32_t k = threadIdx.x; k < K; k += 256) ckb[k] = (float)a.ck[k] + a.beta_bar;
        __syncthreads();
    }
    const uint32_t ph = (uint32_t)PHASE << 16;
    ZT *zc = reinterpret_cast<ZT *>(l.zc);
    unsigned long long acc = 0;
    WLDA_FOR_CHUNKS(l) {
        const uint32_t j = l.chunk_seg[ci], n0 = l.chunk_start[ci];
        const uint32_t s_id = l.ids[j];
        const uint32_t beg = a.segptr[s_id], L = a.segptr[s_id + 1] - beg;
        const uint32_t n1 = min(L, n0 + l.chunk);
        const uint32_t zbase = l.prefix[j];
        const uint32_t *gt = l.tables + l.tab_off[j];
        const uint32_t gcap = l.tab_cap[j];
        if (a.draw_only) {     // initial draw: only publish z for random positioning
            for (uint32_t n = n0 + threadIdx.x; n < n1; n += 256) {
                const uint32_t pos = a.idx ? a.idx[beg + n] : beg + n;
                zc[zbase + n] = (ZT)fld(ld_rec<NW>(a.recs, pos), 0);
            }
            continue;
        }
        if (lds_tab) {
            for (uint32_t k = threadIdx.x; k < K; k += 256) tab[k] = gt[k];
            __syncthreads();
        }
        // columns past the inverse-CDF threshold also gather the counts of
        // their updated z for the word proposals' inverse CDF
        const bool by_cdf = PHASE == PH_WORD && word_cdf(L, K);
        constexpr int PER_THREAD = Tuning::LONG_CHUNK / 256;
        uint32_t zk[PER_THREAD];
#pragma unroll
        for (int bt = 0; bt < PER_THREAD / MH_BATCH; ++bt) {
            const uint32_t nb = n0 + threadIdx.x + bt * 256 * MH_BATCH;
            uint32_t pos[MH_BATCH];
            Rec<NW> rec[MH_BATCH];
            load_positions<MH_BATCH>(a.idx, beg, nb, n1, pos);
#pragma unroll
            for (int u = 0; u < MH_BATCH; ++u) rec[u] = ld_rec<NW>(a.recs, pos[u]);
#pragma unroll
            for (int u = 0; u < MH_BATCH; ++u) {
                const uint32_t n = nb + u * 256;
                if (n >= n1) continue;
                uint32_t s = fld(rec[u], 0);
                const uint4 RA = philox(beg + n, a.iter, ph, 0, a.seed_lo, a.seed_hi);
                const bool asym = PHASE == PH_DOC && a.alpha_k != nullptr;
                if (lds_tab && ck_lds) {
                    // counts and c_k + beta_bar in LDS: each step reads both
                    // topics' (cheaper than keeping the state's in registers)
#pragma unroll
                    for (int i = 1; i <= M; ++i) {
                        const float uacc = unif24(word4(RA, i - 1));
                        const uint32_t c = fld(rec[u], i);
                        const float pc = asym ? a.alpha_k[c] : a.prior;
                        const float ps = asym ? a.alpha_k[s] : a.prior;
                        if (mh_accept_b2(uacc, tab[c], tab[s], pc, ps, ckb[s], ckb[c])) {
                            s = c;
                            ++acc;
                        }
                    }
                } else {
                    // in global memory: the state's count, c_k + beta_bar and
                    // prior are looked up once and carried with it, so the
                    // candidates' lookups do not wait on the MH outcomes
                    uint32_t cs = lds_tab ? tab[s] : gtab_get(gt, gcap, s);
                    float bs = ck_lds ? ckb[s] : (float)a.ck[s] + a.beta_bar;
                    float ps = asym ? a.alpha_k[s] : a.prior;
#pragma unroll
                    for (int i = 1; i <= M; ++i) {
                        const float uacc = unif24(word4(RA, i - 1));
                        const uint32_t c = fld(rec[u], i);
                        const uint32_t cc = lds_tab ? tab[c] : gtab_get(gt, gcap, c);
                        const float bc = ck_lds ? ckb[c] : (float)a.ck[c] + a.beta_bar;
                        const float pc = asym ? a.alpha_k[c] : a.prior;
                        if (mh_accept_b2(uacc, cc, cs, pc, ps, bs, bc)) {
                            s = c;
                            cs = cc;
                            bs = bc;
                            ps = pc;
                            ++acc;
                        }
                    }
                }
                zk[bt * MH_BATCH + u] = s;
                zc[zbase + n] = (ZT)s;
            }
        }
        if (by_cdf) {
            uint32_t *nt = l.tables_new + l.tab_off[j];
            if (lds_tab) {      // chunk histogram in LDS, then one add per topic
                __syncthreads();
                for (uint32_t k = threadIdx.x; k < K; k += 256) tab[k] = 0;
                __syncthreads();
#pragma unroll
                for (int q = 0; q < PER_THREAD; ++q)
                    if (n0 + threadIdx.x + q * 256 < n1) atomicAdd(&tab[zk[q]], 1u);
                __syncthreads();
                for (uint32_t k = threadIdx.x; k < K; k += 256) {
                    const uint32_t c = tab[k];
                    if (c) atomicAdd(&nt[k], c);
                }
            } else {
#pragma unroll
                for (int q = 0; q < PER_THREAD; ++q)
                    if (n0 + threadIdx.x + q * 256 < n1) atomicAdd(&nt[zk[q]], 1u);
            }
        }
        if (lds_tab) __syncthreads();
    }
    add_accepted(a.accepted, acc);
}

// Inclusive prefix sums, in place, of the updated counts of every long word
// past the inverse-CDF threshold (word_cdf): one workgroup per word, tiles of
// 4096 topics.  Where the draw searches them in global memory (K >
// CDF_LDS_MAX) it also writes their guide (the topic at the start of every
// bucket of 2^gs token indices, at most K buckets) over the word's phase-start
// counts, which the MH pass has consumed (the tables are cleared after the
// draw).
template <int M>
__global__ __launch_bounds__(256) void long_cdf_kernel(LongList l, const uint32_t *segptr, uint32_t K) {
    __shared__ uint32_t wsum[4];
    constexpr int PER = 16;
    const bool with_guide = K > Tuning::CDF_LDS_MAX;
    for (uint32_t j = blockIdx.x; j < l.n; j += gridDim.x) {
        const uint32_t s = l.ids[j];
        const uint32_t L = segptr[s + 1] - segptr[s];
        if (!word_cdf(L, K)) continue;
        uint32_t *cnt = l.tables_new + l.tab_off[j];
        uint32_t *guide = l.tables + l.tab_off[j];
        const uint32_t gs = with_guide ? guide_shift(L, K) : 0u;
        const uint32_t nb = with_guide ? (uint32_t)(((uint64_t)L + (1u << gs) - 1) >> gs) : 0u;
        uint32_t carry = 0;
        for (uint32_t t0 = 0; t0 < K; t0 += 256 * PER) {
            const uint32_t k0 = t0 + threadIdx.x * PER;
            uint32_t v[PER], sum = 0;
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                v[i] = k0 + i < K ? cnt[k0 + i] : 0u;
                sum += v[i];
            }
            uint32_t x = sum;
            const uint32_t wl = threadIdx.x & 63;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(x, off, 64);
                if (wl >= (uint32_t)off) x += y;
            }
            if (wl == 63) wsum[threadIdx.x >> 6] = x;
            __syncthreads();
            uint32_t base = carry;
            for (uint32_t w = 0; w < (threadIdx.x >> 6); ++w) base += wsum[w];
            const uint32_t tile = wsum[0] + wsum[1] + wsum[2] + wsum[3];
            uint32_t run = base + x - sum;
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const uint32_t prev = run;      // counts of the topics before k0 + i
                run += v[i];
                if (k0 + i < K) {
                    cnt[k0 + i] = run;
                    // topic k0 + i owns the indices [prev, run): the buckets
                    // starting there point to it
                    if (with_guide) {
                        const uint32_t i1 = (uint32_t)min<uint64_t>(nb, ((uint64_t)run + (1u << gs) - 1) >> gs);
                        for (uint32_t b = (uint32_t)(((uint64_t)prev + (1u << gs) - 1) >> gs); b < i1; ++b)
                            guide[b] = k0 + i;
                    }
                }
            }
            carry += tile;
            __syncthreads();
        }
    }
}

// Walker's alias table (alias sampling; the word phase's BuildAlias over
// C_w) of every long word past the inverse-CDF threshold, over its K topics,
// exact in integers: bin k weighs c_k K against a mean of L, so a draw of a
// uniform bin b and a uniform u in [0, L) that returns b if u < thr_b, else
// alias_b, returns topic k with probability c_k / L.  Built by the
// deterministic two-pointer sweep (Huebschle-Schneider and Sanders, Parallel
// Weighted Random Sampling, ESA 2019): light bins (c K <= L) in topic order
// are topped up by the current heavy bin (c K > L), heavy bins in topic
// order; a heavy bin whose remaining weight r has fallen to L or below keeps
// r and is topped up by the next heavy bin; the bins left when the heavy
// ones run out weigh exactly L.  In place: thr holds the counts on entry and
// ALIAS_DONE | threshold as each bin is finished (the flag keeps the scans
// from reading a finished bin as unfinished); alias receives the alias
// topics.  Sequential, O(K).
constexpr uint32_t ALIAS_DONE = 0x80000000u;
// K up to which a word's table is swept in LDS (8 bytes per topic)
constexpr uint32_t ALIAS_LDS_MAX = 8192;

__device__ __forceinline__ void alias_sweep(uint32_t *thr, uint32_t *al, uint32_t K, uint32_t L) {
    const uint64_t W = L;
    auto light = [&](uint32_t b) {
        const uint32_t v = thr[b];
        return v < ALIAS_DONE && (uint64_t)v * K <= W;
    };
    auto heavy = [&](uint32_t b) {
        const uint32_t v = thr[b];
        return v < ALIAS_DONE && (uint64_t)v * K > W;
    };
    uint32_t i = 0, h = 0;
    while (i < K && !light(i)) ++i;
    while (h < K && !heavy(h)) ++h;
    if (h < K) {
        uint64_t r = (uint64_t)thr[h] * K;
        while (true) {
            if (r > W) {
                if (i >= K) break;      // unreachable: the weights sum to K L
                const uint64_t x = (uint64_t)thr[i] * K;
                thr[i] = ALIAS_DONE | (uint32_t)x;
                al[i] = h;
                r -= W - x;
                do ++i; while (i < K && !light(i));
            } else {
                uint32_t hn = h + 1;
                while (hn < K && !heavy(hn)) ++hn;
                thr[h] = ALIAS_DONE | (uint32_t)r;
                al[h] = hn < K ? hn : h;
                if (hn >= K) break;
                r = (uint64_t)thr[hn] * K - (W - r);
                h = hn;
            }
        }
    }
    for (; i < K; ++i)
        if (light(i)) {                 // weighs exactly L
            thr[i] = ALIAS_DONE | L;
            al[i] = i;
        }
}

// The sweep's table in closed form, built by a whole workgroup.  With the
// light bins in topic order l_1, l_2, ... of deficits L - x and running
// deficit D(k) over the first k of them, and the heavy bins h_1, h_2, ... of
// excesses x - L and running excess E(j), the sweep gives
//   light l_k: thr = x, alias = h_j for the first j with E(j) > D(k-1)
//              (none: x = L, it keeps itself);
//   heavy h_j: thr = L + E(j) - D(k_j), k_j the first k with D(k) >= E(j),
//              alias = h_{j+1}; the last heavy bin: thr = L, itself,
// since h_j is the current heavy bin exactly while D(k-1) < E(j) and its
// remaining weight after the k-th light bin is L + E(j) - D(k).  The running
// sums are block-wide scans, the two searches binary searches: the same
// table as alias_sweep, with every lane busy.  256 threads, 16 topics each.
constexpr uint32_t ALIAS_PAR_MAX = 4096;
constexpr uint32_t ALIAS_PAR_TPT = ALIAS_PAR_MAX / 256;

__device__ __forceinline__ void alias_closed_form(const uint32_t *gcnt, uint32_t *gthr, uint32_t *gal,
                                                  uint32_t K, uint32_t L, uint32_t *sh) {
    // LDS: Darr[K] u64 | Earr[K] u64 | harr[K] u32 | scan: nl[256] u32, sd[256] u64, se[256] u64
    unsigned long long *Darr = reinterpret_cast<unsigned long long *>(sh);
    unsigned long long *Earr = Darr + K;
    uint32_t *harr = reinterpret_cast<uint32_t *>(Earr + K);
    unsigned long long *ssd = reinterpret_cast<unsigned long long *>(harr + ((K + 1) & ~1u));
    unsigned long long *sse = ssd + 256;
    uint32_t *snl = reinterpret_cast<uint32_t *>(sse + 256);
    const uint32_t t = threadIdx.x, k0 = t * ALIAS_PAR_TPT;
    const uint64_t W = L;
    uint32_t c[ALIAS_PAR_TPT];
    uint32_t nl = 0;
    unsigned long long sd = 0, se = 0;
#pragma unroll
    for (uint32_t q = 0; q < ALIAS_PAR_TPT; ++q) {
        const uint32_t k = k0 + q;
        c[q] = k < K ? gcnt[k] : 0u;
        if (k >= K) continue;
        const uint64_t x = (uint64_t)c[q] * K;
        if (x <= W) {
            ++nl;
            sd += W - x;
        } else {
            se += x - W;
        }
    }
    // inclusive scans over the 256 threads, then exclusive bases
    snl[t] = nl;
    ssd[t] = sd;
    sse[t] = se;
    __syncthreads();
    for (uint32_t off = 1; off < 256; off <<= 1) {
        const uint32_t a = t >= off ? snl[t - off] : 0u;
        const unsigned long long b = t >= off ? ssd[t - off] : 0ull, e = t >= off ? sse[t - off] : 0ull;
        __syncthreads();
        snl[t] += a;
        ssd[t] += b;
        sse[t] += e;
        __syncthreads();
    }
    const uint32_t n_light = snl[255], n_heavy = K - n_light;
    uint32_t lr = snl[t] - nl, hr = k0 < K ? k0 - lr : 0u;
    unsigned long long D = ssd[t] - sd, E = sse[t] - se;
#pragma unroll
    for (uint32_t q = 0; q < ALIAS_PAR_TPT; ++q) {
        const uint32_t k = k0 + q;
        if (k >= K) continue;
        const uint64_t x = (uint64_t)c[q] * K;
        if (x <= W) {
            D += W - x;
            Darr[lr++] = D;
        } else {
            E += x - W;
            Earr[hr] = E;
            harr[hr++] = k;
        }
    }
    __syncthreads();
    lr = snl[t] - nl;
    hr = k0 < K ? k0 - lr : 0u;
#pragma unroll
    for (uint32_t q = 0; q < ALIAS_PAR_TPT; ++q) {
        const uint32_t k = k0 + q;
        if (k >= K) continue;
        const uint64_t x = (uint64_t)c[q] * K;
        uint32_t thr, al;
        if (x <= W) {
            const unsigned long long Db = Darr[lr++] - (W - x);   // D(k-1)
            uint32_t lo = 0, hi = n_heavy;                          // first j: Earr[j] > Db
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (Earr[mid] > Db) hi = mid;
                else lo = mid + 1;
            }
            if (lo < n_heavy) {
                thr = (uint32_t)x;
                al = harr[lo];
            } else {
                thr = L;
                al = k;
            }
        } else {
            const uint32_t j = hr++;
            if (j + 1 == n_heavy) {
                thr = L;
                al = k;
            } else {
                const unsigned long long Ej = Earr[j];
                uint32_t lo = 0, hi = n_light;                      // first r: Darr[r] >= Ej
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (Darr[mid] >= Ej) hi = mid;
                    else lo = mid + 1;
                }
                thr = (uint32_t)(W + Ej - Darr[lo]);
                al = harr[j + 1];
            }
        }
        gthr[k] = ALIAS_DONE | thr;
        gal[k] = al;
    }
}

// LDS bytes of alias_closed_form for K topics.
__host__ __device__ inline size_t alias_par_lds(uint32_t K) {
    return 16ull * K + 4ull * ((K + 1) & ~1u) + 256 * (8 + 8 + 4);
}

// The tables of the long words: the updated counts in tables_new become the
// thresholds and the alias topics go to `tables` (the phase-start counts,
// consumed by the MH pass).  K <= ALIAS_PAR_MAX: one 256-thread workgroup per
// word builds the closed form; K <= ALIAS_LDS_MAX: one workgroup per word
// loads its counts into LDS, one lane sweeps there, all write the table back;
// larger K: one thread per word sweeps in global memory.
template <int M>
__global__ __launch_bounds__(256) void long_alias_par_kernel(LongList l, const uint32_t *segptr, uint32_t K) {
    extern __shared__ unsigned long long shq[];      // 8-byte aligned for the running sums
    uint32_t *sh = reinterpret_cast<uint32_t *>(shq);
    for (uint32_t j = blockIdx.x; j < l.n; j += gridDim.x) {
        const uint32_t s_id = l.ids[j];
        const uint32_t L = segptr[s_id + 1] - segptr[s_id];
        if (!word_cdf(L, K)) continue;
        uint32_t *gthr = l.tables_new + l.tab_off[j], *gal = l.tables + l.tab_off[j];
        alias_closed_form(gthr, gthr, gal, K, L, sh);
        __syncthreads();
    }
}

template <int M>
__global__ __launch_bounds__(64) void long_alias_kernel(LongList l, const uint32_t *segptr, uint32_t K,
                                                        uint32_t lds_u) {
    extern __shared__ uint32_t sh[];
    if (lds_u) {
        uint32_t *thr = sh, *al = sh + K;
        for (uint32_t j = blockIdx.x; j < l.n; j += gridDim.x) {
            const uint32_t s_id = l.ids[j];
            const uint32_t L = segptr[s_id + 1] - segptr[s_id];
            if (!word_cdf(L, K)) continue;
            uint32_t *gthr = l.tables_new + l.tab_off[j], *gal = l.tables + l.tab_off[j];
            for (uint32_t k = threadIdx.x; k < K; k += 64) thr[k] = gthr[k];
            __syncthreads();
            if (threadIdx.x == 0) alias_sweep(thr, al, K, L);
            __syncthreads();
            for (uint32_t k = threadIdx.x; k < K; k += 64) {
                gthr[k] = thr[k];
                gal[k] = al[k];
            }
            __syncthreads();
        }
        return;
    }
    const uint32_t j = blockIdx.x * 64 + threadIdx.x;
    if (j >= l.n) return;
    const uint32_t s_id = l.ids[j];
    const uint32_t L = segptr[s_id + 1] - segptr[s_id];
    if (!word_cdf(L, K)) return;
    alias_sweep(l.tables_new + l.tab_off[j], l.tables + l.tab_off[j], K, L);
}

template <int PHASE, int M, int NW, typename ZT, bool ALIAS = false>
__global__ __launch_bounds__(256) void long_draw_kernel(PhaseArgs a, LongList l, uint32_t ck_lds_u,
                                                        uint32_t zero_tables, uint32_t cdf_lds_u) {
    // LDS: [c_k histogram of the new Z (ck_lds) | prefix counts of the
    // current word (cdf_lds, words past the inverse-CDF threshold) | their
    // guide table (bit 1 of cdf_lds_u)]
    extern __shared__ uint32_t ckh[];
    // ck_lds_u: 1 = c_k histogram of the new Z in LDS, 0 = global atomics,
    // 2 = none (long_ck_kernel counts the compact z array instead)
    const bool ck_lds = ck_lds_u == 1, ck_none = ck_lds_u == 2;
    const bool cdf_lds = (cdf_lds_u & 1u) != 0, guided = (cdf_lds_u & 2u) != 0;
    const uint32_t K = a.K;
    uint32_t *cdfl = ckh + (ck_lds ? K : 0);
    uint16_t *guide = reinterpret_cast<uint16_t *>(cdfl + K);
    const uint32_t ph = (uint32_t)PHASE << 16;
    const ZT *zc = reinterpret_cast<const ZT *>(l.zc);
    if (ck_lds) {
        for (uint32_t k = threadIdx.x; k < K; k += 256) ckh[k] = 0;
        __syncthreads();
    }
    WLDA_FOR_CHUNKS(l) {
        const uint32_t j = l.chunk_seg[ci], n0 = l.chunk_start[ci];
        const uint32_t s_id = l.ids[j];
        const uint32_t beg = a.segptr[s_id], L = a.segptr[s_id + 1] - beg;
        const uint32_t n1 = min(L, n0 + l.chunk);
        const ZT *zs = zc + l.prefix[j];
        const bool by_cdf = PHASE == PH_WORD && word_cdf(L, K);
        const uint32_t *cum = l.tables_new + l.tab_off[j];
        uint32_t gs = 0, n_bkt = 0;
        // the guide long_cdf_kernel wrote where the prefix counts stay global
        const uint32_t gs_g = by_cdf && !cdf_lds ? guide_shift(L, K) : 0u;
        const uint32_t nb_g = (uint32_t)(((uint64_t)L + (1u << gs_g) - 1) >> gs_g);
        if (by_cdf && cdf_lds) {
            for (uint32_t k = threadIdx.x; k < K; k += 256) cdfl[k] = cum[k];
            __syncthreads();
        }
        if (by_cdf && guided) {
            // guide buckets of 2^gs token indices, at most GUIDE_MAX of them
            while ((((uint64_t)L + (1u << gs) - 1) >> gs) > GUIDE_MAX) ++gs;
            n_bkt = (uint32_t)(((uint64_t)L + (1u << gs) - 1) >> gs);
            // topic k owns the indices [cum[k-1], cum[k]): the buckets that
            // start there point to it (every bucket is written once)
            for (uint32_t k = threadIdx.x; k < K; k += 256) {
                const uint64_t c0 = k ? cdfl[k - 1] : 0u, c1 = cdfl[k];
                const uint32_t i1 = (uint32_t)min<uint64_t>(n_bkt, (c1 + (1u << gs) - 1) >> gs);
                for (uint32_t i = (uint32_t)((c0 + (1u << gs) - 1) >> gs); i < i1; ++i) guide[i] = (uint16_t)k;
            }
            __syncthreads();
        }
        for (uint32_t nb = n0 + threadIdx.x; nb < n1; nb += 256 * DRAW_BATCH) {
            uint32_t pos[DRAW_BATCH];
            Rec<NW> rec[DRAW_BATCH];
            load_positions<DRAW_BATCH>(a.idx, beg, nb, n1, pos);
            // the record is rebuilt from the updated z alone (compact array,
            // read in chunk order): nothing of the old record survives
#pragma unroll
            for (int u = 0; u < DRAW_BATCH; ++u) {
                rec[u] = rec_zero<NW>();
                set_fld(rec[u], 0, (uint32_t)zs[min(nb + u * 256, n1 - 1)]);
            }
            // all random-positioning reads (or CDF lookups) of the batch are
            // issued before any record is written back
            uint32_t jj[DRAW_BATCH * M] = {};
            uint32_t uu[ALIAS ? DRAW_BATCH * M : 1] = {};
            uint32_t coin = 0;
#pragma unroll
            for (int u = 0; u < DRAW_BATCH; ++u) {
                const uint32_t n = nb + u * 256;
                if (n >= n1) continue;
#pragma unroll
                for (int j = 1; j <= (M + 1) / 2; ++j) {
                    const uint4 RB = philox(beg + n, a.iter, ph | j, 0, a.seed_lo, a.seed_hi);
                    // alias draws: the position inside the bin from the same
                    // call on stream 1
                    uint4 RU = make_uint4(0, 0, 0, 0);
                    if (ALIAS && by_cdf) RU = philox(beg + n, a.iter, ph | j, 1, a.seed_lo, a.seed_hi);
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int i = 2 * j - 1 + h;
                        if (i > M) continue;
                        const uint32_t w = word4(RB, 2 * h + 1);
                        if (take_count_part(unif24(word4(RB, 2 * h)), L, a.mass)) {
                            coin |= 1u << (u * M + i - 1);
                            if (ALIAS && by_cdf) {
                                jj[u * M + i - 1] = dice(w, K);
                                uu[ALIAS ? u * M + i - 1 : 0] = dice(word4(RU, 2 * h + 1), L);
                            } else {
                                jj[u * M + i - 1] = dice(w, L);
                            }
                            if (!by_cdf) set_fld(rec[u], i, (uint32_t)zs[jj[u * M + i - 1]]);
                        } else if (PHASE == PH_DOC && a.alpha_cum) {
                            set_fld(rec[u], i, alpha_prior_topic(a.alpha_cum, K, w));
                        } else {
                            set_fld(rec[u], i, dice(w, K));
                        }
                    }
                }
            }
            if (ALIAS && by_cdf) {
                const uint32_t *thr = l.tables_new + l.tab_off[j];
                const uint32_t *al = l.tables + l.tab_off[j];
#pragma unroll
                for (int d = 0; d < DRAW_BATCH * M; ++d)
                    if ((coin >> d) & 1u) {
                        const uint32_t b = jj[d];
                        set_fld(rec[d / M], d % M + 1, uu[ALIAS ? d : 0] < (thr[b] & ~ALIAS_DONE) ? b : al[b]);
                    }
            } else if (by_cdf) {
                if (guided)
                    cdf_find_guided<DRAW_BATCH * M>(cdfl, guide, gs, n_bkt, K, jj);
                else if (cdf_lds)
                    cdf_find_lds<DRAW_BATCH * M>(cdfl, K, jj);
                else
                    cdf_find_guided_g<DRAW_BATCH * M>(cum, l.tables + l.tab_off[j], gs_g, nb_g, K, jj);
#pragma unroll
                for (int d = 0; d < DRAW_BATCH * M; ++d)
                    if ((coin >> d) & 1u) set_fld(rec[d / M], d % M + 1, jj[d]);
            }
#pragma unroll
            for (int u = 0; u < DRAW_BATCH; ++u) {
                if (nb + u * 256 >= n1) continue;
                st_rec<NW>(a.recs, pos[u], rec[u]);
                const uint32_t z = fld(rec[u], 0);
                if (ck_lds)
                    atomicAdd(&ckh[z], 1u);
                else if (!ck_none)
                    atomicAdd(&a.ck_next[z], 1u);
            }
        }
        if (by_cdf && cdf_lds) __syncthreads();
    }
    if (zero_tables) {
        const size_t nt = l.table_words;
        for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < nt; i += (size_t)gridDim.x * 256)
            l.tables[i] = 0;
    }
    if (ck_lds) {
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < K; k += 256) {
            const uint32_t c = ckh[k];
            if (c) atomicAdd(&a.ck_next[k], c);
        }
    }
}


// The c_k histogram of the long segments' new Z, from the compact array the
// MH pass wrote (every long token's new topic once), for draws that leave it
// out: an LDS histogram per workgroup, eight topics per 16-byte load, flushed
// with one global add per nonzero topic.
template <typename ZT>
__global__ __launch_bounds__(256) void long_ck_kernel(const ZT *zc, uint32_t total, uint32_t K, uint32_t *ck_next) {
    extern __shared__ uint32_t hk[];
    for (uint32_t k = threadIdx.x; k < K; k += 256) hk[k] = 0;
    __syncthreads();
    constexpr uint32_t PER = 16 / sizeof(ZT);
    const uint32_t nvec = total / PER;
    const uint4 *zv = reinterpret_cast<const uint4 *>(zc);
    for (uint32_t v = blockIdx.x * 256 + threadIdx.x; v < nvec; v += gridDim.x * 256) {
        const uint4 q = zv[v];
        const ZT *e = reinterpret_cast<const ZT *>(&q);
#pragma unroll
        for (uint32_t i = 0; i < PER; ++i) atomicAdd(&hk[e[i]], 1u);
    }
    for (uint32_t i = nvec * PER + blockIdx.x * 256 + threadIdx.x; i < total; i += gridDim.x * 256)
        atomicAdd(&hk[zc[i]], 1u);
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < K; k += 256) {
        const uint32_t c = hk[k];
        if (c) atomicAdd(&ck_next[k], c);
    }
}

// --------------------------------------------------------------------------
// Launchers of the kernels above (instantiated per M in wlda_kernels_m.hip)
// --------------------------------------------------------------------------
template <typename Kern>
static hipError_t launch_dyn(Kern k, size_t lds) {
    if (lds > 65536)
        return hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    return hipSuccess;
}

// Blocks are assigned to XCDs round robin: a multiple of 8, enough groups to
// keep every CU busy (max_blocks), never more than the list needs.
inline uint32_t xcd_grid(uint32_t want, uint32_t max_blocks) {
    const uint32_t cap = max_blocks >= 8 ? max_blocks : 8;
    const uint32_t b = want < cap ? want : cap;
    return (b + 7) / 8 * 8;
}

template <int PHASE, int M, int NW, int GROUP, int TPT>
static hipError_t run_seg(const PhaseArgs &a, const SegList &l, uint32_t cap_bound, hipStream_t st) {
    if (l.n == 0) return hipSuccess;
    const bool dense = a.K <= cap_bound;
    const uint32_t cap_max = dense ? 0 : cap_bound;
    const bool packed = !dense && a.K <= PACKED_MAX_K;
    const uint32_t tab_words = dense ? a.K : (packed ? cap_max : 2 * cap_max);
    constexpr int GPB = 256 / GROUP;
    // LDS: the groups' count tables, then, within SEG_LDS_BUDGET, the c_k
    // histogram of the new Z first (each token would otherwise add to it with
    // a global atomic, which costs far more than a gather) and c_k + beta_bar
    // second (else read from global memory, all loads of a segment at once);
    // beyond the budget the old limits hold
    // (the histogram of 16-bit counters above CK_LDS_MAX topics: half the LDS)
    const bool h16 = a.K > Tuning::CK_LDS_MAX;
    const uint64_t tab_bytes = 4ull * GPB * (tab_words + GROUP * TPT), kb = 4ull * a.K;
    const uint64_t hb = h16 ? 4ull * ((a.K + 1) / 2) : kb;
    const uint64_t budget = a.seg_lds_budget;
    bool ckh_lds = tab_bytes + hb <= budget;
    bool ckb_lds = tab_bytes + (ckh_lds ? hb : 0) + kb <= budget;
    if (!ckh_lds) {
        ckh_lds = a.K <= Tuning::CK_LDS_MAX;
        ckb_lds = a.K <= Tuning::CKB_LDS_MAX;
    }
    const size_t lds = (ckh_lds ? hb : 0) + (ckb_lds ? kb : 0) + tab_bytes;
    const uint32_t blocks = xcd_grid((l.n + GPB - 1) / GPB, a.max_blocks);
    const uint32_t ck_flags = (uint32_t)ckh_lds | (uint32_t)ckb_lds << 1 | (uint32_t)(ckh_lds && h16) << 2;
    auto go = [&](auto kern) -> hipError_t {
        hipError_t e = launch_dyn(kern, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), lds, st, a, l, cap_max, (uint32_t)dense, ck_flags);
        return hipGetLastError();
    };
    // the inverse-CDF variant only where a column can be longer than K (then
    // K is small and c_k + beta_bar always sits in LDS); the variant reading
    // c_k + beta_bar from global memory only where it does not
    if constexpr (PHASE == PH_WORD) {
        if (dense && !a.draw_only && a.K < (uint32_t)(GROUP * TPT)) {
            // dense tables of K < GROUP * TPT words always leave room for c_k
            // + beta_bar; there is no variant without it
            if (!ckb_lds) return hipErrorNotSupported;
            return go(seg_kernel<PHASE, M, NW, GROUP, TPT, true, false, false, false>);
        }
    } else {
        if (a.alpha_k) {    // asymmetric alpha: doc-phase variants with alpha_k
            if (packed) {
                if (!ckb_lds) return go(seg_kernel<PHASE, M, NW, GROUP, TPT, false, true, true, true>);
                return go(seg_kernel<PHASE, M, NW, GROUP, TPT, false, false, true, true>);
            }
            if (!ckb_lds) return go(seg_kernel<PHASE, M, NW, GROUP, TPT, false, true, false, true>);
            return go(seg_kernel<PHASE, M, NW, GROUP, TPT, false, false, false, true>);
        }
    }
    if (packed) {
        if (!ckb_lds) return go(seg_kernel<PHASE, M, NW, GROUP, TPT, false, true, true, false>);
        return go(seg_kernel<PHASE, M, NW, GROUP, TPT, false, false, true, false>);
    }
    if (!ckb_lds) return go(seg_kernel<PHASE, M, NW, GROUP, TPT, false, true, false, false>);
    return go(seg_kernel<PHASE, M, NW, GROUP, TPT, false, false, false, false>);
}

// Calls f(std::integral_constant<int, RF>) for the record format rf of M
// proposals per token (see record_format).
template <int M, typename F>
static hipError_t with_rf_m(int rf, F &&f) {
    if constexpr (M <= 4) {
        if (rf < 0) return f(std::integral_constant<int, -(int)(32 / (1 + M))>{});
    }
    if constexpr (M >= 2 && M <= 5) {
        if (rf >= 100) return f(std::integral_constant<int, 100 + (M + 2) / 2>{});
    }
    return f(std::integral_constant<int, (M + 3) / 3>{});
}

// Hash capacity bound of a bin: the power of two >= 2L for its longest segment.
template <int PHASE, int M>
static hipError_t seg_dispatch(const PhaseArgs &a, const SegList &l, int bin, hipStream_t st) {
    return with_rf_m<M>(a.rf, [&](auto rfc) -> hipError_t {
        constexpr int NW = decltype(rfc)::value;
        constexpr int TB = M <= 2 ? Tuning::TPT_BLOCK : Tuning::TPT_BLOCK / 2;
        constexpr int TW = M <= 2 ? Tuning::TPT_WIDE : Tuning::TPT_WIDE / 2;
        constexpr int TS = M <= 2 ? Tuning::TPT_WAVE : Tuning::TPT_WAVE / 2;
        if (bin == BIN_G16) return run_seg<PHASE, M, NW, 16, TS>(a, l, 2 * 16 * TS, st);
        if (bin == BIN_G32) return run_seg<PHASE, M, NW, 32, TS>(a, l, 2 * 32 * TS, st);
        if (bin == BIN_WAVE) return run_seg<PHASE, M, NW, 64, TS>(a, l, 2 * 64 * TS, st);
        if (bin == BIN_WIDE) return run_seg<PHASE, M, NW, 256, TW>(a, l, 2 * 256 * TW, st);
        return run_seg<PHASE, M, NW, 256, TB>(a, l, 2 * 256 * TB, st);
    });
}

template <int PHASE, int M, typename ZT>
static hipError_t long_dispatch_z(const PhaseArgs &a, const LongList &l, hipStream_t st, hipEvent_t *ev) {
    return with_rf_m<M>(a.rf, [&](auto rfc) -> hipError_t {
        constexpr int NW = decltype(rfc)::value;
        const bool lds_tab = a.K <= Tuning::LDS_DENSE_MAX;
        const bool ck_lds = a.K <= Tuning::LONG_CK_LDS_MAX;
        const uint32_t blocks = xcd_grid(l.n_chunks, a.max_blocks);
        hipError_t e;
        if (ev && (e = hipEventRecord(ev[0], st)) != hipSuccess) return e;
        if (!a.draw_only) {
            const size_t lds = lds_tab ? 4ull * a.K : 4ull * 2 * 2 * Tuning::LONG_CHUNK_HASHED;
            e = launch_dyn(long_hist_kernel<PHASE, M, NW>, lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((long_hist_kernel<PHASE, M, NW>), dim3(blocks), dim3(256), lds, st, a, l,
                               (uint32_t)lds_tab);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        if (ev && (e = hipEventRecord(ev[1], st)) != hipSuccess) return e;
        if (PHASE == PH_WORD && !a.draw_only) {
            if ((e = launch_fill_u32(l.tables_new, 0, l.table_words, st)) != hipSuccess) return e;
        }
        {
            const bool mh_tab = lds_tab && !a.draw_only, mh_ck = ck_lds && !a.draw_only;
            const size_t lds = 4ull * ((mh_tab ? a.K : 0) + (mh_ck ? a.K : 0));
            e = launch_dyn(long_mh_kernel<PHASE, M, NW, ZT>, lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((long_mh_kernel<PHASE, M, NW, ZT>), dim3(blocks), dim3(256), lds, st, a, l,
                               (uint32_t)mh_tab, (uint32_t)mh_ck);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        if (ev && (e = hipEventRecord(ev[2], st)) != hipSuccess) return e;
        const bool alias = PHASE == PH_WORD && !a.draw_only && a.word_alias;
        const bool cdf_lds = PHASE == PH_WORD && !alias && a.K <= Tuning::CDF_LDS_MAX;
        if (alias && a.K <= ALIAS_PAR_MAX) {
            const size_t lds = alias_par_lds(a.K);
            if ((e = launch_dyn(long_alias_par_kernel<M>, lds)) != hipSuccess) return e;
            hipLaunchKernelGGL(long_alias_par_kernel<M>, dim3(l.n < 65536 ? l.n : 65536), dim3(256), lds, st, l,
                               a.segptr, a.K);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        } else if (alias) {
            const bool alias_lds = a.K <= ALIAS_LDS_MAX;
            const uint32_t grid = alias_lds ? (l.n < 65536 ? l.n : 65536) : (l.n + 63) / 64;
            hipLaunchKernelGGL(long_alias_kernel<M>, dim3(grid), dim3(64), alias_lds ? 8ull * a.K : 0, st, l,
                               a.segptr, a.K, (uint32_t)alias_lds);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        } else if (PHASE == PH_WORD && !a.draw_only) {
            hipLaunchKernelGGL(long_cdf_kernel<M>, dim3(l.n < 1024 ? l.n : 1024), dim3(256), 0, st, l, a.segptr,
                               a.K);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        // the guide table where K is small enough that building it for every
        // chunk costs less than the binary-search steps it saves (measured:
        // long draw 0.357 -> 0.316 ms at K = 1000, slower at K = 1e4)
        const bool guided = cdf_lds && a.K <= Tuning::GUIDE_K_MAX;
        // where both the c_k histogram and the prefix counts would sit in LDS
        // (4096 < K <= 16384), the histogram comes from a pass over the
        // compact z array instead: the draw then needs half the LDS and runs
        // twice as many workgroups per CU
        const bool ck_split = PHASE == PH_WORD && !a.draw_only && cdf_lds && ck_lds && !guided;
        const bool ck_draw = ck_lds && !ck_split;
        const size_t lds = 4ull * ((ck_draw ? a.K : 0) + (cdf_lds ? a.K : 0) + (guided ? GUIDE_MAX / 2 : 0));
        // the global guides and the alias topics live in the tables until the
        // draw is done: clear them after it instead of inside it
        const bool guides_g = PHASE == PH_WORD && !a.draw_only && !cdf_lds;
        auto draw = [&](auto kern) -> hipError_t {
            hipError_t e2 = launch_dyn(kern, lds);
            if (e2 != hipSuccess) return e2;
            hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), lds, st, a, l, ck_split ? 2u : (uint32_t)ck_draw,
                               (uint32_t)(a.draw_only || guides_g ? 0 : 1),
                               (uint32_t)cdf_lds | (uint32_t)guided << 1);
            return hipGetLastError();
        };
        if constexpr (PHASE == PH_WORD) {
            e = alias ? draw(long_draw_kernel<PHASE, M, NW, ZT, true>) : draw(long_draw_kernel<PHASE, M, NW, ZT>);
        } else {
            e = draw(long_draw_kernel<PHASE, M, NW, ZT>);
        }
        if (e != hipSuccess) return e;
        if (ck_split) {
            const uint32_t gb = a.max_blocks < 256 ? a.max_blocks : 256;
            hipLaunchKernelGGL(long_ck_kernel<ZT>, dim3(gb), dim3(256), 4ull * a.K, st,
                               reinterpret_cast<const ZT *>(l.zc), l.total, a.K, a.ck_next);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        if (guides_g && (e = launch_fill_u32(l.tables, 0, l.table_words, st)) != hipSuccess) return e;
        if (ev) return hipEventRecord(ev[3], st);
        return hipSuccess;
    });
}

template <int PHASE, int M>
static hipError_t long_dispatch(const PhaseArgs &a, const LongList &l, hipStream_t st, hipEvent_t *ev) {
    if (l.n == 0) return hipSuccess;
    if (a.K <= 65535) return long_dispatch_z<PHASE, M, uint16_t>(a, l, st, ev);
    return long_dispatch_z<PHASE, M, uint32_t>(a, l, st, ev);
}

// The histogram pass alone (the log likelihood reads the tables it fills).
template <int PHASE, int M>
static hipError_t long_hist_dispatch(const PhaseArgs &a, const LongList &l, hipStream_t st) {
    if (l.n == 0) return hipSuccess;
    return with_rf_m<M>(a.rf, [&](auto rfc) -> hipError_t {
        constexpr int NW = decltype(rfc)::value;
        const bool lds_dense = a.K <= Tuning::LDS_DENSE_MAX;
        const uint32_t blocks = xcd_grid(l.n_chunks, a.max_blocks);
        const size_t lds = lds_dense ? 4ull * a.K : 4ull * 2 * 2 * Tuning::LONG_CHUNK_HASHED;
        hipError_t e = launch_dyn(long_hist_kernel<PHASE, M, NW>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((long_hist_kernel<PHASE, M, NW>), dim3(blocks), dim3(256), lds, st, a, l,
                           (uint32_t)lds_dense);
        return hipGetLastError();
    });
}

}  // namespace wlda
