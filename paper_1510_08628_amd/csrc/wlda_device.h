// Device arithmetic shared by the sampler and fold-in kernels: the counter-
// based generator and the exact binary32 decisions of one MH step.  Compiled
// without FP contraction, so every implementation of the same definitions
// takes the same decisions bit for bit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wlda {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32 -> 64-bit products mixed into the other lanes, with the Weyl key
// increments between rounds.  The full 64-bit products compile to one
// v_mad_u64_u32 each instead of a mul_hi / mul_lo pair.
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = (uint64_t)0xD2511F53u * c0;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)pb;
        c2 = n2;
        c3 = (uint32_t)pa;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// U(r) = (r >> 8) * 2^-24 on the 2^-24 grid; Dice(r, n) = (r * n) >> 32.
__device__ __forceinline__ float unif24(uint32_t r) { return (float)(r >> 8) * 0x1p-24f; }
__device__ __forceinline__ uint32_t dice(uint32_t r, uint32_t n) { return __umulhi(r, n); }

// Acceptance of Eq. (7): accept iff u * den < num with
//   num = (cnt[c] + prior) * (ck[s] + beta_bar),
//   den = (cnt[s] + prior) * (ck[c] + beta_bar).
// The second form takes ckb[k] = (float)ck[k] + beta_bar precomputed (the
// same binary32 value).
__device__ __forceinline__ bool mh_accept_b(float u, uint32_t cnt_c, uint32_t cnt_s, float prior,
                                            float ckb_s, float ckb_c) {
    const float num = ((float)cnt_c + prior) * ckb_s;
    const float den = ((float)cnt_s + prior) * ckb_c;
    return u * den < num;
}

__device__ __forceinline__ bool mh_accept(float u, uint32_t cnt_c, uint32_t cnt_s, float prior,
                                          uint32_t ck_s, uint32_t ck_c, float beta_bar) {
    return mh_accept_b(u, cnt_c, cnt_s, prior, (float)ck_s + beta_bar, (float)ck_c + beta_bar);
}

// The same with a prior per topic (asymmetric alpha in the doc phase):
// prior_c for the candidate, prior_s for the current state.  With
// prior_c == prior_s == prior the result is that of mh_accept_b.
__device__ __forceinline__ bool mh_accept_b2(float u, uint32_t cnt_c, uint32_t cnt_s, float prior_c,
                                             float prior_s, float ckb_s, float ckb_c) {
    const float num = ((float)cnt_c + prior_c) * ckb_s;
    const float den = ((float)cnt_s + prior_s) * ckb_c;
    return u * den < num;
}

// Prior part of a doc proposal under an asymmetric alpha: topic k with
// probability alpha_k / alpha_bar, given the running sums cum[k] = alpha_0 +
// ... + alpha_k in binary64: x = r 2^-32 cum[K-1] and the smallest k with
// cum[k] > x (one exists, since x < cum[K-1]).  A search whose trip count
// depends on K only.
__device__ __forceinline__ uint32_t alpha_prior_topic(const double *cum, uint32_t K, uint32_t r) {
    const double x = (double)r * 0x1p-32 * cum[K - 1];
    uint32_t base = 0;
    for (uint32_t n = K; n > 1;) {
        const uint32_t half = n >> 1;
        if (cum[base + half - 1] <= x) base += half;
        n -= half;
    }
    return base;
}

// Mixture coin of the proposals (Section 4.3): the count part with
// probability L / (L + mass).
__device__ __forceinline__ bool take_count_part(float u, uint32_t L, float mass) {
    return u * ((float)L + mass) < (float)L;
}

}  // namespace wlda
