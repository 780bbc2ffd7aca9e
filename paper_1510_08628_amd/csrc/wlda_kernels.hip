// gfx950 kernels of the WarpLDA sweep outside the per-M phase kernels:
// initialisation, c_k recount, the log joint likelihood (Section 6.1), the
// point estimates of Eq. (4), and the launchers that hand each phase to the
// translation unit of its M (wlda_kernels_m.hip).
#include "wlda_kernels_impl.h"

namespace wlda {

// --------------------------------------------------------------------------
// Small kernels
// --------------------------------------------------------------------------
__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
        p[i] = v;
}

// z = Dice(K) with the INIT counter (t, 0, 0, 0), t the canonical CSC
// position; proposals cleared.
template <int NW>
__global__ void init_z_kernel(uint64_t *recs, const uint32_t *colidx, uint32_t T, uint32_t K, uint32_t k0,
                              uint32_t k1) {
    for (uint32_t t = blockIdx.x * 256 + threadIdx.x; t < T; t += gridDim.x * 256) {
        const uint4 R = philox(t, 0, (uint32_t)PH_INIT << 16, 0, k0, k1);
        Rec<NW> r = rec_zero<NW>();
        set_fld(r, 0, dice(R.z, K));
        st_rec<NW>(recs, colidx ? colidx[t] : t, r);
    }
}

template <int NW>
__global__ void histogram_z_kernel(const uint64_t *recs, uint32_t T, uint32_t *ck) {
    for (uint32_t t = blockIdx.x * 256 + threadIdx.x; t < T; t += gridDim.x * 256)
        atomicAdd(&ck[fld(ld_rec<NW>(recs, t), 0)], 1u);
}

// --------------------------------------------------------------------------
// Log joint likelihood (Section 6.1), binary64.  One workgroup per segment,
// dense LDS counts (K <= LL_DENSE_MAX).
// --------------------------------------------------------------------------
constexpr uint32_t LL_DENSE_MAX = Tuning::LDS_DENSE_MAX;

__device__ double block_sum(double v) {
    __shared__ double part[4];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0) s = part[0] + part[1] + part[2] + part[3];
    __syncthreads();
    return s;
}

// One workgroup per listed segment: counts in LDS (dense for K <=
// LDS_DENSE_MAX, else an open-addressed table of pow2 >= 2L slots).
template <int NW>
__global__ __launch_bounds__(256) void ll_seg_kernel(const uint64_t *recs, const uint32_t *segptr,
                                                     const uint32_t *idx, const uint32_t *ids,
                                                     uint32_t n_seg, uint32_t K, uint32_t dense_u,
                                                     double prior, double prior_total,
                                                     int length_term, const float *alpha_k, double *out) {
    extern __shared__ uint32_t cnt[];
    const bool dense = dense_u != 0;
    const double lg_prior = lgamma(prior), lg_total = lgamma(prior_total);
    double acc = 0;
    for (uint32_t li = blockIdx.x; li < n_seg; li += gridDim.x) {
        const uint32_t s = ids[li];
        const uint32_t beg = segptr[s], L = segptr[s + 1] - beg;
        const uint32_t cap = dense ? K : pow2_at_least(2 * L);
        uint32_t *key = cnt, *c = dense ? cnt : cnt + cap;
        for (uint32_t k = threadIdx.x; k < cap; k += 256) {
            c[k] = 0;
            if (!dense) key[k] = EMPTY_KEY;
        }
        __syncthreads();
        for (uint32_t n = threadIdx.x; n < L; n += 256) {
            tab_insert(key, c, cap - 1, dense, fld(ld_rec<NW>(recs, idx ? idx[beg + n] : beg + n), 0));
        }
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < cap; k += 256) {
            const uint32_t v = c[k];
            if (!v) continue;
            if (alpha_k) {      // asymmetric alpha: the prior of this topic
                const double pk = (double)alpha_k[dense ? k : key[k]];
                acc += lgamma(pk + (double)v) - lgamma(pk);
            } else {
                acc += lgamma(prior + (double)v) - lg_prior;
            }
        }
        if (length_term && threadIdx.x == 0) acc += lg_total - lgamma(prior_total + (double)L);
        __syncthreads();
    }
    const double sum = block_sum(acc);
    if (threadIdx.x == 0) atomicAdd(out, sum);
}

// LL part of the long segments from their global tables (filled by the
// histogram pass); the tables are zeroed afterwards.
__global__ __launch_bounds__(256) void ll_tables_kernel(LongList l, const uint32_t *segptr, uint32_t K,
                                                        double prior, double prior_total,
                                                        int length_term, const float *alpha_k, double *out) {
    const double lg_prior = lgamma(prior), lg_total = lgamma(prior_total);
    double acc = 0;
    for (uint32_t j = blockIdx.x; j < l.n; j += gridDim.x) {
        uint32_t *base = l.tables + l.tab_off[j];
        const uint32_t cap = l.tab_cap[j];
        const uint32_t nslots = cap ? cap : K;
        uint32_t *c = cap ? base + cap : base;
        for (uint32_t k = threadIdx.x; k < nslots; k += 256) {
            const uint32_t v = c[k];
            if (!v) continue;
            if (alpha_k) {      // asymmetric alpha (hashed keys are topic + 1)
                const double pk = (double)alpha_k[cap ? base[k] - 1 : k];
                acc += lgamma(pk + (double)v) - lgamma(pk);
            } else {
                acc += lgamma(prior + (double)v) - lg_prior;
            }
        }
        if (length_term && threadIdx.x == 0) {
            const uint32_t s = l.ids[j];
            acc += lg_total - lgamma(prior_total + (double)(segptr[s + 1] - segptr[s]));
        }
    }
    const double sum = block_sum(acc);
    if (threadIdx.x == 0) atomicAdd(out, sum);
}

// theta_hat of Eq. (4) (alpha' = alpha + 1): out[d - d0][k] =
// (C_dk + alpha_k) / (L_d + alpha_bar) for documents d0 .. d0 + nd - 1
// (alpha_k = alpha when alpha_k is null).
template <int NW>
__global__ __launch_bounds__(256) void theta_kernel(const uint64_t *recs, const uint32_t *rowptr,
                                                    const uint32_t *rowidx, uint32_t d0, uint32_t nd,
                                                    uint32_t K, float alpha, const float *alpha_k,
                                                    float alpha_bar, float *out) {
    extern __shared__ uint32_t cnt[];
    for (uint32_t d = d0 + blockIdx.x; d < d0 + nd; d += gridDim.x) {
        const uint32_t beg = rowptr[d], L = rowptr[d + 1] - beg;
        for (uint32_t k = threadIdx.x; k < K; k += 256) cnt[k] = 0;
        __syncthreads();
        for (uint32_t n = threadIdx.x; n < L; n += 256)
            atomicAdd(&cnt[fld(ld_rec<NW>(recs, rowidx[beg + n]), 0)], 1u);
        __syncthreads();
        const float den = (float)L + alpha_bar;
        for (uint32_t k = threadIdx.x; k < K; k += 256)
            out[(size_t)(d - d0) * K + k] = ((float)cnt[k] + (alpha_k ? alpha_k[k] : alpha)) / den;
        __syncthreads();
    }
}

// phi_hat of Eq. (4) (beta' = beta + 1): out[w - w0][k] =
// (C_wk + beta) / (C_k + V beta) for words w0 .. w0 + nw - 1, one workgroup per
// word, c_w counted in LDS from the word's column.
template <int NW>
__global__ __launch_bounds__(256) void phi_kernel(const uint64_t *recs, const uint32_t *colptr,
                                                  const uint32_t *colidx, const uint32_t *ck, uint32_t w0,
                                                  uint32_t nw, uint32_t K, float beta, float beta_bar,
                                                  float *out) {
    extern __shared__ uint32_t cnt[];
    for (uint32_t w = w0 + blockIdx.x; w < w0 + nw; w += gridDim.x) {
        const uint32_t beg = colptr[w], L = colptr[w + 1] - beg;
        for (uint32_t k = threadIdx.x; k < K; k += 256) cnt[k] = 0;
        __syncthreads();
        for (uint32_t n = threadIdx.x; n < L; n += 256)
            atomicAdd(&cnt[fld(ld_rec<NW>(recs, colidx ? colidx[beg + n] : beg + n), 0)], 1u);
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < K; k += 256)
            out[(size_t)(w - w0) * K + k] = ((float)cnt[k] + beta) / ((float)ck[k] + beta_bar);
        __syncthreads();
    }
}

__global__ void ll_topics_kernel(const uint32_t *ck, uint32_t K, double beta_bar, double *out) {
    const double lg = lgamma(beta_bar);
    double acc = 0;
    for (uint32_t k = blockIdx.x * 256 + threadIdx.x; k < K; k += gridDim.x * 256)
        if (ck[k]) acc += lg - lgamma(beta_bar + (double)ck[k]);
    const double s = block_sum(acc);
    if (threadIdx.x == 0) atomicAdd(out, s);
}

// --------------------------------------------------------------------------
// Launchers
// --------------------------------------------------------------------------
static int grid_for(uint64_t n, int cap = 8192) {
    uint64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > (uint64_t)cap) b = cap;
    return (int)b;
}

// Calls f(std::integral_constant<int, RF>) for the record format rf.
template <typename F>
static hipError_t with_rf(int rf, F &&f) {
    switch (rf) {
        case -16: return f(std::integral_constant<int, -16>{});
        case -10: return f(std::integral_constant<int, -10>{});
        case -8: return f(std::integral_constant<int, -8>{});
        case -6: return f(std::integral_constant<int, -6>{});
        case 1: return f(std::integral_constant<int, 1>{});
        case 2: return f(std::integral_constant<int, 2>{});
        case 102: return f(std::integral_constant<int, 102>{});
        case 103: return f(std::integral_constant<int, 103>{});
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, uint64_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

hipError_t launch_init_z(uint64_t *recs, const uint32_t *colidx, uint32_t T, uint32_t M, uint32_t K,
                         uint32_t k0, uint32_t k1, hipStream_t st) {
    if (T == 0) return hipSuccess;
    return with_rf(record_format(M, K), [&](auto c) {
        hipLaunchKernelGGL(init_z_kernel<decltype(c)::value>, dim3(grid_for(T)), dim3(256), 0, st, recs, colidx, T,
                           K, k0, k1);
        return hipGetLastError();
    });
}

hipError_t launch_segments(const PhaseArgs &a, uint32_t phase, uint32_t M, const SegList &l, int bin,
                           hipStream_t st) {
    switch (M) {
        case 1: return seg_launch<1>(a, phase, l, bin, st);
        case 2: return seg_launch<2>(a, phase, l, bin, st);
        case 3: return seg_launch<3>(a, phase, l, bin, st);
        case 4: return seg_launch<4>(a, phase, l, bin, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_long_segments(const PhaseArgs &a, uint32_t phase, uint32_t M, const LongList &l,
                                hipStream_t st, hipEvent_t *ev) {
    switch (M) {
        case 1: return long_launch<1>(a, phase, l, st, ev);
        case 2: return long_launch<2>(a, phase, l, st, ev);
        case 3: return long_launch<3>(a, phase, l, st, ev);
        case 4: return long_launch<4>(a, phase, l, st, ev);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_histogram_z(const uint64_t *recs, uint32_t T, uint32_t M, uint32_t K, uint32_t *ck,
                              hipStream_t st) {
    if (T == 0) return hipSuccess;
    return with_rf(record_format(M, K), [&](auto c) {
        hipLaunchKernelGGL(histogram_z_kernel<decltype(c)::value>, dim3(grid_for(T)), dim3(256), 0, st, recs, T, ck);
        return hipGetLastError();
    });
}

hipError_t launch_ll_list(const uint64_t *recs, uint32_t M, const uint32_t *segptr, const uint32_t *idx,
                          const uint32_t *ids, uint32_t n, uint32_t K, double prior, double prior_total,
                          int length_term, double *out, hipStream_t st, const float *alpha_k) {
    if (n == 0) return hipSuccess;
    const bool dense = K <= Tuning::LDS_DENSE_MAX;
    const size_t lds = dense ? 4ull * K : 4ull * 2 * 2 * Tuning::WIDE_MAX;
    const int blocks = n < 4096 ? (int)n : 4096;
    return with_rf(record_format(M, K), [&](auto c) {
        constexpr int RF = decltype(c)::value;
        hipError_t e = launch_dyn(ll_seg_kernel<RF>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(ll_seg_kernel<RF>, dim3(blocks), dim3(256), lds, st, recs, segptr, idx, ids, n, K,
                           (uint32_t)dense, prior, prior_total, length_term, alpha_k, out);
        return hipGetLastError();
    });
}

hipError_t launch_ll_long(const PhaseArgs &a, uint32_t phase, uint32_t M, const LongList &l, double prior,
                          double prior_total, int length_term, double *out, hipStream_t st) {
    if (l.n == 0) return hipSuccess;
    PhaseArgs h = a;
    h.max_blocks = 2048;
    h.draw_only = 0;
    hipError_t e;
    switch (M) {
        case 1: e = long_hist_launch<1>(h, phase, l, st); break;
        case 2: e = long_hist_launch<2>(h, phase, l, st); break;
        case 3: e = long_hist_launch<3>(h, phase, l, st); break;
        case 4: e = long_hist_launch<4>(h, phase, l, st); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ll_tables_kernel, dim3(l.n < 1024 ? l.n : 1024), dim3(256), 0, st, l, a.segptr, a.K, prior,
                       prior_total, length_term, a.alpha_k, out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_fill_u32(l.tables, 0, l.table_words, st);
}

hipError_t launch_theta(const uint64_t *recs, uint32_t M, const uint32_t *rowptr, const uint32_t *idx,
                        uint32_t d0, uint32_t nd, uint32_t K, float alpha, const float *alpha_k,
                        float alpha_bar, float *out, hipStream_t st) {
    if (nd == 0) return hipSuccess;
    if (K > LL_DENSE_MAX) return hipErrorNotSupported;
    const size_t lds = 4ull * K;
    const int blocks = nd < 8192 ? (int)nd : 8192;
    return with_rf(record_format(M, K), [&](auto c) {
        constexpr int RF = decltype(c)::value;
        hipError_t e = launch_dyn(theta_kernel<RF>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(theta_kernel<RF>, dim3(blocks), dim3(256), lds, st, recs, rowptr, idx, d0, nd, K,
                           alpha, alpha_k, alpha_bar, out);
        return hipGetLastError();
    });
}

hipError_t launch_phi(const uint64_t *recs, uint32_t M, const uint32_t *colptr, const uint32_t *colidx,
                      const uint32_t *ck, uint32_t w0, uint32_t nw, uint32_t K, float beta, float beta_bar,
                      float *out, hipStream_t st) {
    if (nw == 0) return hipSuccess;
    if (K > LL_DENSE_MAX) return hipErrorNotSupported;
    const size_t lds = 4ull * K;
    const int blocks = nw < 8192 ? (int)nw : 8192;
    return with_rf(record_format(M, K), [&](auto c) {
        constexpr int RF = decltype(c)::value;
        hipError_t e = launch_dyn(phi_kernel<RF>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(phi_kernel<RF>, dim3(blocks), dim3(256), lds, st, recs, colptr, colidx, ck, w0, nw, K,
                           beta, beta_bar, out);
        return hipGetLastError();
    });
}

hipError_t launch_ll_topics(const uint32_t *ck, uint32_t K, double beta_bar, double *out,
                            hipStream_t st) {
    hipLaunchKernelGGL(ll_topics_kernel, dim3(grid_for(K, 256)), dim3(256), 0, st, ck, K, beta_bar,
                       out);
    return hipGetLastError();
}

}  // namespace wlda