// MLP encoder for the learned fold-in proposal (gfx950).
//
// x = hashed bag of words (bucket of each distinct word, value tf / L), then
//   a1 = b1 + sum_n x_n W1[bucket_n]      (embedding bag, W1: H x 512 bf16)
//   h1 = relu(a1)                         (rounded to bf16 for the next GEMM)
//   a2 = h1 W2 + b2, h2 = relu(a2)        (W2: 512 x 512 bf16, MFMA)
//   z  = h2 W3 + b3, q = softmax(z)       (W3: 512 x K bf16, MFMA)
// trained with the soft cross-entropy -sum_k theta_k log q_k against the
// sampler's own theta_d = (C_dk + alpha) / (L_d + K alpha), by Adam on fp32
// master weights.  Every GEMM takes bf16 operands and accumulates in fp32 on
// the matrix cores (v_mfma_f32_32x32x16_bf16); back-propagated signals are
// rounded to bf16 at the same points as the forward activations.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/warplda.h"

namespace wlda {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t to_bf16(float f) {   // round to nearest even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// C[M x N] (+)= A[M x Kd] B[Kd x N]; bf16 operands addressed by (row, col)
// strides so that transposed operands need no copy; fp32 result.
// 256 threads, 64 x 64 tile, one 32 x 32 MFMA sub-tile per wavefront.
constexpr int GT = 64, GK = 32, GPAD = 8;

__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int Kd, const uint16_t *A,
                                                        long a_rs, long a_cs, const uint16_t *B,
                                                        long b_rs, long b_cs, float *C, int ldc,
                                                        int accumulate) {
    __shared__ uint16_t As[GT][GK + GPAD];
    __shared__ uint16_t Bs[GK][GT + GPAD];
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    f32x16 acc = {};
    for (int k0 = 0; k0 < Kd; k0 += GK) {
        for (int e = threadIdx.x; e < GT * GK; e += 256) {
            const int r = e / GK, c = e % GK;
            const int gr = m0 + r, gc = k0 + c;
            As[r][c] = (gr < M && gc < Kd) ? A[gr * a_rs + gc * a_cs] : (uint16_t)0;
        }
        for (int e = threadIdx.x; e < GK * GT; e += 256) {
            const int r = e / GT, c = e % GT;
            const int gr = k0 + r, gc = n0 + c;
            Bs[r][c] = (gr < Kd && gc < N) ? B[gr * b_rs + gc * b_cs] : (uint16_t)0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; kk += 16) {
            bf16x8 a, b;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                a[e] = __builtin_bit_cast(__bf16, As[wr + (l & 31)][kk + 8 * (l >> 5) + e]);
                b[e] = __builtin_bit_cast(__bf16, Bs[kk + 8 * (l >> 5) + e][wc + (l & 31)]);
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int r = m0 + wr + 8 * (v >> 2) + 4 * (l >> 5) + (v & 3);
        const int c = n0 + wc + (l & 31);
        if (r < M && c < N) {
            float *dst = &C[(long)r * ldc + c];
            *dst = accumulate ? *dst + acc[v] : acc[v];
        }
    }
}

// a1[b][j] = b1[j] + sum_n val_n W1b[idx_n][j]; h1b = bf16(relu(a1))
// One workgroup per document.  Eight features at a time with separate partial
// sums, so eight row reads of W1 are in flight per thread (a single running
// sum serialises one dependent load per feature); the partial sums are added
// in a fixed order, so the result is deterministic.
__global__ __launch_bounds__(256) void embag_fwd_kernel(int H, const uint32_t *rowptr, const uint32_t *idx,
                                                        const float *val, const uint16_t *W1b,
                                                        const float *b1, float *a1, uint16_t *h1b) {
    // The document's nonzeros are split into four contiguous quarters, one
    // per wavefront; for each block of 64 * JPL hidden units every lane
    // accumulates JPL of them (lane, lane + 64, ...) over R rows at a time, so
    // R * JPL row loads are in flight; the four partial sums are then added
    // in a fixed order.
    constexpr int JPL = 8, R = 4, JB = 64 * JPL;
    __shared__ float part[4][JB];
    const int b = blockIdx.x;
    const uint32_t n0 = rowptr[b], n1 = rowptr[b + 1];
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t q = (n1 - n0 + 3) / 4;
    const uint32_t r0 = min(n1, n0 + wave * q), r1 = min(n1, r0 + q);
    for (int jb = 0; jb < H; jb += JB) {
        float acc[JPL];
#pragma unroll
        for (int u = 0; u < JPL; ++u) acc[u] = 0.f;
        // hidden units past H read unit H - 1 (in bounds, never stored), so
        // every load of a batch is issued without a branch
        int jc[JPL];
#pragma unroll
        for (int u = 0; u < JPL; ++u) jc[u] = min(jb + (int)lane + 64 * u, H - 1);
        uint32_t n = r0;
        for (; n + R <= r1; n += R) {
            uint32_t row[R];
            float v[R], w[R][JPL];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                row[r] = idx[n + r];
                v[r] = val[n + r];
            }
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int u = 0; u < JPL; ++u) w[r][u] = from_bf16(W1b[(size_t)row[r] * H + jc[u]]);
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int u = 0; u < JPL; ++u) acc[u] += v[r] * w[r][u];
        }
        for (; n < r1; ++n) {
            const uint32_t row = idx[n];
            const float v = val[n];
#pragma unroll
            for (int u = 0; u < JPL; ++u) acc[u] += v * from_bf16(W1b[(size_t)row * H + jc[u]]);
        }
#pragma unroll
        for (int u = 0; u < JPL; ++u) part[wave][lane + 64 * u] = acc[u];
        __syncthreads();
        for (int jj = threadIdx.x; jj < JB && jb + jj < H; jj += 256) {
            const int j = jb + jj;
            const float sum = b1[j] + ((part[0][jj] + part[1][jj]) + (part[2][jj] + part[3][jj]));
            a1[(size_t)b * H + j] = sum;
            h1b[(size_t)b * H + j] = to_bf16(sum > 0.f ? sum : 0.f);
        }
        __syncthreads();
    }
}

// a = c + bias; hb = bf16(relu(a)); a kept for the ReLU mask
__global__ void bias_relu_kernel(int rows, int cols, const float *c, const float *bias, float *a, uint16_t *hb) {
    const long n = (long)rows * cols;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
        const float v = c[i] + bias[i % cols];
        a[i] = v;
        hb[i] = to_bf16(v > 0.f ? v : 0.f);
    }
}

// logits = c + b3; q = softmax; loss_b = -sum theta log q; g = (q - theta)/B
__global__ __launch_bounds__(256) void softmax_ce_kernel(int K, int B, const float *c, const float *b3,
                                                         const float *theta, float *probs, float *g,
                                                         uint16_t *gb, float *loss_rows) {
    __shared__ float red[4];
    const int b = blockIdx.x;
    const float *z = c + (size_t)b * K;
    float mx = -3.4e38f;
    for (int k = threadIdx.x; k < K; k += 256) mx = fmaxf(mx, z[k] + b3[k]);
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    __syncthreads();
    float s = 0.f;
    for (int k = threadIdx.x; k < K; k += 256) s += expf(z[k] + b3[k] - mx);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    s = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    const float ls = logf(s);
    float lo = 0.f;
    for (int k = threadIdx.x; k < K; k += 256) {
        const float lq = z[k] + b3[k] - mx - ls;
        const float q = expf(lq);
        if (probs) probs[(size_t)b * K + k] = q;
        if (theta) {
            const float t = theta[(size_t)b * K + k];
            lo -= t * lq;
            const float gv = (q - t) / (float)B;
            g[(size_t)b * K + k] = gv;
            gb[(size_t)b * K + k] = to_bf16(gv);
        }
    }
    if (theta && loss_rows) {
        for (int o = 32; o > 0; o >>= 1) lo += __shfl_xor(lo, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lo;
        __syncthreads();
        if (threadIdx.x == 0) loss_rows[b] = red[0] + red[1] + red[2] + red[3];
    }
}

// g = d * [a > 0]; gb = bf16(g)
__global__ void relu_bwd_kernel(long n, const float *d, const float *a, float *g, uint16_t *gb) {
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
        const float v = a[i] > 0.f ? d[i] : 0.f;
        g[i] = v;
        if (gb) gb[i] = to_bf16(v);
    }
}

// Column sums of g (rows x cols) into db: a workgroup owns 32 columns; each
// of its eight row groups sums every eighth row with eight loads in flight,
// and the eight partial sums are added in a fixed order.
__global__ __launch_bounds__(256) void colsum_kernel(int rows, int cols, const float *g, float *db) {
    __shared__ float part[8][32];
    const int c = threadIdx.x & 31, rg = threadIdx.x >> 5;
    const int j = blockIdx.x * 32 + c;
    float s = 0.f;
    if (j < cols) {
        int r = rg;
        for (; r + 56 < rows; r += 64) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = g[(size_t)(r + 8 * u) * cols + j];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; r < rows; r += 8) s += g[(size_t)r * cols + j];
    }
    part[rg][c] = s;
    __syncthreads();
    if (rg == 0 && j < cols) {
        float t = 0.f;
        for (int q = 0; q < 8; ++q) t += part[q][c];
        db[j] = t;
    }
}

// Embedding-bag backward, dW1[u] = sum over the batch's nonzeros (b, u, val)
// of val * g1[b].  The batch (CSR by document) is transposed into lists per
// bucket u (count, exclusive scan, scatter), and one workgroup sums each
// touched bucket's list into its gradient row: no atomics on the H-wide rows.
// A batch with more nonzeros than the list holds (rowptr[B] - rowptr[0] >
// cap, known only on the device; rowptr may be a slice of a larger CSR, with
// offsets into its idx and val) takes the atomic kernel instead; every kernel
// below reads rowptr[0] and rowptr[B] and returns at once when it is not the
// one in charge.
__global__ __launch_bounds__(256) void embag_count_kernel(const uint32_t *rowptr, const uint32_t *idx, uint32_t B,
                                                          uint32_t cap, uint32_t *cnt) {
    if (rowptr[B] - rowptr[0] > cap) return;
    const uint32_t b = blockIdx.x;
    for (uint32_t n = rowptr[b] + threadIdx.x; n < rowptr[b + 1]; n += 256) atomicAdd(&cnt[idx[n]], 1u);
}

// Exclusive scan of cnt[0..nb) into off[0..nb] (off[nb] = total), copied to
// cur; one workgroup of 1024 threads walks tiles of 4096 counts, each thread
// four consecutive ones (coalesced), carrying the running total.
__global__ __launch_bounds__(1024) void embag_scan_kernel(const uint32_t *rowptr, uint32_t B, uint32_t cap,
                                                          uint32_t nb, const uint32_t *cnt, uint32_t *off,
                                                          uint32_t *cur) {
    if (rowptr[B] - rowptr[0] > cap) return;
    __shared__ uint32_t wsum[16];
    const uint32_t wl = threadIdx.x & 63;
    uint32_t carry = 0;
    for (uint32_t t0 = 0; t0 < nb; t0 += 4096) {
        const uint32_t k0 = t0 + threadIdx.x * 4;
        uint32_t v[4], sum = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            v[i] = k0 + i < nb ? cnt[k0 + i] : 0u;
            sum += v[i];
        }
        uint32_t x = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, 64);
            if (wl >= (uint32_t)o) x += y;
        }
        if (wl == 63) wsum[threadIdx.x >> 6] = x;
        __syncthreads();
        uint32_t base = carry, tile = 0;
        for (uint32_t w = 0; w < 16; ++w) {
            if (w < (threadIdx.x >> 6)) base += wsum[w];
            tile += wsum[w];
        }
        uint32_t run = base + x - sum;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (k0 + i < nb) {
                off[k0 + i] = run;
                cur[k0 + i] = run;
            }
            run += v[i];
        }
        carry += tile;
        __syncthreads();
    }
    if (threadIdx.x == 0) off[nb] = carry;
}

__global__ __launch_bounds__(256) void embag_scatter_kernel(const uint32_t *rowptr, const uint32_t *idx,
                                                            const float *val, uint32_t B, uint32_t cap,
                                                            uint32_t *cur, uint2 *list) {
    if (rowptr[B] - rowptr[0] > cap) return;
    const uint32_t b = blockIdx.x;
    for (uint32_t n = rowptr[b] + threadIdx.x; n < rowptr[b + 1]; n += 256) {
        const uint32_t q = atomicAdd(&cur[idx[n]], 1u);
        list[q] = make_uint2(b, __float_as_uint(val[n]));
    }
}

// One workgroup per touched bucket: its list goes through LDS 256 entries at
// a time, and each thread sums its columns with eight g1 rows in flight.
__global__ __launch_bounds__(256) void embag_wgrad_kernel(const uint32_t *rowptr, uint32_t B, uint32_t cap,
                                                          uint32_t nb, int H, const uint32_t *off,
                                                          const uint2 *list, const float *g1, float *dW1) {
    if (rowptr[B] - rowptr[0] > cap) return;
    __shared__ uint2 ent[256];
    for (uint32_t u = blockIdx.x; u < nb; u += gridDim.x) {
        const uint32_t q0 = off[u], q1 = off[u + 1];
        if (q0 == q1) continue;
        // columns of this thread: j = threadIdx.x + 256 c, c < CMAX (H <= 4096)
        constexpr int CMAX = 16;
        float acc[CMAX];
#pragma unroll
        for (int c = 0; c < CMAX; ++c) acc[c] = 0.f;
        for (uint32_t e0 = q0; e0 < q1; e0 += 256) {
            const uint32_t ne = min(256u, q1 - e0);
            __syncthreads();
            if (threadIdx.x < ne) ent[threadIdx.x] = list[e0 + threadIdx.x];
            __syncthreads();
#pragma unroll
            for (int c = 0; c < CMAX; ++c) {
                const int j = threadIdx.x + 256 * c;
                if (j >= H) break;
                uint32_t q = 0;
                for (; q + 8 <= ne; q += 8) {
                    float g[8];
#pragma unroll
                    for (int r = 0; r < 8; ++r) g[r] = g1[(size_t)ent[q + r].x * H + j];
#pragma unroll
                    for (int r = 0; r < 8; ++r) acc[c] += __uint_as_float(ent[q + r].y) * g[r];
                }
                for (; q < ne; ++q) acc[c] += __uint_as_float(ent[q].y) * g1[(size_t)ent[q].x * H + j];
            }
        }
#pragma unroll
        for (int c = 0; c < CMAX; ++c) {
            const int j = threadIdx.x + 256 * c;
            if (j < H) dW1[(size_t)u * H + j] = acc[c];
        }
    }
}

// dW1[idx_n] += val_n * g1[b], one workgroup per document (batches too large
// for the transpose lists only).
__global__ __launch_bounds__(256) void embag_bwd_kernel(int H, const uint32_t *rowptr, const uint32_t *idx,
                                                        const float *val, const float *g1, float *dW1,
                                                        uint32_t B, uint32_t cap) {
    if (rowptr[B] - rowptr[0] <= cap) return;
    const int b = blockIdx.x;
    for (uint32_t n = rowptr[b]; n < rowptr[b + 1]; ++n)
        for (int j = threadIdx.x; j < H; j += 256)
            atomicAdd(&dW1[(size_t)idx[n] * H + j], val[n] * g1[(size_t)b * H + j]);
}

__global__ void adam_kernel(long n, float *w, float *m, float *v, const float *g, uint16_t *wb, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        w[i] = wi;
        if (wb) wb[i] = to_bf16(wi);
    }
}

__global__ void to_bf16_kernel(long n, const float *w, uint16_t *wb) {
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) wb[i] = to_bf16(w[i]);
}

__global__ void zero_f32_kernel(long n, float *p) {
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) p[i] = 0.f;
}

// Learned proposal weights from the encoder's output: w_k = 1 + floor(2^20 *
// ((1 - eps) q_k + eps / K)), stored as running sums (an exact integer CDF).
__global__ __launch_bounds__(256) void probs_to_cdf_kernel(int K, const float *probs, float eps, uint32_t *cdf) {
    __shared__ uint32_t part[256];
    const int b = blockIdx.x;
    const int per = (K + 255) / 256;
    const int k0 = threadIdx.x * per, k1 = min(K, k0 + per);
    uint32_t s = 0;
    for (int k = k0; k < k1; ++k) {
        const float q = (1.f - eps) * probs[(size_t)b * K + k] + eps / (float)K;
        s += 1u + (uint32_t)floorf(q * 1048576.f);
    }
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int t = 0; t < 256; ++t) {
            const uint32_t v = part[t];
            part[t] = run;
            run += v;
        }
    }
    __syncthreads();
    uint32_t run = part[threadIdx.x];
    for (int k = k0; k < k1; ++k) {
        const float q = (1.f - eps) * probs[(size_t)b * K + k] + eps / (float)K;
        run += 1u + (uint32_t)floorf(q * 1048576.f);
        cdf[(size_t)b * K + k] = run;
    }
}

}  // namespace wlda

using namespace wlda;

struct wlda_encoder_s;

// ============================================================================
// Host side
// ============================================================================
struct wlda_encoder_s {
    wlda_encoder_params p{};
    hipStream_t st = nullptr;
    // parameters: fp32 master, Adam moments, gradients, bf16 copies
    float *w[6] = {}, *m[6] = {}, *v[6] = {}, *g[6] = {};
    uint16_t *wb[3] = {};      // W1, W2, W3 in bf16
    long n[6] = {};
    // activations (max_batch rows)
    float *a1 = nullptr, *a2 = nullptr, *c2 = nullptr, *c3 = nullptr, *probs = nullptr, *g3 = nullptr,
          *d2 = nullptr, *g2 = nullptr, *d1 = nullptr, *g1 = nullptr, *loss_rows = nullptr;
    uint16_t *h1b = nullptr, *h2b = nullptr, *g3b = nullptr, *g2b = nullptr;
    // embedding-bag backward: per-bucket counts, offsets, cursors and lists
    uint32_t *tcnt = nullptr, *toff = nullptr, *tcur = nullptr;
    uint2 *tlist = nullptr;
    uint32_t tcap = 0;
    uint64_t steps = 0;
};

namespace wlda {
uint32_t wlda_encoder_get_k(wlda_encoder e) { return e->p.K; }
uint32_t wlda_encoder_get_buckets(wlda_encoder e) { return e->p.buckets; }
uint32_t wlda_encoder_get_max_batch(wlda_encoder e) { return e->p.max_batch; }
void *wlda_encoder_get_stream(wlda_encoder e) { return (void *)e->st; }
}  // namespace wlda

namespace {
constexpr uint64_t EALIGN = 256;
inline uint64_t ea(uint64_t x) { return (x + EALIGN - 1) / EALIGN * EALIGN; }

void param_sizes(const wlda_encoder_params &p, long n[6]) {
    n[0] = (long)p.buckets * p.hidden;   // W1
    n[1] = p.hidden;                     // b1
    n[2] = (long)p.hidden * p.hidden;    // W2
    n[3] = p.hidden;                     // b2
    n[4] = (long)p.hidden * p.K;         // W3
    n[5] = p.K;                          // b3
}

// Nonzeros the embedding-bag backward's transpose lists hold: 4096 per
// document of a full batch, at most 2^22 (a larger batch takes the atomic
// kernel).
uint32_t transpose_cap(const wlda_encoder_params &p) {
    return (uint32_t)std::min<uint64_t>(4096ull * p.max_batch, 1ull << 22);
}

uint64_t enc_bytes(const wlda_encoder_params &p) {
    long n[6];
    param_sizes(p, n);
    uint64_t t = 0;
    for (int i = 0; i < 6; ++i) t += 4 * ea(4ull * n[i]);
    t += ea(2ull * n[0]) + ea(2ull * n[2]) + ea(2ull * n[4]);
    const uint64_t B = p.max_batch, Hd = p.hidden, K = p.K;
    t += 7 * ea(4 * B * Hd) + 3 * ea(4 * B * K) + ea(4 * B) + 3 * ea(2 * B * Hd) + ea(2 * B * K);
    t += 3 * ea(4ull * (p.buckets + 1)) + ea(8ull * transpose_cap(p));
    return t;
}

int grid(long n) { return (int)std::min<long>((n + 255) / 256, 8192); }

hipError_t gemm(hipStream_t st, int M, int N, int Kd, const uint16_t *A, long a_rs, long a_cs,
                const uint16_t *B, long b_rs, long b_cs, float *C, int ldc, int acc) {
    dim3 g((N + GT - 1) / GT, (M + GT - 1) / GT);
    hipLaunchKernelGGL(gemm_bf16_kernel, g, dim3(256), 0, st, M, N, Kd, A, a_rs, a_cs, B, b_rs, b_cs, C, ldc,
                       acc);
    return hipGetLastError();
}

bool valid(const wlda_encoder_params *p) {
    return p && p->buckets >= 1 && p->hidden >= 1 && p->hidden <= 4096 && p->K >= 1 && p->K <= (1u << 20) &&
           p->max_batch >= 1 && p->max_batch <= 65536 && p->lr > 0;
}

// Forward for B rows; leaves activations in the encoder's buffers.
hipError_t forward(wlda_encoder e, uint32_t B, const uint32_t *rowptr, const uint32_t *idx, const float *val) {
    const int Hd = e->p.hidden, K = e->p.K;
    hipStream_t st = e->st;
    hipError_t r;
    hipLaunchKernelGGL(embag_fwd_kernel, dim3(B), dim3(256), 0, st, Hd, rowptr, idx, val, e->wb[0], e->w[1],
                       e->a1, e->h1b);
    if ((r = hipGetLastError())) return r;
    if ((r = gemm(st, B, Hd, Hd, e->h1b, Hd, 1, e->wb[1], Hd, 1, e->c2, Hd, 0))) return r;
    hipLaunchKernelGGL(bias_relu_kernel, dim3(grid((long)B * Hd)), dim3(256), 0, st, (int)B, Hd, e->c2, e->w[3],
                       e->a2, e->h2b);
    if ((r = hipGetLastError())) return r;
    return gemm(st, B, K, Hd, e->h2b, Hd, 1, e->wb[2], K, 1, e->c3, K, 0);
}

// Loss and gradients (no update) for B rows with targets theta.
hipError_t backward(wlda_encoder e, uint32_t B, const uint32_t *rowptr, const uint32_t *idx, const float *val,
                    const float *theta) {
    const int Hd = e->p.hidden, K = e->p.K;
    hipStream_t st = e->st;
    hipError_t r;
    hipLaunchKernelGGL(softmax_ce_kernel, dim3(B), dim3(256), 0, st, K, (int)B, e->c3, e->w[5], theta, e->probs,
                       e->g3, e->g3b, e->loss_rows);
    if ((r = hipGetLastError())) return r;
    // layer 3
    if ((r = gemm(st, Hd, K, B, e->h2b, 1, Hd, e->g3b, K, 1, e->g[4], K, 0))) return r;
    hipLaunchKernelGGL(colsum_kernel, dim3((K + 31) / 32), dim3(256), 0, st, (int)B, K, e->g3, e->g[5]);
    if ((r = gemm(st, B, Hd, K, e->g3b, K, 1, e->wb[2], 1, K, e->d2, Hd, 0))) return r;
    hipLaunchKernelGGL(relu_bwd_kernel, dim3(grid((long)B * Hd)), dim3(256), 0, st, (long)B * Hd, e->d2, e->a2,
                       e->g2, e->g2b);
    // layer 2
    if ((r = gemm(st, Hd, Hd, B, e->h1b, 1, Hd, e->g2b, Hd, 1, e->g[2], Hd, 0))) return r;
    hipLaunchKernelGGL(colsum_kernel, dim3((Hd + 31) / 32), dim3(256), 0, st, (int)B, Hd, e->g2, e->g[3]);
    if ((r = gemm(st, B, Hd, Hd, e->g2b, Hd, 1, e->wb[1], 1, Hd, e->d1, Hd, 0))) return r;
    hipLaunchKernelGGL(relu_bwd_kernel, dim3(grid((long)B * Hd)), dim3(256), 0, st, (long)B * Hd, e->d1, e->a1,
                       e->g1, (uint16_t *)nullptr);
    // layer 1 (embedding bag)
    hipLaunchKernelGGL(colsum_kernel, dim3((Hd + 31) / 32), dim3(256), 0, st, (int)B, Hd, e->g1, e->g[1]);
    hipLaunchKernelGGL(zero_f32_kernel, dim3(grid(e->n[0])), dim3(256), 0, st, e->n[0], e->g[0]);
    const uint32_t nb = e->p.buckets, cap = e->tcap;
    hipLaunchKernelGGL(zero_f32_kernel, dim3(grid(nb)), dim3(256), 0, st, (long)nb, (float *)e->tcnt);
    hipLaunchKernelGGL(embag_count_kernel, dim3(B), dim3(256), 0, st, rowptr, idx, B, cap, e->tcnt);
    hipLaunchKernelGGL(embag_scan_kernel, dim3(1), dim3(1024), 0, st, rowptr, B, cap, nb, e->tcnt, e->toff, e->tcur);
    hipLaunchKernelGGL(embag_scatter_kernel, dim3(B), dim3(256), 0, st, rowptr, idx, val, B, cap, e->tcur,
                       e->tlist);
    hipLaunchKernelGGL(embag_wgrad_kernel, dim3(std::min<uint32_t>(nb, 8192)), dim3(256), 0, st, rowptr, B, cap,
                       nb, Hd, e->toff, e->tlist, e->g1, e->g[0]);
    hipLaunchKernelGGL(embag_bwd_kernel, dim3(B), dim3(256), 0, st, Hd, rowptr, idx, val, e->g1, e->g[0], B, cap);
    return hipGetLastError();
}

hipError_t refresh_bf16(wlda_encoder e) {
    const int map[3] = {0, 2, 4};
    for (int i = 0; i < 3; ++i)
        hipLaunchKernelGGL(to_bf16_kernel, dim3(grid(e->n[map[i]])), dim3(256), 0, e->st, e->n[map[i]],
                           e->w[map[i]], e->wb[i]);
    return hipGetLastError();
}

}  // namespace

extern "C" {

wlda_status wlda_encoder_workspace_bytes(const wlda_encoder_params *p, uint64_t *bytes) {
    if (!valid(p) || !bytes) return WLDA_E_INVALID;
    *bytes = enc_bytes(*p);
    return WLDA_OK;
}

wlda_status wlda_encoder_create(const wlda_encoder_params *p, void *ws, uint64_t ws_bytes, void *stream,
                                wlda_encoder *out) {
    if (!valid(p) || !out) return WLDA_E_INVALID;
    *out = nullptr;
    if (!ws || ((uintptr_t)ws % EALIGN) || ws_bytes < enc_bytes(*p)) return WLDA_E_WORKSPACE;
    wlda_encoder e = new (std::nothrow) wlda_encoder_s();
    if (!e) return WLDA_E_INVALID;
    e->p = *p;
    e->st = (hipStream_t)stream;
    param_sizes(*p, e->n);
    uint8_t *c = (uint8_t *)ws;
    auto take = [&](uint64_t b) { uint8_t *q = c; c += ea(b); return q; };
    for (int i = 0; i < 6; ++i) {
        e->w[i] = (float *)take(4ull * e->n[i]);
        e->m[i] = (float *)take(4ull * e->n[i]);
        e->v[i] = (float *)take(4ull * e->n[i]);
        e->g[i] = (float *)take(4ull * e->n[i]);
    }
    e->wb[0] = (uint16_t *)take(2ull * e->n[0]);
    e->wb[1] = (uint16_t *)take(2ull * e->n[2]);
    e->wb[2] = (uint16_t *)take(2ull * e->n[4]);
    const uint64_t B = p->max_batch, Hd = p->hidden, K = p->K;
    e->a1 = (float *)take(4 * B * Hd);
    e->a2 = (float *)take(4 * B * Hd);
    e->c2 = (float *)take(4 * B * Hd);
    e->d2 = (float *)take(4 * B * Hd);
    e->g2 = (float *)take(4 * B * Hd);
    e->d1 = (float *)take(4 * B * Hd);
    e->g1 = (float *)take(4 * B * Hd);
    e->c3 = (float *)take(4 * B * K);
    e->probs = (float *)take(4 * B * K);
    e->g3 = (float *)take(4 * B * K);
    e->loss_rows = (float *)take(4 * B);
    e->h1b = (uint16_t *)take(2 * B * Hd);
    e->h2b = (uint16_t *)take(2 * B * Hd);
    e->g2b = (uint16_t *)take(2 * B * Hd);
    e->g3b = (uint16_t *)take(2 * B * K);
    e->tcnt = (uint32_t *)take(4ull * (p->buckets + 1));
    e->toff = (uint32_t *)take(4ull * (p->buckets + 1));
    e->tcur = (uint32_t *)take(4ull * (p->buckets + 1));
    e->tcap = transpose_cap(*p);
    e->tlist = (uint2 *)take(8ull * e->tcap);
    hipError_t r = hipSuccess;
    for (int i = 0; i < 6 && !r; ++i) {
        hipLaunchKernelGGL(zero_f32_kernel, dim3(grid(e->n[i])), dim3(256), 0, e->st, e->n[i], e->w[i]);
        hipLaunchKernelGGL(zero_f32_kernel, dim3(grid(e->n[i])), dim3(256), 0, e->st, e->n[i], e->m[i]);
        hipLaunchKernelGGL(zero_f32_kernel, dim3(grid(e->n[i])), dim3(256), 0, e->st, e->n[i], e->v[i]);
        r = hipGetLastError();
    }
    if (!r) r = refresh_bf16(e);
    if (!r) r = hipStreamSynchronize(e->st);
    if (r) {
        delete e;
        return WLDA_E_HIP;
    }
    *out = e;
    return WLDA_OK;
}

wlda_status wlda_encoder_destroy(wlda_encoder e) {
    if (!e) return WLDA_E_INVALID;
    (void)hipStreamSynchronize(e->st);
    delete e;
    return WLDA_OK;
}

wlda_status wlda_encoder_set_weights(wlda_encoder e, const float *const *host) {
    if (!e || !host) return WLDA_E_INVALID;
    hipError_t r = hipSuccess;
    for (int i = 0; i < 6 && !r; ++i) {
        if (!host[i]) return WLDA_E_INVALID;
        r = hipMemcpyAsync(e->w[i], host[i], 4ull * e->n[i], hipMemcpyHostToDevice, e->st);
        if (!r) {
            hipLaunchKernelGGL(zero_f32_kernel, dim3(grid(e->n[i])), dim3(256), 0, e->st, e->n[i], e->m[i]);
            hipLaunchKernelGGL(zero_f32_kernel, dim3(grid(e->n[i])), dim3(256), 0, e->st, e->n[i], e->v[i]);
            r = hipGetLastError();
        }
    }
    if (!r) r = refresh_bf16(e);
    if (!r) r = hipStreamSynchronize(e->st);
    e->steps = 0;
    return r ? WLDA_E_HIP : WLDA_OK;
}

wlda_status wlda_encoder_get_weights(wlda_encoder e, float *const *host) {
    if (!e || !host) return WLDA_E_INVALID;
    hipError_t r = hipSuccess;
    for (int i = 0; i < 6 && !r; ++i)
        if (host[i]) r = hipMemcpyAsync(host[i], e->w[i], 4ull * e->n[i], hipMemcpyDeviceToHost, e->st);
    if (!r) r = hipStreamSynchronize(e->st);
    return r ? WLDA_E_HIP : WLDA_OK;
}

wlda_status wlda_encoder_features(uint32_t buckets, const uint32_t *words, uint32_t L, uint32_t *idx,
                                  float *val, uint32_t *nnz) {
    if (!nnz || buckets == 0 || (L && (!words || !idx || !val))) return WLDA_E_INVALID;
    std::vector<uint32_t> b(L);
    for (uint32_t n = 0; n < L; ++n)
        b[n] = (uint32_t)(((uint64_t)(uint32_t)(words[n] * 0x9E3779B1u) * buckets) >> 32);
    std::sort(b.begin(), b.end());
    uint32_t k = 0;
    for (uint32_t n = 0; n < L;) {
        uint32_t m = n;
        while (m < L && b[m] == b[n]) ++m;
        idx[k] = b[n];
        val[k] = (float)(m - n) / (float)L;
        ++k;
        n = m;
    }
    *nnz = k;
    return WLDA_OK;
}

wlda_status wlda_encoder_features_batch(uint32_t buckets, uint32_t n_docs, const uint64_t *docptr,
                                        const uint32_t *words, uint32_t *rowptr, uint32_t *idx, float *val) {
    if (!docptr || !rowptr || buckets == 0) return WLDA_E_INVALID;
    uint64_t k = 0;
    rowptr[0] = 0;
    for (uint32_t d = 0; d < n_docs; ++d) {
        const uint64_t L = docptr[d + 1] - docptr[d];
        uint32_t nnz = 0;
        if (L >= (1ull << 32)) return WLDA_E_INVALID;
        wlda_status st = wlda_encoder_features(buckets, words + docptr[d], (uint32_t)L, idx + k, val + k, &nnz);
        if (st != WLDA_OK) return st;
        k += nnz;
        if (k >= (1ull << 32)) return WLDA_E_INVALID;
        rowptr[d + 1] = (uint32_t)k;
    }
    return WLDA_OK;
}

wlda_status wlda_encoder_forward(wlda_encoder e, uint32_t B, const uint32_t *rowptr, const uint32_t *idx,
                                 const float *val, float *probs) {
    if (!e || !rowptr || !probs || B > e->p.max_batch) return WLDA_E_INVALID;
    if (B == 0) return WLDA_OK;
    hipError_t r = forward(e, B, rowptr, idx, val);
    if (!r) {
        hipLaunchKernelGGL(softmax_ce_kernel, dim3(B), dim3(256), 0, e->st, (int)e->p.K, (int)B, e->c3, e->w[5],
                           (const float *)nullptr, probs, (float *)nullptr, (uint16_t *)nullptr, (float *)nullptr);
        r = hipGetLastError();
    }
    return r ? WLDA_E_HIP : WLDA_OK;
}

wlda_status wlda_encoder_proposal(wlda_encoder e, uint32_t B, const float *probs, float eps, uint32_t *cdf) {
    if (!e || !probs || !cdf || !(eps > 0) || eps > 1 || (uint64_t)e->p.K * ((1u << 20) + 1) >= (1ull << 32))
        return WLDA_E_INVALID;
    if (B == 0) return WLDA_OK;
    hipLaunchKernelGGL(probs_to_cdf_kernel, dim3(B), dim3(256), 0, e->st, (int)e->p.K, probs, eps, cdf);
    return hipGetLastError() ? WLDA_E_HIP : WLDA_OK;
}

static wlda_status loss_out(wlda_encoder e, uint32_t B, float *loss) {
    if (!loss) return WLDA_OK;
    std::vector<float> h(B);
    if (hipMemcpyAsync(h.data(), e->loss_rows, 4ull * B, hipMemcpyDeviceToHost, e->st) ||
        hipStreamSynchronize(e->st))
        return WLDA_E_HIP;
    double s = 0;
    for (float x : h) s += x;
    *loss = (float)(s / B);
    return WLDA_OK;
}

wlda_status wlda_encoder_gradients(wlda_encoder e, uint32_t B, const uint32_t *rowptr, const uint32_t *idx,
                                   const float *val, const float *theta, float *loss, float *const *host_grads) {
    if (!e || !rowptr || !theta || B == 0 || B > e->p.max_batch) return WLDA_E_INVALID;
    hipError_t r = forward(e, B, rowptr, idx, val);
    if (!r) r = backward(e, B, rowptr, idx, val, theta);
    if (r) return WLDA_E_HIP;
    if (host_grads)
        for (int i = 0; i < 6 && !r; ++i)
            if (host_grads[i]) r = hipMemcpyAsync(host_grads[i], e->g[i], 4ull * e->n[i], hipMemcpyDeviceToHost, e->st);
    if (r || hipStreamSynchronize(e->st)) return WLDA_E_HIP;
    return loss_out(e, B, loss);
}

wlda_status wlda_encoder_train_step(wlda_encoder e, uint32_t B, const uint32_t *rowptr, const uint32_t *idx,
                                    const float *val, const float *theta, float *loss) {
    if (!e || !rowptr || !theta || B == 0 || B > e->p.max_batch) return WLDA_E_INVALID;
    hipError_t r = forward(e, B, rowptr, idx, val);
    if (!r) r = backward(e, B, rowptr, idx, val, theta);
    if (r) return WLDA_E_HIP;
    e->steps++;
    const float c1 = 1.f - std::pow(e->p.beta1, (float)e->steps);
    const float c2 = 1.f - std::pow(e->p.beta2, (float)e->steps);
    const int wbmap[6] = {0, -1, 1, -1, 2, -1};
    for (int i = 0; i < 6; ++i)
        hipLaunchKernelGGL(adam_kernel, dim3(grid(e->n[i])), dim3(256), 0, e->st, e->n[i], e->w[i], e->m[i], e->v[i],
                           e->g[i], wbmap[i] >= 0 ? e->wb[wbmap[i]] : (uint16_t *)nullptr, e->p.lr, e->p.beta1,
                           e->p.beta2, e->p.eps, c1, c2);
    if (hipGetLastError()) return WLDA_E_HIP;
    return loss_out(e, B, loss);
}

}  // extern "C"
