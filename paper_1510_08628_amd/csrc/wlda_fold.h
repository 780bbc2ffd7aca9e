// Fold-in internals shared by the batch fold-in and the server.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/warplda.h"
#include "wlda_internal.h"

namespace wlda {

struct FoldModel {
    const uint32_t *colptr;   // V+1
    const void *zcsc;         // trained z, canonical column order (u16 if K <= 65535)
    const uint32_t *cwk;      // V x K frozen word-topic counts
    const uint32_t *ck;       // K
    uint32_t V, K, M, zc16;
    float a, b, alpha_bar, beta_k, beta_bar;
    uint32_t seed_lo, seed_hi;
};

struct FoldBatch {
    uint32_t n;               // documents in this launch
    const uint32_t *slots;    // slot id of each document
    const uint32_t *off;      // per slot: first token in the pool
    const uint32_t *len;      // per slot: tokens
    const uint32_t *req;      // per slot: request id
    uint32_t *sweep;          // per slot: next sweep (0 = initialise)
    const uint32_t *words;    // pool
    uint32_t *z;              // pool
    uint32_t *pd;             // pool, M x cap (proposal-major)
    uint32_t *pw;             // pool, M x cap
    uint32_t cap;
    const uint32_t *qcdf;     // per slot K running sums of the learned weights (or null)
    uint32_t learned_steps;
    uint32_t max_sweep;       // run only documents with sweep <= max_sweep
    const uint32_t *use_q = nullptr;   // per slot: 1 = learned proposal (null: all use qcdf)
};

constexpr uint32_t FOLD_MAX_TOKENS = 8192;
constexpr uint32_t FOLD_Q_LDS_MAX = 4096;   // learned proposal CDF staged in LDS up to this K

const FoldModel &model_internal(wlda_model m);
const wlda_params &model_params(wlda_model m);
uint32_t wlda_encoder_get_k(wlda_encoder e);
uint32_t wlda_encoder_get_buckets(wlda_encoder e);
uint32_t wlda_encoder_get_max_batch(wlda_encoder e);
void *wlda_encoder_get_stream(wlda_encoder e);
hipError_t fold_launch(const FoldModel &m, const FoldBatch &b, hipStream_t st);
// Held-out log likelihood of the documents of b: hchunk (b.n + 1 entries)
// holds the prefix sums of heldout_chunks(ho_len) over the listed documents,
// n_chunks its last entry; ho_log is scratch indexed like ho_words.
hipError_t fold_heldout(const FoldModel &m, const FoldBatch &b, const uint32_t *ho_off,
                        const uint32_t *ho_len, const uint32_t *ho_words, const uint32_t *hchunk,
                        uint32_t n_chunks, double *ho_log, double alpha, double beta, double *out,
                        hipStream_t st);
uint32_t heldout_chunks(uint32_t n_heldout);

}  // namespace wlda
