// Learned scheduling state shared between the batched launch and the cost
// model's entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace codag {

constexpr int kFeatures = 16;
constexpr int kHidden = 64;
// Parameters of the 16-64-64-1 network, flattened: W1[64][16], b1[64],
// W2[64][64], b2[64], W3[64], b3.
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kHidden * kFeatures;
constexpr int kOffW2 = kOffB1 + kHidden;
constexpr int kOffB2 = kOffW2 + kHidden * kHidden;
constexpr int kOffW3 = kOffB2 + kHidden;
constexpr int kOffB3 = kOffW3 + kHidden;
constexpr int kParams = kOffB3 + 1;  // 5313
// Normalization kept with the parameters: feature means and scales, then the
// target's mean and scale.
constexpr int kNorm = 2 * kFeatures + 2;
constexpr int kSortBuckets = 4096;

struct SchedState {
    bool trained = false;
    float norm_host[kNorm] = {};  // host copy of the normalization
    float *params = nullptr;      // device, kParams
    float *norm = nullptr;        // device, kNorm
    float *adam_m = nullptr, *adam_v = nullptr;  // device, kParams each
    float *grad = nullptr;        // device, kParams
    float *part = nullptr;        // device, segment partial gradients
    uint32_t *hist = nullptr;     // device, kSortBuckets + 1
    // Per-chunk buffers of the learned order, grown on demand (never during
    // graph capture).
    uint32_t cap = 0;
    float *feat = nullptr;      // cap x kFeatures
    float *pred = nullptr;      // cap
    uint32_t *key = nullptr;    // cap
    uint32_t *order = nullptr;  // cap
    // Training buffers, grown on demand.
    uint32_t tcap = 0;
    float *h1 = nullptr, *h2 = nullptr, *g1 = nullptr, *g2 = nullptr;  // tcap x kHidden
    float *e = nullptr;                                                 // tcap
    uint32_t lcap = 0;
    float *losses = nullptr;  // lcap
};

int sched_init(SchedState *s);
void sched_free(SchedState *s);
// Make the per-chunk buffers hold n chunks (not during graph capture).
int sched_reserve(SchedState *s, uint32_t n);
// Enqueue feature extraction, inference and the longest-predicted-first
// sort of n chunks (n <= s->cap); the permutation goes to order_out.
int sched_enqueue_order(SchedState *s, const uint8_t *codecs, const uint8_t *comp,
                        const uint64_t *coff, const uint64_t *ooff, uint32_t n,
                        uint32_t *order_out, hipStream_t st);
// Enqueue a counting sort of n chunks (n <= s->cap) by codec byte: the
// permutation lists every RLE v1 chunk, then every RLE v2 chunk, and so on.
int sched_enqueue_codec_order(SchedState *s, const uint8_t *codecs, uint32_t n, uint32_t *order_out,
                              hipStream_t st);

}  // namespace codag
