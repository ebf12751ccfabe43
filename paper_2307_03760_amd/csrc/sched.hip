// Learned scheduling: a tiny FP32 cost model that predicts each chunk's
// decode time from features readable before decoding, trained on the GPU
// from decode times the decoder itself measures, and used to put the work
// queue of a batched launch in longest-predicted-first order.
//
// Features (16 per chunk, from the chunk's sizes and the header of its first
// Deflate block): log2 compressed and output sizes, their log ratio, codec
// one-hot, first block type one-hot, HLIT/HDIST/HCLEN of a dynamic first
// block, and the distribution of its literal/length code lengths (<= 6, 7-8,
// 9-10, >= 11 bits).
//
// Network: 16 -> 64 -> 64 -> 1 with ReLU, mean squared error on the
// normalized log2 decode time, Adam.  Forward and backward run one sample per
// thread; parameter gradients are sums over samples taken in a fixed order by
// one thread per parameter, so training is deterministic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/codag.h"
#include "deflate.hpp"
#include "internal.hpp"
#include "sched.hpp"

namespace codag {

// ---------------------------------------------------------------------------
// Features: one wave per chunk.
// ---------------------------------------------------------------------------

struct FeatureLds {
    uint16_t cl[1u << kCodeLenBits];
    CodeMeta meta;
    uint16_t sorted[32];
    uint8_t lens[320];
};

constexpr int kFeatWaves = 4;

__global__ void __launch_bounds__(kWave * kFeatWaves)
    chunk_features(const uint8_t *codecs, const uint8_t *comp, const uint64_t *coff,
                   const uint64_t *ooff, uint32_t n, float *feat) {
    __shared__ __align__(16) uint32_t s_ring[kFeatWaves][kRingLdsWords];
    __shared__ __align__(16) uint32_t s_land[kFeatWaves][kLandWords];
    __shared__ __align__(16) FeatureLds s_f[kFeatWaves];
    const uint32_t wave = uni(threadIdx.x / kWave);
    const uint32_t c = blockIdx.x * kFeatWaves + wave;
    if (c >= n) return;
    uint64_t i0 = coff[c], i1 = coff[c + 1], o0 = ooff[c], o1 = ooff[c + 1];
    uint32_t codec = codecs ? uni((uint32_t)codecs[c]) : (uint32_t)CODAG_DEFLATE;
    float in_len = (float)(i1 - i0), out_len = (float)(o1 - o0);
    float f[kFeatures];
#pragma unroll
    for (int k = 0; k < kFeatures; k++) f[k] = 0.f;
    f[0] = log2f(1.f + in_len);
    f[1] = log2f(1.f + out_len);
    f[2] = f[1] - f[0];
    f[3] = codec == CODAG_RLE_V1;
    f[4] = codec == CODAG_RLE_V2;
    f[5] = codec == CODAG_DEFLATE;
    if (codec == CODAG_DEFLATE && i1 > i0 && i1 - i0 < (1u << 28)) {
        InRing in;
        in.init(comp + i0, (uint32_t)(i1 - i0), s_ring[wave], s_land[wave]);
        BitIn bi;
        bi.seek(in, in.skip);
        bi.refill(in);
        uint32_t btype = (uint32_t)(bi.buf >> 1) & 3;
        if (bi.drop(3) && btype < 3) {
            f[6 + btype] = 1.f;
            if (btype == 2) {
                uint32_t hlit, hdist, hclen;
                FeatureLds *fl = &s_f[wave];
                if (read_code_lengths(in, bi, fl->cl, &fl->meta, fl->sorted, fl->lens, hlit,
                                      hdist, hclen) == CODAG_OK) {
                    f[9] = hlit / 286.f;
                    f[10] = hdist / 30.f;
                    f[11] = hclen / 19.f;
                    uint32_t bins[4] = {0, 0, 0, 0}, used = 0;
                    for (uint32_t s = lane(); s < hlit; s += kWave) {
                        uint32_t m = fl->lens[s];
                        if (m) {
                            used++;
                            bins[m <= 6 ? 0 : m <= 8 ? 1 : m <= 10 ? 2 : 3]++;
                        }
                    }
                    // Wave sums of the per-lane counts.
                    for (int off = 32; off >= 1; off >>= 1) {
                        used += __shfl_xor(used, off);
#pragma unroll
                        for (int b = 0; b < 4; b++) bins[b] += __shfl_xor(bins[b], off);
                    }
                    float inv = used ? 1.f / used : 0.f;
#pragma unroll
                    for (int b = 0; b < 4; b++) f[12 + b] = bins[b] * inv;
                }
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
    }
    if (lane() < kFeatures) {
        float v = 0.f;
#pragma unroll
        for (int k = 0; k < kFeatures; k++)
            if ((int)lane() == k) v = f[k];
        feat[(size_t)c * kFeatures + lane()] = v;
    }
}

// ---------------------------------------------------------------------------
// Network.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void load_input(const float *feat, const float *norm, uint32_t i,
                                           float *x) {
#pragma unroll
    for (int k = 0; k < kFeatures; k++)
        x[k] = (feat[(size_t)i * kFeatures + k] - norm[k]) * norm[kFeatures + k];
}

// First layer, fully unrolled so that h1 stays in registers.
__device__ __forceinline__ void layer1(const float *p, const float *x, float *h1) {
#pragma unroll
    for (int j = 0; j < kHidden; j++) {
        float a = p[kOffB1 + j];
#pragma unroll
        for (int k = 0; k < kFeatures; k++) a += p[kOffW1 + j * kFeatures + k] * x[k];
        h1[j] = a > 0.f ? a : 0.f;
    }
}

// Pre-activation of second-layer unit j.
__device__ __forceinline__ float layer2(const float *p, int j, const float *h1) {
    float a = p[kOffB2 + j];
#pragma unroll
    for (int k = 0; k < kHidden; k++) a += p[kOffW2 + j * kHidden + k] * h1[k];
    return a;
}

__device__ __forceinline__ void load_params(const float *params, float *sp) {
    for (int k = threadIdx.x; k < kParams; k += blockDim.x) sp[k] = params[k];
    __syncthreads();
}

__global__ void __launch_bounds__(256)
    mlp_predict(const float *feat, const float *params, const float *norm, uint32_t n, float *pred) {
    __shared__ float sp[kParams];
    load_params(params, sp);
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[kFeatures], h1[kHidden];
    load_input(feat, norm, i, x);
    layer1(sp, x, h1);
    float y = sp[kOffB3];
    for (int j = 0; j < kHidden; j++) {
        float a = layer2(sp, j, h1);
        y += sp[kOffW3 + j] * (a > 0.f ? a : 0.f);
    }
    pred[i] = y * norm[2 * kFeatures + 1] + norm[2 * kFeatures];  // log2 cycles
}

// Forward and backward of one sample per thread.  Stores, row-major per
// sample: H1, H2 (activations), G2, G1 (gradients of e^2 / 2 with respect to
// the pre-activations, where e = y - t) and E = e.  The loss gradient is these
// times 2/n, applied once in the final sums.
__global__ void __launch_bounds__(256)
    mlp_backward(const float *feat, const float *target, const float *params, const float *norm,
                 uint32_t n, float *H1, float *H2, float *G2, float *G1, float *E) {
    __shared__ float sp[kParams];
    load_params(params, sp);
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[kFeatures], h1[kHidden];
    load_input(feat, norm, i, x);
    layer1(sp, x, h1);
    float y = sp[kOffB3];
    for (int j = 0; j < kHidden; j++) {
        float a = layer2(sp, j, h1);
        float h = a > 0.f ? a : 0.f;
        H2[(size_t)i * kHidden + j] = h;
        y += sp[kOffW3 + j] * h;
    }
    float t = (target[i] - norm[2 * kFeatures]) / norm[2 * kFeatures + 1];
    float e = y - t;
    E[i] = e;
    float acc[kHidden];
#pragma unroll
    for (int k = 0; k < kHidden; k++) acc[k] = 0.f;
    for (int j = 0; j < kHidden; j++) {
        float a = layer2(sp, j, h1);  // recomputed rather than kept per j
        float g = a > 0.f ? e * sp[kOffW3 + j] : 0.f;
        G2[(size_t)i * kHidden + j] = g;
#pragma unroll
        for (int k = 0; k < kHidden; k++) acc[k] += sp[kOffW2 + j * kHidden + k] * g;
    }
#pragma unroll
    for (int k = 0; k < kHidden; k++) {
        H1[(size_t)i * kHidden + k] = h1[k];
        G1[(size_t)i * kHidden + k] = h1[k] > 0.f ? acc[k] : 0.f;
    }
}

constexpr int kGradSegments = 64;

// Partial parameter gradients over one fixed segment of the samples (one
// thread per parameter, samples in index order).
__global__ void __launch_bounds__(256)
    mlp_grad_part(const float *feat, const float *norm, uint32_t n, uint32_t seg, const float *H1,
                  const float *H2, const float *G2, const float *G1, const float *E, float *part) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    uint32_t i0 = blockIdx.y * seg, i1 = i0 + seg < n ? i0 + seg : n;
    float g = 0.f;
    if (p < kOffB1) {  // W1[j][k]
        int j = p / kFeatures, k = p % kFeatures;
        float mu = norm[k], sc = norm[kFeatures + k];
        for (uint32_t i = i0; i < i1; i++)
            g += G1[(size_t)i * kHidden + j] * ((feat[(size_t)i * kFeatures + k] - mu) * sc);
    } else if (p < kOffW2) {
        int j = p - kOffB1;
        for (uint32_t i = i0; i < i1; i++) g += G1[(size_t)i * kHidden + j];
    } else if (p < kOffB2) {  // W2[j][k]
        int j = (p - kOffW2) / kHidden, k = (p - kOffW2) % kHidden;
        for (uint32_t i = i0; i < i1; i++) g += G2[(size_t)i * kHidden + j] * H1[(size_t)i * kHidden + k];
    } else if (p < kOffW3) {
        int j = p - kOffB2;
        for (uint32_t i = i0; i < i1; i++) g += G2[(size_t)i * kHidden + j];
    } else if (p < kOffB3) {
        int j = p - kOffW3;
        for (uint32_t i = i0; i < i1; i++) g += E[i] * H2[(size_t)i * kHidden + j];
    } else {
        for (uint32_t i = i0; i < i1; i++) g += E[i];
    }
    part[(size_t)blockIdx.y * kParams + p] = g;
}

// Segment sums in segment order, times 2/n.
__global__ void __launch_bounds__(256) mlp_grad_sum(const float *part, float scale, float *grad) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    float g = 0.f;
    for (int s = 0; s < kGradSegments; s++) g += part[(size_t)s * kParams + p];
    grad[p] = g * scale;
}

// Mean of e^2, summed in a fixed order by one workgroup.
__global__ void __launch_bounds__(256) mlp_loss(const float *E, uint32_t n, float *loss) {
    __shared__ float part[256];
    float a = 0.f;
    for (uint32_t i = threadIdx.x; i < n; i += 256) a += E[i] * E[i];
    part[threadIdx.x] = a;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = part[0] / (float)n;
}

__global__ void __launch_bounds__(256)
    mlp_adam(float *params, const float *grad, float *m, float *v, float lr, float b1, float b2,
             float eps, float c1, float c2) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    float g = grad[p];
    float mp = b1 * m[p] + (1.f - b1) * g;
    float vp = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mp;
    v[p] = vp;
    params[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

__global__ void fill_zero(float *p, uint32_t n) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

// ---------------------------------------------------------------------------
// Longest predicted first: a counting sort on the quantized prediction.
// ---------------------------------------------------------------------------

__global__ void sort_clear(uint32_t *hist) {
    for (int b = threadIdx.x; b <= kSortBuckets; b += blockDim.x) hist[b] = 0;
}

__global__ void sort_keys(const float *pred, uint32_t n, float lo, float hi, uint32_t *key,
                          uint32_t *hist) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float t = (pred[i] - lo) / (hi - lo);
    if (!(t >= 0.f)) t = 0.f;  // also NaN: such chunks go last
    if (t > 1.f) t = 1.f;
    uint32_t k = (kSortBuckets - 1) - (uint32_t)(t * (kSortBuckets - 1));  // descending
    key[i] = k;
    atomicAdd(&hist[k], 1u);
}

// Exclusive prefix sum of the bucket counts (one workgroup).
__global__ void __launch_bounds__(1024) sort_scan(uint32_t *hist) {
    __shared__ uint32_t part[1024];
    const int per = kSortBuckets / 1024;
    uint32_t local[kSortBuckets / 1024];
    uint32_t sum = 0;
    for (int k = 0; k < per; k++) {
        local[k] = hist[threadIdx.x * per + k];
        sum += local[k];
    }
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - sum;
    for (int k = 0; k < per; k++) {
        hist[threadIdx.x * per + k] = run;
        run += local[k];
    }
}

// Codec-grouped order: the key is the chunk's codec byte.
__global__ void sort_keys_codec(const uint8_t *codecs, uint32_t n, uint32_t *key, uint32_t *hist) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = codecs[i];
    key[i] = k;
    atomicAdd(&hist[k], 1u);
}

__global__ void sort_scatter(const uint32_t *key, uint32_t n, uint32_t *hist, uint32_t *order) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    order[atomicAdd(&hist[key[i]], 1u)] = i;
}

}  // namespace codag

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

namespace {

using namespace codag;

template <typename... T>
void free_all(T *&...p) {
    ((p ? (void)hipFree(p) : (void)0), ...);
    ((p = nullptr), ...);
}

void free_chunk_buffers(SchedState *s) {
    free_all(s->feat, s->pred, s->key, s->order);
    s->cap = 0;
}

void free_train_buffers(SchedState *s) {
    free_all(s->h1, s->h2, s->g1, s->g2, s->e);
    s->tcap = 0;
}

int reserve_train(SchedState *s, uint32_t n) {
    if (n <= s->tcap) return CODAG_OK;
    free_train_buffers(s);
    size_t hb = (size_t)n * kHidden * sizeof(float);
    if (hipMalloc(&s->h1, hb) != hipSuccess || hipMalloc(&s->h2, hb) != hipSuccess ||
        hipMalloc(&s->g1, hb) != hipSuccess || hipMalloc(&s->g2, hb) != hipSuccess ||
        hipMalloc(&s->e, (size_t)n * sizeof(float)) != hipSuccess) {
        free_train_buffers(s);
        return CODAG_E_HIP;
    }
    s->tcap = n;
    return CODAG_OK;
}

int reserve_losses(SchedState *s, uint32_t n) {
    if (n <= s->lcap) return CODAG_OK;
    free_all(s->losses);
    s->lcap = 0;
    if (hipMalloc(&s->losses, (size_t)n * sizeof(float)) != hipSuccess) return CODAG_E_HIP;
    s->lcap = n;
    return CODAG_OK;
}

int launched() { return hipGetLastError() == hipSuccess ? CODAG_OK : CODAG_E_HIP; }

int enqueue_features(const uint8_t *codecs, const uint8_t *comp, const uint64_t *coff,
                     const uint64_t *ooff, uint32_t n, float *feat, hipStream_t st) {
    hipLaunchKernelGGL(chunk_features, dim3((n + kFeatWaves - 1) / kFeatWaves),
                       dim3(kWave * kFeatWaves), 0, st, codecs, comp, coff, ooff, n, feat);
    return launched();
}

int enqueue_predict(SchedState *s, const float *feat, uint32_t n, float *pred, hipStream_t st) {
    hipLaunchKernelGGL(mlp_predict, dim3((n + 255) / 256), dim3(256), 0, st, feat, s->params,
                       s->norm, n, pred);
    return launched();
}

// Forward, backward, segment sums and (optionally) the loss at the current
// parameters; the gradient ends in s->grad.
int enqueue_grad(SchedState *s, const float *feat, const float *target, uint32_t n, float *loss,
                 hipStream_t st) {
    hipLaunchKernelGGL(mlp_backward, dim3((n + 255) / 256), dim3(256), 0, st, feat, target,
                       s->params, s->norm, n, s->h1, s->h2, s->g2, s->g1, s->e);
    uint32_t seg = (n + kGradSegments - 1) / kGradSegments;
    hipLaunchKernelGGL(mlp_grad_part, dim3((kParams + 255) / 256, kGradSegments), dim3(256), 0, st,
                       feat, s->norm, n, seg, s->h1, s->h2, s->g2, s->g1, s->e, s->part);
    hipLaunchKernelGGL(mlp_grad_sum, dim3((kParams + 255) / 256), dim3(256), 0, st, s->part,
                       2.f / (float)n, s->grad);
    if (loss) hipLaunchKernelGGL(mlp_loss, dim3(1), dim3(256), 0, st, s->e, n, loss);
    return launched();
}

// splitmix64 (Steele, Lea and Flood 2014), as a seeded source of weights.
uint64_t splitmix64(uint64_t &x) {
    uint64_t z = (x += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

void init_params(uint64_t seed, std::vector<float> &p) {
    p.assign(kParams, 0.f);
    uint64_t x = seed;
    auto fill = [&](int off, int count, int fan_in) {
        double r = std::sqrt(6.0 / fan_in);
        for (int k = 0; k < count; k++) {
            double u = (double)(splitmix64(x) >> 11) * 0x1.0p-53;
            p[off + k] = (float)((2.0 * u - 1.0) * r);
        }
    };
    fill(kOffW1, kHidden * kFeatures, kFeatures);
    fill(kOffW2, kHidden * kHidden, kHidden);
    fill(kOffW3, kHidden, kHidden);
}

void compute_norm(const std::vector<float> &f, const std::vector<float> &t, uint32_t n, float *norm) {
    for (int k = 0; k < kFeatures + 1; k++) {
        double sum = 0, sq = 0;
        for (uint32_t i = 0; i < n; i++) {
            double v = k < kFeatures ? f[(size_t)i * kFeatures + k] : t[i];
            sum += v;
        }
        double mean = sum / n;
        for (uint32_t i = 0; i < n; i++) {
            double v = (k < kFeatures ? f[(size_t)i * kFeatures + k] : t[i]) - mean;
            sq += v * v;
        }
        double sd = std::sqrt(sq / n);
        if (k < kFeatures) {
            norm[k] = (float)mean;
            norm[kFeatures + k] = sd > 1e-12 ? (float)(1.0 / sd) : 0.f;
        } else {
            norm[2 * kFeatures] = (float)mean;
            norm[2 * kFeatures + 1] = sd > 1e-12 ? (float)sd : 1.f;
        }
    }
}

int upload_model(SchedState *s, const float *params, const float *norm, hipStream_t st) {
    if ((params && hipMemcpyAsync(s->params, params, kParams * sizeof(float),
                                  hipMemcpyHostToDevice, st) != hipSuccess) ||
        hipMemcpyAsync(s->norm, norm, kNorm * sizeof(float), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return CODAG_E_HIP;
    std::memcpy(s->norm_host, norm, sizeof(s->norm_host));
    return CODAG_OK;
}

int check_plan(const codag_plan *plan) {
    if (!plan) return CODAG_E_INVALID_ARGUMENT;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return CODAG_E_HIP;
    return dev == plan->device ? CODAG_OK : CODAG_E_INVALID_ARGUMENT;
}

constexpr uint64_t kMaxTrain = 1ull << 24;

}  // namespace

namespace codag {

int sched_init(SchedState *s) {
    if (hipMalloc(&s->params, kParams * sizeof(float)) != hipSuccess ||
        hipMalloc(&s->norm, kNorm * sizeof(float)) != hipSuccess ||
        hipMalloc(&s->adam_m, kParams * sizeof(float)) != hipSuccess ||
        hipMalloc(&s->adam_v, kParams * sizeof(float)) != hipSuccess ||
        hipMalloc(&s->grad, kParams * sizeof(float)) != hipSuccess ||
        hipMalloc(&s->part, (size_t)kGradSegments * kParams * sizeof(float)) != hipSuccess ||
        hipMalloc(&s->hist, (kSortBuckets + 1) * sizeof(uint32_t)) != hipSuccess)
        return CODAG_E_HIP;
    return CODAG_OK;
}

void sched_free(SchedState *s) {
    free_chunk_buffers(s);
    free_train_buffers(s);
    free_all(s->params, s->norm, s->adam_m, s->adam_v, s->grad, s->part, s->hist, s->losses);
    s->lcap = 0;
    s->trained = false;
}

int sched_reserve(SchedState *s, uint32_t n) {
    if (n <= s->cap) return CODAG_OK;
    free_chunk_buffers(s);
    uint32_t cap = n < 1024 ? 1024 : n;
    if (hipMalloc(&s->feat, (size_t)cap * kFeatures * sizeof(float)) != hipSuccess ||
        hipMalloc(&s->pred, (size_t)cap * sizeof(float)) != hipSuccess ||
        hipMalloc(&s->key, (size_t)cap * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&s->order, (size_t)cap * sizeof(uint32_t)) != hipSuccess) {
        free_chunk_buffers(s);
        return CODAG_E_HIP;
    }
    s->cap = cap;
    return CODAG_OK;
}

int sched_enqueue_codec_order(SchedState *s, const uint8_t *codecs, uint32_t n, uint32_t *order_out,
                              hipStream_t st) {
    if (n > s->cap) return CODAG_E_INVALID_ARGUMENT;
    uint32_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(sort_clear, dim3(1), dim3(1024), 0, st, s->hist);
    hipLaunchKernelGGL(sort_keys_codec, dim3(blocks), dim3(256), 0, st, codecs, n, s->key, s->hist);
    hipLaunchKernelGGL(sort_scan, dim3(1), dim3(1024), 0, st, s->hist);
    hipLaunchKernelGGL(sort_scatter, dim3(blocks), dim3(256), 0, st, s->key, n, s->hist, order_out);
    return launched();
}

int sched_enqueue_order(SchedState *s, const uint8_t *codecs, const uint8_t *comp,
                        const uint64_t *coff, const uint64_t *ooff, uint32_t n,
                        uint32_t *order_out, hipStream_t st) {
    if (n > s->cap) return CODAG_E_INVALID_ARGUMENT;
    int rc = enqueue_features(codecs, comp, coff, ooff, n, s->feat, st);
    if (!rc) rc = enqueue_predict(s, s->feat, n, s->pred, st);
    if (rc) return rc;
    float my = s->norm_host[2 * kFeatures], sy = s->norm_host[2 * kFeatures + 1];
    float lo = my - 4.f * sy, hi = my + 4.f * sy;
    if (!(hi > lo)) hi = lo + 1.f;
    uint32_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(sort_clear, dim3(1), dim3(1024), 0, st, s->hist);
    hipLaunchKernelGGL(sort_keys, dim3(blocks), dim3(256), 0, st, s->pred, n, lo, hi, s->key,
                       s->hist);
    hipLaunchKernelGGL(sort_scan, dim3(1), dim3(1024), 0, st, s->hist);
    hipLaunchKernelGGL(sort_scatter, dim3(blocks), dim3(256), 0, st, s->key, n, s->hist, order_out);
    return launched();
}

}  // namespace codag

extern "C" {

int codag_sched_features(codag_plan *plan, const uint8_t *codecs, const uint8_t *comp_buf,
                         const uint64_t *chunk_offsets, const uint64_t *out_offsets,
                         uint64_t n_chunks, float *feat, void *stream) {
    int st = check_plan(plan);
    if (st) return st;
    if (n_chunks == 0) return CODAG_OK;
    if (n_chunks >= (1ull << 32) - 64 || !comp_buf || !chunk_offsets || !out_offsets || !feat)
        return CODAG_E_INVALID_ARGUMENT;
    return enqueue_features(codecs, comp_buf, chunk_offsets, out_offsets, (uint32_t)n_chunks, feat,
                            static_cast<hipStream_t>(stream));
}

int codag_sched_set_params(codag_plan *plan, const float *params, const float *norm) {
    int st = check_plan(plan);
    if (st) return st;
    if (!params || !norm) return CODAG_E_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lock(plan->mu);
    st = upload_model(&plan->sched, params, norm, nullptr);
    if (st) return st;
    plan->sched.trained = true;
    plan->have_key = false;  // a captured learned order would still be valid, but be safe
    return CODAG_OK;
}

int codag_sched_get_params(const codag_plan *plan, float *params, float *norm) {
    int st = check_plan(plan);
    if (st) return st;
    if (!plan->sched.trained) return CODAG_E_INVALID_ARGUMENT;
    if (params && hipMemcpy(params, plan->sched.params, kParams * sizeof(float),
                            hipMemcpyDeviceToHost) != hipSuccess)
        return CODAG_E_HIP;
    if (norm) std::memcpy(norm, plan->sched.norm_host, sizeof(plan->sched.norm_host));
    return CODAG_OK;
}

namespace {
// Saved model layout: magic, format version, the three sizes, the packed
// parameters and the normalization (little-endian floats), then a 64-bit
// FNV-1a hash of everything before it.
constexpr char kBlobMagic[8] = {'C', 'O', 'D', 'A', 'G', 'M', 'L', 'P'};
constexpr uint32_t kBlobVersion = 1;
constexpr size_t kBlobHeader = 8 + 4 * 4;
static_assert(CODAG_SCHED_BLOB_BYTES == kBlobHeader + 4 * (kParams + kNorm) + 8, "blob size");

uint64_t fnv1a64(const uint8_t *p, size_t n) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (size_t i = 0; i < n; i++) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}
}  // namespace

int codag_sched_save(const codag_plan *plan, void *buf, size_t cap, size_t *len) {
    int st = check_plan(plan);
    if (st) return st;
    if (len) *len = CODAG_SCHED_BLOB_BYTES;
    if (!buf || cap < CODAG_SCHED_BLOB_BYTES) return CODAG_E_INVALID_ARGUMENT;
    if (!plan->sched.trained) return CODAG_E_INVALID_ARGUMENT;
    std::vector<float> params(kParams), norm(kNorm);
    st = codag_sched_get_params(plan, params.data(), norm.data());
    if (st) return st;
    uint8_t *b = static_cast<uint8_t *>(buf);
    const uint32_t hdr[4] = {kBlobVersion, (uint32_t)kFeatures, (uint32_t)kParams, (uint32_t)kNorm};
    std::memcpy(b, kBlobMagic, 8);
    std::memcpy(b + 8, hdr, sizeof(hdr));
    std::memcpy(b + kBlobHeader, params.data(), 4 * kParams);
    std::memcpy(b + kBlobHeader + 4 * kParams, norm.data(), 4 * kNorm);
    const size_t body = kBlobHeader + 4 * (kParams + kNorm);
    const uint64_t h = fnv1a64(b, body);
    std::memcpy(b + body, &h, 8);
    return CODAG_OK;
}

int codag_sched_load(codag_plan *plan, const void *buf, size_t len) {
    int st = check_plan(plan);
    if (st) return st;
    if (!buf || len != CODAG_SCHED_BLOB_BYTES) return CODAG_E_INVALID_ARGUMENT;
    const uint8_t *b = static_cast<const uint8_t *>(buf);
    uint32_t hdr[4];
    std::memcpy(hdr, b + 8, sizeof(hdr));
    if (std::memcmp(b, kBlobMagic, 8) != 0 || hdr[0] != kBlobVersion || hdr[1] != (uint32_t)kFeatures ||
        hdr[2] != (uint32_t)kParams || hdr[3] != (uint32_t)kNorm)
        return CODAG_E_INVALID_ARGUMENT;
    const size_t body = kBlobHeader + 4 * (kParams + kNorm);
    uint64_t h;
    std::memcpy(&h, b + body, 8);
    if (h != fnv1a64(b, body)) return CODAG_E_INVALID_ARGUMENT;
    std::vector<float> params(kParams), norm(kNorm);
    std::memcpy(params.data(), b + kBlobHeader, 4 * kParams);
    std::memcpy(norm.data(), b + kBlobHeader + 4 * kParams, 4 * kNorm);
    for (float v : params)
        if (!std::isfinite(v)) return CODAG_E_INVALID_ARGUMENT;
    for (float v : norm)
        if (!std::isfinite(v)) return CODAG_E_INVALID_ARGUMENT;
    return codag_sched_set_params(plan, params.data(), norm.data());
}

int codag_sched_train(codag_plan *plan, const float *feat, const float *target, uint64_t n,
                      int steps, float lr, uint64_t seed, float *losses, void *stream) {
    int st = check_plan(plan);
    if (st) return st;
    if (!feat || !target || n < 2 || n >= kMaxTrain || steps < 0 || steps > 1000000 ||
        !(lr >= 0.f) || !std::isfinite(lr))
        return CODAG_E_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lock(plan->mu);
    SchedState *s = &plan->sched;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (seed) {
        std::vector<float> f((size_t)n * kFeatures), t(n), p;
        if (hipMemcpyAsync(f.data(), feat, f.size() * sizeof(float), hipMemcpyDeviceToHost, hs) !=
                hipSuccess ||
            hipMemcpyAsync(t.data(), target, t.size() * sizeof(float), hipMemcpyDeviceToHost, hs) !=
                hipSuccess ||
            hipStreamSynchronize(hs) != hipSuccess)
            return CODAG_E_HIP;
        float norm[kNorm];
        compute_norm(f, t, (uint32_t)n, norm);
        init_params(seed, p);
        if ((st = upload_model(s, p.data(), norm, hs))) return st;
        s->trained = true;
    } else if (!s->trained) {
        return CODAG_E_INVALID_ARGUMENT;
    }
    plan->have_key = false;
    if ((st = reserve_train(s, (uint32_t)n))) return st;
    if (losses && (st = reserve_losses(s, (uint32_t)std::max(steps, 1)))) return st;
    uint32_t pb = (kParams + 255) / 256;
    hipLaunchKernelGGL(fill_zero, dim3(pb), dim3(256), 0, hs, s->adam_m, (uint32_t)kParams);
    hipLaunchKernelGGL(fill_zero, dim3(pb), dim3(256), 0, hs, s->adam_v, (uint32_t)kParams);
    const double b1 = 0.9, b2 = 0.999;
    for (int k = 1; k <= steps; k++) {
        if ((st = enqueue_grad(s, feat, target, (uint32_t)n, losses ? s->losses + (k - 1) : nullptr,
                               hs)))
            return st;
        float c1 = (float)(1.0 - std::pow(b1, k)), c2 = (float)(1.0 - std::pow(b2, k));
        hipLaunchKernelGGL(mlp_adam, dim3(pb), dim3(256), 0, hs, s->params, s->grad, s->adam_m,
                           s->adam_v, lr, (float)b1, (float)b2, 1e-8f, c1, c2);
        if ((st = launched())) return st;
    }
    if (losses && steps > 0 &&
        hipMemcpyAsync(losses, s->losses, (size_t)steps * sizeof(float), hipMemcpyDeviceToHost,
                       hs) != hipSuccess)
        return CODAG_E_HIP;
    return hipStreamSynchronize(hs) == hipSuccess ? CODAG_OK : CODAG_E_HIP;
}

int codag_sched_grad(codag_plan *plan, const float *feat, const float *target, uint64_t n,
                     float *grad, float *loss, void *stream) {
    int st = check_plan(plan);
    if (st) return st;
    if (!feat || !target || n < 1 || n >= kMaxTrain) return CODAG_E_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lock(plan->mu);
    SchedState *s = &plan->sched;
    if (!s->trained) return CODAG_E_INVALID_ARGUMENT;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if ((st = reserve_train(s, (uint32_t)n)) || (st = reserve_losses(s, 1))) return st;
    if ((st = enqueue_grad(s, feat, target, (uint32_t)n, s->losses, hs))) return st;
    if ((grad && hipMemcpyAsync(grad, s->grad, kParams * sizeof(float), hipMemcpyDeviceToHost,
                                hs) != hipSuccess) ||
        (loss && hipMemcpyAsync(loss, s->losses, sizeof(float), hipMemcpyDeviceToHost, hs) !=
                     hipSuccess))
        return CODAG_E_HIP;
    return hipStreamSynchronize(hs) == hipSuccess ? CODAG_OK : CODAG_E_HIP;
}

int codag_sched_predict(codag_plan *plan, const float *feat, uint64_t n, float *pred,
                        void *stream) {
    int st = check_plan(plan);
    if (st) return st;
    if (n == 0) return CODAG_OK;
    if (!feat || !pred || n >= (1ull << 32) - 64) return CODAG_E_INVALID_ARGUMENT;
    if (!plan->sched.trained) return CODAG_E_INVALID_ARGUMENT;
    return enqueue_predict(&plan->sched, feat, (uint32_t)n, pred, static_cast<hipStream_t>(stream));
}

int codag_sched_order(codag_plan *plan, const uint8_t *codecs, const uint8_t *comp_buf,
                      const uint64_t *chunk_offsets, const uint64_t *out_offsets,
                      uint64_t n_chunks, uint32_t *order, void *stream) {
    int st = check_plan(plan);
    if (st) return st;
    if (n_chunks == 0) return CODAG_OK;
    if (n_chunks >= (1ull << 32) - 64 || !comp_buf || !chunk_offsets || !out_offsets || !order)
        return CODAG_E_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lock(plan->mu);
    SchedState *s = &plan->sched;
    if (!s->trained) return CODAG_E_INVALID_ARGUMENT;
    if ((st = sched_reserve(s, (uint32_t)n_chunks))) return st;
    return sched_enqueue_order(s, codecs, comp_buf, chunk_offsets, out_offsets, (uint32_t)n_chunks,
                               order, static_cast<hipStream_t>(stream));
}

}  // extern "C"
