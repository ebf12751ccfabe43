// Batched launch: thousands of mixed-codec chunks in one persistent kernel.
//
// The grid holds a fixed number of resident waves per CU; each wave takes
// the next position of a device-side work queue (one atomic add per chunk),
// maps it through an optional order array, and decodes that chunk with the
// chunk's codec using the same per-wave decoders as the plain launch.  The
// queue order is the scheduler's lever: with chunks of very uneven cost, the
// order decides how much idle time the last waves leave at the end.  The
// sequence (queue reset, optional scheduling kernels, decode) can be captured
// once in a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/codag.h"
#include "decode.hpp"
#include "internal.hpp"
#include "sched.hpp"

namespace codag {

__global__ void reset_queue(uint32_t *head) {
    if (threadIdx.x == 0) *head = 0;
}

// Each wave claims `claim` consecutive queue positions at a time (one
// atomic add for several small chunks) until the queue is empty.  Every
// store of a per-chunk result is made by all lanes with the same value (a
// one-lane branch inside this loop would make the compiler treat the loop
// as divergent).
template <int TB, uint32_t H, int WPB>
__global__ void __launch_bounds__(kWave * WPB)
    decode_batch(const uint8_t *codecs, const uint8_t *comp, const uint64_t *coff, uint8_t *out,
                 const uint64_t *ooff, uint32_t n, const uint32_t *order, uint32_t *head,
                 uint32_t claim, int32_t *status, unsigned long long *err, uint64_t *ticks) {
    __shared__ __align__(16) uint32_t s_ring[WPB][kRingLdsWords];
    __shared__ __align__(16) uint32_t s_land[WPB][kLandWords];
    __shared__ __align__(16) WaveScratch<CODAG_DEFLATE, TB, H> s_scratch[WPB];
    const uint32_t wave = uni(threadIdx.x / kWave);
    uint32_t idx = 0, last = 0;
    for (;;) {
        if (idx == last) {
            // Lane 0 adds; the others add zero, so lane 0's old value is the
            // claimed position whatever order the lanes' adds are applied in.
            idx = uni(atomicAdd(head, lane() == 0 ? claim : 0u));
            if (idx >= n) break;
            last = min(idx + claim, n);
        }
        const uint32_t q = idx++;
        uint32_t c = order ? uni(order[q]) : q;
        if (c >= n) {  // not a permutation: report the queue position
            atomicMin(err, (unsigned long long)error_key(q, CODAG_E_INVALID_ARGUMENT));
            continue;
        }
        uint32_t codec = uni((uint32_t)codecs[c]);
        uint64_t t0 = __builtin_amdgcn_s_memtime();
        int st;
        if (codec == CODAG_RLE_V1)
            st = decode_one<CODAG_RLE_V1, TB, H>(
                comp, coff, out, ooff, c, s_ring[wave], s_land[wave],
                reinterpret_cast<WaveScratch<CODAG_RLE_V1, TB, H> *>(&s_scratch[wave]));
        else if (codec == CODAG_RLE_V2)
            st = decode_one<CODAG_RLE_V2, TB, H>(
                comp, coff, out, ooff, c, s_ring[wave], s_land[wave],
                reinterpret_cast<WaveScratch<CODAG_RLE_V2, TB, H> *>(&s_scratch[wave]));
        else if (codec == CODAG_DEFLATE)
            st = decode_one<CODAG_DEFLATE, TB, H>(comp, coff, out, ooff, c, s_ring[wave],
                                                  s_land[wave], &s_scratch[wave]);
        else if (codec == CODAG_LZ4)
            st = decode_one<CODAG_LZ4, TB, H>(
                comp, coff, out, ooff, c, s_ring[wave], s_land[wave],
                reinterpret_cast<WaveScratch<CODAG_LZ4, TB, H> *>(&s_scratch[wave]));
        else
            st = CODAG_E_INVALID_ARGUMENT;
        uint64_t t1 = __builtin_amdgcn_s_memtime();
        if (ticks) ticks[c] = t1 - t0;
        if (status) status[c] = st;
        if (st != CODAG_OK) atomicMin(err, (unsigned long long)error_key(c, st));
    }
}

template <int TB, uint32_t H>
constexpr uint32_t batch_lds_per_wave() {
    return (uint32_t)(4 * kRingLdsWords + 4 * kLandWords + sizeof(WaveScratch<CODAG_DEFLATE, TB, H>));
}

}  // namespace codag

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

using namespace codag;

namespace {

constexpr uint32_t kLdsPerCu = 160 * 1024;
constexpr int kBatchTB = 9;  // default Deflate literal/length table bits in the batched kernel
constexpr int kVgprWavesPerSimd = 5;  // the decoders use up to 92 VGPRs

template <int TB>
uint32_t lds_per_wave_tb(int hist_kib) {
    return hist_kib == 16  ? batch_lds_per_wave<TB, 16384>()
           : hist_kib == 8 ? batch_lds_per_wave<TB, 8192>()
                           : batch_lds_per_wave<TB, 4096>();
}

uint32_t lds_per_wave(int hist_kib, int tb) {
    return tb == 10 ? lds_per_wave_tb<10>(hist_kib) : lds_per_wave_tb<9>(hist_kib);
}

int max_waves_per_cu(int hist_kib, int tb, int wpb) {
    int by_lds = (int)(kLdsPerCu / (lds_per_wave(hist_kib, tb) * wpb)) * wpb;
    return std::max(wpb, std::min({by_lds, 4 * kVgprWavesPerSimd, 16}));
}

}  // namespace

namespace {

void drop_graph(codag_plan *p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    p->have_key = false;
}

int resolve_opts(const codag_batch_opts *in, codag_batch_opts *o) {
    codag_batch_opts r{};
    if (in) r = *in;
    if (r.waves_per_block == 0) r.waves_per_block = 2;
    if (r.lit_table_bits == 0) r.lit_table_bits = kBatchTB;
    if (r.history_kib == 0) r.history_kib = 4;
    if (r.waves_per_block != 1 && r.waves_per_block != 2 && r.waves_per_block != 4)
        return CODAG_E_INVALID_ARGUMENT;
    if (r.chunks_per_claim == 0) r.chunks_per_claim = 1;
    if (r.lit_table_bits != 9 && r.lit_table_bits != 10) return CODAG_E_INVALID_ARGUMENT;
    if (r.history_kib != 4 && r.history_kib != 8 && r.history_kib != 16) return CODAG_E_INVALID_ARGUMENT;
    if (r.order < CODAG_ORDER_INDEX || r.order > CODAG_ORDER_CODEC) return CODAG_E_INVALID_ARGUMENT;
    if (r.chunks_per_claim < 1 || r.chunks_per_claim > 64) return CODAG_E_INVALID_ARGUMENT;
    if (r.waves_per_cu < 0 || r.waves_per_cu > 64) return CODAG_E_INVALID_ARGUMENT;
    if (r.waves_per_cu == 0)
        r.waves_per_cu = max_waves_per_cu(r.history_kib, r.lit_table_bits, r.waves_per_block);
    *o = r;
    return CODAG_OK;
}

template <int TB, uint32_t H, int WPB>
void launch_decode(codag_plan *p, const BatchArgs &a, const uint32_t *order, unsigned long long *err,
                   hipStream_t s) {
    uint32_t blocks = (uint32_t)std::max<int64_t>(1, ((int64_t)p->num_cus * p->opts.waves_per_cu) / WPB);
    hipLaunchKernelGGL((decode_batch<TB, H, WPB>), dim3(blocks), dim3(kWave * WPB), 0, s, a.codecs,
                       a.comp, a.coff, a.out, a.ooff, (uint32_t)a.n, order, p->head,
                       (uint32_t)p->opts.chunks_per_claim, a.status, err, a.ticks);
}

template <int TB>
void launch_decode_tb(codag_plan *p, const BatchArgs &a, const uint32_t *order,
                      unsigned long long *err, hipStream_t s) {
    const int h = p->opts.history_kib;
    switch (p->opts.waves_per_block) {
        case 1:
            h == 16 ? launch_decode<TB, 16384, 1>(p, a, order, err, s)
            : h == 8 ? launch_decode<TB, 8192, 1>(p, a, order, err, s)
                     : launch_decode<TB, 4096, 1>(p, a, order, err, s);
            break;
        case 4:
            h == 16 ? launch_decode<TB, 16384, 4>(p, a, order, err, s)
            : h == 8 ? launch_decode<TB, 8192, 4>(p, a, order, err, s)
                     : launch_decode<TB, 4096, 4>(p, a, order, err, s);
            break;
        default:
            h == 16 ? launch_decode<TB, 16384, 2>(p, a, order, err, s)
            : h == 8 ? launch_decode<TB, 8192, 2>(p, a, order, err, s)
                     : launch_decode<TB, 4096, 2>(p, a, order, err, s);
    }
}

// Enqueue the whole sequence on s.
int enqueue(codag_plan *p, const BatchArgs &a, unsigned long long *err, hipStream_t s) {
    hipLaunchKernelGGL(reset_queue, dim3(1), dim3(kWave), 0, s, p->head);
    const uint32_t *order = nullptr;
    if (p->opts.order == CODAG_ORDER_GIVEN) {
        order = a.order;
    } else if (p->opts.order == CODAG_ORDER_LEARNED && p->sched.trained) {
        int st = sched_enqueue_order(&p->sched, a.codecs, a.comp, a.coff, a.ooff, (uint32_t)a.n,
                                     p->sched.order, s);
        if (st) return st;
        order = p->sched.order;
    } else if (p->opts.order == CODAG_ORDER_CODEC) {
        int st = sched_enqueue_codec_order(&p->sched, a.codecs, (uint32_t)a.n, p->sched.order, s);
        if (st) return st;
        order = p->sched.order;
    }
    if (p->opts.lit_table_bits == 10)
        launch_decode_tb<10>(p, a, order, err, s);
    else
        launch_decode_tb<9>(p, a, order, err, s);
    return hipGetLastError() == hipSuccess ? CODAG_OK : CODAG_E_HIP;
}

int run_batch(codag_plan *p, const BatchArgs &a, hipStream_t s) {
    DeviceState *ds = nullptr;
    int st = device_state(&ds);
    if (st) return st;
    // The scheduler's per-chunk buffers are sized here, never during capture.
    if (((p->opts.order == CODAG_ORDER_LEARNED && p->sched.trained) ||
         p->opts.order == CODAG_ORDER_CODEC) &&
        (st = sched_reserve(&p->sched, (uint32_t)a.n)))
        return st;
    if (!p->opts.use_graph) return enqueue(p, a, ds->err, s);
    if (!(p->have_key && p->key == a)) {
        drop_graph(p);
        if (hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return CODAG_E_HIP;
        st = enqueue(p, a, ds->err, p->capture);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(p->capture, &g);
        if (st || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return st ? st : CODAG_E_HIP;
        }
        p->graph = g;
        if (hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            drop_graph(p);
            return CODAG_E_HIP;
        }
        p->key = a;
        p->have_key = true;
    }
    return hipGraphLaunch(p->exec, s) == hipSuccess ? CODAG_OK : CODAG_E_HIP;
}

// Autotune results kept for the process, keyed by the device's
// architecture, its CU count and the shape of the chunk array: the share of
// each codec in eighths, log2 of the mean output bytes per chunk and of the
// chunk count, and the plan's queue order.
struct TuneEntry {
    std::string key;
    codag_batch_opts opts;
    double ms;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;

int tune_key(codag_plan *p, const uint8_t *codecs, const uint64_t *ooff, uint64_t n, hipStream_t s,
             std::string &key) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, p->device) != hipSuccess) return CODAG_E_HIP;
    std::vector<uint8_t> c(n);
    uint64_t o[2] = {0, 0};
    if (hipMemcpyAsync(c.data(), codecs, n, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&o[0], ooff, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&o[1], ooff + n, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return CODAG_E_HIP;
    uint64_t count[6] = {0, 0, 0, 0, 0, 0};
    for (uint8_t v : c) count[v <= CODAG_LZ4 ? v : 0]++;
    const uint64_t mean = o[1] > o[0] ? (o[1] - o[0]) / n : 0;
    char buf[384];
    int len = std::snprintf(buf, sizeof(buf), "%s cus=%d mix=", prop.gcnArchName, p->num_cus);
    for (int k = 0; k < 6; k++)
        len += std::snprintf(buf + len, sizeof(buf) - len, "%s%d", k ? "," : "",
                             (int)((8 * count[k] + n / 2) / n));
    std::snprintf(buf + len, sizeof(buf) - len, " out=2^%d n=2^%d order=%d",
                  mean ? 63 - __builtin_clzll(mean) : 0, 63 - __builtin_clzll(n), p->opts.order);
    key = buf;
    for (char &ch : key)
        if (ch == '|' || ch == '\n') ch = '_';
    return CODAG_OK;
}

// The tuned knobs of a cached configuration, laid over the plan's own.
void apply_tuned(const codag_batch_opts &t, codag_batch_opts *o) {
    o->history_kib = t.history_kib;
    o->lit_table_bits = t.lit_table_bits;
    o->waves_per_block = t.waves_per_block;
    o->chunks_per_claim = t.chunks_per_claim;
    o->waves_per_cu = t.waves_per_cu;
    if (o->order == CODAG_ORDER_INDEX) o->order = t.order;
}

int check_args(codag_plan *plan, const uint8_t *codecs, const uint8_t *comp, const uint64_t *coff,
               uint8_t *out, const uint64_t *ooff, uint64_t n, const uint32_t *order) {
    if (!plan) return CODAG_E_INVALID_ARGUMENT;
    if (n == 0) return CODAG_OK;
    if (n >= (1ull << 32) - 64) return CODAG_E_INVALID_ARGUMENT;
    if (!codecs || !comp || !coff || !out || !ooff) return CODAG_E_INVALID_ARGUMENT;
    if (plan->opts.order == CODAG_ORDER_GIVEN && !order) return CODAG_E_INVALID_ARGUMENT;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return CODAG_E_HIP;
    if (dev != plan->device) return CODAG_E_INVALID_ARGUMENT;
    return CODAG_OK;
}

}  // namespace

extern "C" {

int codag_plan_create(codag_plan **plan, const codag_batch_opts *opts) {
    if (!plan) return CODAG_E_INVALID_ARGUMENT;
    *plan = nullptr;
    auto *p = new codag_plan();
    if (hipGetDevice(&p->device) != hipSuccess ||
        hipDeviceGetAttribute(&p->num_cus, hipDeviceAttributeMultiprocessorCount, p->device) !=
            hipSuccess) {
        delete p;
        return CODAG_E_HIP;
    }
    int st = resolve_opts(opts, &p->opts);
    if (st) {
        delete p;
        return st;
    }
    if (hipMalloc(&p->head, sizeof(uint32_t)) != hipSuccess ||
        hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking) != hipSuccess) {
        codag_plan_destroy(p);
        return CODAG_E_HIP;
    }
    st = sched_init(&p->sched);
    if (st) {
        codag_plan_destroy(p);
        return st;
    }
    *plan = p;
    return CODAG_OK;
}

void codag_plan_destroy(codag_plan *plan) {
    if (!plan) return;
    (void)hipDeviceSynchronize();
    drop_graph(plan);
    sched_free(&plan->sched);
    if (plan->head) (void)hipFree(plan->head);
    if (plan->capture) (void)hipStreamDestroy(plan->capture);
    delete plan;
}

int codag_plan_get_opts(const codag_plan *plan, codag_batch_opts *opts) {
    if (!plan || !opts) return CODAG_E_INVALID_ARGUMENT;
    *opts = plan->opts;
    return CODAG_OK;
}

int codag_plan_set_opts(codag_plan *plan, const codag_batch_opts *opts) {
    if (!plan) return CODAG_E_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lock(plan->mu);
    codag_batch_opts r;
    int st = resolve_opts(opts, &r);
    if (st) return st;
    plan->opts = r;
    drop_graph(plan);
    return CODAG_OK;
}

int codag_decompress_batch(codag_plan *plan, const uint8_t *codecs, const uint8_t *comp_buf,
                           const uint64_t *chunk_offsets, uint8_t *out_buf,
                           const uint64_t *out_offsets, uint64_t n_chunks,
                           int32_t *chunk_status, const uint32_t *order,
                           uint64_t *chunk_ticks, void *stream) {
    int st = check_args(plan, codecs, comp_buf, chunk_offsets, out_buf, out_offsets, n_chunks, order);
    if (st || n_chunks == 0) return st;
    std::lock_guard<std::mutex> lock(plan->mu);
    BatchArgs a{codecs, comp_buf, chunk_offsets, out_buf, out_offsets, n_chunks,
                chunk_status, plan->opts.order == CODAG_ORDER_GIVEN ? order : nullptr, chunk_ticks};
    return run_batch(plan, a, static_cast<hipStream_t>(stream));
}

int codag_autotune(codag_plan *plan, const uint8_t *codecs, const uint8_t *comp_buf,
                   const uint64_t *chunk_offsets, uint8_t *out_buf, const uint64_t *out_offsets,
                   uint64_t n_chunks, const uint32_t *order, int reps, double *best_ms,
                   void *stream) {
    int st = check_args(plan, codecs, comp_buf, chunk_offsets, out_buf, out_offsets, n_chunks, order);
    if (st) return st;
    if (reps < 1 || reps > 1000) return CODAG_E_INVALID_ARGUMENT;
    if (n_chunks == 0) return CODAG_OK;
    std::lock_guard<std::mutex> lock(plan->mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const codag_batch_opts base = plan->opts;
    std::string key;
    if ((st = tune_key(plan, codecs, out_offsets, n_chunks, s, key))) return st;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        for (const TuneEntry &e : g_tune) {
            if (e.key != key) continue;
            codag_batch_opts o = base, r;
            apply_tuned(e.opts, &o);
            if (resolve_opts(&o, &r)) break;  // stale entry: tune again
            r.use_graph = base.use_graph;
            plan->opts = r;
            drop_graph(plan);
            if (best_ms) *best_ms = e.ms;
            return CODAG_OK;
        }
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return CODAG_E_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return CODAG_E_HIP;
    }
    double best = 1e30;
    codag_batch_opts best_opts = base;
    auto trial = [&](codag_batch_opts o) -> int {
        codag_batch_opts r;
        if (resolve_opts(&o, &r)) return CODAG_OK;
        plan->opts = r;
        plan->opts.use_graph = 0;
        BatchArgs a{codecs, comp_buf, chunk_offsets, out_buf, out_offsets, n_chunks, nullptr,
                    r.order == CODAG_ORDER_GIVEN ? order : nullptr, nullptr};
        int rc = run_batch(plan, a, s);  // warm-up
        if (rc) return rc;
        std::vector<float> t;
        for (int k = 0; k < reps; k++) {
            if (hipEventRecord(e0, s) != hipSuccess) return CODAG_E_HIP;
            rc = run_batch(plan, a, s);
            if (rc) return rc;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                return CODAG_E_HIP;
            float ms = 0;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return CODAG_E_HIP;
            t.push_back(ms);
        }
        std::sort(t.begin(), t.end());
        double med = t[t.size() / 2];
        if (med < best) {
            best = med;
            best_opts = r;
            best_opts.use_graph = base.use_graph;
        }
        return CODAG_OK;
    };
    // Coordinate search: window size, Deflate table bits, waves per
    // workgroup, chunks per queue claim, codec-grouped against index order
    // (when the plan's order is the index order), then the number of
    // resident waves per CU.
    for (int hist : {4, 8, 16}) {
        if (st) break;
        codag_batch_opts o = base;
        o.history_kib = hist;
        o.waves_per_cu = 0;
        st = trial(o);
    }
    for (int tb : {9, 10}) {
        if (st) break;
        codag_batch_opts o = best_opts;
        o.lit_table_bits = tb;
        o.waves_per_cu = 0;
        st = trial(o);
    }
    for (int wpb : {1, 2, 4}) {
        if (st) break;
        codag_batch_opts o = best_opts;
        o.waves_per_block = wpb;
        o.waves_per_cu = 0;
        st = trial(o);
    }
    for (int claim : {1, 2, 4}) {
        if (st) break;
        codag_batch_opts o = best_opts;
        o.chunks_per_claim = claim;
        o.waves_per_cu = 0;
        st = trial(o);
    }
    if (base.order == CODAG_ORDER_INDEX) {
        for (int ord : {CODAG_ORDER_INDEX, CODAG_ORDER_CODEC}) {
            if (st) break;
            codag_batch_opts o = best_opts;
            o.order = ord;
            o.waves_per_cu = 0;
            st = trial(o);
        }
    }
    if (!st) {
        int top = max_waves_per_cu(best_opts.history_kib, best_opts.lit_table_bits,
                                   best_opts.waves_per_block);
        for (int w = top - 2 * best_opts.waves_per_block; w >= std::max(4, top / 2) && !st;
             w -= 2 * best_opts.waves_per_block) {
            codag_batch_opts o = best_opts;
            o.waves_per_cu = w;
            st = trial(o);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    plan->opts = best_opts;
    drop_graph(plan);
    if (best_ms) *best_ms = best;
    if (!st) {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune.push_back(TuneEntry{key, best_opts, best});
    }
    return st;
}

int codag_autotune_cache_save(char *buf, size_t cap, size_t *len) {
    std::string text;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        for (const TuneEntry &e : g_tune) {
            char line[160];
            std::snprintf(line, sizeof(line), "|%d|%d|%d|%d|%d|%d|%.6f\n", e.opts.history_kib,
                          e.opts.lit_table_bits, e.opts.waves_per_block, e.opts.chunks_per_claim,
                          e.opts.waves_per_cu, e.opts.order, e.ms);
            text += e.key;
            text += line;
        }
    }
    if (len) *len = text.size() + 1;
    if (!buf || cap < text.size() + 1) return CODAG_E_INVALID_ARGUMENT;
    std::memcpy(buf, text.c_str(), text.size() + 1);
    return CODAG_OK;
}

int codag_autotune_cache_load(const char *text) {
    if (!text) return CODAG_E_INVALID_ARGUMENT;
    std::vector<TuneEntry> add;
    const char *p = text;
    while (*p) {
        const char *nl = std::strchr(p, '\n');
        if (!nl) return CODAG_E_INVALID_ARGUMENT;
        std::string line(p, nl);
        p = nl + 1;
        const size_t bar = line.find('|');
        if (bar == 0 || bar == std::string::npos) return CODAG_E_INVALID_ARGUMENT;
        TuneEntry e{};
        e.key = line.substr(0, bar);
        int nread = 0;
        if (std::sscanf(line.c_str() + bar, "|%d|%d|%d|%d|%d|%d|%lf%n", &e.opts.history_kib,
                        &e.opts.lit_table_bits, &e.opts.waves_per_block, &e.opts.chunks_per_claim,
                        &e.opts.waves_per_cu, &e.opts.order, &e.ms, &nread) != 7 ||
            (size_t)nread != line.size() - bar || !(e.ms >= 0))
            return CODAG_E_INVALID_ARGUMENT;
        codag_batch_opts r;
        if (e.opts.waves_per_cu < 1 || resolve_opts(&e.opts, &r)) return CODAG_E_INVALID_ARGUMENT;
        add.push_back(e);
    }
    std::lock_guard<std::mutex> g(g_tune_mu);
    for (TuneEntry &e : add) {
        auto it = std::find_if(g_tune.begin(), g_tune.end(), [&](const TuneEntry &x) { return x.key == e.key; });
        if (it != g_tune.end())
            *it = e;
        else
            g_tune.push_back(e);
    }
    return CODAG_OK;
}

void codag_autotune_cache_clear(void) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune.clear();
}

}  // extern "C"
