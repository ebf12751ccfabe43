// Host-side state shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "../../include/codag.h"
#include "sched.hpp"

namespace codag {

constexpr int kMaxDevices = 64;

struct DeviceState {
    unsigned long long *err = nullptr;  // first-error word: (chunk << 4) | -status, then a result slot
    void *scratch = nullptr;            // this device's static scratch array
};

extern std::mutex g_mu;
extern DeviceState g_dev[kMaxDevices];

// The current device's state, created on first use.
int device_state(DeviceState **out);

// Group-parallel RLE v1 (few chunks): index, decode and status passes on s.
// The passes share a device workspace of rle_v1_split_workspace(n) bytes
// (every byte written before it is read, so it needs no clearing): the
// caller's, or with workspace == NULL one from the stream-ordered allocator.
int launch_rle_v1_split(const uint8_t *comp, const uint64_t *coff, uint8_t *out,
                        const uint64_t *ooff, uint32_t n, int32_t *status, unsigned long long *err,
                        hipStream_t s, void *workspace);
size_t rle_v1_split_workspace(uint32_t n);
constexpr uint64_t kSplitMaxChunks = 256;
// Per chunk: 32 range records of 16 bytes and two 8-byte error keys.
constexpr size_t kSplitWorkspacePerChunk = 32 * 16 + 2 * 8;

// Group-parallel RLE v2 (index pass, one decoding wave per range, status
// pass), the same way; workspace rle_v2_split_workspace(n) bytes.
int launch_rle_v2_split(const uint8_t *comp, const uint64_t *coff, uint8_t *out,
                        const uint64_t *ooff, uint32_t n, int32_t *status, unsigned long long *err,
                        hipStream_t s, void *workspace);
size_t rle_v2_split_workspace(uint32_t n);
constexpr uint64_t kSplitV2MaxChunks = 2048;
// Per chunk: 8 range starts of 8 bytes, the stop value and padding (16
// bytes), two 8-byte error keys.
constexpr size_t kSplitV2WorkspacePerChunk = 8 * 8 + 16 + 2 * 8;

// The decoding-unit ablations (codag_opts.variant != 0), on stream s.
int launch_variant(int variant, int codec, const uint8_t *comp, const uint64_t *coff, uint8_t *out,
                   const uint64_t *ooff, uint32_t n, int32_t *status, unsigned long long *err,
                   hipStream_t s);

// Byte RLE and RLE element types other than signed 8-byte values (one wave
// per chunk), on stream s.
int launch_typed(int codec, int elem_bytes, bool is_unsigned, const uint8_t *comp, const uint64_t *coff,
                 uint8_t *out, const uint64_t *ooff, uint32_t n, int32_t *status,
                 unsigned long long *err, uint64_t *ticks, hipStream_t s);

// Arguments of one batched launch (a captured graph is reused while they
// stay the same).
struct BatchArgs {
    const uint8_t *codecs;
    const uint8_t *comp;
    const uint64_t *coff;
    uint8_t *out;
    const uint64_t *ooff;
    uint64_t n;
    int32_t *status;
    const uint32_t *order;
    uint64_t *ticks;
    bool operator==(const BatchArgs &o) const { return std::memcmp(this, &o, sizeof(*this)) == 0; }
};

}  // namespace codag

struct codag_plan {
    int device = 0;
    int num_cus = 0;
    codag_batch_opts opts{};
    uint32_t *head = nullptr;  // queue position counter
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    codag::BatchArgs key{};
    bool have_key = false;
    codag::SchedState sched;       // learned cost model and its buffers
    std::mutex mu;
};
