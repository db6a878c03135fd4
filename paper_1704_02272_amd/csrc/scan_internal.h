// Shapes and scratch of the tiled scan kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pfac_impl.h"

namespace pfac {

constexpr uint32_t kThreads = 1024;  // workgroup: 16 waves sharing one LDS image
constexpr uint32_t kWaves = kThreads / 64;
constexpr uint32_t kStep = 1024;     // bytes a wave streams per step: 64 lanes x 16
constexpr uint32_t kSpan = 16384;    // bytes per work unit (a wave's ticket)
constexpr uint32_t kQCap = 1088;     // survivor queue: 63 left over + a whole step
constexpr uint32_t kHCap = 256;      // hit queue (starts with a match) per span
constexpr uint32_t kWaveLds = (kQCap + kHCap) * 2;  // bytes of LDS per wave
static_assert(kSpan <= 65536, "span-local starts are 16-bit");
static_assert(kWaveLds % 16 == 0, "wave regions stay 16-byte aligned");

__host__ __device__ inline size_t image_bytes(const DevTable &t) { return ((size_t)t.lds_words * 4 + 15) & ~(size_t)15; }

// Decoupled look-back state of one scan (device memory, owned by a workspace).
//   word[t]   one 64-bit word per span: epoch (bits 44..63) | flag (42..43) | value (0..41)
//             flag 1: value = matches in span t; flag 2: value = matches in spans 0..t.
//             Flag and value share one word, so publishing and reading need only relaxed
//             device-scope atomics: no fence, no L2 write-back or invalidate per tile.
//   ctrl[0]   span ticket   ctrl[1] waves done   ctrl[2] epoch (1 .. 2^20 - 1)
//   ctrl[3]   error bits (1: a bounded wait expired, 2: count past 2^42)
// The last wave of a launch writes the count, resets the ticket and the done count
// and advances the epoch, so a later launch (or a replayed graph) needs no host-side
// reset; words of an older epoch never match. The host clears the words before the epoch
// could wrap (kEpochPeriod launches).
constexpr uint32_t kEpochBits = 20;
constexpr uint64_t kEpochPeriod = (1u << kEpochBits) - 2;
constexpr uint64_t kValueMask = (1ull << 42) - 1;
struct TileState {
    uint64_t *word;
    uint32_t *ctrl;
};

// Count value that reports a device-side error (the host maps it to a status).
constexpr uint64_t kCountTimeout = ~0ull;
constexpr uint64_t kCountOverflow = ~0ull - 1;

size_t scan_lds_bytes(const DevTable &t);
// grid = 0: as many workgroups as fit on the device at once.
int launch_tiled(const DevTable &t, const uint8_t *text, uint64_t n, const uint64_t *offsets,
                 uint32_t n_packets, uint64_t *keys, uint64_t cap, uint64_t *d_count,
                 const TileState &ts, uint32_t grid, hipStream_t s);

}  // namespace pfac
