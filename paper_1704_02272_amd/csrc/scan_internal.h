// Shapes and scratch of the tiled scan kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pfac_impl.h"

namespace pfac {

constexpr uint32_t kThreads = 512;             // workgroup size (8 waves of 64)
constexpr uint32_t kWaves = kThreads / 64;
constexpr uint32_t kTile = 16384;              // start positions per tile
constexpr uint32_t kHalo = 256;                // text staged past the tile end
static_assert(kTile / 32 == kThreads, "one survivor-bitmap word per lane");
static_assert(kTile % (16 * kThreads) == 0, "whole prefilter rounds");

// Decoupled look-back state of one scan (device memory, owned by a workspace).
//   word[t]   one 64-bit word per tile: epoch (bits 44..63) | flag (42..43) | value (0..41)
//             flag 1: value = matches in tile t; flag 2: value = matches in tiles 0..t.
//             Flag and value share one word, so publishing and reading need only relaxed
//             device-scope atomics: no fence, no L2 write-back or invalidate per tile.
//   ctrl[0]   tile ticket   ctrl[1] workgroups done   ctrl[2] epoch (1 .. 2^20 - 1)
//   ctrl[3]   error bits (1: a bounded wait expired, 2: count past 2^42)
// The last workgroup of a launch writes the count, resets the ticket and the done count
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
uint32_t scan_grid(const DevTable &t, uint64_t n_tiles);
int launch_tiled(const DevTable &t, const uint8_t *text, uint64_t n, const uint64_t *offsets,
                 uint32_t n_packets, uint64_t *keys, uint64_t cap, uint64_t *d_count,
                 const TileState &ts, uint32_t grid, hipStream_t s);

}  // namespace pfac
