// Kernel launchers (device code lives in kernels_*.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pfac_impl.h"

namespace pfac {

// Plain scan (one lane per start, trie in HBM, count pass + emit pass).
int launch_plain(const DevTable &t, const uint8_t *text, uint64_t n, uint64_t *keys,
                 uint64_t cap, uint64_t *d_count, uint64_t *block_counts,
                 uint64_t *block_offsets, hipStream_t s);
uint64_t plain_blocks(uint64_t n);

// Histogram of prefix depths (walk steps before a missing transition, capped at cap,
// 1 <= cap <= 63) of every start of text[0 .. n) into hist[0 .. cap], zeroed first.
int launch_prefix_hist(const DevTable &t, const uint8_t *text, uint64_t n, uint32_t cap, uint64_t *hist,
                       uint32_t cus, hipStream_t s);

// Store one value to device memory (graph-capture safe: a kernel, not a memset).
int launch_set_u64(uint64_t *dst, uint64_t value, hipStream_t s);

// Free the scratch the automaton keeps for `stream` on every device (after the stream
// has drained). Owners of streams they destroy call it first, so scratch keyed by a
// stream's address never outlives the stream.
void release_stream(pfac_automaton *a, void *stream);
// Number of per-stream scratch areas the automaton holds (all devices).
size_t workspace_count(pfac_automaton *a);
// Upload the table to the current device if needed and size `stream`'s scratch for
// scans of up to n bytes, so later scans of that size allocate nothing.
int reserve_stream(pfac_automaton *a, void *stream, uint64_t n);

}  // namespace pfac
