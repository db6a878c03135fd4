// Scan kernels over the compressed trie of Section 3.2 (device code in scan_kernels.h):
// the same walk, with pattern ids found by the rank of the spelled string.
#include "scan_kernels.h"

namespace pfac {

int launch_tiled_merged(const DevTable &t, const uint8_t *text, uint64_t n, const uint64_t *offsets,
                        uint32_t n_packets, uint64_t *keys, uint64_t cap, uint64_t *d_count, const SpanOut &so,
                        const TileState &ts, const uint64_t *sizes, uint32_t grid, uint32_t span_log2,
                        uint32_t lane_bytes, hipStream_t s) {
    return launch_tiled_t<true>(t, text, n, offsets, n_packets, keys, cap, d_count, so, ts, sizes, grid, span_log2,
                                lane_bytes, s);
}

}  // namespace pfac
