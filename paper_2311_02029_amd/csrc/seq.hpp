// Sequence-set kernels shared by the index build and the read path: packing
// ASCII into bit planes, and tiled minimizer extraction.
#pragma once

#include "runtime.hpp"

namespace mt {

// Bit planes of a sequence set (layout described in device.hpp).
struct PackedSeqs {
    DBuf<u64x2> lohi;
    DBuf<u64> nb;
    DBuf<u64> blk_off;  // n + 1: first block of each sequence
    u64 n = 0;
    u64 blocks_cap = 0;
};

// Packs `in` (device ASCII) into planes.  The offsets are checked first (a
// synchronizing step): a sequence longer than len_limit fails with
// len_message, malformed offsets with MT_EINVAL.  Bad bytes raise
// ERR_BAD_BYTE in d_flags; has_n (nullable, n entries, zeroed by the caller)
// receives 1 for sequences containing N.
void pack_sequences(const mt_seqs &in, u64 len_limit, u32 len_flag, const char *len_message, PackedSeqs &out,
                    u32 *d_flags, u32 *has_n, hipStream_t s);

// Tiled minimizer extraction.  plan() sizes the tiles and counts the
// minimizers of every tile; after the caller has read n_tiles / n_min back
// (tile_off[n] and min_off[n_tiles]), emit() writes them in sequence order.
struct MinimizerPlan {
    int tile = 0;
    DBuf<u64> tile_off;   // n + 1
    DBuf<u32> tile_map;   // tile -> sequence
    DBuf<u32> tile_count;
    DBuf<u64> tile_bits;  // TILE / 64 words of chosen starts per tile
    DBuf<u64> min_off;    // n_tiles + 1 (allocated for the tile bound)
    u64 tiles_cap = 0;
};
void minimizer_plan(const mt_seqs &in, const PackedSeqs &ps, u32 k, u32 w, int tile, MinimizerPlan &mp,
                    hipStream_t s);
void minimizer_emit(const mt_seqs &in, const PackedSeqs &ps, u32 k, u32 w, MinimizerPlan &mp, u64 *out_x,
                    u32 *out_seq, u32 *out_pos, hipStream_t s);

// Copies `count` values from device to host and waits for the stream.
void read_back(hipStream_t s, const void *dev, void *host, size_t bytes);

}  // namespace mt
