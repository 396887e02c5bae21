// tile_layout.hpp -- sizes of the mesh fine pass's LDS block, shared by the
// kernel (kernels_fwd.hip) and the bounds-checked CPU model of its index
// arithmetic (tests/cpu_models/tile_lds_model.cpp).  Plain C++: no HIP types.
//
// One 64-lane wave rasterizes one 8x8 tile.  Per chunk of faces it keeps, in
// LDS, the chunk's tile records (kTileRecBytes each); lane j reads record j's
// pixel mask and a bit transpose across the wave gives every lane the
// chunk's faces that may cover its pixel (bit j = record j).  After the last
// chunk the same block, with kSpareBytes more, is reused to stage the
// fragments for coalesced stores (kStageG1 slots of ids and depths, then
// kStageG2 slots of barycentrics and distances, per pass).
#pragma once

namespace rast {
namespace tile_layout {

constexpr int kLanes = 64;         // wave width, one lane per tile pixel
constexpr int kChunk = 64;         // faces per chunk: the gather takes one list entry per lane, and
                                   // the transpose one record per lane
constexpr int kTileRecBytes = 96;  // a face as the tile pass keeps it
constexpr int kStageG1 = 16;       // slots per staging pass for ids and depths
constexpr int kStageG2 = 8;        // slots per staging pass for barycentrics and distances
constexpr int kRecBytes = kChunk * kTileRecBytes;
constexpr int kSpareBytes = 4096;  // room the write-out staging needs beyond the records
constexpr int kLdsBytes = kRecBytes + kSpareBytes;

static_assert(kChunk == kLanes, "the chunk gather gives every lane exactly one entry of the bin list, and the "
                                "transpose one record per lane");

// Staging footprint in 4-byte words for a queue of kb slots.
constexpr int stage_words_g1(int kb) { return 2 * kLanes * ((kb < kStageG1 ? kb : kStageG1) + 1); }
constexpr int stage_words_g2(int kb) {
    return kLanes * (3 * (kb < kStageG2 ? kb : kStageG2) + 1) + kLanes * ((kb < kStageG2 ? kb : kStageG2) + 1);
}
static_assert(4 * stage_words_g1(64) <= kLdsBytes, "id/depth staging exceeds the tile LDS");
static_assert(4 * stage_words_g2(64) <= kLdsBytes, "bary/dist staging exceeds the tile LDS");

}  // namespace tile_layout
}  // namespace rast
