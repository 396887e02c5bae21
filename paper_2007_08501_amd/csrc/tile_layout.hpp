// tile_layout.hpp -- sizes of the mesh fine pass's LDS block, shared by the
// kernel (kernels_fwd.hip) and the bounds-checked CPU model of its index
// arithmetic (tests/cpu_models/tile_lds_model.cpp).  Plain C++: no HIP types.
//
// One 64-lane wave rasterizes one 8x8 tile.  Per chunk of faces it keeps, in
// LDS, the chunk's tile records (kTileRecBytes each) and one byte list per
// lane (entry i of lane l at byte i * kLanes + l); after the last chunk the
// same block is reused to stage the fragments for coalesced stores
// (kStageG1 slots of ids and depths, then kStageG2 slots of barycentrics and
// distances, per pass).
#pragma once

namespace rast {
namespace tile_layout {

constexpr int kLanes = 64;         // wave width, one lane per tile pixel
constexpr int kChunk = 64;         // faces per chunk: the gather takes one list entry per lane
constexpr int kTileRecBytes = 96;  // a face as the tile pass keeps it
constexpr int kStageG1 = 16;       // slots per staging pass for ids and depths
constexpr int kStageG2 = 8;        // slots per staging pass for barycentrics and distances
constexpr int kRecBytes = kChunk * kTileRecBytes;
constexpr int kListBytes = kChunk * kLanes;
constexpr int kLdsBytes = kRecBytes + kListBytes;

static_assert(kChunk == kLanes, "the chunk gather gives every lane exactly one entry of the bin list");

// Staging footprint in 4-byte words for a queue of kb slots.
constexpr int stage_words_g1(int kb) { return 2 * kLanes * ((kb < kStageG1 ? kb : kStageG1) + 1); }
constexpr int stage_words_g2(int kb) {
    return kLanes * (3 * (kb < kStageG2 ? kb : kStageG2) + 1) + kLanes * ((kb < kStageG2 ? kb : kStageG2) + 1);
}
static_assert(4 * stage_words_g1(64) <= kLdsBytes, "id/depth staging exceeds the tile LDS");
static_assert(4 * stage_words_g2(64) <= kLdsBytes, "bary/dist staging exceeds the tile LDS");

}  // namespace tile_layout
}  // namespace rast
