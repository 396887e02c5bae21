// tile_lds_model.cpp -- bounds-checked CPU model of the index arithmetic of
// the mesh fine pass's LDS block (one 64-lane wave per 8x8 tile).
//
// The model replays, for every lane of the wave, the offsets the tile pass
// computes into its LDS block -- the compaction of a chunk's face records
// (a lane's rank among the lanes that keep a face), lane j's read of record
// j's pixel mask, the bit transpose across the wave (the same six butterfly
// stages as the kernel's), the records read back through the bits of every
// lane's word, and the staging offsets of the fragment write-out for every
// queue size -- against the block sizes of tile_layout.hpp, which the kernel
// uses as well.  The transpose is also checked against its definition.
// Every access goes through a checked accessor; the program is built with
// AddressSanitizer and UndefinedBehaviorSanitizer.
//
//   tile_lds_model [chunk]   chunk: faces per chunk (default: the kernel's);
//                            a chunk narrower than the wave shows what goes
//                            wrong when 64 lanes gather into a smaller block
// Exit status 0: every offset in bounds; 1: an out-of-bounds offset (printed).
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2007_08501_amd/csrc/tile_layout.hpp"

namespace tl = rast::tile_layout;

struct Block {
    int chunk;           // records in the block
    size_t rec_bytes;    // chunk * kTileRecBytes
    std::vector<unsigned char> mem;
    std::vector<uint64_t> mask;  // each record's pixel mask (a field of the record)
    explicit Block(int c)
        : chunk(c), rec_bytes((size_t)c * tl::kTileRecBytes), mem(rec_bytes + tl::kSpareBytes), mask(c) {}
};

// The kernel's transpose: row i of the 64x64 bit matrix in lane i.
static void transpose64(uint64_t (&x)[tl::kLanes]) {
    static const uint64_t kLow[6] = {0x5555555555555555ull, 0x3333333333333333ull, 0x0f0f0f0f0f0f0f0full,
                                     0x00ff00ff00ff00ffull, 0x0000ffff0000ffffull, 0x00000000ffffffffull};
    for (int s = 5; s >= 0; --s) {
        const int j = 1 << s;
        const uint64_t m = kLow[s];
        uint64_t y[tl::kLanes];
        for (int l = 0; l < tl::kLanes; ++l) y[l] = x[l ^ j];
        for (int l = 0; l < tl::kLanes; ++l)
            x[l] = (l & j) ? ((x[l] & ~m) | ((y[l] & ~m) >> j)) : ((x[l] & m) | ((y[l] & m) << j));
    }
}

static int fail(const char* what, long long idx, long long limit, int lane) {
    std::printf("OUT OF BOUNDS: %s index %lld, limit %lld (lane %d)\n", what, idx, limit, lane);
    return 1;
}

// One chunk of up to `chunk` list entries gathered by 64 lanes, each lane
// keeping its face with probability keep_p; `cov` decides which kept faces'
// boxes cover which lane's pixel.
static int chunk_pass(Block& B, long long c0, long long cnt, std::mt19937_64& rng, double keep_p, double cov_p) {
    std::bernoulli_distribution keep_d(keep_p), cov_d(cov_p);
    // 1. gather: lane l takes list entry c0 + l; compaction by rank among keepers
    uint64_t kept = 0;
    for (int lane = 0; lane < tl::kLanes; ++lane) {
        const bool in_list = c0 + lane < cnt;
        if (in_list && keep_d(rng)) kept |= 1ull << lane;
    }
    for (int lane = 0; lane < tl::kLanes; ++lane) {
        if (!((kept >> lane) & 1ull)) continue;
        const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        const int dst = __builtin_popcountll(kept & lt);
        if (dst >= B.chunk) return fail("chunk record", dst, B.chunk, lane);
        const size_t off = (size_t)dst * tl::kTileRecBytes;
        B.mem.at(off) = (unsigned char)dst;  // first byte of the record
    }
    const int m = __builtin_popcountll(kept);
    // 2. lane j < m reads record j's pixel mask; the transpose hands lane p
    //    the faces whose masks hold pixel p
    uint64_t row[tl::kLanes], word[tl::kLanes];
    for (int j = 0; j < m; ++j) {
        uint64_t mk = 0;
        for (int lane = 0; lane < tl::kLanes; ++lane)
            if (cov_d(rng)) mk |= 1ull << lane;
        if (j >= B.chunk) return fail("record mask", j, B.chunk, j);
        B.mask.at(j) = mk;
    }
    for (int lane = 0; lane < tl::kLanes; ++lane) {
        if (lane < m && lane >= B.chunk) return fail("record mask read", lane, B.chunk, lane);
        row[lane] = word[lane] = lane < m ? B.mask.at(lane) : 0ull;
    }
    transpose64(word);
    // 3. read back: every bit of a lane's word names a record of this chunk,
    //    and the words are the transpose of the rows
    for (int lane = 0; lane < tl::kLanes; ++lane) {
        for (int i = 0; i < tl::kLanes; ++i) {
            const bool bit = (word[lane] >> i) & 1ull;
            if (bit != (bool)((row[i] >> lane) & 1ull)) {
                std::printf("TRANSPOSE: lane %d bit %d\n", lane, i);
                return 1;
            }
            if (bit && i >= m) return fail("record named by a lane's word", i, m, lane);
            if (bit) (void)B.mem.at((size_t)i * tl::kTileRecBytes);  // the record the test reads
        }
    }
    return 0;
}

// Staging offsets of the fragment write-out for a queue of kb slots (the
// kernel's two passes: ids and depths kStageG1 slots at a time, then
// barycentrics and distances kStageG2 slots at a time), in 4-byte words.
static int staging(const Block& B, int kb) {
    const long long words = (long long)B.mem.size() / 4;
    {
        const int G = kb < tl::kStageG1 ? kb : tl::kStageG1, S = G + 1;
        for (int lane = 0; lane < tl::kLanes; ++lane)
            for (int k = 0; k < G; ++k) {
                const long long sid = (long long)lane * S + k, sz = 64LL * S + lane * S + k;
                if (sid >= words) return fail("id staging", sid, words, lane);
                if (sz >= words) return fail("depth staging", sz, words, lane);
            }
    }
    {
        const int G = kb < tl::kStageG2 ? kb : tl::kStageG2, SB = 3 * G + 1, SD = G + 1;
        for (int lane = 0; lane < tl::kLanes; ++lane)
            for (int k = 0; k < G; ++k) {
                const long long sb = (long long)lane * SB + 3 * k + 2, sd = 64LL * SB + lane * SD + k;
                if (sb >= words) return fail("bary staging", sb, words, lane);
                if (sd >= words) return fail("dist staging", sd, words, lane);
            }
    }
    return 0;
}

int main(int argc, char** argv) {
    const int chunk = argc > 1 ? std::atoi(argv[1]) : tl::kChunk;
    if (chunk <= 0 || chunk > tl::kLanes) {
        std::printf("chunk must be in 1..%d\n", tl::kLanes);
        return 2;
    }
    Block B(chunk);
    std::mt19937_64 rng(12345);
    // bins of many sizes, the chunk loop stepping by `chunk` as the kernel does
    const long long counts[] = {0, 1, 7, 47, 48, 63, 64, 65, 100, 127, 128, 129, 480, 1000};
    const double keeps[] = {0.05, 0.5, 1.0};
    const double covs[] = {0.1, 0.6, 1.0};
    for (long long cnt : counts)
        for (double kp : keeps)
            for (double cp : covs)
                for (long long c0 = 0; c0 < cnt; c0 += chunk)
                    if (chunk_pass(B, c0, cnt, rng, kp, cp)) return 1;
    for (int kb : {1, 2, 4, 8, 16, 32, 64})
        if (staging(B, kb)) return 1;
    std::printf("ok: chunk %d, LDS block %zu bytes, every offset in bounds\n", chunk, B.mem.size());
    return 0;
}
