// tile_lds_model.cpp -- bounds-checked CPU model of the index arithmetic of
// the mesh fine pass's LDS block (one 64-lane wave per 8x8 tile).
//
// The model replays, for every lane of the wave, the offsets the tile pass
// computes into its LDS block -- the compaction of a chunk's face records
// (a lane's rank among the lanes that keep a face), the per-lane byte lists
// (entry i of lane l at byte i * 64 + l), the records read back through those
// lists, and the staging offsets of the fragment write-out for every queue
// size -- against the block sizes of tile_layout.hpp, which the kernel uses
// as well.  Every access goes through a checked accessor; the program is
// built with AddressSanitizer and UndefinedBehaviorSanitizer.
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
    size_t list_bytes;   // chunk * kLanes
    std::vector<unsigned char> mem;
    explicit Block(int c)
        : chunk(c), rec_bytes((size_t)c * tl::kTileRecBytes), list_bytes((size_t)c * tl::kLanes),
          mem(rec_bytes + list_bytes) {}
};

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
    // 2. per-lane byte lists of the kept faces whose boxes cover the lane's pixel
    std::vector<std::vector<int>> cov(m, std::vector<int>(tl::kLanes));
    for (int j = 0; j < m; ++j)
        for (int lane = 0; lane < tl::kLanes; ++lane) cov[j][lane] = cov_d(rng);
    std::vector<int> nl(tl::kLanes, 0);
    for (int lane = 0; lane < tl::kLanes; ++lane) {
        for (int j = 0; j < m; ++j) {
            if (!cov[j][lane]) continue;
            const long long off = (long long)tl::kLanes * nl[lane] + lane;
            if (off >= (long long)B.list_bytes) return fail("lane list", off, (long long)B.list_bytes, lane);
            B.mem.at(B.rec_bytes + (size_t)off) = (unsigned char)j;
            ++nl[lane];
        }
    }
    // 3. read back: every list entry names a record of this chunk
    for (int lane = 0; lane < tl::kLanes; ++lane) {
        for (int i = 0; i < nl[lane]; ++i) {
            const int j = B.mem.at(B.rec_bytes + (size_t)tl::kLanes * i + lane);
            if (j >= m) return fail("record named by a list", j, m, lane);
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
