// Shared pieces of the paths that advance many pairs per launch (batched solves, serving):
// table builders, grow-only buffers, and the choice and tiling of the K-iteration tile launches
// over the current levels of several pairs.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <iterator>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "runtime.hpp"

namespace flowmi {

constexpr int kBatchNt = 1025;   // general tile kernel of the multi-pair levels (1024 threads, small tiles)
constexpr int kNq = 8;           // per-XCD sub-queues of the work-queue order

enum { ORDER_TABLE = 0, ORDER_QUEUE = 1 };

struct StageChoice {
    int K = 0;                   // iterations per tile launch (>= iters: the whole warp in one launch)
    int ew = 64;                 // extended tile width target
    int order = ORDER_TABLE;
    int nt = 1024;               // pDR / ALG1 stages: tile work-group code (see pdr_tb_capacity)
    int tnt = kBatchNt;          // ADMM stages: tile work-group code (kBatchNt or a wave-row code, table order)
};

// One multi-item launch of an elementwise body: items and block offsets at byte offsets of a table.
struct BLaunch {
    size_t items = 0, off = 0;
    int n = 0, total = 0;
};

// Host-side builder of a device table: typed arrays at 256-byte aligned offsets.
struct TableBuilder {
    std::vector<char> h;
    template <typename T> size_t put(const std::vector<T>& v) {
        const size_t o = (h.size() + 255) & ~(size_t)255;
        h.resize(o + std::max<size_t>(1, v.size() * sizeof(T)), 0);
        if (!v.empty()) std::memcpy(h.data() + o, v.data(), v.size() * sizeof(T));
        return o;
    }
    // items plus their block-offset prefix (blocks[k] work-groups for item k)
    template <typename T> BLaunch launch(const std::vector<T>& items, const std::vector<int>& blocks) {
        BLaunch L;
        std::vector<int> off(items.size() + 1, 0);
        for (size_t k = 0; k < items.size(); ++k) off[k + 1] = off[k] + blocks[k];
        L.items = put(items);
        L.off = put(off);
        L.n = (int)items.size();
        L.total = off.back();
        return L;
    }
};

// Grow-only device buffer (growing synchronises the device: the old contents may be in use).
struct DevBuf {
    char* d = nullptr;
    size_t bytes = 0;
    flow_status ensure(size_t need, const char* what);
    void release();
};

// Grow-only pinned host buffer.
struct PinnedBuf {
    char* h = nullptr;
    size_t bytes = 0;
    flow_status ensure(size_t need);
    void release();
};

// First-fit allocator over offsets [0, cap) (the serving arena; callers round sizes up to 256 bytes):
// the free ranges sorted by offset, adjacent free ranges merged on release.
struct RangeAlloc {
    size_t cap = 0;
    std::map<size_t, size_t> free_;   // offset -> size
    void reset(size_t c) {
        cap = c;
        free_.clear();
        if (c) free_[0] = c;
    }
    bool alloc(size_t n, size_t& off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            off = it->first;
            const size_t rest = it->second - n;
            free_.erase(it);
            if (rest) free_[off + n] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

inline int launches_per_warp(int iters, int K) { return iters <= 0 ? 0 : (iters + K - 1) / K; }

// Level shapes (H, W) that one tile launch covers.
using Shapes = std::vector<std::pair<int, int>>;
// Every shape takes tiles of ADMM tile code nt for exactly K iterations with width target ew (or
// fits one tile).
bool shapes_fit(const Shapes& s, bool hw, int K, int ew, int nt = kBatchNt);
bool shapes_all_resident(const Shapes& s, bool hw, int nt = kBatchNt);
// Built-in choice: the whole warp in one launch where every level fits one general tile; else
// wave-row tiles, of 48 rows and 9 iterations per launch when the levels hold a million pixels or
// more (many rounds of work-groups), of 32 rows and 8 iterations otherwise (more, shorter tiles).
StageChoice default_stage_choice(const Shapes& s, bool hw, int iters);
// Lower K (and fall back to width 64) until every shape fits; a wave-row code runs in table order,
// and falls back to kBatchNt where a shape takes none of its tiles.
StageChoice fit_stage_choice(StageChoice c, const Shapes& s, bool hw);
// Tiles of one level for a choice, naming descriptor `desc`.
void level_tiles(int H, int W, bool hw, const StageChoice& ch, int desc, std::vector<TbTile>& out);
// The K-iteration launches of one warp over `ntiles` tiles (table at `tiles`, descriptors at
// `descs`, launch direction 0, 1, 0, ... starting from `dir0`); queue order uses kNq counters per
// launch from `counters` (zeroed by the caller).  With `ntiles_dev` the kernels read the tile count
// there instead (launches that a graph replays over changing tables).  Returns the direction after
// the launches.
int enqueue_tile_warp(const TbTile* tiles, int ntiles, int grid, const TbLevel* descs, const StageChoice& ch,
                      const flow_params& p, int at_slot, int dir0, unsigned* counters, hipStream_t s,
                      const int* ntiles_dev = nullptr);
int tile_grid(const StageChoice& ch, int ntiles);
// pDR / ALG1: every level of an H x W pair with `levels` levels takes 1024-thread tiles at one
// iteration per launch (with many sweeps the pDR halo can outgrow a tile).
bool pd_pair_tileable(int H, int W, int levels, const flow_params& p);
// pDR / ALG1 choice over levels of several pairs sharing K-iteration launches: 1024-thread tiles,
// the whole warp per launch where every level fits one tile, else the plain path's built-in K
// lowered until every level takes tiles (0 if none does).
int pd_shared_k(const Shapes& s, const flow_params& p);
// Checks of one caller pair (shape, pitches, device extents); `who` prefixes messages.
flow_status validate_pair(const flow_pair& q, const flow_params& p, const std::string& who);

}  // namespace flowmi
