// P-RASTER on the host cores: the paper's parallel RASTER (Section 3.5,
// Algorithms 2 and 3), as a multi-core CPU baseline beside the GPU library.
//
// Steps, in the paper's order:
//   1. The input is cut into unsorted batches, one per thread; each thread
//      projects its points (Section 3.2: binary64 product, truncation toward
//      zero) and counts them per tile in a map of its own.
//   2. The per-thread maps are joined.  Here the join is parallel: each thread
//      splits its map by vertical slice (kx range), and the owner of a slice
//      merges the pieces of that slice from every thread.  The paper joins the
//      maps sequentially and names that join as its projection bottleneck.
//   3. Tiles with fewer than tau points are dropped (Algorithm 1).
//   4. Each vertical slice is clustered on its own thread (Algorithm 2):
//      connected components over the 8-neighbourhood within the slice.  A
//      component with a tile in a column next to a slice border is a join
//      candidate; the others are kept when they hold at least mu tiles.
//   5. Join candidates are merged across borders (Algorithm 3) with a
//      union-find over the candidates, visiting the borders right to left; a
//      merged cluster is kept when it holds at least mu tiles.  This gives the
//      same clusters as the paper's iterative join, since the partition of the
//      significant tiles into connected components is unique.
// Output rows (kx, ky, count, label_x, label_y), sorted by tile, where the
// label is the lexicographically smallest tile of the cluster.
//
// Slices are evenly spaced between the smallest and largest kx seen, one per
// thread (Section 3.5 suggests taking the range from the data rather than
// from fixed GPS bounds).
//
// Build: g++ -O3 -std=c++17 -pthread -fPIC -shared.  No dependency on the GPU
// library or the CPU oracle.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <new>
#include <thread>
#include <vector>

namespace {

constexpr int kOk = 0, kInval = -1, kRange = -2, kNoMem = -3;

// A tile as one word: each coordinate with its sign bit flipped, x in the
// high half.  Unsigned order of the words is the (kx, ky) order, and with
// |k| <= 2^31 - 2 a word is never all ones.
inline uint64_t pack(int32_t x, int32_t y) {
    return ((uint64_t)((uint32_t)x ^ 0x80000000u) << 32) | ((uint32_t)y ^ 0x80000000u);
}
inline int32_t unpack_x(uint64_t k) { return (int32_t)((uint32_t)(k >> 32) ^ 0x80000000u); }
inline int32_t unpack_y(uint64_t k) { return (int32_t)((uint32_t)k ^ 0x80000000u); }

inline uint64_t mix64(uint64_t z) {  // the SplitMix64 finaliser (Steele et al.)
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Open-addressing map from a packed tile to a 32-bit value; the all-ones
// word marks an empty slot.
struct TileMap {
    static constexpr uint64_t kEmpty = ~0ull;
    std::vector<uint64_t> key;
    std::vector<uint32_t> val;
    uint64_t mask = 0, used = 0;

    void init(uint64_t want) {
        uint64_t c = 16;
        while (c < 2 * want) c <<= 1;
        key.assign(c, kEmpty);
        val.assign(c, 0);
        mask = c - 1;
        used = 0;
    }
    void grow() {
        std::vector<uint64_t> ok;
        std::vector<uint32_t> ov;
        ok.swap(key);
        ov.swap(val);
        init(ok.size());
        for (size_t i = 0; i < ok.size(); ++i)
            if (ok[i] != kEmpty) add(ok[i], ov[i]);
    }
    void add(uint64_t k, uint32_t v) {
        if (2 * (used + 1) > mask + 1) grow();
        uint64_t p = mix64(k) & mask;
        while (key[p] != kEmpty && key[p] != k) p = (p + 1) & mask;
        if (key[p] == kEmpty) {
            key[p] = k;
            val[p] = v;
            ++used;
        } else {
            val[p] += v;
        }
    }
    // value of k, or UINT32_MAX when absent
    uint32_t find(uint64_t k) const {
        uint64_t p = mix64(k) & mask;
        while (key[p] != kEmpty) {
            if (key[p] == k) return val[p];
            p = (p + 1) & mask;
        }
        return UINT32_MAX;
    }
};

struct Piece {
    const void* pts;
    int64_t begin, end;
    int dtype;
};

inline double coord(const void* pts, int dtype, int64_t i, int c) {
    return dtype == 1 ? (double)((const float*)pts)[2 * i + c] : ((const double*)pts)[2 * i + c];
}

// tile of one coordinate; false when the product is not finite or its
// truncation falls outside +-(2^31 - 2)
inline bool tile_of(double v, double s, int32_t* k) {
    const double p = v * s;
    if (!(std::fabs(p) < 2147483647.0)) return false;
    *k = (int32_t)std::trunc(p);
    return true;
}

struct Timer {
    std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
    double lap() {
        const auto n = std::chrono::steady_clock::now();
        const double d = std::chrono::duration<double>(n - t).count();
        t = n;
        return d;
    }
};

// Runs f(0) ... f(threads - 1) on their own threads; an allocation failure in
// any of them is rethrown here after all have ended.
template <typename F>
void parallel(int threads, F&& f) {
    std::vector<std::thread> pool;
    std::atomic<bool> nomem{false};
    pool.reserve(threads);
    for (int t = 0; t < threads; ++t)
        pool.emplace_back([&f, &nomem, t] {
            try {
                f(t);
            } catch (const std::bad_alloc&) {
                nomem = true;
            }
        });
    for (auto& th : pool) th.join();
    if (nomem) throw std::bad_alloc();
}

struct UnionFind {
    std::vector<uint32_t> parent;
    explicit UnionFind(size_t n) : parent(n) {
        for (size_t i = 0; i < n; ++i) parent[i] = (uint32_t)i;
    }
    uint32_t root(uint32_t a) {
        while (parent[a] != a) {
            parent[a] = parent[parent[a]];
            a = parent[a];
        }
        return a;
    }
    void join(uint32_t a, uint32_t b) {
        a = root(a);
        b = root(b);
        if (a != b) parent[std::max(a, b)] = std::min(a, b);
    }
};

// One vertical slice after counting: its significant tiles and components.
struct Slice {
    int32_t lo = 0, hi = 0;       // kx range [lo, hi)
    std::vector<uint64_t> tile;   // significant tiles
    std::vector<uint32_t> count;
    TileMap index;                // tile -> position in `tile`
    std::vector<uint32_t> comp;   // per tile: local component
    std::vector<uint32_t> comp_size;
    std::vector<uint64_t> comp_min;  // smallest packed tile
    std::vector<uint8_t> comp_border;
    uint32_t first_global = 0;    // global id of component 0 among all slices
};


}  // namespace

extern "C" {

struct praster_result {
    std::vector<int64_t> kx, ky, lx, ly;
    std::vector<uint64_t> count;
    int64_t clusters = 0;
    int64_t distinct = 0;
    int64_t significant = 0;
    int64_t join_candidates = 0;  // components next to a slice border
    double seconds[5] = {0, 0, 0, 0, 0};  // project, join + threshold, slice clustering, border join, output
};

// chunks: nchunks pointers to (counts[c], 2) row-major arrays of dtype
// (1 = float32, 2 = float64).  threads >= 1.  Returns 0, -1 (bad argument),
// -2 (a coordinate out of range) or -3 (out of memory); *out is set on
// success only.
int praster_cluster(const void* const* chunks, const int64_t* counts, int nchunks, int dtype, double scale,
                    uint64_t tau, uint64_t mu, int threads, praster_result** out) {
    if (!out || nchunks < 0 || (nchunks > 0 && (!chunks || !counts)) || (dtype != 1 && dtype != 2) ||
        !(scale > 0.0) || !std::isfinite(scale) || tau == 0 || mu == 0 || threads < 1)
        return kInval;
    *out = nullptr;
    try {
        Timer tm;
        std::unique_ptr<praster_result> r(new praster_result());
        // 1. batches: each chunk cut into `threads` ranges, dealt round-robin
        std::vector<Piece> pieces;
        for (int c = 0; c < nchunks; ++c) {
            if (counts[c] < 0 || (counts[c] > 0 && !chunks[c])) return kInval;
            const int64_t step = (counts[c] + threads - 1) / threads;
            for (int64_t b = 0; b < counts[c]; b += std::max<int64_t>(step, 1))
                pieces.push_back(Piece{chunks[c], b, std::min(counts[c], b + step), dtype});
        }
        std::vector<TileMap> local(threads);
        std::vector<int32_t> tmin(threads, INT32_MAX), tmax(threads, INT32_MIN);
        std::atomic<bool> bad{false};
        parallel(threads, [&](int t) {
            TileMap& m = local[t];
            m.init(1 << 16);
            int32_t mn = INT32_MAX, mx = INT32_MIN;
            for (size_t q = t; q < pieces.size(); q += threads) {
                const Piece& pc = pieces[q];
                for (int64_t i = pc.begin; i < pc.end; ++i) {
                    int32_t kx, ky;
                    if (!tile_of(coord(pc.pts, pc.dtype, i, 0), scale, &kx) ||
                        !tile_of(coord(pc.pts, pc.dtype, i, 1), scale, &ky)) {
                        bad = true;
                        return;
                    }
                    mn = std::min(mn, kx);
                    mx = std::max(mx, kx);
                    m.add(pack(kx, ky), 1);
                }
            }
            tmin[t] = mn;
            tmax[t] = mx;
        });
        if (bad) return kRange;
        r->seconds[0] = tm.lap();
        const int32_t gmin = *std::min_element(tmin.begin(), tmin.end());
        const int32_t gmax = *std::max_element(tmax.begin(), tmax.end());
        std::vector<Slice> slices(threads);
        if (gmin <= gmax) {
            // 2. slices of equal kx width; each thread splits its map by slice,
            // then each slice owner merges its pieces
            const int64_t span = (int64_t)gmax - gmin + 1;
            const int64_t width = (span + threads - 1) / threads;
            for (int s = 0; s < threads; ++s) {
                slices[s].lo = (int32_t)std::min<int64_t>((int64_t)gmin + s * width, (int64_t)gmax + 1);
                slices[s].hi = (int32_t)std::min<int64_t>((int64_t)gmin + (s + 1) * width, (int64_t)gmax + 1);
            }
            std::vector<std::vector<std::vector<std::pair<uint64_t, uint32_t>>>> parts(
                threads, std::vector<std::vector<std::pair<uint64_t, uint32_t>>>(threads));
            parallel(threads, [&](int t) {
                const TileMap& m = local[t];
                for (size_t i = 0; i <= m.mask; ++i)
                    if (m.key[i] != TileMap::kEmpty)
                        parts[t][((int64_t)unpack_x(m.key[i]) - gmin) / width].emplace_back(m.key[i], m.val[i]);
            });
            local.clear();
            local.shrink_to_fit();
            std::vector<int64_t> distinct(threads, 0);
            parallel(threads, [&](int s) {
                size_t total = 0;
                for (int t = 0; t < threads; ++t) total += parts[t][s].size();
                TileMap merged;
                merged.init(std::max<size_t>(total / 2, 16));
                for (int t = 0; t < threads; ++t) {
                    for (const auto& kv : parts[t][s]) merged.add(kv.first, kv.second);
                    std::vector<std::pair<uint64_t, uint32_t>>().swap(parts[t][s]);
                }
                distinct[s] = (int64_t)merged.used;
                // 3. significance
                Slice& sl = slices[s];
                for (size_t i = 0; i <= merged.mask; ++i)
                    if (merged.key[i] != TileMap::kEmpty && merged.val[i] >= tau) {
                        sl.tile.push_back(merged.key[i]);
                        sl.count.push_back(merged.val[i]);
                    }
            });
            for (int s = 0; s < threads; ++s) {
                r->distinct += distinct[s];
                r->significant += (int64_t)slices[s].tile.size();
            }
            r->seconds[1] = tm.lap();
            // 4. components inside each slice (breadth-first search)
            parallel(threads, [&](int s) {
                Slice& sl = slices[s];
                const size_t n = sl.tile.size();
                sl.index.init(std::max<size_t>(n, 16));
                for (size_t i = 0; i < n; ++i) sl.index.add(sl.tile[i], (uint32_t)i);
                sl.comp.assign(n, UINT32_MAX);
                std::vector<uint32_t> queue;
                for (size_t i = 0; i < n; ++i) {
                    if (sl.comp[i] != UINT32_MAX) continue;
                    const uint32_t c = (uint32_t)sl.comp_size.size();
                    uint32_t size = 0;
                    uint64_t best = UINT64_MAX;
                    bool border = false;
                    queue.clear();
                    queue.push_back((uint32_t)i);
                    sl.comp[i] = c;
                    for (size_t h = 0; h < queue.size(); ++h) {
                        const uint32_t u = queue[h];
                        ++size;
                        best = std::min(best, sl.tile[u]);
                        const int32_t x = unpack_x(sl.tile[u]), y = unpack_y(sl.tile[u]);
                        if ((s > 0 && x == sl.lo) || (s + 1 < threads && x == sl.hi - 1)) border = true;
                        for (int dx = -1; dx <= 1; ++dx)
                            for (int dy = -1; dy <= 1; ++dy) {
                                if (dx == 0 && dy == 0) continue;
                                const int64_t nx = (int64_t)x + dx, ny = (int64_t)y + dy;
                                if (nx < sl.lo || nx >= sl.hi || ny < INT32_MIN || ny > INT32_MAX) continue;
                                const uint32_t v = sl.index.find(pack((int32_t)nx, (int32_t)ny));
                                if (v != UINT32_MAX && sl.comp[v] == UINT32_MAX) {
                                    sl.comp[v] = c;
                                    queue.push_back(v);
                                }
                            }
                    }
                    sl.comp_size.push_back(size);
                    sl.comp_min.push_back(best);
                    sl.comp_border.push_back(border ? 1 : 0);
                }
            });
            r->seconds[2] = tm.lap();
            // 5. join across borders, right to left, over all components
            // (components away from borders are their own roots)
            uint32_t total = 0;
            for (int s = 0; s < threads; ++s) {
                for (uint8_t b : slices[s].comp_border) r->join_candidates += b;
                slices[s].first_global = total;
                total += (uint32_t)slices[s].comp_size.size();
            }
            UnionFind uf(total);
            for (int s = threads - 1; s >= 1; --s) {
                Slice& right = slices[s];
                Slice& left = slices[s - 1];
                if (right.tile.empty() || left.tile.empty() || left.hi != right.lo) continue;
                for (size_t i = 0; i < right.tile.size(); ++i) {
                    const int32_t x = unpack_x(right.tile[i]), y = unpack_y(right.tile[i]);
                    if (x != right.lo) continue;
                    for (int dy = -1; dy <= 1; ++dy) {
                        const int64_t ny = (int64_t)y + dy;
                        if (ny < INT32_MIN || ny > INT32_MAX) continue;
                        const uint32_t v = left.index.find(pack(x - 1, (int32_t)ny));
                        if (v != UINT32_MAX)
                            uf.join(right.first_global + right.comp[i], left.first_global + left.comp[v]);
                    }
                }
            }
            std::vector<uint64_t> size(total, 0), best(total, UINT64_MAX);
            for (int s = 0; s < threads; ++s)
                for (size_t c = 0; c < slices[s].comp_size.size(); ++c) {
                    const uint32_t g = uf.root(slices[s].first_global + (uint32_t)c);
                    size[g] += slices[s].comp_size[c];
                    best[g] = std::min(best[g], slices[s].comp_min[c]);
                }
            for (uint32_t g = 0; g < total; ++g)
                if (uf.root(g) == g && size[g] >= mu) ++r->clusters;
            r->seconds[3] = tm.lap();
            // output: kept tiles of each slice, sorted per slice in parallel;
            // slices are kx ranges in order, so the concatenation is sorted
            std::vector<std::vector<std::pair<uint64_t, uint32_t>>> rows(threads);
            parallel(threads, [&](int s) {
                Slice& sl = slices[s];
                for (size_t i = 0; i < sl.tile.size(); ++i) {
                    const uint32_t g = uf.root(sl.first_global + sl.comp[i]);
                    if (size[g] >= mu) rows[s].emplace_back(sl.tile[i], (uint32_t)i);
                }
                std::sort(rows[s].begin(), rows[s].end());
            });
            size_t t_out = 0;
            for (int s = 0; s < threads; ++s) t_out += rows[s].size();
            r->kx.resize(t_out);
            r->ky.resize(t_out);
            r->lx.resize(t_out);
            r->ly.resize(t_out);
            r->count.resize(t_out);
            std::vector<size_t> base(threads, 0);
            for (int s = 1; s < threads; ++s) base[s] = base[s - 1] + rows[s - 1].size();
            parallel(threads, [&](int s) {
                const Slice& sl = slices[s];
                size_t o = base[s];
                for (const auto& kv : rows[s]) {
                    const uint32_t i = kv.second;
                    const uint32_t g = uf.root(sl.first_global + sl.comp[i]);
                    r->kx[o] = unpack_x(sl.tile[i]);
                    r->ky[o] = unpack_y(sl.tile[i]);
                    r->count[o] = sl.count[i];
                    r->lx[o] = unpack_x(best[g]);
                    r->ly[o] = unpack_y(best[g]);
                    ++o;
                }
            });
            r->seconds[4] = tm.lap();
        }
        *out = r.release();
        return kOk;
    } catch (const std::bad_alloc&) {
        return kNoMem;
    }
}

int64_t praster_num_tiles(const praster_result* r) { return r ? (int64_t)r->kx.size() : 0; }

// stats: distinct tiles, significant tiles, clusters, join candidates;
// seconds: the five phases
void praster_stats(const praster_result* r, int64_t* stats, double* seconds) {
    if (!r) return;
    if (stats) {
        stats[0] = r->distinct;
        stats[1] = r->significant;
        stats[2] = r->clusters;
        stats[3] = r->join_candidates;
    }
    if (seconds) std::memcpy(seconds, r->seconds, sizeof r->seconds);
}

// copies the rows into caller arrays of praster_num_tiles elements each
void praster_rows(const praster_result* r, int64_t* kx, int64_t* ky, uint64_t* count, int64_t* lx, int64_t* ly) {
    if (!r) return;
    const size_t t = r->kx.size();
    std::memcpy(kx, r->kx.data(), t * sizeof(int64_t));
    std::memcpy(ky, r->ky.data(), t * sizeof(int64_t));
    std::memcpy(count, r->count.data(), t * sizeof(uint64_t));
    std::memcpy(lx, r->lx.data(), t * sizeof(int64_t));
    std::memcpy(ly, r->ly.data(), t * sizeof(int64_t));
}

void praster_free(praster_result* r) { delete r; }

}  // extern "C"
