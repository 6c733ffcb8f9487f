// RASTER CPU oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, single-threaded implementation of contraction clustering
// (Ulm et al., "Contraction Clustering (RASTER)", Algorithm 1 with Section 3.2
// for the projection and Section 3.6 for chunked input).  It exists to check
// the GPU path, and only the test suite, the package smoke check and the
// benchmark's CPU-baseline leg may load it.  The product library never links
// or calls it, and the two share no source: this file has its own projection,
// its own tile representation (a pair of signed 64-bit integers rather than a
// packed 64-bit key), its own std::unordered_map accumulator and a stack-based
// depth-first agglomeration in the order Algorithm 1 gives.
//
// Readings taken where the paper is silent or loose (each also listed in the
// design notes):
//   * project(x, y) = (trunc(fl(x*s)), trunc(fl(y*s))): one IEEE-754 binary64
//     product, rounded to nearest, truncated toward zero (Section 3.2 speaks of
//     truncating, and of scaling up and converting to integers).  FP32 input is
//     widened to binary64 exactly before the product.
//   * A point whose product is not finite or whose magnitude is at least
//     2^31 - 1 is a range error (tile coordinates must fit |k| <= 2^31 - 2);
//     the whole chunk is then rejected and the stream fails.
//   * Three-dimensional points (Section 3.6 generalises the method to d
//     dimensions): the same projection per coordinate, |k| <= 2^20 - 2, and
//     the neighbourhood taken over all three coordinates (26 tiles at
//     Chebyshev 1, 6 at Manhattan 1: 3^d - 1 and 2d).
//   * Significant means count >= tau (Algorithm 1 removes tiles whose count is
//     below tau).  tau = 0 and mu = 0 are invalid arguments.
//   * neighbors(u, delta) holds the tiles at Chebyshev distance 1 to delta
//     (metric 0) or Manhattan distance 1 to delta (metric 1) from u
//     (Section 3.2 names both metrics and a distance delta; the paper's own
//     code uses Chebyshev 1, the eight adjacent tiles, which is the default
//     here).  Only significant tiles are taken into a cluster.
//   * Optional 2x2 post-step (Section 3.6, Figure 4, for points spread over the
//     tiles around a grid corner): a tile with fewer than tau points is also
//     significant when the four tiles of some 2x2 square containing it hold at
//     least tau points together.  Only tiles holding points are retained; the
//     squares are summed over the counts before any tile is removed.
//   * A cluster is kept when it holds at least mu tiles.
//   * Each kept tile is reported with its count and the lexicographically
//     smallest (kx, ky) of its cluster as the cluster's label; output is sorted
//     by (kx, ky).
//
// Build: g++ -O2 -ffp-contract=off -fPIC -shared (no fast-math).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <unordered_map>
#include <unordered_set>
#include <utility>
#include <vector>

namespace {

constexpr int kOK = 0;
constexpr int kInval = -1;
constexpr int kRange = -2;
constexpr int kState = -5;

// A tile of the 2-D grid (z = 0) or of the 3-D grid (Section 3.6 generalises
// the method to d dimensions).  Order is lexicographic in (x, y, z).
struct Tile {
    int64_t x, y, z = 0;
    bool operator==(const Tile& o) const { return x == o.x && y == o.y && z == o.z; }
    bool operator<(const Tile& o) const {
        return x < o.x || (x == o.x && (y < o.y || (y == o.y && z < o.z)));
    }
};

struct TileHash {
    size_t operator()(const Tile& t) const {
        // std::hash of each coordinate, combined; any hash gives the same result.
        size_t a = std::hash<int64_t>()(t.x);
        size_t b = std::hash<int64_t>()(t.y);
        size_t c = std::hash<int64_t>()(t.z);
        a ^= b + 0x9e3779b97f4a7c15ULL + (a << 6) + (a >> 2);
        return a ^ (c + 0x9e3779b97f4a7c15ULL + (a << 6) + (a >> 2));
    }
};

// Largest magnitude of a scaled coordinate, exclusive: tile coordinates must
// fit |k| <= 2^31 - 2 in 2-D and |k| <= 2^20 - 2 in 3-D (three coordinates
// share one 64-bit key on the GPU).
constexpr double kBound2d = 2147483647.0;
constexpr double kBound3d = 1048575.0;

// Section 3.2: scale the coordinate and truncate it to an integer.
int project_coord(double v, double scale, double bound, int64_t* k) {
    double p = v * scale;
    if (!(std::fabs(p) < bound)) return kRange;  // also rejects NaN and Inf
    *k = (int64_t)std::trunc(p);
    return kOK;
}

struct OracleStream {
    double scale;
    uint64_t tau, mu;
    int32_t metric = 0;  // 0: Chebyshev, 1: Manhattan
    int64_t delta = 1;
    bool window = false;  // the 2x2 post-step
    int32_t dims = 2;     // coordinates per point and per tile: 2 or 3
    double bound = kBound2d;
    bool failed = false;
    bool finished = false;
    uint64_t n_points = 0;
    // acc: tile -> number of points projected onto it (Algorithm 1, contraction).
    std::unordered_map<Tile, uint64_t, TileHash> acc;
    // results filled by finish()
    uint64_t distinct = 0, significant = 0, components = 0, clusters = 0;
    std::vector<Tile> out_tile;
    std::vector<uint64_t> out_count;
    std::vector<Tile> out_label;
};

double point_coord(const void* pts, int dtype, int dims, int64_t i, int c) {
    if (dtype == 1) return (double)((const float*)pts)[dims * i + c];
    return ((const double*)pts)[dims * i + c];
}

}  // namespace

extern "C" {

// s = 10^p for an integer precision p in [0, 15]; every intermediate is an
// integer below 2^53, so the product is exact.
double oracle_scale_for_precision(int32_t p) {
    double s = 1.0;
    for (int i = 0; i < p; ++i) s *= 10.0;
    return s;
}

// Projection alone, for pinning the tile keys: writes kx[i], ky[i].
// dtype: 1 = float32 pairs, 2 = float64 pairs (row-major (n, 2)).
int oracle_project(const void* pts, int64_t n, int32_t dtype, double scale,
                   int64_t* kx, int64_t* ky) {
    if (n < 0 || (dtype != 1 && dtype != 2) || (n > 0 && (!pts || !kx || !ky))) return kInval;
    for (int64_t i = 0; i < n; ++i) {
        if (project_coord(point_coord(pts, dtype, 2, i, 0), scale, kBound2d, &kx[i]) != kOK) return kRange;
        if (project_coord(point_coord(pts, dtype, 2, i, 1), scale, kBound2d, &ky[i]) != kOK) return kRange;
    }
    return kOK;
}

// The same for three-dimensional points (row-major (n, 3)), each coordinate
// projected alone; tiles must satisfy |k| <= 2^20 - 2.
int oracle_project3(const void* pts, int64_t n, int32_t dtype, double scale,
                    int64_t* kx, int64_t* ky, int64_t* kz) {
    if (n < 0 || (dtype != 1 && dtype != 2) || (n > 0 && (!pts || !kx || !ky || !kz))) return kInval;
    int64_t* out[3] = {kx, ky, kz};
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c)
            if (project_coord(point_coord(pts, dtype, 3, i, c), scale, kBound3d, &out[c][i]) != kOK) return kRange;
    return kOK;
}

// metric: 0 = Chebyshev, 1 = Manhattan; 1 <= delta <= 64; window: 0 or 1
// (the 2x2 post-step, 2-D only); dims: 2 or 3.
void* oracle_begin_ex(double scale, uint64_t tau, uint64_t mu, int32_t metric, int64_t delta, int32_t window,
                      int32_t dims) {
    if (!(scale > 0.0) || !std::isfinite(scale) || tau == 0 || mu == 0) return nullptr;
    if ((metric != 0 && metric != 1) || delta < 1 || delta > 64 || (window != 0 && window != 1)) return nullptr;
    if ((dims != 2 && dims != 3) || (dims == 3 && window == 1)) return nullptr;
    OracleStream* s = new OracleStream();
    s->scale = scale;
    s->tau = tau;
    s->mu = mu;
    s->metric = metric;
    s->delta = delta;
    s->window = window == 1;
    s->dims = dims;
    s->bound = dims == 3 ? kBound3d : kBound2d;
    return s;
}

void* oracle_begin(double scale, uint64_t tau, uint64_t mu) { return oracle_begin_ex(scale, tau, mu, 0, 1, 0, 2); }

// Contraction over one chunk of points (Algorithm 1, first loop).  Chunks may
// come in any number and order (Section 3.6).  The chunk is checked first, so a
// range error leaves the accumulator untouched and marks the stream failed.
int oracle_feed(void* h, const void* pts, int64_t n, int32_t dtype) {
    OracleStream* s = (OracleStream*)h;
    if (!s) return kInval;
    if (s->failed || s->finished) return kState;
    if (n < 0 || (dtype != 1 && dtype != 2) || (n > 0 && !pts)) return kInval;
    std::vector<Tile> keys((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        Tile t;
        if (project_coord(point_coord(pts, dtype, s->dims, i, 0), s->scale, s->bound, &t.x) != kOK ||
            project_coord(point_coord(pts, dtype, s->dims, i, 1), s->scale, s->bound, &t.y) != kOK ||
            (s->dims == 3 &&
             project_coord(point_coord(pts, dtype, s->dims, i, 2), s->scale, s->bound, &t.z) != kOK)) {
            s->failed = true;
            return kRange;
        }
        keys[(size_t)i] = t;
    }
    for (const Tile& t : keys) {
        auto it = s->acc.find(t);
        if (it == s->acc.end()) s->acc.emplace(t, 1);
        else it->second += 1;
    }
    s->n_points += (uint64_t)n;
    return kOK;
}

// Number of distinct tiles seen so far (before the significance filter).
int64_t oracle_num_tiles(void* h) {
    OracleStream* s = (OracleStream*)h;
    return s ? (int64_t)s->acc.size() : -1;
}

// Every (kx, ky[, kz], count) of the accumulator, sorted by tile; call before
// finish().  Arrays must hold oracle_num_tiles() entries; kz may be NULL.
int oracle_tile_counts(void* h, int64_t* kx, int64_t* ky, int64_t* kz, uint64_t* count) {
    OracleStream* s = (OracleStream*)h;
    if (!s) return kInval;
    if (s->finished) return kState;
    std::vector<std::pair<Tile, uint64_t>> all(s->acc.begin(), s->acc.end());
    std::sort(all.begin(), all.end(),
              [](const std::pair<Tile, uint64_t>& a, const std::pair<Tile, uint64_t>& b) {
                  return a.first < b.first;
              });
    for (size_t i = 0; i < all.size(); ++i) {
        kx[i] = all[i].first.x;
        ky[i] = all[i].first.y;
        if (kz) kz[i] = all[i].first.z;
        count[i] = all[i].second;
    }
    return kOK;
}

// Significance filter and agglomeration (Algorithm 1, second loop and the
// while-loop), then the mu filter.
int oracle_finish(void* h) {
    OracleStream* s = (OracleStream*)h;
    if (!s) return kInval;
    if (s->failed || s->finished) return kState;
    s->finished = true;
    s->distinct = s->acc.size();

    // With the 2x2 post-step: tiles below tau that lie in a 2x2 square of
    // tiles holding at least tau points together, found on the full counts.
    std::unordered_set<Tile, TileHash> by_square;
    if (s->window) {
        auto count_of = [&](int64_t x, int64_t y) -> uint64_t {
            auto it = s->acc.find(Tile{x, y});
            return it == s->acc.end() ? 0 : it->second;
        };
        for (const auto& kv : s->acc) {
            if (kv.second >= s->tau) continue;
            const Tile& t = kv.first;
            // the four squares holding t have their lower-left corner at
            // (t.x - a, t.y - b) for a, b in {0, 1}
            for (int64_t a = 0; a <= 1 && !by_square.count(t); ++a)
                for (int64_t b = 0; b <= 1; ++b) {
                    const int64_t x0 = t.x - a, y0 = t.y - b;
                    const uint64_t sum = count_of(x0, y0) + count_of(x0 + 1, y0) + count_of(x0, y0 + 1) +
                                         count_of(x0 + 1, y0 + 1);
                    if (sum >= s->tau) {
                        by_square.insert(t);
                        break;
                    }
                }
        }
    }

    // Remove every tile whose count is below tau (unless a square keeps it).
    for (auto it = s->acc.begin(); it != s->acc.end();) {
        if (it->second < s->tau && !by_square.count(it->first)) it = s->acc.erase(it);
        else ++it;
    }
    s->significant = s->acc.size();

    // sigma := keys of acc (the significant tiles).
    std::unordered_set<Tile, TileHash> sigma;
    sigma.reserve(s->acc.size());
    for (const auto& kv : s->acc) sigma.insert(kv.first);

    std::vector<std::vector<Tile>> kept;
    while (!sigma.empty()) {
        Tile t = *sigma.begin();
        sigma.erase(sigma.begin());
        std::vector<Tile> cluster;
        std::vector<Tile> visit{t};
        while (!visit.empty()) {
            Tile u = visit.back();
            visit.pop_back();
            cluster.push_back(u);
            // ns = neighbours of u that are still in sigma; drop them from
            // sigma and queue them for the visit.
            const int64_t d = s->delta;
            const int64_t dz_max = s->dims == 3 ? d : 0;
            for (int64_t dx = -d; dx <= d; ++dx) {
                for (int64_t dy = -d; dy <= d; ++dy) {
                    for (int64_t dz = -dz_max; dz <= dz_max; ++dz) {
                        if (dx == 0 && dy == 0 && dz == 0) continue;
                        if (s->metric == 1 && std::llabs(dx) + std::llabs(dy) + std::llabs(dz) > d) continue;
                        Tile v{u.x + dx, u.y + dy, u.z + dz};
                        auto it = sigma.find(v);
                        if (it != sigma.end()) {
                            sigma.erase(it);
                            visit.push_back(v);
                        }
                    }
                }
            }
        }
        s->components += 1;
        if (cluster.size() >= s->mu) kept.push_back(std::move(cluster));
    }
    s->clusters = kept.size();

    std::vector<std::pair<Tile, Tile>> rows;  // (tile, label)
    for (const auto& c : kept) {
        Tile lab = c[0];
        for (const Tile& t : c)
            if (t < lab) lab = t;
        for (const Tile& t : c) rows.emplace_back(t, lab);
    }
    std::sort(rows.begin(), rows.end(),
              [](const std::pair<Tile, Tile>& a, const std::pair<Tile, Tile>& b) {
                  return a.first < b.first;
              });
    s->out_tile.resize(rows.size());
    s->out_label.resize(rows.size());
    s->out_count.resize(rows.size());
    for (size_t i = 0; i < rows.size(); ++i) {
        s->out_tile[i] = rows[i].first;
        s->out_label[i] = rows[i].second;
        s->out_count[i] = s->acc.at(rows[i].first);
    }
    return kOK;
}

// stats[0..6] = n points, distinct tiles, significant tiles, components of the
// significant tiles, kept clusters, output tiles, failed flag.
int oracle_stats(void* h, int64_t* stats) {
    OracleStream* s = (OracleStream*)h;
    if (!s) return kInval;
    stats[0] = (int64_t)s->n_points;
    stats[1] = (int64_t)(s->finished ? s->distinct : s->acc.size());
    stats[2] = (int64_t)s->significant;
    stats[3] = (int64_t)s->components;
    stats[4] = (int64_t)s->clusters;
    stats[5] = (int64_t)s->out_tile.size();
    stats[6] = s->failed ? 1 : 0;
    return kOK;
}

// Output rows after finish(): tile, count and label tile, sorted by tile;
// kz and label_z (3-D) may be NULL.
int oracle_result(void* h, int64_t* kx, int64_t* ky, int64_t* kz, uint64_t* count,
                  int64_t* label_x, int64_t* label_y, int64_t* label_z) {
    OracleStream* s = (OracleStream*)h;
    if (!s) return kInval;
    if (!s->finished) return kState;
    for (size_t i = 0; i < s->out_tile.size(); ++i) {
        kx[i] = s->out_tile[i].x;
        ky[i] = s->out_tile[i].y;
        count[i] = s->out_count[i];
        label_x[i] = s->out_label[i].x;
        label_y[i] = s->out_label[i].y;
        if (kz) kz[i] = s->out_tile[i].z;
        if (label_z) label_z[i] = s->out_label[i].z;
    }
    return kOK;
}

// Point counts of chosen tiles only: count[q] = number of points whose tile
// (Section 3.2) is (qx[q], qy[q]).  Lets a test check single tiles of an input
// far too large for the full accumulator.  Accumulates into `count`, so it can
// be called once per chunk.
int oracle_count_tiles(const void* pts, int64_t n, int32_t dtype, double scale, const int64_t* qx,
                       const int64_t* qy, int64_t nq, uint64_t* count) {
    if (n < 0 || nq < 0 || (dtype != 1 && dtype != 2)) return kInval;
    std::unordered_map<Tile, int64_t, TileHash> where;
    where.reserve((size_t)nq * 2);
    for (int64_t q = 0; q < nq; ++q) where.emplace(Tile{qx[q], qy[q]}, q);
    for (int64_t i = 0; i < n; ++i) {
        Tile t;
        if (project_coord(point_coord(pts, dtype, 2, i, 0), scale, kBound2d, &t.x) != kOK ||
            project_coord(point_coord(pts, dtype, 2, i, 1), scale, kBound2d, &t.y) != kOK)
            return kRange;
        auto it = where.find(t);
        if (it != where.end()) count[it->second] += 1;
    }
    return kOK;
}

void oracle_free(void* h) { delete (OracleStream*)h; }

}  // extern "C"
