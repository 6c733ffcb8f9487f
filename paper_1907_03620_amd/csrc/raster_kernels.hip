// gfx950 kernels of the RASTER hot path (Algorithm 1 of the RASTER paper):
//   contraction   -- projection (Section 3.2) fused with per-tile counting in
//                    an open-addressing device table, then a prefix-scan
//                    compaction of the tiles holding at least tau points;
//   agglomeration -- union-find connected components over the eight-neighbour
//                    adjacency of significant tiles (Section 3.2, Chebyshev
//                    distance 1), then the mu filter and the min-key label.
//
// Everything is integer work except one binary64 product per coordinate.  The
// file is compiled with -ffp-contract=off and without fast-math so that the
// product is the correctly rounded IEEE one.
//
// Wavefront size is 64.  Counters that many lanes bump are aggregated per
// wave with a ballot before the single global atomic.

#include <hip/hip_ext.h>

#include "raster_internal.h"

namespace rst {
namespace {

// ---------------------------------------------------------------- helpers ---

// 32-bit integer mixer "lowbias32" (C. Wellons, "Prospecting for hash
// functions", 2018): a bijection whose output bits each depend on every input
// bit.  Only 32-bit multiplies: a 64-bit one costs four of them on the VALU.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Fibonacci-hashing multiplier, floor(2^32 / golden ratio), odd.
constexpr uint32_t kGolden32 = 0x9e3779b9u;

// Hash that picks a key's partition (and coarse bucket): that of its
// super-tile.  Top bits are used.
__device__ __forceinline__ uint32_t place_hash(uint64_t key) {
    const uint32_t sx = (uint32_t)(key >> 32) >> kSuperLog2, sy = (uint32_t)key >> kSuperLog2;
    return mix32(sx * kGolden32 + sy);
}

// The same for three-dimensional keys (three biased 21-bit coordinates, x
// highest): the super-tile is the 4x4x4 cube of tiles holding the key, 64
// tiles as in two dimensions.
__device__ __forceinline__ uint32_t place_hash3(uint64_t key) {
    constexpr uint64_t f = (1ull << 21) - 1;
    const uint32_t sx = (uint32_t)(key >> 42) >> 2, sy = (uint32_t)((key >> 21) & f) >> 2;
    const uint32_t sz = (uint32_t)(key & f) >> 2;
    return mix32((sx * kGolden32 + sy) * kGolden32 + sz);
}

__device__ __forceinline__ uint32_t place_of(uint64_t key, uint32_t d3) {
    return d3 ? place_hash3(key) : place_hash(key);
}

// Hash that picks a key's home slot inside its partition.  Low bits are used.
// Tiles near each other never share a hash: x * kGolden32 + y (mod 2^32) takes
// distinct values on any window of 2^14 x 2^17 tiles (checked exhaustively).
__device__ __forceinline__ uint32_t slot_hash(uint64_t key) {
    return mix32((uint32_t)(key >> 32) * kGolden32 + (uint32_t)key);
}

// Distinct-tile sketch (HyperLogLog, Flajolet, Fusy, Gandouet and Meunier,
// AofA 2007) over a fixed 1/64 of the tiles: those whose slot hash has its
// low 6 bits zero.  Register = the top kHllLog2 hash bits, rank = 1 + the
// leading zeros of hash bits [6, 32 - kHllLog2).  Returns false for a tile
// outside the sample.
__device__ __forceinline__ bool hll_from_hash(uint32_t h, uint32_t& reg, uint32_t& rank) {
    constexpr uint32_t rank_bits = 26 - kHllLog2;
    if (h & 63u) return false;
    const uint32_t rest = (h >> 6) & ((1u << rank_bits) - 1);
    rank = rest ? (uint32_t)__clz(rest) - (32 - rank_bits) + 1 : rank_bits + 1;
    reg = h >> (32 - kHllLog2);
    return true;
}
__device__ __forceinline__ bool hll_sample(uint64_t key, uint32_t& reg, uint32_t& rank) {
    return hll_from_hash(slot_hash(key), reg, rank);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (1ull << lane_id()) - 1ull;
}

// Relaxed read of an LDS word that other lanes may be updating; unlike a
// volatile read it compiles to an LDS load, not a generic one that also waits
// for outstanding global loads.
__device__ __forceinline__ uint64_t lds_load_relaxed(uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Workgroups are dispatched to the 8 XCDs round-robin by index, and each XCD
// has its own L2.  For a pass over n items whose random accesses stay near
// the item (table slices and union-find words of neighbouring tiles), each
// XCD takes one contiguous eighth of [0, n) and its workgroups stride over
// it, so every slice is fetched into one L2 only.  Covers [0, n) exactly once
// for any grid; a grid that is not a multiple of 8 falls back to a plain
// grid stride.
constexpr uint32_t kXcds = 8;
struct XcdSpan {
    uint64_t lo, hi;      // this XCD's items
    uint64_t first, step; // this thread's first item and stride
};
__device__ __forceinline__ XcdSpan xcd_span(uint64_t n) {
    if (gridDim.x % kXcds != 0)
        return {0, n, blockIdx.x * (uint64_t)blockDim.x + threadIdx.x, (uint64_t)gridDim.x * blockDim.x};
    const uint32_t x = blockIdx.x % kXcds, w = blockIdx.x / kXcds;
    const uint64_t lo = n * x / kXcds, hi = n * (x + 1) / kXcds;
    return {lo, hi, lo + (uint64_t)w * blockDim.x + threadIdx.x, (uint64_t)(gridDim.x / kXcds) * blockDim.x};
}

__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Device-scope relaxed accesses for words other workgroups modify during the
// same kernel (union-find parents and sizes).  They bypass the per-XCD L2, so
// every read sees the device-coherent value.
__device__ __forceinline__ uint32_t ld_relaxed(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane) {
    uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// Adds every thread's `v` to *ctr with one atomic per workgroup (a single
// counter word hit once per wave would serialise hundreds of thousands of
// same-address atomics).  Every thread of the workgroup must call it, once,
// at a point all of them reach.
__device__ __forceinline__ void block_count_add64(unsigned long long* ctr, unsigned long long v) {
    __shared__ unsigned long long part64[16];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if (lane_id() == 0) part64[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < (int)((blockDim.x + 63) >> 6); ++i) t += part64[i];
        if (t) atomicAdd(ctr, t);
    }
}

// Sum of v over the workgroup, valid in thread 0.
__device__ __forceinline__ uint32_t block_total32(uint32_t v) {
    __shared__ uint32_t tot32[16];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if (lane_id() == 0) tot32[w] = v;
    __syncthreads();
    uint32_t t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)((blockDim.x + 63) >> 6); ++i) t += tot32[i];
    return t;
}

// The same for a 32-bit word.
__device__ __forceinline__ void block_count_add32(uint32_t* dst, uint32_t v) {
    __shared__ uint32_t part32[16];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if (lane_id() == 0) part32[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int i = 0; i < (int)((blockDim.x + 63) >> 6); ++i) t += part32[i];
        if (t) atomicAdd(dst, t);
    }
}

__device__ __forceinline__ void block_count_add(unsigned long long* ctr, uint32_t v) {
    __shared__ uint32_t part[16];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if (lane_id() == 0) part[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < (int)((blockDim.x + 63) >> 6); ++i) t += part[i];
        if (t) atomicAdd(ctr, t);
    }
}

// Projection of Section 3.2: one binary64 product per coordinate, truncated
// toward zero.  Returns false (range error) unless both tiles satisfy
// |k| <= 2^31 - 2, which also rejects NaN and infinities.  The key is the
// biased pair (kx + 2^31, ky + 2^31) packed high/low.
__device__ __forceinline__ bool tile_key(double x, double y, double s, uint64_t& key) {
    const double px = x * s;
    const double py = y * s;
    if (!(fabs(px) < 2147483647.0) || !(fabs(py) < 2147483647.0)) return false;
    const uint32_t bx = (uint32_t)(int32_t)px + 0x80000000u;
    const uint32_t by = (uint32_t)(int32_t)py + 0x80000000u;
    key = ((uint64_t)bx << 32) | by;
    return true;
}

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <typename T> struct Pair;
template <> struct Pair<double> {
    using V = f64x2;
};
template <> struct Pair<float> {
    using V = f32x2;
};

template <typename T>
__device__ __forceinline__ void load_point(const T* pts, int64_t i, double& x, double& y) {
    using V = typename Pair<T>::V;
    // points are in device (global) memory: saying so lets the compiler use
    // global loads, not generic ones, when the pointer came from memory
    const __attribute__((address_space(1))) V* g = (const __attribute__((address_space(1))) V*)(pts);
    const V v = __builtin_nontemporal_load(g + i);
    x = (double)v.x;  // FP32 widens exactly
    y = (double)v.y;
}

// Three-dimensional rows (Section 3.6 generalises the method to d
// dimensions) are a point type of their own, so that the counting kernels,
// templated on the point type, take them as they are.  A 3-D key packs the
// three biased coordinates k + 2^20 (21 bits each, |k| <= 2^20 - 2) as x:y:z
// from the high bits: unsigned key order is the lexicographic tile order, and
// no valid key reaches kEmptyKey.  The table, binning, scan and union-find
// code treat keys as opaque, so they serve both.
template <typename E> struct Pt3 {
    E c[3];
};
template <typename P> struct PtDims {
    static constexpr int value = 2;
};
template <typename E> struct PtDims<Pt3<E>> {
    static constexpr int value = 3;
};

constexpr uint32_t kBias3 = 1u << 20;
constexpr uint64_t kField3 = (1ull << 21) - 1;

__device__ __forceinline__ bool tile_key3(double x, double y, double z, double s, uint64_t& key) {
    const double px = x * s;
    const double py = y * s;
    const double pz = z * s;
    if (!(fabs(px) < 1048575.0) || !(fabs(py) < 1048575.0) || !(fabs(pz) < 1048575.0)) return false;
    const uint64_t bx = (uint32_t)((int32_t)px + (int32_t)kBias3);
    const uint64_t by = (uint32_t)((int32_t)py + (int32_t)kBias3);
    const uint64_t bz = (uint32_t)((int32_t)pz + (int32_t)kBias3);
    key = (bx << 42) | (by << 21) | bz;
    return true;
}

template <typename P>
__device__ __forceinline__ void load_xyz(const P* pts, int64_t i, double& x, double& y, double& z) {
    load_point(pts, i, x, y);
    z = 0.0;
}

template <typename E>
__device__ __forceinline__ void load_xyz(const Pt3<E>* pts, int64_t i, double& x, double& y, double& z) {
    const __attribute__((address_space(1))) E* g = (const __attribute__((address_space(1))) E*)(pts);
    x = (double)__builtin_nontemporal_load(g + 3 * i);
    y = (double)__builtin_nontemporal_load(g + 3 * i + 1);
    z = (double)__builtin_nontemporal_load(g + 3 * i + 2);
}

template <typename P>
__device__ __forceinline__ bool point_key(double x, double y, double z, double s, uint64_t& key) {
    if constexpr (PtDims<P>::value == 3) return tile_key3(x, y, z, s, key);
    else return tile_key(x, y, s, key);
}

__device__ __forceinline__ uint32_t job_of_tile(const uint32_t* tile_prefix, uint32_t njobs, uint32_t t) {
    uint32_t lo = 0, hi = njobs;  // find the last j with tile_prefix[j] <= t
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (tile_prefix[mid] <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Contiguous range of work tiles of one persistent workgroup, and the job of
// its first tile.  Consecutive tiles mostly belong to one job, so the job is
// found once and then advanced at job boundaries (tile_prefix has njobs + 1
// entries, the last one the tile total); and at any moment the workgroups
// work on many jobs, not all on one job's buckets.
struct TileRange {
    uint32_t lo, hi, job;
};

__device__ __forceinline__ TileRange tile_range(const uint32_t* tile_prefix, uint32_t njobs, uint32_t tiles) {
    const uint32_t per = (tiles + gridDim.x - 1) / gridDim.x;
    TileRange r;
    r.lo = min(blockIdx.x * per, tiles);
    r.hi = min(r.lo + per, tiles);
    r.job = r.lo < r.hi ? job_of_tile(tile_prefix, njobs, r.lo) : 0u;
    return r;
}

__device__ __forceinline__ uint32_t advance_job(const uint32_t* tile_prefix, uint32_t job, uint32_t t) {
    while (tile_prefix[job + 1] <= t) ++job;  // skips jobs without tiles
    return job;
}

__device__ __forceinline__ bool job_point_key(const JobInfo& J, int64_t i, uint64_t& key) {
    double x, y;
    if (J.dtype == 1) load_point(static_cast<const float*>(J.pts), i, x, y);
    else load_point(static_cast<const double*>(J.pts), i, x, y);
    return tile_key(x, y, J.scale, key);
}

enum AddResult : int { ADD_FOUND = 0, ADD_NEW = 1, ADD_FULL = 2 };

// ---- key frame of a two-dimensional table ----------------------------------
//
// A key inside the table's frame (a window of 2^20 x 2^20 tiles) is described
// by h, a bijective mix of its super-tile's 34-bit position in the frame, and
// its 32-bit entry: the low 26 bits of h and the key's 6-bit position inside
// the super-tile.  The top 8 bits of h (the coarse bucket) and the entry give
// the key back.  The mix is a multiplication by an odd constant, whose top
// bits (partition and coarse bucket) depend on every bit of the position,
// then a xor-shift that brings them down into the entry; both are
// invertible modulo 2^34.
constexpr uint64_t kFrameStMask = (1ull << kFrameStBits) - 1;
constexpr uint64_t kFrameMul = 0x2c1b3c6d5ull, kFrameMulInv = 0x1eea1427dull;
static_assert(((kFrameMul * kFrameMulInv) & ((1ull << 34) - 1)) == 1, "inverse modulo 2^34");
constexpr uint32_t kFrameSide = 1u << kFrameLog2;
constexpr uint32_t kFrameStSide = kFrameLog2 - 3;  // bits of one super-tile coordinate

__device__ __forceinline__ uint64_t frame_mix(uint64_t v) {
    v = (v * kFrameMul) & kFrameStMask;
    return v ^ (v >> 17);
}

__device__ __forceinline__ uint64_t frame_unmix(uint64_t h) {
    h ^= h >> 17;  // its own inverse on 34 bits
    return (h * kFrameMulInv) & kFrameStMask;
}

// Home slot of entry e inside its partition (before masking to the partition
// size): 12 bits of h, with the 64 positions inside the super-tile spread
// over the partition by a step of 65.
__device__ __forceinline__ uint32_t frame_home(uint32_t e) { return (e >> 6) ^ ((e & 63u) * 65u); }

// h and entry of a key; false for a key outside the frame.
__device__ __forceinline__ bool frame_code(uint64_t key, uint32_t fx, uint32_t fy, uint64_t& h, uint32_t& e) {
    const uint32_t rx = (uint32_t)(key >> 32) - fx, ry = (uint32_t)key - fy;
    if ((rx | ry) >= kFrameSide) return false;
    h = frame_mix(((uint64_t)(rx >> 3) << kFrameStSide) | (ry >> 3));
    e = ((uint32_t)(h & ((1u << kFrameHLow) - 1)) << 6) | ((rx & 7u) << 3) | (ry & 7u);
    return true;
}

// The key of entry e in coarse bucket cb.
__device__ __forceinline__ uint64_t frame_key(uint32_t cb, uint32_t e, uint32_t fx, uint32_t fy) {
    const uint64_t st = frame_unmix(((uint64_t)cb << kFrameHLow) | (e >> 6));
    const uint32_t rx = ((uint32_t)(st >> kFrameStSide) << 3) | ((e >> 3) & 7u);
    const uint32_t ry = ((uint32_t)(st & ((1u << kFrameStSide) - 1)) << 3) | (e & 7u);
    return ((uint64_t)(fx + rx) << 32) | (uint32_t)(fy + ry);
}

// Home slot of a key: partition from the placement hash of its super-tile
// (or from h inside a frame), slot inside the partition from the key's own
// hash (or the entry's).
__device__ __forceinline__ uint64_t home_slot(uint64_t key, const Geo& g) {
    uint64_t h;
    uint32_t e;
    if (g.framed && frame_code(key, g.fx, g.fy, h, e)) {
        const uint64_t part = g.p_log2 ? (h >> (kFrameStBits - g.p_log2)) : 0;
        return (part << g.cp_log2) | (frame_home(e) & ((1u << g.cp_log2) - 1));
    }
    const uint64_t part = g.p_log2 ? (place_of(key, g.d3) >> (32 - g.p_log2)) : 0;
    return (part << g.cp_log2) | (slot_hash(key) & ((1u << g.cp_log2) - 1));
}

// Next probe position: linear, wrapping inside the partition.
__device__ __forceinline__ uint64_t next_slot(uint64_t s, const Geo& g) {
    const uint64_t m = (1ull << g.cp_log2) - 1;
    return (s & ~m) | ((s + 1) & m);
}

// Adds `inc` to the count of `key`, inserting the key into an empty slot of
// its probe window if it is not there yet.  Keys are only ever written once
// (empty -> key), so a stale read can only show a slot as empty; the
// compare-and-swap then returns the true occupant.
__device__ __forceinline__ int table_add(Slot* tab, const Geo& g, uint64_t key, uint32_t inc) {
    uint64_t pos = home_slot(key, g);
    for (uint32_t p = 0; p < kMaxProbe; ++p) {
        Slot* sl = tab + pos;
        uint64_t cur = ld_relaxed(&sl->key);
        if (cur == kEmptyKey) {
            cur = atomicCAS(reinterpret_cast<unsigned long long*>(&sl->key), (unsigned long long)kEmptyKey,
                            (unsigned long long)key);
            if (cur == kEmptyKey) {
                atomicAdd(&sl->count, inc);
                return ADD_NEW;
            }
        }
        if (cur == key) {
            atomicAdd(&sl->count, inc);
            return ADD_FOUND;
        }
        pos = next_slot(pos, g);
    }
    return ADD_FULL;
}

// Read-only lookup; returns the slot index or ~0 when the key is absent.
__device__ __forceinline__ uint64_t table_find(const Slot* tab, const Geo& g, uint64_t key) {
    uint64_t pos = home_slot(key, g);
    for (uint32_t p = 0; p < kMaxProbe; ++p) {
        const uint64_t cur = tab[pos].key;
        if (cur == key) return pos;
        if (cur == kEmptyKey) return ~0ull;
        pos = next_slot(pos, g);
    }
    return ~0ull;
}

// Appends (key, count) records of the lanes with `pred` to the spill buffer;
// one atomic per wave reserves the positions.  Reached by the whole wave.
__device__ __forceinline__ void spill_push(const SpillBuf& sp, unsigned long long* ctr, bool pred,
                                           uint64_t key, uint32_t count) {
    const uint64_t b = __ballot(pred);
    if (b == 0) return;
    const int leader = __ffsll((long long)b) - 1;
    uint64_t base = 0;
    if (lane_id() == leader) base = atomicAdd(&ctr[C_SPILLED], (unsigned long long)__popcll(b));
    base = readlane64(base, leader);
    if (pred) {
        const uint64_t idx = base + __popcll(b & lanemask_lt());
        if (idx < sp.cap) {
            sp.keys[idx] = key;
            sp.counts[idx] = count;
        } else {
            atomicOr(&ctr[C_ERROR], (unsigned long long)kErrSpillOverflow);
        }
    }
}

// ------------------------------------------------------------ contraction ---

__global__ void k_fill_table(Slot* tab, uint64_t cap) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < cap;
         i += (uint64_t)gridDim.x * blockDim.x) {
        Slot s;
        s.key = kEmptyKey;
        s.count = 0;
        s.aux = kNotSignificant;
        tab[i] = s;
    }
}

__global__ void k_zero_u64(uint64_t* p, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Direct counting: every point goes straight to the device table.  A
// workgroup covers blockDim * ITEMS consecutive points; lane t of the group
// takes points base + t + j * blockDim so each load instruction is coalesced.
template <typename T, int ITEMS>
__global__ void k_count_direct(const T* __restrict__ pts, int64_t n, double scale, Slot* tab,
                               const Geo g, SpillBuf sp, unsigned long long* ctr) {
    const int64_t base = (int64_t)blockIdx.x * blockDim.x * ITEMS + threadIdx.x;
    uint64_t key[ITEMS];
    uint32_t valid = 0;
    bool bad = false;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = base + (int64_t)j * blockDim.x;
        key[j] = 0;
        if (i < n) {
            double x, y, z;
            load_xyz(pts, i, x, y, z);
            if (point_key<T>(x, y, z, scale, key[j])) valid |= 1u << j;
            else bad = true;
        }
    }
    if (bad) atomicOr(&ctr[C_ERROR], (unsigned long long)kErrRange);
    uint32_t fresh = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        int r = ADD_FOUND;
        if (valid & (1u << j)) {
            r = table_add(tab, g, key[j], 1u);
            fresh += (r == ADD_NEW);
        }
        spill_push(sp, ctr, r == ADD_FULL, key[j], 1u);
    }
    block_count_add(&ctr[C_INSERTED], fresh);
}

// Counting with LDS pre-aggregation: a workgroup first combines equal tiles
// of `sweeps` consecutive tiles of points in a small LDS hash table, then adds
// each distinct tile once to the device table.  Points whose tile finds no
// room in LDS go straight to the device table.  Pays off when a few hot tiles
// take a large share of the points.
template <typename T, int ITEMS>
__global__ void k_count_preagg(const T* __restrict__ pts, int64_t n, double scale, Slot* tab,
                               const Geo g, SpillBuf sp, unsigned long long* ctr, int lds_log2,
                               int sweeps) {
    extern __shared__ unsigned char smem[];
    const uint32_t L = 1u << lds_log2;
    uint64_t* lkey = reinterpret_cast<uint64_t*>(smem);
    uint32_t* lcnt = reinterpret_cast<uint32_t*>(lkey + L);
    for (uint32_t s = threadIdx.x; s < L; s += blockDim.x) {
        lkey[s] = kEmptyKey;
        lcnt[s] = 0;
    }
    __syncthreads();
    bool bad = false;
    uint32_t fresh = 0;
    const int64_t span = (int64_t)blockDim.x * ITEMS;
    for (int sw = 0; sw < sweeps; ++sw) {
        const int64_t base = ((int64_t)blockIdx.x * sweeps + sw) * span + threadIdx.x;
        if (base - threadIdx.x >= n) break;  // uniform across the workgroup
        uint64_t key[ITEMS];
        uint32_t valid = 0;
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int64_t i = base + (int64_t)j * blockDim.x;
            key[j] = 0;
            if (i < n) {
                double x, y, z;
                load_xyz(pts, i, x, y, z);
                if (point_key<T>(x, y, z, scale, key[j])) valid |= 1u << j;
                else bad = true;
            }
        }
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            int r = ADD_FOUND;
            if (valid & (1u << j)) {
                const uint64_t k = key[j];
                uint32_t pos = (slot_hash(k) >> 16) & (L - 1);
                bool done = false;
                for (int p = 0; p < 8 && !done; ++p) {
                    uint64_t cur = lds_load_relaxed(&lkey[pos]);
                    if (cur == kEmptyKey) cur = atomicCAS(reinterpret_cast<unsigned long long*>(&lkey[pos]),
                                                          (unsigned long long)kEmptyKey, (unsigned long long)k);
                    if (cur == kEmptyKey || cur == k) {
                        atomicAdd(&lcnt[pos], 1u);
                        done = true;
                    }
                    pos = (pos + 1) & (L - 1);
                }
                if (!done) {
                    r = table_add(tab, g, k, 1u);
                    fresh += (r == ADD_NEW);
                }
            }
            spill_push(sp, ctr, r == ADD_FULL, key[j], 1u);
        }
    }
    if (bad) atomicOr(&ctr[C_ERROR], (unsigned long long)kErrRange);
    __syncthreads();
    for (uint32_t s0 = 0; s0 < L; s0 += blockDim.x) {
        const uint32_t s = s0 + threadIdx.x;
        int r = ADD_FOUND;
        uint64_t k = kEmptyKey;
        uint32_t c = 0;
        if (s < L) {
            k = lkey[s];
            c = lcnt[s];
            if (k != kEmptyKey) {
                r = table_add(tab, g, k, c);
                fresh += (r == ADD_NEW);
            }
        }
        spill_push(sp, ctr, r == ADD_FULL, k, c);
    }
    block_count_add(&ctr[C_INSERTED], fresh);
}

__global__ void k_insert_records(const uint64_t* keys, const uint32_t* counts, uint64_t n, Slot* tab,
                                 const Geo g, SpillBuf sp, unsigned long long* ctr) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t n_round = (n + 63) / 64 * 64;  // whole waves iterate together
    uint32_t fresh = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_round; i += stride) {
        int r = ADD_FOUND;
        uint64_t k = 0;
        uint32_t c = 0;
        if (i < n) {
            k = keys[i];
            c = counts[i];
            r = table_add(tab, g, k, c);
        }
        fresh += (r == ADD_NEW);
        spill_push(sp, ctr, r == ADD_FULL, k, c);
    }
    block_count_add(&ctr[C_INSERTED], fresh);
}

__global__ void k_rehash(const Slot* from, uint64_t from_cap, Slot* to, const Geo to_g, SpillBuf sp,
                         unsigned long long* ctr) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t n_round = (from_cap + 63) / 64 * 64;  // whole waves iterate together
    uint32_t fresh = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_round; i += stride) {
        int r = ADD_FOUND;
        uint64_t k = kEmptyKey;
        uint32_t c = 0;
        if (i < from_cap) {
            const Slot s = from[i];
            k = s.key;
            c = s.count;
            if (k != kEmptyKey) r = table_add(to, to_g, k, c);
        }
        fresh += (r == ADD_NEW);
        spill_push(sp, ctr, r == ADD_FULL, k, c);
    }
    block_count_add(&ctr[C_INSERTED], fresh);
}

// ------------------------------------------------------ binned contraction ---
//
// The per-point count update is the hot loop of the method.  Done directly it
// costs one device-scope atomic per point, and those are executed at a single
// memory-side point at a few tens of billions per second.  The binned path
// instead routes every key to the workgroup that owns its table partition:
//   level 1: project the points and append each key to one of 128 coarse
//            buckets (top 7 hash bits), in runs written by one workgroup;
//   level 2: split each coarse bucket into its partitions;
//   update : one workgroup per partition loads the 4096-slot slice into LDS,
//            adds every key with LDS atomics and writes the slice back.
// All traffic is then sequential HBM streams plus one table read and write
// per group of chunks.

constexpr int BIN_THREADS = 512;
constexpr int BIN_ITEMS = (int)kBinTile / BIN_THREADS;  // 8

struct BinScratch {
    uint64_t key[kBinTile];
    uint32_t hist[kMaxFine];
    uint32_t off[kMaxFine];
    uint32_t base[kMaxFine];
    uint32_t total;
};

// Bucket of a key: the log2 nb bits of its placement hash that end top_bits
// from the top, so buckets refine in step with partitions.
__device__ __forceinline__ uint32_t bucket_of(uint64_t key, uint32_t top_bits, uint32_t nb, uint32_t d3) {
    return top_bits ? (place_of(key, d3) >> (32 - top_bits)) & (nb - 1) : 0u;
}

// Scatters this tile's valid keys into nb buckets: bucket b's keys are
// appended at out[b * stride + cursor[b] ...].  A key past its bucket's
// capacity (cap <= stride) goes straight into the table instead.  The bucket of a
// key is bucket_of(key, top_bits, nb, D3).  S.hist must be zero on entry (and a
// barrier passed); every thread of the workgroup calls.
template <bool D3>
__device__ void bin_tile(BinScratch& S, const uint64_t (&key)[BIN_ITEMS], const uint16_t (&bucket)[BIN_ITEMS],
                         uint32_t valid, uint32_t nb, uint32_t top_bits, uint64_t* out, uint64_t stride,
                         uint64_t cap, uint32_t* cursor, Slot* tab, const Geo& g, const SpillBuf& sp, unsigned long long* ctr,
                         uint32_t& fresh) {
    uint32_t rank[BIN_ITEMS];
#pragma unroll
    for (int j = 0; j < BIN_ITEMS; ++j) {
        rank[j] = 0;
        if (valid & (1u << j)) rank[j] = atomicAdd(&S.hist[bucket[j]], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const uint32_t per = (nb + 63) / 64;
        const uint32_t lo = threadIdx.x * per;
        uint32_t sum = 0;
        for (uint32_t q = 0; q < per; ++q)
            if (lo + q < nb) sum += S.hist[lo + q];
        uint32_t inc = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t v = __shfl_up(inc, o);
            if (lane_id() >= o) inc += v;
        }
        uint32_t ex = inc - sum;
        for (uint32_t q = 0; q < per; ++q)
            if (lo + q < nb) {
                S.off[lo + q] = ex;
                ex += S.hist[lo + q];
            }
        if (threadIdx.x == 63) S.total = inc;
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nb; b += BIN_THREADS)
        S.base[b] = S.hist[b] ? atomicAdd(&cursor[b], S.hist[b]) : 0u;
#pragma unroll
    for (int j = 0; j < BIN_ITEMS; ++j) {
        if (valid & (1u << j)) {
            const uint32_t p = S.off[bucket[j]] + rank[j];
            S.key[p] = key[j];
        }
    }
    __syncthreads();
    const uint32_t total = S.total;
    for (uint32_t q0 = 0; q0 < total; q0 += BIN_THREADS) {
        const uint32_t q = q0 + threadIdx.x;
        int r = ADD_FOUND;
        uint64_t k = 0;
        if (q < total) {
            k = S.key[q];
            const uint32_t b = bucket_of(k, top_bits, nb, D3);
            const uint64_t dst = (uint64_t)S.base[b] + (q - S.off[b]);
            if (dst < cap) {
                out[(uint64_t)b * stride + dst] = k;
            } else {
                // no table yet (not filled): the key waits in the spill buffer
                r = tab ? table_add(tab, g, k, 1u) : ADD_FULL;
                fresh += (r == ADD_NEW);
            }
        }
        spill_push(sp, ctr, r == ADD_FULL, k, 1u);
    }
}

__device__ __forceinline__ void add_fresh(unsigned long long* ctr, uint32_t fresh) {
    block_count_add(&ctr[C_INSERTED], fresh);
}

// hll, if not null, receives the hll_sample sketch of the keys: kHllReps
// replicas of the registers (one per workgroup index modulo kHllReps, so
// that the merges of many workgroups do not meet on a few cache lines).
// (SKETCH is a template parameter so that the sketch's LDS does not cost the
// other calls occupancy.)
template <typename T, bool SKETCH>
__global__ __launch_bounds__(BIN_THREADS) void k_bin_points(const T* __restrict__ pts, int64_t n, double scale,
                                                            uint64_t* bin1, uint64_t cap1, uint32_t* cursor1,
                                                            Slot* tab, const Geo g, SpillBuf sp,
                                                            unsigned long long* ctr, uint32_t* hll) {
    __shared__ BinScratch S;
    __shared__ uint32_t sk[SKETCH ? (1u << kHllLog2) : 1u];
    for (uint32_t b = threadIdx.x; b < kCoarse; b += BIN_THREADS) S.hist[b] = 0;
    if (SKETCH)
        for (uint32_t b = threadIdx.x; b < (1u << kHllLog2); b += BIN_THREADS) sk[b] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kBinTile + threadIdx.x;
    uint64_t key[BIN_ITEMS];
    uint16_t bucket[BIN_ITEMS];
    uint32_t valid = 0;
    bool bad = false;
    // all loads first, so that they are in flight together
    double x[BIN_ITEMS], y[BIN_ITEMS], z[BIN_ITEMS];
#pragma unroll
    for (int j = 0; j < BIN_ITEMS; ++j) {
        const int64_t i = base + (int64_t)j * BIN_THREADS;
        x[j] = 0.0;
        y[j] = 0.0;
        z[j] = 0.0;
        if (i < n) load_xyz(pts, i, x[j], y[j], z[j]);
    }
#pragma unroll
    for (int j = 0; j < BIN_ITEMS; ++j) {
        const int64_t i = base + (int64_t)j * BIN_THREADS;
        key[j] = 0;
        bucket[j] = 0;
        if (i < n) {
            if (point_key<T>(x[j], y[j], z[j], scale, key[j])) {
                valid |= 1u << j;
                bucket[j] = (uint16_t)bucket_of(key[j], kCoarseLog2, kCoarse, PtDims<T>::value == 3);
                uint32_t reg, rank;
                if (SKETCH && hll_sample(key[j], reg, rank)) atomicMax(&sk[reg], rank);
            } else {
                bad = true;
            }
        }
    }
    if (bad) atomicOr(&ctr[C_ERROR], (unsigned long long)kErrRange);
    uint32_t fresh = 0;
    const uint32_t r = blockIdx.x % kBinRep;
    bin_tile<PtDims<T>::value == 3>(S, key, bucket, valid, kCoarse, kCoarseLog2, bin1 + (uint64_t)r * kCoarse * cap1,
                                    cap1, cap1,
             cursor1 + r * kCoarse, tab, g, sp, ctr, fresh);
    add_fresh(ctr, fresh);
    if (SKETCH) {
        __syncthreads();  // every sampled key is registered
        uint32_t* rep = hll + ((uint64_t)(blockIdx.x % kHllReps) << kHllLog2);
        for (uint32_t b = threadIdx.x; b < (1u << kHllLog2); b += BIN_THREADS)
            if (sk[b]) atomicMax(rep + b, sk[b]);
    }
}

// Level 2: workgroup (l1, seg) splits keys [seg * kBinTile, ...) of coarse
// list l1 = (replica r, bucket b1) into replica r of that bucket's partition
// lists.  Segments vary fastest with the workgroup index: the workgroups in
// flight at once then append to the lists of a few dozen coarse lists, whose
// open partial lines stay in L2 until complete, while the replicas keep the
// cursor lines they update apart.
template <bool D3>
__global__ __launch_bounds__(BIN_THREADS) void k_bin_keys(const uint64_t* __restrict__ bin1, uint64_t cap1,
                                                          const uint32_t* cursor1, uint32_t segs, uint64_t* bin2,
                                                          uint64_t cap2, uint32_t* cursor2, Slot* tab, const Geo g,
                                                          SpillBuf sp, unsigned long long* ctr) {
    __shared__ BinScratch S;
    const uint32_t l1 = blockIdx.x / segs;
    const uint32_t seg = blockIdx.x % segs;
    const uint32_t r = l1 / kCoarse, b1 = l1 % kCoarse;
    const uint64_t cnt = min((uint64_t)cursor1[l1], cap1);
    const uint64_t start = (uint64_t)seg * kBinTile;
    if (start >= cnt) return;  // uniform across the workgroup
    const uint32_t fine_log2 = g.p_log2 - kCoarseLog2;
    const uint32_t nb = 1u << fine_log2;
    for (uint32_t b = threadIdx.x; b < nb; b += BIN_THREADS) S.hist[b] = 0;
    __syncthreads();
    uint64_t key[BIN_ITEMS];
    uint16_t bucket[BIN_ITEMS];
    uint32_t valid = 0;
    const uint64_t* src = bin1 + (uint64_t)l1 * cap1;
    // all loads first, so that they are in flight together
#pragma unroll
    for (int j = 0; j < BIN_ITEMS; ++j) {
        const uint64_t i = start + (uint64_t)j * BIN_THREADS + threadIdx.x;
        key[j] = 0;
        if (i < cnt) key[j] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int j = 0; j < BIN_ITEMS; ++j) {
        const uint64_t i = start + (uint64_t)j * BIN_THREADS + threadIdx.x;
        bucket[j] = 0;
        if (i < cnt) {
            bucket[j] = (uint16_t)bucket_of(key[j], g.p_log2, nb, D3);
            valid |= 1u << j;
        }
    }
    uint32_t fresh = 0;
    // partition lists are stored partition-major (a partition's replicas
    // side by side), their cursors replica-major
    const uint64_t first = (uint64_t)b1 << fine_log2;
    bin_tile<D3>(S, key, bucket, valid, nb, g.p_log2, bin2 + (first * kBinRep + r) * cap2, kBinRep * cap2, cap2,
             cursor2 + ((uint64_t)r << g.p_log2) + first, tab, g, sp, ctr,
             fresh);
    add_fresh(ctr, fresh);
}

constexpr int AGG_THREADS = 512;
constexpr uint32_t kPartSlots = 1u << kPartLog2;

// LDS version of table_add over one partition slice (same probe sequence as
// the device table, so slots stay where a device-table probe looks for them).
// Continues from position pos, whose word was read as cur (possibly stale:
// a stale empty only sends the key through the compare-and-swap).
__device__ __forceinline__ int lds_add_from(uint64_t* lkey, uint32_t* lcnt, uint64_t key, uint32_t pos,
                                            uint64_t cur) {
    for (uint32_t p = 0; p < kMaxProbe; ++p) {
        if (p) cur = lds_load_relaxed(&lkey[pos]);
        if (cur == kEmptyKey) {
            cur = atomicCAS(reinterpret_cast<unsigned long long*>(&lkey[pos]), (unsigned long long)kEmptyKey,
                            (unsigned long long)key);
            if (cur == kEmptyKey) {
                atomicAdd(&lcnt[pos], 1u);
                return ADD_NEW;
            }
        }
        if (cur == key) {
            atomicAdd(&lcnt[pos], 1u);
            return ADD_FOUND;
        }
        pos = (pos + 1) & (kPartSlots - 1);
    }
    return ADD_FULL;
}

// One workgroup per partition: load the slice, add its keys, store it back.
// Keys are fetched AGG_BATCH per thread at a time so that many loads are in
// flight before the LDS work that depends on them.
constexpr int AGG_BATCH = 8;

// The NL key lists of one partition: list i holds min(count[i * cstride], cap)
// keys at src + i * lstride, read as one concatenated range.  The sizes are
// loaded once, into registers.
template <int NL>
struct PartLists {
    const uint64_t* src;
    uint64_t lstride;
    uint32_t size[NL];
    uint32_t total;
    __device__ PartLists(const uint64_t* s, uint64_t ls, const uint32_t* count, uint64_t cstride, uint64_t cap)
        : src(s), lstride(ls), total(0) {
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            size[i] = (uint32_t)min((uint64_t)count[i * cstride], cap);
            total += size[i];
        }
    }
    __device__ uint32_t size_of(uint32_t li) const {
        uint32_t v = 0;
#pragma unroll
        for (int i = 0; i < NL; ++i)
            if ((uint32_t)i == li) v = size[i];
        return v;
    }
};

// Adds the L.total keys of the lists L to one 4096-slot partition through LDS.
// With load false the table holds no key yet, and the slice starts empty
// without being read.  With whole (a table not filled yet) every slot of the
// slice is written, the empty ones too; with write false (no entries: the
// slice was read only to be counted) none is.
template <int NL>
__device__ __forceinline__ void aggregate_partition(const PartLists<NL>& L, Slot* part, bool load, uint64_t* lkey,
                                                    uint32_t* lcnt, const SpillBuf& sp,
                                                    unsigned long long* spill_ctr, uint32_t& fresh,
                                                    bool whole = false, bool write = true) {
    constexpr int PER = (int)kPartSlots / AGG_THREADS;
    const uint32_t cnt = L.total;
    if (load) {
        Slot v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) v[u] = part[u * AGG_THREADS + threadIdx.x];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            lkey[u * AGG_THREADS + threadIdx.x] = v[u].key;
            lcnt[u * AGG_THREADS + threadIdx.x] = v[u].count;
        }
    } else {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            lkey[u * AGG_THREADS + threadIdx.x] = kEmptyKey;
            lcnt[u * AGG_THREADS + threadIdx.x] = 0;
        }
    }
    __syncthreads();
    // a thread's positions only grow, so it walks the lists once: list li
    // covers positions [lo, hi) of the concatenation
    uint32_t li = 0, lo = 0, hi = L.size[0];
    constexpr uint32_t STEP = AGG_THREADS * AGG_BATCH;
    // The keys of batch q0: addresses first (positions past the end clamped
    // to the last key), then all loads unconditionally, so that no load waits
    // for another.  Needs q0 < cnt.
    auto fetch = [&](uint32_t q0, uint64_t (&k)[AGG_BATCH]) {
        const uint64_t* at[AGG_BATCH];
#pragma unroll
        for (int u = 0; u < AGG_BATCH; ++u) {
            const uint32_t q = min(q0 + u * AGG_THREADS + threadIdx.x, cnt - 1);
            while (q >= hi) {
                ++li;
                lo = hi;
                hi += L.size_of(li);
            }
            at[u] = L.src + li * L.lstride + (q - lo);
        }
#pragma unroll
        for (int u = 0; u < AGG_BATCH; ++u) k[u] = __builtin_nontemporal_load(at[u]);
    };
    // software pipeline: the next batch's loads are in flight while this
    // batch is added in LDS
    uint64_t k[AGG_BATCH], next[AGG_BATCH];
    if (cnt > 0) fetch(0, next);
    for (uint32_t q0 = 0; q0 < cnt; q0 += STEP) {
#pragma unroll
        for (int u = 0; u < AGG_BATCH; ++u) k[u] = next[u];
        if (q0 + STEP < cnt) fetch(q0 + STEP, next);  // uniform across the workgroup
#pragma unroll
        for (int u = 0; u < AGG_BATCH; ++u)
            if (q0 + u * AGG_THREADS + threadIdx.x >= cnt) k[u] = kEmptyKey;
        // home-slot reads of all keys together; most keys find themselves
        // there, and only the others walk the probe sequence
        uint32_t pos[AGG_BATCH];
        uint64_t cur[AGG_BATCH];
#pragma unroll
        for (int u = 0; u < AGG_BATCH; ++u) {
            pos[u] = slot_hash(k[u]) & (kPartSlots - 1);
            cur[u] = k[u] != kEmptyKey ? lds_load_relaxed(&lkey[pos[u]]) : kEmptyKey;
        }
#pragma unroll
        for (int u = 0; u < AGG_BATCH; ++u) {
            int r = ADD_FOUND;
            if (k[u] != kEmptyKey) {
                if (cur[u] == k[u]) {
                    atomicAdd(&lcnt[pos[u]], 1u);
                } else {
                    r = lds_add_from(lkey, lcnt, k[u], pos[u], cur[u]);
                    fresh += (r == ADD_NEW);
                }
            }
            spill_push(sp, spill_ctr, r == ADD_FULL, k[u], 1u);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const uint32_t s = u * AGG_THREADS + threadIdx.x;
        const uint64_t k = lkey[s];
        if (write && (whole || k != kEmptyKey)) {
            Slot v;
            v.key = k;
            v.count = lcnt[s];  // 0 in an empty slot
            v.aux = kNotSignificant;
            part[s] = v;
        }
    }
}

// At least 6 waves per SIMD: the LDS slice allows three workgroups of 8 waves
// per CU, and this holds the registers (the next batch's keys included) to
// what three need.
// With whole (a table not filled yet: no key in it) every workgroup writes
// its whole slice, which fills the table.  With cn.partials (the final
// update) every workgroup also counts its partition for the significance
// scan (AggCount), reading the slice even when it got no entries.
__global__ __launch_bounds__(AGG_THREADS, 6) void k_aggregate(const uint64_t* __restrict__ bin2, uint64_t cap2,
                                                           const uint32_t* cursor2, Slot* tab, SpillBuf sp,
                                                           unsigned long long* ctr, bool whole, AggCount cn) {
    __shared__ uint64_t lkey[kPartSlots];
    __shared__ uint32_t lcnt[kPartSlots];
    const uint64_t p = blockIdx.x;
    const uint64_t parts = gridDim.x;
    const PartLists<kBinRep> L(bin2 + p * kBinRep * cap2, cap2, cursor2 + p, parts, cap2);
    if (L.total == 0 && !whole && !cn.partials) return;  // uniform across the workgroup
    uint32_t fresh = 0;
    aggregate_partition(L, tab + (p << kPartLog2), !whole && ctr[C_TABLE_KEYS] != 0, lkey, lcnt, sp, ctr, fresh,
                        whole, whole || L.total != 0);
    add_fresh(ctr, fresh);
    if (cn.partials) {
        // the slice in LDS is final: each thread counts the slots it wrote
        constexpr int PER = (int)kPartSlots / AGG_THREADS;
        uint32_t sig = 0;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t sl = u * AGG_THREADS + threadIdx.x;
            sig += lkey[sl] != kEmptyKey && lcnt[sl] >= cn.tau;
        }
        // (the occupied slots and their sum are totalled by the scatter pass:
        // totalling them here as well made this kernel much slower)
        block_count_add32(cn.partials + (p >> cn.blk_shift), sig);
    }
}

// ---- framed binned contraction (two-dimensional tables with a key frame) -----
//
// The same two binning levels and LDS update as above, moving 4-byte entries
// (frame_code) instead of 8-byte keys.  Level 1 uses kFrameCoarse coarse
// buckets (the top 8 bits of h) and work tiles of kFBinTile points; level 2
// splits each coarse list by the next bits of h, which are the top bits of
// the entry, so it needs no hashing.  Keys outside the frame, and entries past
// a full list, go straight into the table, or into the spill buffer while the
// table is not filled yet (tab == nullptr).

// Points per thread of the framed level 1.  16 (an 8192-point tile, three
// workgroups per CU) and 8 (a 4096-point tile, four per CU) measure the same;
// the larger tile takes half the cursor atomics.
constexpr int kFBinItems1 = 16;
constexpr uint32_t kFBinTile = 8192;  // level 2's work tile
constexpr int FBIN_ITEMS = (int)kFBinTile / BIN_THREADS;  // 16

struct FBinCommon {
    uint32_t ent[kFBinTile];
    uint32_t hist[kMaxFine];
    uint32_t off[kMaxFine];
    uint32_t base[kMaxFine];
    uint32_t total;
};
// Level 1: ITEMS points per thread, kFrameCoarse buckets.
template <int ITEMS>
struct FBinScratch1 {
    uint32_t ent[BIN_THREADS * ITEMS];
    uint8_t bkt[BIN_THREADS * ITEMS];  // the coarse bucket of each staged entry
    uint32_t hist[kFrameCoarse];
    uint32_t off[kFrameCoarse];
    uint32_t base[kFrameCoarse];
    uint32_t total;
};

// Scatters this tile's valid entries into nb buckets, as bin_tile does for
// keys.  Level 1 (L1) buckets are coarse buckets, taken from S.bkt on the way
// out; level-2 buckets are (e >> 6) >> sub_shift, inside coarse bucket cb.
template <bool L1, int ITEMS, typename Scratch>
__device__ void fbin_tile(Scratch& S, const uint32_t (&ent)[ITEMS], const uint16_t (&bucket)[ITEMS],
                          uint32_t valid, uint32_t nb, uint32_t sub_shift, uint32_t cb, uint32_t* out,
                          uint64_t stride, uint64_t cap, uint32_t* cursor, Slot* tab, const Geo& g,
                          const SpillBuf& sp, unsigned long long* ctr, uint32_t& fresh) {
    uint32_t rank[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        rank[j] = 0;
        if (valid & (1u << j)) rank[j] = atomicAdd(&S.hist[bucket[j]], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const uint32_t per = (nb + 63) / 64;
        const uint32_t lo = threadIdx.x * per;
        uint32_t sum = 0;
        for (uint32_t q = 0; q < per; ++q)
            if (lo + q < nb) sum += S.hist[lo + q];
        uint32_t inc = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t v = __shfl_up(inc, o);
            if (lane_id() >= o) inc += v;
        }
        uint32_t ex = inc - sum;
        for (uint32_t q = 0; q < per; ++q)
            if (lo + q < nb) {
                S.off[lo + q] = ex;
                ex += S.hist[lo + q];
            }
        if (threadIdx.x == 63) S.total = inc;
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nb; b += BIN_THREADS)
        S.base[b] = S.hist[b] ? atomicAdd(&cursor[b], S.hist[b]) : 0u;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        if (valid & (1u << j)) {
            const uint32_t p = S.off[bucket[j]] + rank[j];
            S.ent[p] = ent[j];
            if constexpr (L1) S.bkt[p] = (uint8_t)bucket[j];
        }
    }
    __syncthreads();
    const uint32_t total = S.total;
    for (uint32_t q0 = 0; q0 < total; q0 += BIN_THREADS) {
        const uint32_t q = q0 + threadIdx.x;
        int r = ADD_FOUND;
        uint64_t k = 0;
        if (q < total) {
            const uint32_t e = S.ent[q];
            uint32_t b;
            if constexpr (L1) b = S.bkt[q];
            else b = (e >> 6) >> sub_shift;
            const uint64_t dst = (uint64_t)S.base[b] + (q - S.off[b]);
            if (dst < cap) {
                out[(uint64_t)b * stride + dst] = e;
            } else {
                k = frame_key(L1 ? b : cb, e, g.fx, g.fy);
                r = tab ? table_add(tab, g, k, 1u) : ADD_FULL;
                fresh += (r == ADD_NEW);
            }
        }
        spill_push(sp, ctr, r == ADD_FULL, k, 1u);
    }
}

template <typename T, bool SKETCH, int ITEMS>
__global__ __launch_bounds__(BIN_THREADS) void k_bin_points_f(const T* __restrict__ pts, int64_t n, double scale,
                                                              uint32_t* bin1, uint64_t cap1, uint32_t* cursor1,
                                                              Slot* tab, const Geo g, SpillBuf sp,
                                                              unsigned long long* ctr, uint32_t* hll) {
    constexpr uint32_t TILE = BIN_THREADS * ITEMS;
    __shared__ FBinScratch1<ITEMS> S;
    __shared__ uint32_t sk[SKETCH ? (1u << kHllLog2) : 1u];
    for (uint32_t b = threadIdx.x; b < kFrameCoarse; b += BIN_THREADS) S.hist[b] = 0;
    if (SKETCH)
        for (uint32_t b = threadIdx.x; b < (1u << kHllLog2); b += BIN_THREADS) sk[b] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * TILE + threadIdx.x;
    uint32_t ent[ITEMS];
    uint16_t bucket[ITEMS];
    uint32_t valid = 0, rare = 0, fresh = 0;
    bool bad = false;
    constexpr int HALF = ITEMS > 8 ? ITEMS / 2 : ITEMS;
#pragma unroll
    for (int h0 = 0; h0 < ITEMS; h0 += HALF) {
        // the loads of half the items first, so that they are in flight together
        double x[HALF], y[HALF];
#pragma unroll
        for (int j = 0; j < HALF; ++j) {
            const int64_t i = base + (int64_t)(h0 + j) * BIN_THREADS;
            x[j] = 0.0;
            y[j] = 0.0;
            if (i < n) load_point(pts, i, x[j], y[j]);
        }
        // Keys inside the frame without branches (the projection of
        // tile_key, then frame_code); points outside the frame wait for the
        // pass below, and range errors only raise the flag.
#pragma unroll
        for (int j = 0; j < HALF; ++j) {
            const int jj = h0 + j;
            const bool in = base + (int64_t)jj * BIN_THREADS < n;
            const double px = x[j] * scale, py = y[j] * scale;
            const bool ok = fabs(px) < 2147483647.0 && fabs(py) < 2147483647.0;
            const uint32_t bx = (uint32_t)(int32_t)(ok ? px : 0.0) + 0x80000000u;
            const uint32_t by = (uint32_t)(int32_t)(ok ? py : 0.0) + 0x80000000u;
            const uint32_t rx = bx - g.fx, ry = by - g.fy;
            const bool inside = ok && (rx | ry) < kFrameSide;
            const uint64_t h = frame_mix(((uint64_t)((rx >> 3) & ((1u << kFrameStSide) - 1)) << kFrameStSide) |
                                         ((ry >> 3) & ((1u << kFrameStSide) - 1)));
            const uint32_t e = ((uint32_t)(h & ((1u << kFrameHLow) - 1)) << 6) | ((rx & 7u) << 3) | (ry & 7u);
            ent[jj] = e;
            bucket[jj] = (uint16_t)(h >> kFrameHLow);
            valid |= (in && inside ? 1u : 0u) << jj;
            rare |= (in && ok && !inside ? 1u : 0u) << jj;
            bad |= in && !ok;
            // the sketch takes the mixed h with the position in the
            // super-tile spread over 32 bits: no second hash
            uint32_t reg, rank;
            if (SKETCH && in && inside && hll_from_hash((uint32_t)h ^ ((e & 63u) * kGolden32), reg, rank))
                atomicMax(&sk[reg], rank);
        }
    }
    // Points whose tiles lie outside the frame: read again and put straight
    // into the table (with the key's own sketch hash).
    if (__ballot(rare != 0)) {  // uniform across the wave
#pragma unroll 1
        for (int jj = 0; jj < ITEMS; ++jj) {
            int r = ADD_FOUND;
            uint64_t key = 0;
            if ((rare >> jj) & 1u) {
                double x, y;
                load_point(pts, base + (int64_t)jj * BIN_THREADS, x, y);
                (void)tile_key(x, y, scale, key);  // in range: checked above
                uint32_t reg, rank;
                if (SKETCH && hll_sample(key, reg, rank)) atomicMax(&sk[reg], rank);
                // no table yet (not filled): the key waits in the spill buffer
                r = tab ? table_add(tab, g, key, 1u) : ADD_FULL;
                fresh += (r == ADD_NEW);
            }
            spill_push(sp, ctr, r == ADD_FULL, key, 1u);
        }
    }
    if (bad) atomicOr(&ctr[C_ERROR], (unsigned long long)kErrRange);
    const uint32_t rep = blockIdx.x % kBinRep;
    fbin_tile<true, ITEMS>(S, ent, bucket, valid, kFrameCoarse, 0u, 0u, bin1 + (uint64_t)rep * kFrameCoarse * cap1,
                           cap1, cap1, cursor1 + rep * kFrameCoarse, tab, g, sp, ctr, fresh);
    add_fresh(ctr, fresh);
    if (SKETCH) {
        __syncthreads();  // every sampled key is registered
        uint32_t* rp = hll + ((uint64_t)(blockIdx.x % kHllReps) << kHllLog2);
        for (uint32_t b = threadIdx.x; b < (1u << kHllLog2); b += BIN_THREADS)
            if (sk[b]) atomicMax(rp + b, sk[b]);
    }
}

// Level 2: workgroup (l1, seg) splits entries [seg * kFBinTile, ...) of
// coarse list l1 = (replica r, bucket b1) into replica r of that bucket's
// partition lists (stored as in the unframed binning).
__global__ __launch_bounds__(BIN_THREADS) void k_bin_keys_f(const uint32_t* __restrict__ bin1, uint64_t cap1,
                                                            const uint32_t* cursor1, uint32_t segs, uint32_t* bin2,
                                                            uint64_t cap2, uint32_t* cursor2, Slot* tab, const Geo g,
                                                            SpillBuf sp, unsigned long long* ctr) {
    __shared__ FBinCommon S;
    const uint32_t l1 = blockIdx.x / segs;
    const uint32_t seg = blockIdx.x % segs;
    const uint32_t r = l1 / kFrameCoarse, b1 = l1 % kFrameCoarse;
    const uint64_t cnt = min((uint64_t)cursor1[l1], cap1);
    const uint64_t start = (uint64_t)seg * kFBinTile;
    if (start >= cnt) return;  // uniform across the workgroup
    const uint32_t fine_log2 = g.p_log2 - kFrameCoarseLog2;
    const uint32_t nb = 1u << fine_log2;
    const uint32_t sub_shift = kFrameHLow - fine_log2;
    for (uint32_t b = threadIdx.x; b < nb; b += BIN_THREADS) S.hist[b] = 0;
    __syncthreads();
    uint32_t ent[FBIN_ITEMS];
    uint16_t bucket[FBIN_ITEMS];
    uint32_t valid = 0;
    const uint32_t* src = bin1 + (uint64_t)l1 * cap1;
    // all loads first, so that they are in flight together
#pragma unroll
    for (int j = 0; j < FBIN_ITEMS; ++j) {
        const uint64_t i = start + (uint64_t)j * BIN_THREADS + threadIdx.x;
        ent[j] = 0;
        // plain loads: non-temporal ones made this pass and the update that
        // reads its lists slower (1.02 and 1.0 ms against 0.94 and 0.95)
        if (i < cnt) ent[j] = src[i];
    }
#pragma unroll
    for (int j = 0; j < FBIN_ITEMS; ++j) {
        const uint64_t i = start + (uint64_t)j * BIN_THREADS + threadIdx.x;
        bucket[j] = (uint16_t)((ent[j] >> 6) >> sub_shift);
        if (i < cnt) valid |= 1u << j;
    }
    uint32_t fresh = 0;
    const uint64_t first = (uint64_t)b1 << fine_log2;
    fbin_tile<false, FBIN_ITEMS>(S, ent, bucket, valid, nb, sub_shift, b1, bin2 + (first * kBinRep + r) * cap2,
                                 kBinRep * cap2, cap2, cursor2 + ((uint64_t)r << g.p_log2) + first, tab, g, sp, ctr,
                                 fresh);
    add_fresh(ctr, fresh);
}

// One workgroup per partition adds its entries to the slice in LDS.  A slot
// is claimed by a 64-bit word, 1 << 32 | entry (0: empty), and counted in its
// own 32-bit word, so that the count updates spread over all LDS banks.  When
// the table already held keys the slice is read first; a slot holding a key
// outside the frame gets the word 2 << 32, which no entry matches, and is not
// written back.
constexpr int FAGG_BATCH = 8;

template <int NL>
struct PartEntries {
    const uint32_t* src;
    uint64_t lstride;
    uint32_t size[NL];
    uint32_t total;
    __device__ PartEntries(const uint32_t* s, uint64_t ls, const uint32_t* count, uint64_t cstride, uint64_t cap)
        : src(s), lstride(ls), total(0) {
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            size[i] = (uint32_t)min((uint64_t)count[i * cstride], cap);
            total += size[i];
        }
    }
    __device__ uint32_t size_of(uint32_t li) const {
        uint32_t v = 0;
#pragma unroll
        for (int i = 0; i < NL; ++i)
            if ((uint32_t)i == li) v = size[i];
        return v;
    }
};

struct FAggLds {
    uint64_t word[kPartSlots];
    uint32_t cnt[kPartSlots];
};
constexpr uint64_t kClaimed = 1ull << 32, kForeign = 2ull << 32;

__device__ __forceinline__ void aggregate_entries(const PartEntries<kBinRep>& L, Slot* part, uint32_t cb, const Geo& g,
                                                  bool load, FAggLds& A, const SpillBuf& sp, unsigned long long* ctr,
                                                  uint32_t& fresh, bool whole) {
    constexpr int PER = (int)kPartSlots / AGG_THREADS;
    if (load) {
        Slot v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) v[u] = part[u * AGG_THREADS + threadIdx.x];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t sl = u * AGG_THREADS + threadIdx.x;
            uint64_t w = 0, h;
            uint32_t e, c = 0;
            if (v[u].key != kEmptyKey) {
                c = v[u].count;
                w = frame_code(v[u].key, g.fx, g.fy, h, e) ? (kClaimed | e) : kForeign;
            }
            A.word[sl] = w;
            A.cnt[sl] = c;
        }
    } else {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            A.word[u * AGG_THREADS + threadIdx.x] = 0;
            A.cnt[u * AGG_THREADS + threadIdx.x] = 0;
        }
    }
    __syncthreads();
    const uint32_t cnt = L.total;
    uint32_t li = 0, lo = 0, hi = L.size[0];
    constexpr uint32_t STEP = AGG_THREADS * FAGG_BATCH;
    auto fetch = [&](uint32_t q0, uint32_t (&k)[FAGG_BATCH]) {
        const uint32_t* at[FAGG_BATCH];
#pragma unroll
        for (int u = 0; u < FAGG_BATCH; ++u) {
            const uint32_t q = min(q0 + u * AGG_THREADS + threadIdx.x, cnt - 1);
            while (q >= hi) {
                ++li;
                lo = hi;
                hi += L.size_of(li);
            }
            at[u] = L.src + li * L.lstride + (q - lo);
        }
#pragma unroll
        for (int u = 0; u < FAGG_BATCH; ++u) k[u] = __builtin_nontemporal_load(at[u]);
    };
    uint32_t k[FAGG_BATCH], next[FAGG_BATCH];
    fetch(0, next);
    for (uint32_t q0 = 0; q0 < cnt; q0 += STEP) {
#pragma unroll
        for (int u = 0; u < FAGG_BATCH; ++u) k[u] = next[u];
        if (q0 + STEP < cnt) fetch(q0 + STEP, next);  // uniform across the workgroup
        // home-slot reads of all entries together; most entries find
        // themselves there, and only the others walk the probe sequence
        uint32_t pos[FAGG_BATCH];
        uint64_t cur[FAGG_BATCH];
#pragma unroll
        for (int u = 0; u < FAGG_BATCH; ++u) {
            pos[u] = frame_home(k[u]) & (kPartSlots - 1);
            cur[u] = q0 + u * AGG_THREADS + threadIdx.x < cnt ? lds_load_relaxed(&A.word[pos[u]]) : 0;
        }
#pragma unroll
        for (int u = 0; u < FAGG_BATCH; ++u) {
            const bool have = q0 + u * AGG_THREADS + threadIdx.x < cnt;
            int r = ADD_FOUND;
            if (have) {
                const uint64_t want = kClaimed | k[u];
                uint32_t ps = pos[u];
                uint64_t c = cur[u];
                r = ADD_FULL;
                for (uint32_t step = 0; step < kMaxProbe; ++step) {
                    if (step) c = lds_load_relaxed(&A.word[ps]);
                    if (c == 0) {
                        c = atomicCAS(reinterpret_cast<unsigned long long*>(&A.word[ps]), 0ull,
                                      (unsigned long long)want);
                        if (c == 0) {
                            atomicAdd(&A.cnt[ps], 1u);
                            r = ADD_NEW;
                            break;
                        }
                    }
                    if (c == want) {
                        atomicAdd(&A.cnt[ps], 1u);
                        r = ADD_FOUND;
                        break;
                    }
                    ps = (ps + 1) & (kPartSlots - 1);
                }
                fresh += (r == ADD_NEW);
            }
            const uint64_t key = r == ADD_FULL ? frame_key(cb, k[u], g.fx, g.fy) : 0;
            spill_push(sp, ctr, r == ADD_FULL, key, 1u);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const uint32_t sl = u * AGG_THREADS + threadIdx.x;
        const uint64_t w = A.word[sl];
        if ((w >> 32) == 1 || (whole && w == 0)) {
            Slot v;
            v.key = w ? frame_key(cb, (uint32_t)w, g.fx, g.fy) : kEmptyKey;
            v.count = A.cnt[sl];  // 0 in an empty slot
            v.aux = kNotSignificant;
            part[sl] = v;
        }
    }
}

__global__ __launch_bounds__(AGG_THREADS, 6) void k_aggregate_f(const uint32_t* __restrict__ bin2, uint64_t cap2,
                                                                const uint32_t* cursor2, Slot* tab, const Geo g,
                                                                SpillBuf sp, unsigned long long* ctr, bool whole) {
    __shared__ FAggLds A;
    const uint64_t p = blockIdx.x;
    const uint64_t parts = gridDim.x;
    const PartEntries<kBinRep> L(bin2 + p * kBinRep * cap2, cap2, cursor2 + p, parts, cap2);
    if (L.total == 0 && !whole) return;  // uniform across the workgroup
    Slot* part = tab + (p << kPartLog2);
    const uint32_t cb = (uint32_t)(p >> (g.p_log2 - kFrameCoarseLog2));
    uint32_t fresh = 0;
    aggregate_entries(L, part, cb, g, !whole && ctr[C_TABLE_KEYS] != 0, A, sp, ctr, fresh, whole);
    add_fresh(ctr, fresh);
}

// The same update with 4-byte claim words, for tables with at least 512
// partitions: a partition's entries then share their top p_log2 - 8 bits
// (the partition's bits below its coarse bucket), so an entry whose top bit
// differs from theirs marks an empty slot and another one a slot holding a
// key outside the frame.
//
// Each entry looks at its home slot and the next one, which hold about 90%
// of the entries of a partition filled to half its slots.  The others are
// deferred to a ring of the wave's own in LDS and walk their probe sequences
// 64 at a time, one per lane, so that a wave does not run the longest walk
// of each of its entries.  The slice and the rings take 36 KB of LDS, which
// lets four workgroups share a CU.
constexpr uint32_t AGG_RING = 128;  // deferred entries per wave (at most 127 wait)
static_assert(AGG_RING * (AGG_THREADS / 64) * 4 >= 64 * 8, "the rings hold the census bits afterwards");
struct FAggLds32 {
    uint32_t ent[kPartSlots];
    uint32_t cnt[kPartSlots];
    uint32_t ring[AGG_THREADS / 64][AGG_RING];
};

__global__ __launch_bounds__(AGG_THREADS, 8) void k_aggregate_f32(const uint32_t* __restrict__ bin2, uint64_t cap2,
                                                                  const uint32_t* cursor2, Slot* tab, const Geo g,
                                                                  SpillBuf sp, unsigned long long* ctr,
                                                                  AggCensus cen, bool whole, AggCount cn) {
    __shared__ FAggLds32 A;
    const uint64_t p = blockIdx.x;
    const uint64_t parts = gridDim.x;
    const PartEntries<kBinRep> L(bin2 + p * kBinRep * cap2, cap2, cursor2 + p, parts, cap2);
    if (L.total == 0 && !cen.rec && !whole && !cn.partials) return;  // uniform across the workgroup
    const bool load = !whole && ctr[C_TABLE_KEYS] != 0;
    Slot* part = tab + (p << kPartLog2);
    const uint32_t fine = g.p_log2 - kFrameCoarseLog2;  // >= 1 here
    const uint32_t cb = (uint32_t)(p >> fine);
    const uint32_t top = (uint32_t)(p & ((1u << fine) - 1)) << (32 - fine);
    const uint32_t kEmpty = top ^ 0x80000000u, kAlien = kEmpty ^ 1u;  // never an entry of this partition
    constexpr int PER = (int)kPartSlots / AGG_THREADS;
    if (load) {
        Slot v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) v[u] = part[u * AGG_THREADS + threadIdx.x];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t sl = u * AGG_THREADS + threadIdx.x;
            uint64_t h;
            uint32_t e = kEmpty, c = 0;
            if (v[u].key != kEmptyKey) {
                c = v[u].count;
                if (!frame_code(v[u].key, g.fx, g.fy, h, e)) e = kAlien;
            }
            A.ent[sl] = e;
            A.cnt[sl] = c;
        }
    } else {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            A.ent[u * AGG_THREADS + threadIdx.x] = kEmpty;
            A.cnt[u * AGG_THREADS + threadIdx.x] = 0;
        }
    }
    __syncthreads();
    uint32_t* ring = A.ring[threadIdx.x >> 6];
    const uint32_t lane = lane_id();
    const uint64_t lt = lanemask_lt();
    uint32_t head = 0, tail = 0;  // the wave's ring (uniform across the wave)
    uint32_t fresh = 0;
    // Up to 64 deferred entries, one per lane, walk their probe sequences from
    // the home slot (a lost claim may have filled the first two slots with
    // other keys since they were read).
    auto drain = [&]() {
        const uint32_t n = min(tail - head, 64u);
        bool act = lane < n;
        const uint32_t e = act ? ring[(head + lane) & (AGG_RING - 1)] : 0u;
        head += n;
        uint32_t ps = frame_home(e) & (kPartSlots - 1);
        for (uint32_t step = 0; act && step < kMaxProbe; ++step) {
            uint32_t c = __hip_atomic_load(&A.ent[ps], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (c == kEmpty) {
                c = atomicCAS(&A.ent[ps], kEmpty, e);
                fresh += (c == kEmpty);
            }
            if (c == kEmpty || c == e) {
                atomicAdd(&A.cnt[ps], 1u);
                act = false;
            } else {
                ps = (ps + 1) & (kPartSlots - 1);
            }
        }
        // still active: no slot within the probe limit
        spill_push(sp, ctr, act, act ? frame_key(cb, e, g.fx, g.fy) : 0, 1u);
    };
    // One entry at its first two slots; true when it has to walk further.
    auto first_two = [&](uint32_t e, uint32_t h, uint32_t c0, uint32_t c1) {
        uint32_t s = h, c = c0;
        if (c != e && c != kEmpty) {
            s = (h + 1) & (kPartSlots - 1);
            c = c1;
        }
        if (c != e && c != kEmpty) return true;
        if (c == kEmpty) {
            c = atomicCAS(&A.ent[s], kEmpty, e);
            if (c == kEmpty) {
                ++fresh;
                c = e;
            }
        }
        if (c != e) return true;
        atomicAdd(&A.cnt[s], 1u);
        return false;
    };
    // Batches of STEP entries, list by list: (li, q0) is uniform across the
    // workgroup, and the next batch's loads are in flight while this one is
    // added.
    constexpr uint32_t STEP = AGG_THREADS * FAGG_BATCH;
    uint32_t li = 0, q0 = 0;
    while (li < kBinRep && L.size_of(li) == 0) ++li;
    auto fetch = [&](uint32_t bl, uint32_t bq, uint32_t (&k)[FAGG_BATCH]) {
        const uint32_t n_l = L.size_of(bl);
        const uint32_t* src = L.src + bl * L.lstride;
#pragma unroll
        for (int u = 0; u < FAGG_BATCH; ++u) {
            const uint32_t q = bq + u * AGG_THREADS + threadIdx.x;
            k[u] = __builtin_nontemporal_load(src + min(q, n_l - 1));
        }
    };
    uint32_t k[FAGG_BATCH], next[FAGG_BATCH];
    if (li < kBinRep) fetch(li, q0, next);
    while (li < kBinRep) {
        const uint32_t n_l = L.size_of(li), bq = q0;
#pragma unroll
        for (int u = 0; u < FAGG_BATCH; ++u) k[u] = next[u];
        q0 += STEP;
        if (q0 >= n_l) {
            q0 = 0;
            do ++li;
            while (li < kBinRep && L.size_of(li) == 0);
        }
        if (li < kBinRep) fetch(li, q0, next);
        // the first two slots of every entry read together
        uint32_t hs[FAGG_BATCH], c0[FAGG_BATCH], c1[FAGG_BATCH];
#pragma unroll
        for (int u = 0; u < FAGG_BATCH; ++u) {
            hs[u] = frame_home(k[u]) & (kPartSlots - 1);
            c0[u] = __hip_atomic_load(&A.ent[hs[u]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            c1[u] = __hip_atomic_load(&A.ent[(hs[u] + 1) & (kPartSlots - 1)], __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
        }
#pragma unroll
        for (int u = 0; u < FAGG_BATCH; ++u) {
            const bool have = bq + u * AGG_THREADS + threadIdx.x < n_l;
            const bool defer = have && first_two(k[u], hs[u], c0[u], c1[u]);
            const uint64_t b = __ballot(defer);
            if (b) {  // uniform across the wave
                if (defer) ring[(tail + (uint32_t)__popcll(b & lt)) & (AGG_RING - 1)] = k[u];
                tail += (uint32_t)__popcll(b);
                if (tail - head >= 64) {
                    // the ring's entries are written by other lanes of this wave
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    drain();
                }
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    while (tail != head) drain();
    __syncthreads();
    // the rings are free now: their first 512 bytes take the census bits
    uint64_t* wbits = reinterpret_cast<uint64_t*>(&A.ring[0][0]);
    uint32_t occ = 0, sum = 0;  // (a table holds fewer than 2^32 points)
    uint32_t sig = 0;           // significant slots, for the threshold's scan (cn)
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const uint32_t sl = u * AGG_THREADS + threadIdx.x;
        const uint32_t e = A.ent[sl], c = A.cnt[sl];
        if (cen.img) {
            // the final update writes the slice image (the table itself only
            // if keys spill afterwards: k_image_to_table)
            cen.img[(p << kPartLog2) + sl] = make_uint2(e, c);
        } else if ((L.total && e != kEmpty && e != kAlien) || (whole && e == kEmpty)) {
            // (whole: a table not filled yet takes every slot, the empty ones too)
            Slot v;
            v.key = e != kEmpty ? frame_key(cb, e, g.fx, g.fy) : kEmptyKey;
            v.count = c;
            v.aux = kNotSignificant;
            part[sl] = v;
        }
        if (cn.partials) sig += e != kEmpty && c >= cn.tau;  // (keys outside the frame too)
        if (cen.rec) {
            // the wave's 64 slots u * AGG_THREADS + 64 w + lane form word 8 u + w
            occ += e != kEmpty;
            sum += e != kEmpty ? c : 0u;
            const uint64_t b = __ballot(e != kEmpty && c >= cen.tau);
            if (lane_id() == 0) wbits[u * (AGG_THREADS / 64) + (threadIdx.x >> 6)] = b;
        }
    }
    add_fresh(ctr, fresh);
    if (cen.rec) {
        __syncthreads();
        if (threadIdx.x < 64) {
            const uint64_t b = wbits[threadIdx.x];
            const uint32_t lo = (uint32_t)__popc((uint32_t)b), c = (uint32_t)__popcll(b);
            uint32_t inc = c;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t t = __shfl_up(inc, o);
                if (lane_id() >= (uint32_t)o) inc += t;
            }
            uint2* r = cen.rec + (p << 7) + 2 * threadIdx.x;
            r[0] = make_uint2((uint32_t)b, inc - c);
            r[1] = make_uint2((uint32_t)(b >> 32), inc - c + lo);
            if (threadIdx.x == 63) cen.ptotal[p] = inc;
        }
        // the partition's occupied slots and count sum beside its total: the
        // scan of the totals adds them up (atomics per workgroup on two
        // counter words made this kernel slower)
        const uint32_t o = block_total32(occ), c = block_total32(sum);
        if (threadIdx.x == 0) {
            cen.ptotal[parts + p] = o;
            cen.ptotal[2 * parts + p] = c;
        }
    }
    // the threshold's counting pass (AggCount), as in k_aggregate
    if (cn.partials) block_count_add32(cn.partials + (p >> cn.blk_shift), sig);
}

// Fallback: every entry held in the coarse lists goes straight to the table.
__global__ void k_drain_bins_f(const uint32_t* bin1, uint64_t cap1, const uint32_t* cursor1, Slot* tab, const Geo g,
                               SpillBuf sp, unsigned long long* ctr) {
    const uint64_t total = (uint64_t)kBinRep * kFrameCoarse * cap1;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t n_round = (total + 63) / 64 * 64;
    uint32_t fresh = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_round; i += stride) {
        int r = ADD_FOUND;
        uint64_t k = 0;
        if (i < total) {
            const uint64_t b = i / cap1, q = i % cap1;
            if (q < min((uint64_t)cursor1[b], cap1)) {
                k = frame_key((uint32_t)(b % kFrameCoarse), bin1[i], g.fx, g.fy);
                r = table_add(tab, g, k, 1u);
                fresh += (r == ADD_NEW);
            }
        }
        spill_push(sp, ctr, r == ADD_FULL, k, 1u);
    }
    add_fresh(ctr, fresh);
}

// Tile bounding box of points [0, n) over the points with a valid tile: each
// workgroup writes {min bx, max bx, min by, max by} (biased) of its points to
// part[4 * blockIdx.x ...], then k_bbox_merge folds the parts into out.
constexpr int kBboxBlocks = 256;
static_assert(kBboxWords == 4 + 4 * kBboxBlocks, "box scratch holds one part per workgroup");

template <typename T>
__global__ __launch_bounds__(256) void k_key_bbox(const T* __restrict__ pts, int64_t n, double scale, uint32_t* part) {
    __shared__ uint32_t red[4][4];
    uint32_t v[4] = {~0u, 0u, ~0u, 0u};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double x, y;
        load_point(pts, i, x, y);
        uint64_t key;
        if (tile_key(x, y, scale, key)) {
            const uint32_t bx = (uint32_t)(key >> 32), by = (uint32_t)key;
            v[0] = min(v[0], bx);
            v[1] = max(v[1], bx);
            v[2] = min(v[2], by);
            v[3] = max(v[3], by);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        v[0] = min(v[0], (uint32_t)__shfl_xor((int)v[0], o));
        v[1] = max(v[1], (uint32_t)__shfl_xor((int)v[1], o));
        v[2] = min(v[2], (uint32_t)__shfl_xor((int)v[2], o));
        v[3] = max(v[3], (uint32_t)__shfl_xor((int)v[3], o));
    }
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0)
        for (int c = 0; c < 4; ++c) red[w][c] = v[c];
    __syncthreads();
    if (threadIdx.x < 4) {
        const int c = threadIdx.x;
        uint32_t r = red[0][c];
        for (int q = 1; q < 4; ++q) r = (c & 1) ? max(r, red[q][c]) : min(r, red[q][c]);
        part[4 * blockIdx.x + c] = r;
    }
}

__global__ void k_bbox_merge(const uint32_t* part, int parts, uint32_t* out) {
    if (threadIdx.x < 4) {
        const int c = threadIdx.x;
        uint32_t r = (c & 1) ? 0u : ~0u;
        for (int b = 0; b < parts; ++b) r = (c & 1) ? max(r, part[4 * b + c]) : min(r, part[4 * b + c]);
        out[c] = r;
    }
}

// ---- binned counting for batches ----------------------------------------------
//
// The same two binning levels and LDS update, over every job of a batch at
// once.  Each job owns 2^(p_log2 - cshift) coarse buckets (a coarse bucket
// names its job) and its partitions in the arena; a work tile of level 1 holds
// kBinTile points of one job.  Persistent grids read every size from Dims.

__global__ __launch_bounds__(BIN_THREADS) void k_bbin_points(JobView jv, const uint32_t* tile_prefix, uint64_t* bin1,
                                                             uint32_t* cursor1, Slot* tab) {
    __shared__ BinScratch S;
    const uint32_t tiles = jv.dims->tiles, njobs = jv.dims->njobs;
    const uint64_t cap1 = jv.dims->cap1;
    const SpillBuf none{nullptr, nullptr, 0};
    const TileRange tr = tile_range(tile_prefix, njobs, tiles);
    uint32_t job = tr.job;
    for (uint32_t t = tr.lo; t < tr.hi; ++t) {
        job = advance_job(tile_prefix, job, t);
        const JobInfo& J = jv.jobs[job];
        const Geo g = job_geo(J);  // batch jobs are two-dimensional
        const uint32_t top = g.p_log2 - J.cshift;  // coarse bits of the hash
        const uint32_t nb = 1u << top;
        for (uint32_t b = threadIdx.x; b < nb; b += BIN_THREADS) S.hist[b] = 0;
        __syncthreads();
        const int64_t base = (int64_t)(t - J.first_tile) * kBinTile + threadIdx.x;
        uint64_t key[BIN_ITEMS];
        uint16_t bucket[BIN_ITEMS];
        uint32_t valid = 0;
        bool bad = false;
        // all loads first, indices clamped (a tile holds at least one point of
        // its job) and results masked, so that they are in flight together
        double x[BIN_ITEMS], y[BIN_ITEMS];
        if (J.dtype == 1) {
#pragma unroll
            for (int j = 0; j < BIN_ITEMS; ++j)
                load_point(static_cast<const float*>(J.pts), min(base + (int64_t)j * BIN_THREADS, J.n - 1), x[j], y[j]);
        } else {
#pragma unroll
            for (int j = 0; j < BIN_ITEMS; ++j)
                load_point(static_cast<const double*>(J.pts), min(base + (int64_t)j * BIN_THREADS, J.n - 1), x[j],
                           y[j]);
        }
#pragma unroll
        for (int j = 0; j < BIN_ITEMS; ++j) {
            const int64_t i = base + (int64_t)j * BIN_THREADS;
            key[j] = 0;
            bucket[j] = 0;
            if (i < J.n) {
                if (tile_key(x[j], y[j], J.scale, key[j])) {
                    valid |= 1u << j;
                    bucket[j] = (uint16_t)bucket_of(key[j], top, nb, false);
                } else {
                    bad = true;
                }
            }
        }
        unsigned long long* jc = jv.job_ctr + (uint64_t)job * kCounterWords;
        if (bad) atomicOr(&jc[C_ERROR], (unsigned long long)kErrRange);
        uint32_t fresh = 0;
        bin_tile<false>(S, key, bucket, valid, nb, top, bin1 + (uint64_t)J.cbase * cap1, cap1, cap1, cursor1 + J.cbase,
                 tab + J.slot_base, g, none, jc, fresh);
        __syncthreads();  // S is reused by the next tile
    }
}

__global__ __launch_bounds__(BIN_THREADS) void k_bbin_keys(JobView jv, const uint32_t* cjob, const uint64_t* bin1,
                                                           const uint32_t* cursor1, uint64_t* bin2,
                                                           uint32_t* cursor2, Slot* tab) {
    __shared__ BinScratch S;
    const uint64_t cap1 = jv.dims->cap1;
    const uint32_t segs = jv.dims->segs;
    const uint32_t ncoarse = jv.dims->ncoarse;
    const uint64_t work = (uint64_t)ncoarse * segs;
    const SpillBuf none{nullptr, nullptr, 0};
    // segment-major: workgroups running together take different coarse
    // buckets, so their cursor updates land on different partitions' lines
    for (uint64_t w = blockIdx.x; w < work; w += gridDim.x) {
        const uint32_t c = (uint32_t)(w % ncoarse);
        const uint32_t seg = (uint32_t)(w / ncoarse);
        const uint64_t cnt = min((uint64_t)cursor1[c], cap1);
        const uint64_t start = (uint64_t)seg * kBinTile;
        if (start >= cnt) continue;  // uniform across the workgroup
        const uint32_t job = cjob[c];
        const JobInfo& J = jv.jobs[job];
        const Geo g = job_geo(J);  // batch jobs are two-dimensional
        const uint32_t nb = 1u << J.cshift;
        for (uint32_t b = threadIdx.x; b < nb; b += BIN_THREADS) S.hist[b] = 0;
        __syncthreads();
        uint64_t key[BIN_ITEMS];
        uint16_t bucket[BIN_ITEMS];
        uint32_t valid = 0;
        const uint64_t* src = bin1 + (uint64_t)c * cap1;
        // all loads first (indices clamped below cnt > start, results masked)
#pragma unroll
        for (int j = 0; j < BIN_ITEMS; ++j)
            key[j] = __builtin_nontemporal_load(src + min(start + (uint64_t)j * BIN_THREADS + threadIdx.x, cnt - 1));
#pragma unroll
        for (int j = 0; j < BIN_ITEMS; ++j) {
            const uint64_t i = start + (uint64_t)j * BIN_THREADS + threadIdx.x;
            bucket[j] = 0;
            if (i < cnt) {
                bucket[j] = (uint16_t)bucket_of(key[j], g.p_log2, nb, false);
                valid |= 1u << j;
            } else {
                key[j] = 0;
            }
        }
        uint32_t fresh = 0;
        const uint64_t first = (uint64_t)(c - J.cbase) << J.cshift;  // job-local partition
        bin_tile<false>(S, key, bucket, valid, nb, g.p_log2, bin2 + J.bin2_base + first * J.cap2, J.cap2, J.cap2,
                 cursor2 + J.part_base + first, tab + J.slot_base, g, none,
                 jv.job_ctr + (uint64_t)job * kCounterWords, fresh);
        __syncthreads();
    }
}

__global__ __launch_bounds__(AGG_THREADS) void k_bagg(JobView jv, const uint64_t* __restrict__ bin2,
                                                      const uint32_t* cursor2, Slot* tab) {
    __shared__ uint64_t lkey[kPartSlots];
    __shared__ uint32_t lcnt[kPartSlots];
    const uint64_t parts = jv.dims->slots >> kPartLog2;
    const SpillBuf none{nullptr, nullptr, 0};
    for (uint64_t p = blockIdx.x; p < parts; p += gridDim.x) {
        const JobInfo& J = jv.jobs[jv.part_job[p]];
        const PartLists<1> L(bin2 + J.bin2_base + (p - J.part_base) * J.cap2, 0, cursor2 + p, 0, J.cap2);
        // keys past a bucket's capacity were added to the table directly, so
        // the slice is read
        if (L.total == 0) continue;  // uniform across the workgroup
        uint32_t fresh = 0;
        aggregate_partition(L, tab + (p << kPartLog2), true, lkey, lcnt, none,
                            jv.job_ctr + (uint64_t)jv.part_job[p] * kCounterWords, fresh);
        __syncthreads();
    }
}

// Fallback: every key held in the coarse buckets goes straight to the table.
__global__ void k_drain_bins(const uint64_t* bin1, uint64_t cap1, const uint32_t* cursor1, Slot* tab, const Geo g,
                             SpillBuf sp, unsigned long long* ctr) {
    const uint64_t total = (uint64_t)kBinRep * kCoarse * cap1;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t n_round = (total + 63) / 64 * 64;
    uint32_t fresh = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_round; i += stride) {
        int r = ADD_FOUND;
        uint64_t k = 0;
        if (i < total) {
            const uint64_t b = i / cap1, q = i % cap1;
            if (q < min((uint64_t)cursor1[b], cap1)) {
                k = bin1[i];
                r = table_add(tab, g, k, 1u);
                fresh += (r == ADD_NEW);
            }
        }
        spill_push(sp, ctr, r == ADD_FULL, k, 1u);
    }
    add_fresh(ctr, fresh);
}

__global__ void k_fill_words(uint64_t* p, uint64_t n, uint64_t v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_snapshot_keys(unsigned long long* ctr) {
    if (threadIdx.x == 0) ctr[C_TABLE_KEYS] = ctr[C_INSERTED];
}

__global__ void k_zero_u32(uint32_t* p, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ---------------------------------------------------------------- scans ----
//
// Stream compaction in three passes over a fixed grid of kScanBlocks
// workgroups.  Workgroup b owns a contiguous range of indices, cut into tiles
// of SCAN_TILE = 256 threads x 16 items (thread t takes tile offsets
// t + 256 j).  Pass 1 counts flagged indices per range, pass 2 scans the
// kScanBlocks partial counts, pass 3 recomputes the flags and writes every
// flagged index to its position.  Positions follow index order, so the
// compaction is stable.

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;
constexpr int SCAN_WAVES = SCAN_THREADS / 64;

__device__ __forceinline__ void block_range(uint64_t N, uint64_t& lo, uint64_t& hi) {
    uint64_t per = (N + gridDim.x - 1) / gridDim.x;
    per = (per + SCAN_TILE - 1) / SCAN_TILE * SCAN_TILE;
    lo = (uint64_t)blockIdx.x * per;
    hi = lo + per;
    if (lo > N) lo = N;
    if (hi > N) hi = N;
}

// Sum of a per-thread value over the workgroup (SCAN_THREADS threads).
template <typename V>
__device__ __forceinline__ V block_sum(V v, V* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if (lane_id() == 0) red[w] = v;
    __syncthreads();
    V t = 0;
    for (int i = 0; i < SCAN_WAVES; ++i) t += red[i];
    return t;
}

// Positions of the flagged items of one tile.  `bits` holds this lane's flags
// (bit j for item j).  Returns the tile's flagged count; pos_j gives item j's
// exclusive position within the tile (only meaningful when bit j is set).
struct TileScratch {
    uint32_t cnt[SCAN_ITEMS][SCAN_WAVES];
    uint32_t total;
};

__device__ __forceinline__ uint32_t tile_positions(uint32_t bits, uint32_t (&pos)[SCAN_ITEMS],
                                                   TileScratch& ts) {
    const int w = threadIdx.x >> 6;
    const uint64_t lt = lanemask_lt();
    uint32_t within[SCAN_ITEMS];
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const uint64_t b = __ballot((bits >> j) & 1u);
        within[j] = __popcll(b & lt);
        if (lane_id() == 0) ts.cnt[j][w] = __popcll(b);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int j = 0; j < SCAN_ITEMS; ++j)
            for (int q = 0; q < SCAN_WAVES; ++q) {
                const uint32_t c = ts.cnt[j][q];
                ts.cnt[j][q] = run;
                run += c;
            }
        ts.total = run;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) pos[j] = ts.cnt[j][w] + within[j];
    const uint32_t total = ts.total;
    __syncthreads();  // scratch is reused by the next tile
    return total;
}

// Exclusive scan of kScanBlocks partial counts by one workgroup of 1024
// threads; the total goes to *total_out.
__global__ __launch_bounds__(1024) void k_scan_partials(uint32_t* partials, unsigned long long* total_out) {
    constexpr int PER = kScanBlocks / 1024;
    __shared__ uint32_t wsum[16];
    uint32_t v[PER];
    uint32_t local = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        v[k] = partials[threadIdx.x * PER + k];
        local += v[k];
    }
    // inclusive scan of `local` across the workgroup
    uint32_t inc = local;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(inc, off);
        if (lane_id() >= off) inc += o;
    }
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) wsum[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int i = 0; i < 16; ++i) {
            const uint32_t c = wsum[i];
            wsum[i] = run;
            run += c;
        }
        *total_out = run;
    }
    __syncthreads();
    uint32_t ex = wsum[w] + inc - local;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        partials[threadIdx.x * PER + k] = ex;
        ex += v[k];
    }
}

// ---- significance scan (Algorithm 1: drop tiles with fewer than tau points) --
//
// Scan tiles are 4096 slots, the size of a table partition, so with several
// jobs every scan tile belongs to exactly one job (its tau, its counters).

__device__ __forceinline__ uint32_t job_of_slot(const JobView& jv, bool multi, uint64_t slot) {
    return multi ? jv.part_job[slot >> kPartLog2] : 0u;
}

// Key and count of the slots of one scan tile (t0 < hi).  The loads are
// unconditional -- items past hi re-read slot hi - 1 and are then marked
// empty -- so that all of them are in flight together.
__device__ __forceinline__ void load_slots(const Slot* tab, uint64_t t0, uint64_t hi, uint64_t (&key)[SCAN_ITEMS],
                                           uint32_t (&cnt)[SCAN_ITEMS]) {
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const uint64_t i = min(t0 + (uint64_t)j * SCAN_THREADS + threadIdx.x, hi - 1);
        key[j] = tab[i].key;
        cnt[j] = tab[i].count;
    }
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j)
        if (t0 + (uint64_t)j * SCAN_THREADS + threadIdx.x >= hi) key[j] = kEmptyKey;
}

// Marks of the 2x2 post-step for the slots of one scan tile: aux ==
// kSquareKeep (set by k_square_part) makes a slot significant whatever its
// count.  Items past hi read slot hi - 1; the caller masks them by key.
__device__ __forceinline__ void load_square_marks(const Slot* tab, uint64_t t0, uint64_t hi,
                                                  bool (&mark)[SCAN_ITEMS]) {
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j)
        mark[j] = tab[min(t0 + (uint64_t)j * SCAN_THREADS + threadIdx.x, hi - 1)].aux == kSquareKeep;
}

template <bool SQUARE>
__global__ __launch_bounds__(SCAN_THREADS) void k_threshold_count(const Slot* tab, JobView jv, uint32_t* partials,
                                                                  unsigned long long* ctr) {
    __shared__ unsigned long long red[SCAN_WAVES];
    const uint64_t N = jv.dims->slots;
    const bool multi = jv.part_job != nullptr;
    uint64_t lo, hi;
    block_range(N, lo, hi);
    unsigned long long sig = 0, occ = 0, sum = 0;
    for (uint64_t t0 = lo; t0 < hi; t0 += SCAN_TILE) {
        const uint32_t job = job_of_slot(jv, multi, t0);
        const uint32_t tau = jv.jobs[job].tau;
        unsigned long long occ_t = 0, sum_t = 0;
        uint64_t key[SCAN_ITEMS];
        uint32_t cnt[SCAN_ITEMS];
        bool mark[SCAN_ITEMS] = {};
        load_slots(tab, t0, hi, key, cnt);
        if (SQUARE) load_square_marks(tab, t0, hi, mark);
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            if (key[j] != kEmptyKey) {
                occ_t += 1;
                sum_t += cnt[j];
                sig += (cnt[j] >= tau || mark[j]);
            }
        }
        occ += occ_t;
        sum += sum_t;
        if (multi) {
            occ_t = block_sum(occ_t, red);
            sum_t = block_sum(sum_t, red);
            if (threadIdx.x == 0) {
                if (occ_t) atomicAdd(&jv.job_ctr[(uint64_t)job * kCounterWords + C_DISTINCT], occ_t);
                if (sum_t) atomicAdd(&jv.job_ctr[(uint64_t)job * kCounterWords + C_SUM], sum_t);
            }
        }
    }
    sig = block_sum(sig, red);
    occ = block_sum(occ, red);
    sum = block_sum(sum, red);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = (uint32_t)sig;
        if (occ) atomicAdd(&ctr[C_DISTINCT], occ);
        if (sum) atomicAdd(&ctr[C_SUM], sum);
    }
}

// TOTALS (one job whose final update did the counting pass): the occupied
// slots and their count sum go to ctr[C_DISTINCT] and ctr[C_SUM] here.
template <bool SQUARE, bool TOTALS = false>
__global__ __launch_bounds__(SCAN_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_threshold_scatter(Slot* tab, JobView jv, const uint32_t* offsets,
                                                                    uint64_t* s_key, uint32_t* s_count,
                                                                    uint32_t* size, unsigned long long* ctr) {
    __shared__ TileScratch ts;
    __shared__ unsigned long long red[SCAN_WAVES];
    const uint64_t N = jv.dims->slots;
    const bool multi = jv.part_job != nullptr;
    uint64_t lo, hi;
    block_range(N, lo, hi);
    uint64_t run = offsets[blockIdx.x];
    uint32_t occ = 0, sum = 0;  // (a table holds fewer than 2^32 points)
    for (uint64_t t0 = lo; t0 < hi; t0 += SCAN_TILE) {
        const uint32_t job = job_of_slot(jv, multi, t0);
        const uint32_t tau = jv.jobs[job].tau;
        uint32_t bits = 0;
        uint64_t key[SCAN_ITEMS];
        uint32_t cnt[SCAN_ITEMS];
        bool mark[SCAN_ITEMS] = {};
        load_slots(tab, t0, hi, key, cnt);
        if (SQUARE) load_square_marks(tab, t0, hi, mark);
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            if (key[j] != kEmptyKey && (cnt[j] >= tau || mark[j])) bits |= 1u << j;
            if (TOTALS && key[j] != kEmptyKey) {
                occ += 1;
                sum += cnt[j];
            }
        }
        uint32_t pos[SCAN_ITEMS];
        const uint32_t total = tile_positions(bits, pos, ts);
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            const uint64_t i = t0 + (uint64_t)j * SCAN_THREADS + threadIdx.x;
            if (key[j] == kEmptyKey) continue;
            if (bits & (1u << j)) {
                const uint64_t p = run + pos[j];
                s_key[p] = key[j];
                s_count[p] = cnt[j];
                size[p] = 0;
                if (multi) jv.s_job[p] = job;
                tab[i].aux = (uint32_t)p;
            }  // other slots hold kNotSignificant (fill and update passes write it; the 2x2 pass marks only
               // slots that become significant here)
        }
        run += total;
    }
    if (TOTALS) {
        const unsigned long long o = block_sum((unsigned long long)occ, red);
        const unsigned long long c = block_sum((unsigned long long)sum, red);
        if (threadIdx.x == 0) {
            if (o) atomicAdd(&ctr[C_DISTINCT], o);
            if (c) atomicAdd(&ctr[C_SUM], c);
        }
    }
}

// ---- export of all (key, count) pairs, for checking the contraction ---------

__global__ __launch_bounds__(SCAN_THREADS) void k_export_count(const Slot* tab, uint64_t cap, uint32_t* partials,
                                                               unsigned long long* ctr) {
    __shared__ unsigned long long red[SCAN_WAVES];
    uint64_t lo, hi;
    block_range(cap, lo, hi);
    unsigned long long occ = 0;
    for (uint64_t t0 = lo; t0 < hi; t0 += SCAN_TILE)
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            const uint64_t i = t0 + (uint64_t)j * SCAN_THREADS + threadIdx.x;
            if (i < hi && tab[i].key != kEmptyKey) occ += 1;
        }
    occ = block_sum(occ, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = (uint32_t)occ;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_export_scatter(const Slot* tab, uint64_t cap,
                                                                 const uint32_t* offsets, uint64_t* keys,
                                                                 uint32_t* counts, uint64_t out_cap) {
    __shared__ TileScratch ts;
    uint64_t lo, hi;
    block_range(cap, lo, hi);
    uint64_t run = offsets[blockIdx.x];
    for (uint64_t t0 = lo; t0 < hi; t0 += SCAN_TILE) {
        uint32_t bits = 0;
        uint64_t key[SCAN_ITEMS];
        uint32_t cnt[SCAN_ITEMS];
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            const uint64_t i = t0 + (uint64_t)j * SCAN_THREADS + threadIdx.x;
            key[j] = kEmptyKey;
            cnt[j] = 0;
            if (i < hi) {
                const Slot s = tab[i];
                key[j] = s.key;
                cnt[j] = s.count;
                if (s.key != kEmptyKey) bits |= 1u << j;
            }
        }
        uint32_t pos[SCAN_ITEMS];
        const uint32_t total = tile_positions(bits, pos, ts);
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            if (!(bits & (1u << j))) continue;
            const uint64_t p = run + pos[j];
            if (p < out_cap) {
                keys[p] = key[j];
                counts[p] = cnt[j];
            }
        }
        run += total;
    }
}

// ---------------------------------------------------------- agglomeration ---
//
// Connected components of the significant tiles under 8-adjacency, as a
// union-find forest over compact indices in which every parent has a smaller
// tile key than its child.  The root of a component is then its smallest
// tile, so the label comes for free.  Four passes:
//   link  : each tile looks up its four backward neighbours (x-1, y-1),
//           (x-1, y), (x-1, y+1), (x, y-1) -- the ones with smaller keys -- and
//           points at the smallest significant one; it also records them.
//           Forward neighbours are covered because each forward edge is a
//           backward edge of the other tile.
//   jump  : every tile replaces its parent by its root.
//   merge : for every recorded neighbour in a different tree, the two trees
//           are united with a device-scope compare-and-swap hook.
//   finish: every tile takes its final root; component sizes and roots are
//           counted.
// Link, jump and finish write only words no other thread hooks in the same
// kernel, so they use ordinary cached accesses; merge, where concurrent hooks
// happen, reads parents at device scope.

constexpr uint32_t kNoNeighbour = 0xFFFFFFFFu;

// Walk bound: every chain is far shorter, so hitting it means corrupt state;
// the walk then stops and raises kErrInternal instead of spinning.
constexpr uint32_t kUfMaxSteps = 1u << 24;

// Root walk with path halving, ordinary loads and stores.  Only for kernels
// in which no thread hooks (parents only move to ancestors).
__device__ __forceinline__ uint32_t uf_root_cached(uint32_t* parent, uint32_t x, uint32_t s, bool& bad) {
    for (uint32_t it = 0; it < kUfMaxSteps; ++it) {
        const uint32_t p = parent[x];
        if (p >= s) break;
        if (p == x) return x;
        const uint32_t gp = parent[p];
        if (gp >= s) break;
        if (gp == p) return p;
        parent[x] = gp;
        x = gp;
    }
    bad = true;
    return x;
}

// Root walk at device scope, for the merge kernel where hooks run concurrently.
__device__ __forceinline__ uint32_t uf_root(uint32_t* parent, uint32_t x, uint32_t s, bool& bad) {
    for (uint32_t it = 0; it < kUfMaxSteps; ++it) {
        const uint32_t p = ld_relaxed(parent + x);
        if (p >= s) break;
        if (p == x) return x;
        x = p;
    }
    bad = true;
    return x;
}

// Hooks the trees of a and b together: the root with the larger key goes
// under the other root.  A failed compare-and-swap continues from the parent
// value it returned, which has a strictly smaller key.
__device__ __forceinline__ void uf_unite(uint32_t* parent, const uint64_t* key, uint32_t a, uint32_t b, uint32_t s,
                                         bool& bad) {
    a = uf_root(parent, a, s, bad);
    b = uf_root(parent, b, s, bad);
    for (uint32_t it = 0; it < kUfMaxSteps; ++it) {
        if (bad || a == b) return;
        if (key[a] < key[b]) {
            const uint32_t t = a;
            a = b;
            b = t;
        }
        const uint32_t old = atomicCAS(parent + a, a, b);
        if (old == a) return;
        if (old >= s) {
            bad = true;
            return;
        }
        a = uf_root(parent, old, s, bad);
        b = uf_root(parent, b, s, bad);
    }
    bad = true;
}

// 2x2 post-step (Section 3.6, for points spread over the tiles around a grid
// corner): a slot below tau whose tile lies in a 2x2 square of tiles that hold
// at least tau points together gets aux = kSquareKeep, which the threshold
// scan then counts as significant.  One workgroup per table partition with the
// slice's keys and counts in LDS; the counts of the eight surrounding tiles are
// read there when they share the partition, else from the device table.  Only
// counts are read, and only aux is written, so the order of the partitions
// does not matter.  In a batch each partition belongs to the job part_job
// names, whose table starts at its slot_base.
constexpr int SQUARE_THREADS = 512;
constexpr uint32_t SQUARE_RING = 128;  // light slots queued per wave (at most 127 wait)

// The light tiles of a slice are queued in a ring of their wave's and
// checked 64 at a time, one per lane (a slice-wide list would take 8 KB of
// LDS and leave room for two workgroups per CU instead of three; six waves
// per SIMD, so that three fit the registers too).
__global__ __launch_bounds__(SQUARE_THREADS, 6) void k_square_part(Slot* tab, JobView jv) {
    __shared__ uint64_t lkey[kPartSlots];
    __shared__ uint32_t lcnt[kPartSlots];
    __shared__ uint16_t ring[SQUARE_THREADS / 64][SQUARE_RING];
    const bool multi = jv.part_job != nullptr;
    const uint64_t parts = multi ? jv.dims->slots >> kPartLog2 : (jv.jobs[0].cap + kPartSlots - 1) >> kPartLog2;
    const uint32_t w = threadIdx.x >> 6, lane = lane_id();
    const uint64_t lt = lanemask_lt();
    uint16_t* rw = ring[w];
    for (uint64_t p = blockIdx.x; p < parts; p += gridDim.x) {
        // the partition's job: its table starts at slot_base (a whole number
        // of partitions), so job-local partition jp holds slots base.. of it
        const JobInfo& J = jv.jobs[multi ? jv.part_job[p] : 0u];
        const uint32_t tau = J.tau;
        const Geo g = job_geo(J);  // the step is two-dimensional
        const uint32_t psize = (uint32_t)min<uint64_t>(J.cap, kPartSlots);
        Slot* jt = tab + J.slot_base;
        const uint64_t jp = p - (J.slot_base >> kPartLog2);
        const uint64_t base = jp << kPartLog2;
        __syncthreads();  // the previous partition's slice is no longer read
        for (uint32_t u = threadIdx.x; u < psize; u += SQUARE_THREADS) {
            const Slot v = jt[base + u];
            lkey[u] = v.key;
            lcnt[u] = v.count;
        }
        __syncthreads();
        // marks slot u when a 2x2 square holding its tile reaches tau
        auto check = [&](uint32_t u) {
            const uint32_t bx = (uint32_t)(lkey[u] >> 32);
            const uint32_t by = (uint32_t)lkey[u];
            // the eight surrounding tiles, q = 3 (dx + 1) + (dy + 1) without
            // the centre: the home slots of those in other partitions are
            // loaded together first (key and count in one 16-byte load), and
            // only a key that is neither there nor an empty slot walks on
            uint64_t nk[9], pos[9];
            bool in[9], remote[9];
            Slot hv[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int64_t x = (int64_t)bx + (q / 3 - 1), y = (int64_t)by + (q % 3 - 1);
                in[q] = q != 4 && x >= 2 && x <= 0xFFFFFFFEll && y >= 2 && y <= 0xFFFFFFFEll;
                nk[q] = ((uint64_t)(uint32_t)x << 32) | (uint32_t)y;
                pos[q] = in[q] ? home_slot(nk[q], g) : 0;
                remote[q] = in[q] && (pos[q] >> kPartLog2) != jp;
                if (remote[q]) hv[q] = jt[pos[q]];
            }
            uint64_t c[3][3];  // counts of the tiles (bx + dx, by + dy), [dx + 1][dy + 1]
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                uint64_t n_cnt = 0;
                if (q == 4) {
                    n_cnt = lcnt[u];
                } else if (in[q] && !remote[q]) {
                    uint32_t lp = (uint32_t)(pos[q] - base);
                    for (uint32_t step = 0; step < kMaxProbe; ++step) {
                        const uint64_t cur = lkey[lp];
                        if (cur == nk[q]) {
                            n_cnt = lcnt[lp];
                            break;
                        }
                        if (cur == kEmptyKey) break;
                        lp = (lp + 1) & (psize - 1);
                    }
                } else if (remote[q]) {
                    if (hv[q].key == nk[q]) {
                        n_cnt = hv[q].count;
                    } else if (hv[q].key != kEmptyKey) {
                        // the rest of the probe sequence, as table_find walks it
                        uint64_t at = pos[q];
                        for (uint32_t step = 1; step < kMaxProbe; ++step) {
                            at = next_slot(at, g);
                            const Slot v = jt[at];
                            if (v.key == nk[q]) {
                                n_cnt = v.count;
                                break;
                            }
                            if (v.key == kEmptyKey) break;
                        }
                    }
                }
                c[q / 3][q % 3] = n_cnt;
            }
            bool keep = false;
#pragma unroll
            for (int a = 0; a <= 1; ++a)
#pragma unroll
                for (int b = 0; b <= 1; ++b)
                    keep |= c[a][b] + c[a + 1][b] + c[a][b + 1] + c[a + 1][b + 1] >= (uint64_t)tau;
            if (keep) jt[base + u].aux = kSquareKeep;
        };
        // the wave's chunks of 64 slots, every eighth chunk of the slice
        // (uniform across the wave, as are head and tail)
        uint32_t head = 0, tail = 0;
        for (uint32_t u0 = w * 64; u0 < psize; u0 += SQUARE_THREADS) {
            const uint32_t u = u0 + lane;
            const bool light = u < psize && lkey[u] != kEmptyKey && lcnt[u] < tau;
            const uint64_t b = __ballot(light);
            if (light) rw[(tail + (uint32_t)__popcll(b & lt)) & (SQUARE_RING - 1)] = (uint16_t)u;
            tail += (uint32_t)__popcll(b);
            if (tail - head >= 64) {
                // the ring's entries are written by other lanes of this wave
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                check(rw[(head + lane) & (SQUARE_RING - 1)]);
                head += 64;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (tail != head && lane < tail - head) check(rw[(head + lane) & (SQUARE_RING - 1)]);
    }
}

// Link pass: parent = the significant backward neighbour with the smallest
// key (or the tile itself), nbr = the compact indices of all significant
// backward neighbours ((x-1, y-1), (x-1, y), (x-1, y+1), (x, y-1); with the
// forward ones seen from the other side they cover all eight).  One
// workgroup per table partition: the slice is read into LDS once, and with
// super-tile placement most neighbours share the tile's partition and are
// probed there; only the others are probed in the device table.
//
// GENERAL: the offsets come from the rounds of `grp` (a larger or Manhattan
// neighbourhood, or the 3-D one with D3) instead of the four fixed ones; each
// round writes its own record of four words, and the parent (the smallest-key
// neighbour over all the group's offsets) is written by the first group only.
constexpr int LINK_THREADS = 512;

template <bool GENERAL, bool D3 = false>
__global__ __launch_bounds__(LINK_THREADS) void k_link_part(const Slot* tab, JobView jv, uint32_t* parent,
                                                            uint32_t* nbr, unsigned long long* ctr, NbrGroup grp) {
    __shared__ uint64_t lkey[kPartSlots];
    __shared__ uint32_t laux[kPartSlots];
    __shared__ uint16_t list[kPartSlots];
    __shared__ uint32_t nlist;
    const uint32_t s = (uint32_t)ctr[C_SIGNIFICANT];
    const bool multi = jv.part_job != nullptr;
    const uint64_t parts = (jv.dims->slots + kPartSlots - 1) >> kPartLog2;
    // rounds of this launch: nbr holds one record of four words per round
    const uint32_t rounds = GENERAL ? grp.nrounds : 1u;
    bool bad = false;
    for (uint64_t p = blockIdx.x; p < parts; p += gridDim.x) {
        const JobInfo& J = jv.jobs[multi ? jv.part_job[p] : 0u];
        const Geo g = job_geo(J, D3);
        const uint32_t psize = (uint32_t)min<uint64_t>(J.cap, kPartSlots);  // a power of two
        const uint64_t base = p << kPartLog2;
        if (threadIdx.x == 0) nlist = 0;
        __syncthreads();  // also orders the previous partition's LDS reads before the overwrite
        // slice into LDS, all loads in flight at once
        constexpr int PER = (int)kPartSlots / LINK_THREADS;
        {
            Slot v[PER];
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const uint32_t u = k * LINK_THREADS + threadIdx.x;
                if (u < psize) v[k] = tab[base + u];
            }
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const uint32_t u = k * LINK_THREADS + threadIdx.x;
                if (u < psize) {
                    lkey[u] = v[k].key;
                    laux[u] = v[k].aux;
                }
            }
        }
        // local indices of the significant slots into list
        for (uint32_t u0 = 0; u0 < psize; u0 += LINK_THREADS) {
            const uint32_t u = u0 + threadIdx.x;
            const bool sig = u < psize && lkey[u] != kEmptyKey && laux[u] != kNotSignificant;
            const uint64_t b = __ballot(sig);
            uint32_t wbase = 0;
            if (lane_id() == 0 && b) wbase = atomicAdd(&nlist, (uint32_t)__popcll(b));
            wbase = __shfl(wbase, 0);
            if (sig) list[wbase + __popcll(b & lanemask_lt())] = (uint16_t)u;
        }
        __syncthreads();
        const uint32_t nl = nlist;
        const Slot* jt = tab + J.slot_base;
        for (uint32_t t = threadIdx.x; t < nl; t += LINK_THREADS) {
            const uint32_t u = list[t];
            const uint64_t key = lkey[u];
            const uint32_t i = laux[u];
            if (i >= s) {
                bad = true;
                continue;
            }
            const uint32_t bx = (uint32_t)(key >> 32);
            const uint32_t by = (uint32_t)key;
            uint32_t best = i;
            uint64_t best_key = key;
#pragma unroll 1
            for (uint32_t r = 0; r < rounds; ++r) {
                const NbrRound& nr = grp.r[r];
                uint64_t nk[4];
                bool want[4];
                if (!GENERAL) {
                    // valid biased coordinates lie in [2, 2^32 - 2]
                    const bool left = bx > 2u;
                    const bool down = by > 2u;
                    const bool up = by < 0xFFFFFFFEu;
                    nk[0] = ((uint64_t)(bx - 1) << 32) | (uint32_t)(by - 1);
                    want[0] = left && down;
                    nk[1] = ((uint64_t)(bx - 1) << 32) | by;
                    want[1] = left;
                    nk[2] = ((uint64_t)(bx - 1) << 32) | (uint32_t)(by + 1);
                    want[2] = left && up;
                    nk[3] = ((uint64_t)bx << 32) | (uint32_t)(by - 1);
                    want[3] = down;
                } else if (!D3) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int64_t x = (int64_t)bx + nr.dx[q];
                        const int64_t y = (int64_t)by + nr.dy[q];
                        want[q] = q < (int)nr.count && x >= 2 && x <= 0xFFFFFFFEll && y >= 2 && y <= 0xFFFFFFFEll;
                        nk[q] = want[q] ? (((uint64_t)(uint32_t)x << 32) | (uint32_t)y) : key;
                    }
                } else {
                    // 3-D keys: biased fields of 21 bits, valid in [2, 2^21 - 2]
                    const int64_t x0 = (int64_t)(key >> 42), y0 = (int64_t)((key >> 21) & kField3);
                    const int64_t z0 = (int64_t)(key & kField3);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int64_t x = x0 + nr.dx[q], y = y0 + nr.dy[q], z = z0 + nr.dz[q];
                        const int64_t hi = (int64_t)kField3 - 1;
                        want[q] = q < (int)nr.count && x >= 2 && x <= hi && y >= 2 && y <= hi && z >= 2 && z <= hi;
                        nk[q] = want[q] ? (((uint64_t)x << 42) | ((uint64_t)y << 21) | (uint64_t)z) : key;
                    }
                }
                // first probes: device-table loads for the other partitions are
                // issued together, LDS probes need no wait
                // (home slot and the next one: a probe walk mostly ends there)
                uint64_t pos[4];
                bool local[4];
                Slot v[4], w[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    pos[q] = home_slot(nk[q], g);
                    local[q] = ((J.slot_base + pos[q]) >> kPartLog2) == p;
                    if (want[q] && !local[q]) {
                        v[q] = jt[pos[q]];
                        w[q] = jt[next_slot(pos[q], g)];
                    }
                }
                uint32_t j[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    j[q] = kNoNeighbour;
                    if (!want[q]) continue;
                    uint32_t aux = kNotSignificant;
                    if (local[q]) {
                        uint32_t lp = (uint32_t)(J.slot_base + pos[q] - base);
                        for (uint32_t step = 0; step < kMaxProbe; ++step) {
                            const uint64_t cur = lkey[lp];
                            if (cur == nk[q]) {
                                aux = laux[lp];
                                break;
                            }
                            if (cur == kEmptyKey) break;
                            lp = (lp + 1) & (psize - 1);
                        }
                    } else {
                        if (v[q].key != nk[q] && v[q].key != kEmptyKey) {
                            // second probe already loaded
                            pos[q] = next_slot(pos[q], g);
                            v[q] = w[q];
                            uint32_t steps = 2;
                            while (v[q].key != nk[q] && v[q].key != kEmptyKey && steps < kMaxProbe) {
                                pos[q] = next_slot(pos[q], g);
                                v[q] = jt[pos[q]];
                                ++steps;
                            }
                        }
                        if (v[q].key == nk[q]) aux = v[q].aux;
                    }
                    if (aux != kNotSignificant) {
                        if (aux >= s) {
                            bad = true;
                        } else {
                            j[q] = aux;
                            if (nk[q] < best_key) {
                                best_key = nk[q];
                                best = aux;
                            }
                        }
                    }
                }
                uint4 rec;
                rec.x = j[0];
                rec.y = j[1];
                rec.z = j[2];
                rec.w = j[3];
                reinterpret_cast<uint4*>(nbr)[(uint64_t)i * rounds + r] = rec;
            }
            if (!GENERAL || grp.set_parent) parent[i] = best;
        }
    }
    if (bad) atomicOr(&ctr[C_ERROR], (unsigned long long)kErrInternal);
}

// ---- framed tables: census of the significant slots, then the link pass ----
//
// For a framed single table of at least 512 partitions (Chebyshev distance 1,
// two dimensions) the compact index of a significant tile -- its rank among
// the significant slots in slot order (Algorithm 1: the tiles kept by the
// tau test) -- is computed where it is needed instead of being written into
// every slot.  The census gives every 32 slots of the table one 8-byte
// record: their significance bits and the number of significant slots before
// them.  It counts within census blocks (runs of whole partitions) first; a
// scan of the block totals and a pass over the records make the counts
// global.  The link pass then reads each slice once: it writes the compact
// arrays of its partition and finds the neighbours, local ones through the
// slice in LDS and the others through the table and one census record.

constexpr int CENSUS_THREADS = 512;
constexpr uint32_t kCensusRecLog2 = 5;                       // 32 slots per record
constexpr uint32_t kCensusPartRecs = kPartSlots >> kCensusRecLog2;  // 128

__host__ __device__ inline uint32_t census_blk_shift(uint32_t p_log2) {
    constexpr uint32_t scan_log2 = 11;  // kScanBlocks == 2^11
    static_assert((1u << scan_log2) == (uint32_t)kScanBlocks, "census blocks");
    return p_log2 > scan_log2 ? p_log2 - scan_log2 : 0u;
}

template <bool SQUARE>
__device__ __forceinline__ bool slot_significant(const Slot& v, uint32_t tau) {
    return v.key != kEmptyKey && (v.count >= tau || (SQUARE && v.aux == kSquareKeep));
}

// rec[r] = (bits of slots 32 r .. 32 r + 31, significant slots before them
// in their census block); boff[b] = the total of census block b.
template <bool SQUARE>
__global__ __launch_bounds__(CENSUS_THREADS) void k_census_framed(const Slot* tab, const Geo g, uint32_t tau,
                                                                  uint2* rec, uint32_t* boff,
                                                                  unsigned long long* ctr) {
    __shared__ uint64_t wbits[64];
    __shared__ uint32_t ptotal;
    __shared__ unsigned long long red[CENSUS_THREADS / 64][2];
    const uint64_t parts = 1ull << g.p_log2;
    const uint64_t ppb = 1ull << census_blk_shift(g.p_log2);
    const uint64_t p0 = (uint64_t)blockIdx.x * ppb;
    const uint32_t w = threadIdx.x >> 6;
    uint32_t run = 0;
    unsigned long long occ = 0, sum = 0;
    for (uint64_t p = p0; p < p0 + ppb && p < parts; ++p) {
        constexpr int PER = (int)kPartSlots / CENSUS_THREADS;
        const Slot* sl = tab + (p << kPartLog2);
        Slot v[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) v[k] = sl[k * CENSUS_THREADS + threadIdx.x];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const bool o = v[k].key != kEmptyKey;
            occ += o;
            sum += o ? v[k].count : 0u;
            // the wave's 64 slots k * CENSUS_THREADS + 64 w + lane form word 8 k + w
            const uint64_t b = __ballot(slot_significant<SQUARE>(v[k], tau));
            if (lane_id() == 0) wbits[k * (CENSUS_THREADS / 64) + w] = b;
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            const uint64_t b = wbits[threadIdx.x];
            const uint32_t lo = (uint32_t)__popc((uint32_t)b), c = (uint32_t)__popcll(b);
            uint32_t inc = c;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t t = __shfl_up(inc, o);
                if (lane_id() >= (uint32_t)o) inc += t;
            }
            const uint32_t before = run + inc - c;
            uint2* r = rec + (p << 7) + 2 * threadIdx.x;
            r[0] = make_uint2((uint32_t)b, before);
            r[1] = make_uint2((uint32_t)(b >> 32), before + lo);
            if (threadIdx.x == 63) ptotal = inc;
        }
        __syncthreads();
        run += ptotal;
    }
    for (int o = 32; o > 0; o >>= 1) {
        occ += __shfl_xor(occ, o);
        sum += __shfl_xor(sum, o);
    }
    if (lane_id() == 0) {
        red[w][0] = occ;
        red[w][1] = sum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long to = 0, ts = 0;
        for (int i = 0; i < CENSUS_THREADS / 64; ++i) {
            to += red[i][0];
            ts += red[i][1];
        }
        boff[blockIdx.x] = run;
        if (to) atomicAdd(&ctr[C_DISTINCT], to);
        if (ts) atomicAdd(&ctr[C_SUM], ts);
    }
}

// Exclusive scan of n words in place by one workgroup of 1024 threads (each
// takes a run of ceil(n / 1024)); the total goes to *total_out.
// With ctr, also the sums of stat[0, n) and stat[n, 2n) (a census's occupied
// slots and count sums per partition) go to ctr[C_DISTINCT] and ctr[C_SUM].
__global__ __launch_bounds__(1024) void k_scan_u32(uint32_t* v, uint32_t n, unsigned long long* total_out,
                                                   const uint32_t* stat, unsigned long long* ctr) {
    __shared__ uint32_t wsum[16];
    if (ctr) {
        uint32_t o = 0, c = 0;
        for (uint32_t i = threadIdx.x; i < n; i += 1024) {
            o += stat[i];
            c += stat[n + i];
        }
        o = block_total32(o);
        c = block_total32(c);
        if (threadIdx.x == 0) {
            ctr[C_DISTINCT] = o;
            ctr[C_SUM] = c;
        }
    }
    const uint32_t per = (n + 1023) / 1024;
    const uint32_t lo = min(threadIdx.x * per, n), hi = min(lo + per, n);
    uint32_t local = 0;
    constexpr uint32_t kRun = 16;  // runs up to this long are loaded all at once
    uint32_t run[kRun];
    if (per <= kRun) {
#pragma unroll
        for (uint32_t k = 0; k < kRun; ++k) run[k] = lo + k < hi ? v[lo + k] : 0u;
#pragma unroll
        for (uint32_t k = 0; k < kRun; ++k) local += run[k];
    } else {
        for (uint32_t i = lo; i < hi; ++i) local += v[i];
    }
    uint32_t inc = local;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(inc, off);
        if (lane_id() >= (uint32_t)off) inc += o;
    }
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) wsum[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int i = 0; i < 16; ++i) {
            const uint32_t c = wsum[i];
            wsum[i] = run;
            run += c;
        }
        *total_out = run;
    }
    __syncthreads();
    uint32_t ex = wsum[w] + inc - local;
    if (per <= kRun) {
#pragma unroll
        for (uint32_t k = 0; k < kRun; ++k)
            if (lo + k < hi) {
                v[lo + k] = ex;
                ex += run[k];
            }
    } else {
        for (uint32_t i = lo; i < hi; ++i) {
            const uint32_t c = v[i];
            v[i] = ex;
            ex += c;
        }
    }
}

// Adds each census block's offset (boff after the scan) to its records.
__global__ void k_census_offsets(uint2* rec, uint64_t nrec, const uint32_t* boff, uint32_t blk_shift) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nrec;
         i += (uint64_t)gridDim.x * blockDim.x)
        rec[i].y += boff[(i >> 7) >> blk_shift];
}

// Compact index of the significant slot at `pos` from its census record.
__device__ __forceinline__ uint32_t census_index(uint2 r, uint64_t pos) {
    return r.y + (uint32_t)__popc(r.x & ((1u << (pos & 31)) - 1u));
}

// The eight-neighbour link pass over the census (as k_link_part<false, false>
// for the rest): the slice is held in LDS as 4-byte entries (with the empty
// and foreign markers of k_aggregate_f32) and the local ranks of its
// significant slots.  At most 80 VGPRs, so that six waves per SIMD hide the
// device-table probes.  With IMG the slices come from the image the final
// update wrote (entry and count per slot, 8 bytes instead of 16), and so do
// the probes for neighbours inside the frame; keys outside the frame are
// still found in the table.  A null table (never filled: every key went
// through the binning into the image) holds no such keys.
//
// With manh (Manhattan distance 1) only the two backward neighbours that
// share an edge with the tile are looked up, (-1, 0) and (0, -1).
template <bool SQUARE, bool IMG>
__global__ __launch_bounds__(LINK_THREADS, 6) void k_link_census(const Slot* tab, const uint2* img, const Geo g,
                                                              uint32_t tau, bool manh, const uint2* rec, uint64_t* s_key,
                                                              uint32_t* s_count, uint32_t* size, uint32_t* parent,
                                                              uint32_t* nbr, unsigned long long* ctr) {
    __shared__ uint32_t lent[kPartSlots];
    __shared__ uint16_t lrank[kPartSlots];  // rank among the partition's significant slots, kNoRank if none
    __shared__ uint16_t list[kPartSlots];   // slot of each rank
    // parent of each rank: itself (no backward neighbour), the rank of a
    // parent in this partition, or kFar | the compact index of one outside
    __shared__ uint32_t lpar[kPartSlots];
    constexpr uint32_t kFar = 0x80000000u;
    constexpr uint16_t kNoRank = 0xFFFFu;
    const uint32_t s = (uint32_t)ctr[C_SIGNIFICANT];
    const uint64_t parts = 1ull << g.p_log2;
    const uint32_t fine = g.p_log2 - kFrameCoarseLog2;  // >= 1 here
    const uint32_t w = threadIdx.x >> 6;
    if (ctr[C_SIGNIFICANT] >= kFar) {  // compact indices need 31 bits here; uniform across the grid
        if (threadIdx.x == 0) atomicOr(&ctr[C_ERROR], (unsigned long long)kErrInternal);
        return;
    }
    const uint64_t lt = lanemask_lt();
    bool bad = false;
    for (uint64_t p = blockIdx.x; p < parts; p += gridDim.x) {
        const uint64_t base = p << kPartLog2;
        const uint32_t cb = (uint32_t)(p >> fine);
        const uint32_t top = (uint32_t)(p & ((1u << fine) - 1)) << (32 - fine);
        const uint32_t kEmpty = top ^ 0x80000000u, kAlien = kEmpty ^ 1u;  // never an entry of this partition
        const uint2 last = rec[(p << 7) + kCensusPartRecs - 1];
        const uint32_t poff = rec[p << 7].y;
        const uint32_t nl = last.y + (uint32_t)__popc(last.x) - poff;
        __syncthreads();  // the previous partition's LDS reads are done
        constexpr int PER = (int)kPartSlots / LINK_THREADS;
        {
            Slot v[IMG ? 1 : PER];
            uint2 iv[IMG ? PER : 1];
            uint32_t wz[PER];  // census counts before this wave's words, loaded with the slice
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                if constexpr (IMG) iv[k] = img[base + k * LINK_THREADS + threadIdx.x];
                else v[k] = tab[base + k * LINK_THREADS + threadIdx.x];
                const uint32_t word = (uint32_t)__builtin_amdgcn_readfirstlane(k * (LINK_THREADS / 64) + w);
                wz[k] = rec[(p << 7) + 2 * word].y;
            }
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const uint32_t u = k * LINK_THREADS + threadIdx.x;
                uint32_t e = kEmpty, cnt;
                bool sig;
                if constexpr (IMG) {
                    e = iv[k].x;
                    cnt = iv[k].y;
                    sig = e != kEmpty && cnt >= tau;
                } else {
                    uint64_t h;
                    if (v[k].key != kEmptyKey && !frame_code(v[k].key, g.fx, g.fy, h, e)) e = kAlien;
                    cnt = v[k].count;
                    sig = slot_significant<SQUARE>(v[k], tau);
                }
                lent[u] = e;
                const uint64_t b = __ballot(sig);
                const uint32_t r = wz[k] - poff + (uint32_t)__popcll(b & lt);
                lrank[u] = sig ? (uint16_t)r : kNoRank;
                if (sig) {
                    list[r] = (uint16_t)u;
                    lpar[r] = r;
                    const uint64_t i = (uint64_t)poff + r;
                    if (i < s) {
                        if constexpr (IMG)
                            s_key[i] = e != kAlien ? frame_key(cb, e, g.fx, g.fy) : tab[base + u].key;
                        else
                            s_key[i] = v[k].key;
                        s_count[i] = cnt;
                        size[i] = 0;
                    } else {
                        bad = true;
                    }
                }
            }
        }
        __syncthreads();
        for (uint32_t t = threadIdx.x; t < nl; t += LINK_THREADS) {
            const uint32_t u = list[t];
            const uint32_t i = poff + t;
            if (i >= s) {
                bad = true;
                continue;
            }
            const uint32_t eu = lent[u];
            const uint64_t key = eu != kAlien ? frame_key(cb, eu, g.fx, g.fy) : tab[base + u].key;
            const uint32_t bx = (uint32_t)(key >> 32), by = (uint32_t)key;
            // valid biased coordinates lie in [2, 2^32 - 2]
            const bool left = bx > 2u, down = by > 2u, up = by < 0xFFFFFFFEu;
            uint64_t nk[4];
            bool want[4];
            nk[0] = ((uint64_t)(bx - 1) << 32) | (uint32_t)(by - 1);
            want[0] = left && down && !manh;
            nk[1] = ((uint64_t)(bx - 1) << 32) | by;
            want[1] = left;
            nk[2] = ((uint64_t)(bx - 1) << 32) | (uint32_t)(by + 1);
            want[2] = left && up && !manh;
            nk[3] = ((uint64_t)bx << 32) | (uint32_t)(by - 1);
            want[3] = down;
            // Loads for the neighbours in other partitions issued together:
            // the keys of the home slot and the next one, and the home slot's
            // census record, whose bit tells significance (no counts read).
            // Neighbours in this partition are probed in LDS meanwhile.
            uint64_t pos[4];
            uint32_t e[4];
            uint2 cr[4];
            bool local[4], framed[4];
            // IMG: a0/a1 hold entries (4 bytes) and pq the neighbour's
            // partition; otherwise k0/k1 hold keys
            uint32_t a0[IMG ? 4 : 1], a1[IMG ? 4 : 1], pq[IMG ? 4 : 1];
            uint64_t k0[IMG ? 1 : 4], k1[IMG ? 1 : 4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint64_t h;
                framed[q] = frame_code(nk[q], g.fx, g.fy, h, e[q]);
                const uint64_t part_q = h >> (kFrameStBits - g.p_log2);
                local[q] = framed[q] && part_q == p;
                pos[q] = home_slot(nk[q], g);
                if constexpr (IMG) {
                    pq[q] = (uint32_t)part_q;
                    if (want[q] && !local[q] && framed[q]) {
                        a0[q] = img[pos[q]].x;
                        a1[q] = img[next_slot(pos[q], g)].x;
                        cr[q] = rec[pos[q] >> kCensusRecLog2];
                    }
                } else {
                    if (want[q] && !local[q]) {
                        k0[q] = tab[pos[q]].key;
                        k1[q] = tab[next_slot(pos[q], g)].key;
                        cr[q] = rec[pos[q] >> kCensusRecLog2];
                    }
                }
            }
            uint32_t j[4];
            uint32_t best = i;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                j[q] = kNoNeighbour;
                if (!want[q]) continue;
                if (local[q]) {
                    uint32_t lp = (uint32_t)(pos[q] - base);
                    for (uint32_t step = 0; step < kMaxProbe; ++step) {
                        const uint32_t cur = lent[lp];
                        if (cur == e[q]) {
                            const uint16_t r = lrank[lp];
                            if (r != kNoRank) j[q] = poff + r;
                            break;
                        }
                        if (cur == kEmpty) break;
                        lp = (lp + 1) & (kPartSlots - 1);
                    }
                } else if (IMG && framed[q]) {
                    // the neighbour's partition marks its empty slots by its own value
                    const uint32_t none = ((pq[IMG ? q : 0] & ((1u << fine) - 1)) << (32 - fine)) ^ 0x80000000u;
                    const uint64_t home = pos[q];
                    uint32_t ce = a0[IMG ? q : 0];
                    if (ce != e[q] && ce != none) {
                        pos[q] = next_slot(pos[q], g);
                        ce = a1[IMG ? q : 0];
                        uint32_t steps = 2;
                        while (ce != e[q] && ce != none && steps < kMaxProbe) {
                            pos[q] = next_slot(pos[q], g);
                            ce = img[pos[q]].x;
                            ++steps;
                        }
                    }
                    if (ce == e[q]) {
                        uint2 r = cr[q];
                        if ((pos[q] >> kCensusRecLog2) != (home >> kCensusRecLog2)) r = rec[pos[q] >> kCensusRecLog2];
                        if ((r.x >> (pos[q] & 31)) & 1u) j[q] = census_index(r, pos[q]);
                    }
                } else if (!IMG || tab) {
                    // keys outside the frame (IMG: not loaded ahead) are in the
                    // table; with the image and no table (never filled) there
                    // are none
                    const uint64_t home = pos[q];
                    uint64_t ck = IMG ? tab[pos[q]].key : k0[IMG ? 0 : q];
                    if (ck != nk[q] && ck != kEmptyKey) {
                        pos[q] = next_slot(pos[q], g);
                        ck = IMG ? tab[pos[q]].key : k1[IMG ? 0 : q];
                        uint32_t steps = 2;
                        while (ck != nk[q] && ck != kEmptyKey && steps < kMaxProbe) {
                            pos[q] = next_slot(pos[q], g);
                            ck = tab[pos[q]].key;
                            ++steps;
                        }
                    }
                    if (ck == nk[q]) {
                        uint2 r = IMG ? rec[pos[q] >> kCensusRecLog2] : cr[q];
                        if ((pos[q] >> kCensusRecLog2) != (home >> kCensusRecLog2)) r = rec[pos[q] >> kCensusRecLog2];
                        if ((r.x >> (pos[q] & 31)) & 1u) j[q] = census_index(r, pos[q]);
                    }
                }
                if (j[q] != kNoNeighbour) {
                    if (j[q] >= s) {
                        bad = true;
                        j[q] = kNoNeighbour;
                    } else if (best == i) {
                        // backward neighbours come in increasing key order; the
                        // parent edge is in the forest already, so the merge
                        // pass need not see it
                        best = j[q];
                        j[q] = kNoNeighbour;
                    }
                }
            }
            uint4 out;
            out.x = j[0];
            out.y = j[1];
            out.z = j[2];
            out.w = j[3];
            reinterpret_cast<uint4*>(nbr)[i] = out;
            lpar[t] = best == i ? t : best - poff < nl ? best - poff : kFar | best;
        }
        __syncthreads();
        // parent = the end of the tile's chain of parents inside the partition
        // (its root, or the first parent outside), so that the jump pass
        // only follows the links between partitions
        for (uint32_t t = threadIdx.x; t < nl; t += LINK_THREADS) {
            const uint32_t i = poff + t;
            if (i >= s) continue;
            uint32_t x = t, v = lpar[t];
            for (uint32_t step = 0; step < nl && !(v & kFar) && v != x; ++step) {
                if (v >= nl) {  // never a rank of this partition
                    bad = true;
                    break;
                }
                x = v;
                v = lpar[x];
            }
            parent[i] = v & kFar ? v & ~kFar : poff + x;
        }
    }
    if (bad) atomicOr(&ctr[C_ERROR], (unsigned long long)kErrInternal);
}

// Parents after this pass are roots or, where a concurrent path-halving write
// lands after the root is stored, ancestors; merge and compress only need
// ancestors.
__global__ void k_jump(uint32_t* parent, unsigned long long* ctr) {
    const uint32_t s = (uint32_t)ctr[C_SIGNIFICANT];
    bool bad = false;
    const XcdSpan span = xcd_span(s);
    for (uint64_t i = span.first; i < span.hi; i += span.step)
        parent[i] = uf_root_cached(parent, (uint32_t)i, s, bad);
    if (bad) atomicOr(&ctr[C_ERROR], (unsigned long long)kErrInternal);
}

// Unites every tile with the neighbours recorded by one link launch: `recs`
// records of four words per tile.
__global__ void k_merge(const uint32_t* nbr, uint32_t recs, const uint64_t* s_key, uint32_t* parent,
                        unsigned long long* ctr) {
    const uint32_t s = (uint32_t)ctr[C_SIGNIFICANT];
    bool bad = false;
    const XcdSpan span = xcd_span(s);
    for (uint64_t i = span.first; i < span.hi; i += span.step) {
        // After the jump pass parents are roots; a tile whose recorded
        // neighbours share its root needs no hook.  These first reads may be
        // stale within this kernel: an equal value still proves the two tiles
        // are connected, and a differing one only costs a redundant unite.
        const uint32_t ri = __hip_atomic_load(parent + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll 1
        for (uint32_t r = 0; r < recs; ++r) {
            const uint4 rec = reinterpret_cast<const uint4*>(nbr)[i * recs + r];
            const uint32_t j[4] = {rec.x, rec.y, rec.z, rec.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (j[q] == kNoNeighbour) continue;
                if (__hip_atomic_load(parent + j[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == ri) continue;
                uf_unite(parent, s_key, (uint32_t)i, j[q], s, bad);
            }
        }
    }
    if (bad) atomicOr(&ctr[C_ERROR], (unsigned long long)kErrInternal);
}

// Final roots into root[] (a separate array: path halving by other threads
// keeps rewriting parent words with ancestors that need not be roots), the
// root count, and component sizes counted up to mu: a member adds itself only
// while the size it reads is below mu.  Reads only ever under-state the size,
// so the final value is below mu exactly when the component has fewer than mu
// tiles.
__global__ void k_compress(JobView jv, uint32_t* parent, uint32_t* root, uint32_t* size, unsigned long long* ctr) {
    const uint32_t s = (uint32_t)ctr[C_SIGNIFICANT];
    const bool multi = jv.part_job != nullptr;
    // a plain grid stride: the size counters take memory-side atomics, which
    // run faster spread over all of [0, s) than gathered per XCD
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t s_round = ((uint64_t)s + 63) / 64 * 64;  // whole waves run the same trip count
    bool bad = false;
    uint32_t roots = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < s_round; i += stride) {
        if (i < s) {
            const uint32_t r = uf_root_cached(parent, (uint32_t)i, s, bad);
            root[i] = r;
            const uint32_t mu = jv.jobs[multi ? jv.s_job[i] : 0u].mu;
            if (ld_relaxed(size + r) < mu) atomicAdd(size + r, 1u);
            roots += (r == (uint32_t)i);
        }
    }
    block_count_add(&ctr[C_COMPONENTS], roots);
    if (bad) atomicOr(&ctr[C_ERROR], (unsigned long long)kErrInternal);
}

// The same for the census path, one workgroup per partition: the roots of
// the partition's significant tiles are counted in LDS first, so that a
// component's size takes one memory-side atomic per partition it touches
// instead of one per tile (the partition's compact range comes from the
// census records).
__global__ __launch_bounds__(512) void k_compress_census(const uint2* rec, uint64_t parts, uint32_t mu,
                                                         uint32_t* parent, uint32_t* root, uint32_t* size,
                                                         unsigned long long* ctr) {
    __shared__ uint32_t hroot[kPartSlots];  // a partition has at most kPartSlots tiles, so as many roots
    __shared__ uint32_t hcnt[kPartSlots];
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    const uint32_t s = (uint32_t)ctr[C_SIGNIFICANT];
    bool bad = false;
    uint32_t roots = 0;
    for (uint64_t p = blockIdx.x; p < parts; p += gridDim.x) {
        const uint2 last = rec[(p << 7) + kCensusPartRecs - 1];
        const uint32_t poff = rec[p << 7].y;
        const uint32_t nl = last.y + (uint32_t)__popc(last.x) - poff;
        __syncthreads();  // the previous partition's counts are out
        for (uint32_t u = threadIdx.x; u < kPartSlots; u += blockDim.x) {
            hroot[u] = kNone;
            hcnt[u] = 0;
        }
        __syncthreads();
        for (uint32_t t = threadIdx.x; t < nl; t += blockDim.x) {
            const uint32_t i = poff + t;
            if (i >= s) {
                bad = true;
                continue;
            }
            const uint32_t r = uf_root_cached(parent, i, s, bad);
            root[i] = r;
            roots += (r == i);
            uint32_t h = mix32(r) & (kPartSlots - 1);
            for (uint32_t step = 0; step < kPartSlots; ++step) {
                uint32_t cur = __hip_atomic_load(&hroot[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (cur == kNone) cur = atomicCAS(&hroot[h], kNone, r);
                if (cur == kNone || cur == r) {
                    atomicAdd(&hcnt[h], 1u);
                    break;
                }
                h = (h + 1) & (kPartSlots - 1);
            }
        }
        __syncthreads();
        for (uint32_t u = threadIdx.x; u < kPartSlots; u += blockDim.x) {
            const uint32_t r = hroot[u];
            if (r != kNone && ld_relaxed(size + r) < mu) atomicAdd(size + r, hcnt[u]);
        }
    }
    block_count_add(&ctr[C_COMPONENTS], roots);
    if (bad) atomicOr(&ctr[C_ERROR], (unsigned long long)kErrInternal);
}

// Writes the keys of a slice image back into the table (for a table that
// has to grow after an update that wrote only the image).
__global__ void k_image_to_table(const uint2* img, Slot* tab, const Geo g) {
    const uint32_t fine = g.p_log2 - kFrameCoarseLog2;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < g.cap;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t p = i >> kPartLog2;
        const uint32_t top = (uint32_t)(p & ((1u << fine) - 1)) << (32 - fine);
        const uint32_t kEmpty = top ^ 0x80000000u, kAlien = kEmpty ^ 1u;
        const uint2 v = img[i];
        if (v.x != kEmpty && v.x != kAlien) {
            Slot sl;
            sl.key = frame_key((uint32_t)(p >> fine), v.x, g.fx, g.fy);
            sl.count = v.y;
            sl.aux = kNotSignificant;
            tab[i] = sl;
        }
    }
}

// ---- mu filter (Algorithm 1: keep clusters of at least mu tiles) -----------

// Root, mu and root size of the items of one scan tile (t0 < hi <= s).  Each
// round of loads is unconditional (indices clamped, results masked) so that
// it is in flight for all items at once.  Items past hi read as root s.
__device__ __forceinline__ void filter_items(const JobView& jv, bool multi, uint32_t mu0, const uint32_t* root,
                                             const uint32_t* size, uint64_t s, uint64_t t0, uint64_t hi,
                                             uint32_t (&rt)[SCAN_ITEMS], uint32_t (&mu)[SCAN_ITEMS],
                                             uint32_t (&sz)[SCAN_ITEMS]) {
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const uint64_t i = min(t0 + (uint64_t)j * SCAN_THREADS + threadIdx.x, hi - 1);
        rt[j] = root[i];
        mu[j] = multi ? jv.s_job[i] : mu0;  // the job id, for now
    }
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        if (t0 + (uint64_t)j * SCAN_THREADS + threadIdx.x >= hi) rt[j] = (uint32_t)s;
        sz[j] = size[min((uint64_t)rt[j], s - 1)];
        if (multi) mu[j] = jv.jobs[mu[j]].mu;
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_filter_count(JobView jv, const uint32_t* root, const uint32_t* size,
                                                               uint32_t* partials, unsigned long long* ctr) {
    __shared__ unsigned long long red[SCAN_WAVES];
    const uint64_t s = ctr[C_SIGNIFICANT];
    const bool multi = jv.part_job != nullptr;
    const uint32_t mu0 = jv.jobs[0].mu;
    uint64_t lo, hi;
    block_range(s, lo, hi);
    unsigned long long keep = 0, kept_roots = 0;
    for (uint64_t t0 = lo; t0 < hi; t0 += SCAN_TILE) {
        uint32_t rt[SCAN_ITEMS], mu[SCAN_ITEMS], sz[SCAN_ITEMS];
        filter_items(jv, multi, mu0, root, size, s, t0, hi, rt, mu, sz);
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            const uint64_t i = t0 + (uint64_t)j * SCAN_THREADS + threadIdx.x;
            const bool k = i < hi && rt[j] < s && sz[j] >= mu[j];
            keep += k;
            kept_roots += (k && rt[j] == (uint32_t)i);
        }
    }
    keep = block_sum(keep, red);
    kept_roots = block_sum(kept_roots, red);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = (uint32_t)keep;
        if (kept_roots) atomicAdd(&ctr[C_CLUSTERS], kept_roots);
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_filter_scatter(JobView jv, const uint64_t* s_key,
                                                                 const uint32_t* s_count, const uint32_t* root,
                                                                 const uint32_t* size, const uint32_t* offsets,
                                                                 const unsigned long long* ctr, int32_t* out_kx,
                                                                 int32_t* out_ky, int32_t* out_kz,
                                                                 uint32_t* out_count, uint64_t* out_label,
                                                                 uint32_t* out_job) {
    __shared__ TileScratch ts;
    const uint64_t s = ctr[C_SIGNIFICANT];
    const bool multi = jv.part_job != nullptr;
    const uint32_t mu0 = jv.jobs[0].mu;
    uint64_t lo, hi;
    block_range(s, lo, hi);
    uint64_t run = offsets[blockIdx.x];
    for (uint64_t t0 = lo; t0 < hi; t0 += SCAN_TILE) {
        uint32_t bits = 0;
        uint32_t rt[SCAN_ITEMS], mu[SCAN_ITEMS], sz[SCAN_ITEMS];
        filter_items(jv, multi, mu0, root, size, s, t0, hi, rt, mu, sz);
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            const uint64_t i = t0 + (uint64_t)j * SCAN_THREADS + threadIdx.x;
            if (i < hi && rt[j] < s && sz[j] >= mu[j]) bits |= 1u << j;
        }
        uint32_t pos[SCAN_ITEMS];
        const uint32_t total = tile_positions(bits, pos, ts);
        // row data of all items loaded together (indices clamped), then
        // the kept rows written
        uint64_t key[SCAN_ITEMS], label[SCAN_ITEMS];
        uint32_t cnt[SCAN_ITEMS];
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            const uint64_t i = min(t0 + (uint64_t)j * SCAN_THREADS + threadIdx.x, hi - 1);
            key[j] = s_key[i];
            cnt[j] = s_count[i];
            label[j] = s_key[min((uint64_t)rt[j], s - 1)];
        }
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            if (!(bits & (1u << j))) continue;
            const uint64_t i = t0 + (uint64_t)j * SCAN_THREADS + threadIdx.x;
            const uint64_t p = run + pos[j];
            if (out_kz) {  // 3-D keys (uniform across the grid)
                out_kx[p] = (int32_t)(key[j] >> 42) - (int32_t)kBias3;
                out_ky[p] = (int32_t)((key[j] >> 21) & kField3) - (int32_t)kBias3;
                out_kz[p] = (int32_t)(key[j] & kField3) - (int32_t)kBias3;
            } else {
                out_kx[p] = (int32_t)((uint32_t)(key[j] >> 32) - 0x80000000u);
                out_ky[p] = (int32_t)((uint32_t)key[j] - 0x80000000u);
            }
            out_count[p] = cnt[j];
            out_label[p] = label[j];
            if (multi) out_job[p] = jv.s_job[i];
        }
        run += total;
    }
}

// Writes a one-job descriptor (passed by value with the launch) to device
// memory, so that a caller needs no host-to-device copy for it.
__global__ void k_store_job(Dims d, JobInfo j, Dims* d_dims, JobInfo* d_job) {
    *d_dims = d;
    *d_job = j;
}

// ---- distinct-tile sketch of one point set -------------------------------------
//
// The hll_sample sketch of n points into kHllReps register replicas (one per
// workgroup index modulo kHllReps).  Range errors are left to the counting
// pass.
template <typename T>
__global__ __launch_bounds__(256) void k_points_hll(const T* __restrict__ pts, int64_t n, double scale,
                                                    uint32_t* hll) {
    constexpr int U = 16;
    uint32_t* rep = hll + ((uint64_t)(blockIdx.x % kHllReps) << kHllLog2);
    for (int64_t i0 = (int64_t)blockIdx.x * U * blockDim.x; i0 < n; i0 += (int64_t)gridDim.x * U * blockDim.x) {
        // loads of all items first (indices clamped, results masked)
        double x[U], y[U], z[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            load_xyz(pts, min(i0 + (int64_t)u * blockDim.x + threadIdx.x, n - 1), x[u], y[u], z[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            uint64_t key;
            uint32_t r, rank;
            if (i0 + (int64_t)u * blockDim.x + threadIdx.x < n && point_key<T>(x[u], y[u], z[u], scale, key) &&
                hll_sample(key, r, rank))
                atomicMax(rep + r, rank);
        }
    }
}

// ---- distinct-tile estimate per job (batches) ---------------------------------
//
// The hll_sample sketch of each job's tiles, so that its table can be sized
// before counting.  Reads every point once; range errors are left to the
// counting pass.

// One work tile of k_batch_hll in the job's point type: loads of all items
// first (indices clamped, results masked), then the sampled keys.
template <typename T>
__device__ __forceinline__ void hll_tile(const T* pts, int64_t base, int64_t end, double scale, uint32_t* reg) {
    constexpr int U = 16;
    for (int64_t i0 = base; i0 < end; i0 += (int64_t)U * blockDim.x) {
        double x[U], y[U];
#pragma unroll
        for (int u = 0; u < U; ++u) load_point(pts, min(i0 + (int64_t)u * blockDim.x + threadIdx.x, end - 1), x[u], y[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            uint64_t key;
            if (i0 + (int64_t)u * blockDim.x + threadIdx.x >= end || !tile_key(x[u], y[u], scale, key)) continue;
            uint32_t r, rank;
            if (hll_sample(key, r, rank)) atomicMax(reg + r, rank);
        }
    }
}

__global__ __launch_bounds__(256) void k_batch_hll(JobView jv, const uint32_t* tile_prefix, uint32_t tile,
                                                   uint32_t* hll) {
    const uint32_t tiles = jv.dims->tiles, njobs = jv.dims->njobs;
    const TileRange tr = tile_range(tile_prefix, njobs, tiles);
    uint32_t job = tr.job;
    for (uint32_t t = tr.lo; t < tr.hi; ++t) {
        job = advance_job(tile_prefix, job, t);
        const JobInfo& J = jv.jobs[job];
        const int64_t base = (int64_t)(t - J.first_tile) * tile;
        const int64_t end = min(base + (int64_t)tile, J.n);
        uint32_t* reg = hll + ((uint64_t)job << kHllLog2);
        if (J.dtype == 1) hll_tile(static_cast<const float*>(J.pts), base, end, J.scale, reg);
        else hll_tile(static_cast<const double*>(J.pts), base, end, J.scale, reg);
    }
}

// ---- per-point labels (the second projection pass of Section 4.1) ---------------
//
// A lookup table of a result's tiles: cap (a power of two) slots of two words
// {biased key, value}, empty key UINT64_MAX, home slot from the slot hash,
// linear probing over the whole table.  The value is the cluster label
// (per-point labels) or, with ROWS, the tile's row in the result (per-tile
// point lists).  Every point is then projected again and its tile looked up.

template <bool ROWS>
__global__ void k_label_table(const int32_t* kx, const int32_t* ky, const int32_t* kz, const uint64_t* label,
                              uint64_t t, uint64_t* tab, uint64_t cap) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < t;
         i += (uint64_t)gridDim.x * blockDim.x) {
        // rows of a 3-D result (kz given) take the 3-D key
        const uint64_t key =
            kz ? ((uint64_t)(uint32_t)(kx[i] + (int32_t)kBias3) << 42) |
                     ((uint64_t)(uint32_t)(ky[i] + (int32_t)kBias3) << 21) | (uint32_t)(kz[i] + (int32_t)kBias3)
               : ((uint64_t)((uint32_t)kx[i] + 0x80000000u) << 32) | ((uint32_t)ky[i] + 0x80000000u);
        uint64_t pos = slot_hash(key) & (cap - 1);
        // the keys are distinct and the table is at most half full: a free
        // slot is always found
        while (atomicCAS(reinterpret_cast<unsigned long long*>(tab + 2 * pos), (unsigned long long)kEmptyKey,
                         (unsigned long long)key) != kEmptyKey)
            pos = (pos + 1) & (cap - 1);
        tab[2 * pos + 1] = ROWS ? i : label[i];
    }
}

template <typename P>
__global__ __launch_bounds__(256) void k_point_labels(const P* __restrict__ pts, int64_t n, double scale,
                                                      const uint64_t* __restrict__ tab, uint64_t cap,
                                                      uint64_t* __restrict__ out, unsigned long long* err) {
    // One slot is {key, label}, 16-byte aligned, read by a single 16-byte load:
    // the label arrives with the key compare instead of a second round trip.
    typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
    const u64x2* __restrict__ slots = reinterpret_cast<const u64x2*>(tab);
    constexpr int U = 8;
    bool bad = false;
    for (int64_t i0 = (int64_t)blockIdx.x * U * blockDim.x; i0 < n; i0 += (int64_t)gridDim.x * U * blockDim.x) {
        // loads of all items first (indices clamped, results masked)
        double x[U], y[U], z[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            load_xyz(pts, min(i0 + (int64_t)u * blockDim.x + threadIdx.x, n - 1), x[u], y[u], z[u]);
        uint64_t key[U], pos[U];
        u64x2 cur[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            key[u] = 0;
            ok[u] = point_key<P>(x[u], y[u], z[u], scale, key[u]);
            pos[u] = slot_hash(key[u]) & (cap - 1);
            cur[u] = slots[pos[u]];  // first probes together; a bad key's probe is discarded
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + (int64_t)u * blockDim.x + threadIdx.x;
            if (i >= n) continue;
            uint64_t lab = kEmptyKey;  // -1: the point is on no kept tile
            if (!ok[u]) {
                bad = true;
            } else {
                // the table is at most half full: the walk ends at the key or an empty slot
                while (cur[u].x != key[u] && cur[u].x != kEmptyKey) {
                    pos[u] = (pos[u] + 1) & (cap - 1);
                    cur[u] = slots[pos[u]];
                }
                if (cur[u].x == key[u]) lab = cur[u].y;
            }
            out[i] = lab;
        }
    }
    if (bad) atomicOr(err, (unsigned long long)kErrRange);
}

// ---- per-tile point lists (RASTER', Section 3.4) -----------------------------
//
// The points of every kept tile, gathered after clustering by a second pass
// over the points: the row of each point's tile is looked up in a ROWS table
// and counted; the count's old value is the point's rank within its row.  The
// counts are scanned into row offsets and every point written to offset +
// rank.  Within a row the order is that of the counting atomics (a tile's
// points form a set).

constexpr uint32_t kNoRow = 0xFFFFFFFFu;

template <typename P>
__global__ __launch_bounds__(256) void k_point_rows(const P* __restrict__ pts, int64_t n, double scale,
                                                    const uint64_t* __restrict__ tab, uint64_t cap,
                                                    uint32_t* __restrict__ row_of,
                                                    uint32_t* __restrict__ rank, uint32_t* count,
                                                    unsigned long long* err) {
    typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
    const u64x2* __restrict__ slots = reinterpret_cast<const u64x2*>(tab);
    constexpr int U = 8;
    bool bad = false;
    for (int64_t i0 = (int64_t)blockIdx.x * U * blockDim.x; i0 < n; i0 += (int64_t)gridDim.x * U * blockDim.x) {
        double x[U], y[U], z[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            load_xyz(pts, min(i0 + (int64_t)u * blockDim.x + threadIdx.x, n - 1), x[u], y[u], z[u]);
        uint64_t key[U], pos[U];
        u64x2 cur[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            key[u] = 0;
            ok[u] = point_key<P>(x[u], y[u], z[u], scale, key[u]);
            pos[u] = slot_hash(key[u]) & (cap - 1);
            cur[u] = slots[pos[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + (int64_t)u * blockDim.x + threadIdx.x;
            if (i >= n) continue;
            uint32_t row = kNoRow, k = 0;
            if (!ok[u]) {
                bad = true;
            } else {
                while (cur[u].x != key[u] && cur[u].x != kEmptyKey) {
                    pos[u] = (pos[u] + 1) & (cap - 1);
                    cur[u] = slots[pos[u]];
                }
                if (cur[u].x == key[u]) {
                    row = (uint32_t)cur[u].y;
                    k = atomicAdd(count + row, 1u);
                }
            }
            row_of[i] = row;
            rank[i] = k;
        }
    }
    if (bad) atomicOr(err, (unsigned long long)kErrRange);
}

// pass 1 of the row-offset scan: the sum of each workgroup's range of counts
__global__ __launch_bounds__(SCAN_THREADS) void k_rows_sum(const uint32_t* count, uint64_t t, uint32_t* partials) {
    __shared__ uint32_t red[SCAN_WAVES];
    uint64_t lo, hi;
    block_range(t, lo, hi);
    uint32_t sum = 0;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += SCAN_THREADS) sum += count[i];
    sum = block_sum(sum, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = sum;
}

// pass 3: start[i] = points on rows before i (start[t] = all of them).  Each
// thread takes SCAN_ITEMS consecutive rows of a tile.
__global__ __launch_bounds__(SCAN_THREADS) void k_rows_start(const uint32_t* count, uint64_t t,
                                                             const uint32_t* partials,
                                                             const unsigned long long* total, uint64_t* start) {
    __shared__ uint32_t wsum[SCAN_WAVES];
    uint64_t lo, hi;
    block_range(t, lo, hi);
    uint64_t run = partials[blockIdx.x];
    for (uint64_t t0 = lo; t0 < hi; t0 += SCAN_TILE) {
        const uint64_t first = t0 + (uint64_t)threadIdx.x * SCAN_ITEMS;
        uint32_t v[SCAN_ITEMS];
        uint32_t mine = 0;
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            v[j] = first + j < hi ? count[first + j] : 0u;
            mine += v[j];
        }
        // exclusive scan of the per-thread sums over the workgroup
        uint32_t inc = mine;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off);
            if (lane_id() >= off) inc += o;
        }
        const int w = threadIdx.x >> 6;
        if (lane_id() == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t before = 0, tile_total = 0;
        for (int q = 0; q < SCAN_WAVES; ++q) {
            if (q < w) before += wsum[q];
            tile_total += wsum[q];
        }
        __syncthreads();  // wsum is reused by the next tile
        uint64_t at = run + before + inc - mine;
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            if (first + j < hi) start[first + j] = at;
            at += v[j];
        }
        run += tile_total;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) start[t] = *total;
}

// Each point on a kept tile goes to its row's offset plus its rank.  Rows,
// ranks and offsets of U items are loaded before the first store.
__global__ __launch_bounds__(256) void k_scatter_rows(const uint32_t* __restrict__ row_of,
                                                      const uint32_t* __restrict__ rank, int64_t n,
                                                      const uint64_t* __restrict__ start,
                                                      uint64_t* __restrict__ out) {
    constexpr int U = 8;
    for (int64_t i0 = (int64_t)blockIdx.x * U * blockDim.x; i0 < n; i0 += (int64_t)gridDim.x * U * blockDim.x) {
        uint32_t r[U], k[U];
        uint64_t at[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = min(i0 + (int64_t)u * blockDim.x + threadIdx.x, n - 1);
            r[u] = row_of[i];
            k[u] = rank[i];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) at[u] = r[u] != kNoRow ? start[r[u]] : 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + (int64_t)u * blockDim.x + threadIdx.x;
            if (i < n && r[u] != kNoRow) out[at[u] + k[u]] = (uint64_t)i;
        }
    }
}

// ---- per-job ranges and statistics (batches) ----------------------------------

__global__ void k_bounds(const uint32_t* seg_job, const unsigned long long* n_dev, uint32_t* start, uint32_t* end) {
    const uint64_t n = *n_dev;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t j = seg_job[i];
        if (i == 0 || seg_job[i - 1] != j) start[j] = (uint32_t)i;
        if (i + 1 == n || seg_job[i + 1] != j) end[j] = (uint32_t)(i + 1);
    }
}

// One workgroup per job: roots and kept roots among the job's compact tiles.
// Workgroups per job of the statistics pass; the job's range is shared
// between them round-robin.
constexpr uint32_t kJobStatSplit = 8;

__global__ __launch_bounds__(SCAN_THREADS) void k_job_stats(JobView jv, const uint32_t* root, const uint32_t* size,
                                                            const uint32_t* s_start, const uint32_t* s_end,
                                                            const uint32_t* o_start, const uint32_t* o_end) {
    __shared__ unsigned long long red[SCAN_WAVES];
    const uint32_t job = blockIdx.x / kJobStatSplit, part = blockIdx.x % kJobStatSplit;
    if (job >= jv.dims->njobs) return;  // uniform
    const uint32_t mu = jv.jobs[job].mu;
    const uint32_t a = s_start[job], b = s_end[job];
    unsigned long long comps = 0, kept = 0;
    for (uint32_t i = a + part * SCAN_THREADS + threadIdx.x; i < b; i += kJobStatSplit * SCAN_THREADS) {
        if (root[i] == i) {
            comps += 1;
            kept += (size[i] >= mu);
        }
    }
    comps = block_sum(comps, red);
    kept = block_sum(kept, red);
    if (threadIdx.x == 0) {
        unsigned long long* c = jv.job_ctr + (uint64_t)job * kCounterWords;
        if (comps) atomicAdd(&c[C_COMPONENTS], comps);
        if (kept) atomicAdd(&c[C_CLUSTERS], kept);
        if (part == 0) {
            c[C_SIGNIFICANT] = b - a;
            c[C_TILES] = o_end[job] - o_start[job];
        }
    }
}

// ---- batched counting: every job's points in one launch -----------------------

__global__ void k_fill_dims(Slot* tab, const Dims* dims) {
    const uint64_t cap = dims->slots;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < cap;
         i += (uint64_t)gridDim.x * blockDim.x) {
        Slot v;
        v.key = kEmptyKey;
        v.count = 0;
        v.aux = kNotSignificant;
        tab[i] = v;
    }
}

// Work tile t holds blockDim * ITEMS consecutive points of one job.  With
// lds_log2 > 0 the tile's keys are first combined in an LDS hash table and
// each distinct tile of the work tile is added once.
template <int ITEMS>
__global__ void k_batch_count(JobView jv, const uint32_t* tile_prefix, Slot* tab, int lds_log2) {
    extern __shared__ unsigned char smem[];
    const uint32_t tiles = jv.dims->tiles, njobs = jv.dims->njobs;
    const uint32_t L = lds_log2 > 0 ? (1u << lds_log2) : 0u;
    uint64_t* lkey = reinterpret_cast<uint64_t*>(smem);
    uint32_t* lcnt = reinterpret_cast<uint32_t*>(lkey + L);
    for (uint32_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const uint32_t job = job_of_tile(tile_prefix, njobs, t);
        const JobInfo& J = jv.jobs[job];
        Slot* jt = tab + J.slot_base;
        const Geo g = job_geo(J);  // batch jobs are two-dimensional
        unsigned long long* jc = jv.job_ctr + (uint64_t)job * kCounterWords;
        const int64_t base = (int64_t)(t - J.first_tile) * blockDim.x * ITEMS;
        if (L) {
            for (uint32_t q = threadIdx.x; q < L; q += blockDim.x) {
                lkey[q] = kEmptyKey;
                lcnt[q] = 0;
            }
            __syncthreads();
        }
        bool bad = false;
        uint32_t full = 0;
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int64_t i = base + (int64_t)j * blockDim.x + threadIdx.x;
            if (i >= J.n) continue;
            uint64_t k;
            if (!job_point_key(J, i, k)) {
                bad = true;
                continue;
            }
            bool done = false;
            if (L) {
                uint32_t pos = (slot_hash(k) >> 16) & (L - 1);
                for (int p = 0; p < 8 && !done; ++p) {
                    uint64_t cur = lds_load_relaxed(&lkey[pos]);
                    if (cur == kEmptyKey)
                        cur = atomicCAS(reinterpret_cast<unsigned long long*>(&lkey[pos]),
                                        (unsigned long long)kEmptyKey, (unsigned long long)k);
                    if (cur == kEmptyKey || cur == k) {
                        atomicAdd(&lcnt[pos], 1u);
                        done = true;
                    }
                    pos = (pos + 1) & (L - 1);
                }
            }
            if (!done) full += (table_add(jt, g, k, 1u) == ADD_FULL);
        }
        if (L) {
            __syncthreads();
            for (uint32_t q = threadIdx.x; q < L; q += blockDim.x) {
                const uint64_t k = lkey[q];
                if (k != kEmptyKey) full += (table_add(jt, g, k, lcnt[q]) == ADD_FULL);
            }
            __syncthreads();
        }
        if (bad) atomicOr(&jc[C_ERROR], (unsigned long long)kErrRange);
        if (full) atomicAdd(&jc[C_SPILLED], (unsigned long long)full);
    }
}

int grid_for(uint64_t work, int block, int max_blocks) {
    uint64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > (uint64_t)max_blocks) g = max_blocks;
    return (int)g;
}

// Persistent grids for the data-dependent passes: enough waves to fill 256
// CUs several times over.
constexpr int kPersistBlocks = 256 * 8;

// A launch timed by the events of `span` (recorded from the kernel's own
// dispatch) or untimed.
template <typename F, typename... Args>
void launch_k(F kernel, dim3 grid, dim3 block, uint32_t lds, hipStream_t stream, const KernelSpan& span,
              Args... args) {
    if (span.a)
        hipExtLaunchKernelGGL(kernel, grid, block, lds, stream, span.a, span.b, 0u, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, stream, args...);
}

template <typename T, int ITEMS>
hipError_t launch_count_t(const T* pts, int64_t n, double scale, Slot* tab, const Geo g, SpillBuf sp,
                          unsigned long long* ctr, const KernelTuning& tu, hipStream_t stream,
                          const KernelSpan& span) {
    const int block = tu.block;
    if (tu.preagg_slots > 0) {
        int lds_log2 = 0;
        while ((1 << lds_log2) < tu.preagg_slots) ++lds_log2;
        const int sweeps = tu.preagg_tiles > 0 ? tu.preagg_tiles : 1;
        const int64_t per_block = (int64_t)block * ITEMS * sweeps;
        const int64_t grid = (n + per_block - 1) / per_block;
        const size_t lds = (size_t)(1u << lds_log2) * (sizeof(uint64_t) + sizeof(uint32_t));
        launch_k(k_count_preagg<T, ITEMS>, dim3((unsigned)grid), dim3(block), (uint32_t)lds, stream, span, pts, n,
                 scale, tab, g, sp, ctr, lds_log2, sweeps);
    } else {
        const int64_t per_block = (int64_t)block * ITEMS;
        const int64_t grid = (n + per_block - 1) / per_block;
        launch_k(k_count_direct<T, ITEMS>, dim3((unsigned)grid), dim3(block), 0u, stream, span, pts, n, scale, tab, g,
                 sp, ctr);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_count_items(const T* pts, int64_t n, double scale, Slot* tab, const Geo g, SpillBuf sp,
                              unsigned long long* ctr, const KernelTuning& tu, hipStream_t stream,
                              const KernelSpan& span) {
    switch (tu.items) {
        case 1: return launch_count_t<T, 1>(pts, n, scale, tab, g, sp, ctr, tu, stream, span);
        case 2: return launch_count_t<T, 2>(pts, n, scale, tab, g, sp, ctr, tu, stream, span);
        case 4: return launch_count_t<T, 4>(pts, n, scale, tab, g, sp, ctr, tu, stream, span);
        case 8: return launch_count_t<T, 8>(pts, n, scale, tab, g, sp, ctr, tu, stream, span);
        default: return launch_count_t<T, 16>(pts, n, scale, tab, g, sp, ctr, tu, stream, span);
    }
}

}  // namespace

// ------------------------------------------------------------- launchers ---

hipError_t launch_fill_table(Slot* tab, uint64_t cap, hipStream_t stream) {
    hipLaunchKernelGGL(k_fill_table, dim3(grid_for(cap, 256, 65536)), dim3(256), 0, stream, tab, cap);
    return hipGetLastError();
}

hipError_t launch_zero_u64(uint64_t* p, uint64_t n, hipStream_t stream) {
    hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(n, 256, 65536)), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* p, uint64_t n, hipStream_t stream) {
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(n, 256, 65536)), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t launch_project_count(const void* pts, int64_t n, int dtype, double scale, Slot* tab, uint64_t cap,
                                 SpillBuf spill, unsigned long long* ctr, const KernelTuning& tu,
                                 hipStream_t stream, int dims, Frame frame, const KernelSpan& span) {
    if (n <= 0) return hipSuccess;
    const Geo g = make_geo(cap, dims == 3, frame);
    if (dims == 3) {
        if (dtype == 1)
            return launch_count_items(static_cast<const Pt3<float>*>(pts), n, scale, tab, g, spill, ctr, tu, stream,
                                      span);
        return launch_count_items(static_cast<const Pt3<double>*>(pts), n, scale, tab, g, spill, ctr, tu, stream,
                                  span);
    }
    if (dtype == 1)
        return launch_count_items(static_cast<const float*>(pts), n, scale, tab, g, spill, ctr, tu, stream, span);
    return launch_count_items(static_cast<const double*>(pts), n, scale, tab, g, spill, ctr, tu, stream, span);
}

hipError_t launch_bin_points(const void* pts, int64_t n, int dtype, double scale, uint64_t* bin1, uint64_t cap1,
                             uint32_t* cursor1, Slot* tab, uint64_t cap, SpillBuf spill, unsigned long long* ctr,
                             uint32_t* hll, hipStream_t stream, int dims, const KernelSpan& span) {
    if (n <= 0) return hipSuccess;
    const Geo g = make_geo(cap, dims == 3);
    const unsigned grid = (unsigned)((n + kBinTile - 1) / kBinTile);
    auto go = [&](auto kernel, const auto* p) {
        launch_k(kernel, dim3(grid), dim3(BIN_THREADS), 0u, stream, span, p, n, scale, bin1, cap1, cursor1, tab, g,
                 spill, ctr, hll);
    };
    if (dims == 3) {
        const Pt3<float>* pf = static_cast<const Pt3<float>*>(pts);
        const Pt3<double>* pd = static_cast<const Pt3<double>*>(pts);
        if (dtype == 1) {
            if (hll) go(k_bin_points<Pt3<float>, true>, pf);
            else go(k_bin_points<Pt3<float>, false>, pf);
        } else {
            if (hll) go(k_bin_points<Pt3<double>, true>, pd);
            else go(k_bin_points<Pt3<double>, false>, pd);
        }
        return hipGetLastError();
    }
    const float* pf = static_cast<const float*>(pts);
    const double* pd = static_cast<const double*>(pts);
    if (dtype == 1) {
        if (hll) go(k_bin_points<float, true>, pf);
        else go(k_bin_points<float, false>, pf);
    } else {
        if (hll) go(k_bin_points<double, true>, pd);
        else go(k_bin_points<double, false>, pd);
    }
    return hipGetLastError();
}

hipError_t launch_bin_keys(const uint64_t* bin1, uint64_t cap1, const uint32_t* cursor1, uint64_t* bin2,
                           uint64_t cap2, uint32_t* cursor2, Slot* tab, uint64_t cap, SpillBuf spill,
                           unsigned long long* ctr, hipStream_t stream, bool d3, const KernelSpan& span) {
    const Geo g = make_geo(cap, d3);
    if (!binned_geometry(g)) return hipErrorInvalidValue;
    const uint64_t lists2 = (uint64_t)kBinRep << g.p_log2;
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(lists2, 256, 4096)), dim3(256), 0, stream, cursor2, lists2);
    const uint32_t segs = (uint32_t)((cap1 + kBinTile - 1) / kBinTile);
    const dim3 grid(kBinRep * kCoarse * segs);
    if (d3)
        launch_k(k_bin_keys<true>, grid, dim3(BIN_THREADS), 0u, stream, span, bin1, cap1, cursor1, segs, bin2, cap2,
                 cursor2, tab, g, spill, ctr);
    else
        launch_k(k_bin_keys<false>, grid, dim3(BIN_THREADS), 0u, stream, span, bin1, cap1, cursor1, segs, bin2, cap2,
                 cursor2, tab, g, spill, ctr);
    return hipGetLastError();
}

hipError_t launch_aggregate(const uint64_t* bin2, uint64_t cap2, const uint32_t* cursor2, uint32_t* cursor1,
                            Slot* tab, uint64_t cap, SpillBuf spill, unsigned long long* ctr, hipStream_t stream,
                            const KernelSpan& span, bool whole, const AggCount& count) {
    const Geo g = make_geo(cap);  // the update only needs the partition count
    if (!binned_geometry(g)) return hipErrorInvalidValue;
    if (count.partials && count.blk_shift != scan_block_shift(cap)) return hipErrorInvalidValue;
    const uint64_t parts = 1ull << g.p_log2;
    hipLaunchKernelGGL(k_snapshot_keys, dim3(1), dim3(64), 0, stream, ctr);
    if (count.partials)
        hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(kScanBlocks, 256, 64)), dim3(256), 0, stream, count.partials,
                           (uint64_t)kScanBlocks);
    launch_k(k_aggregate, dim3((unsigned)parts), dim3(AGG_THREADS), 0u, stream, span, bin2, cap2, cursor2, tab, spill,
             ctr, whole, count);
    hipLaunchKernelGGL(k_zero_u32, dim3(4), dim3(256), 0, stream, cursor1, (uint64_t)kBinRep * kCoarse);
    return hipGetLastError();
}

hipError_t launch_drain_bins(uint64_t* bin1, uint64_t cap1, uint32_t* cursor1, Slot* tab, uint64_t cap,
                             SpillBuf spill, unsigned long long* ctr, hipStream_t stream, bool d3) {
    hipLaunchKernelGGL(k_drain_bins, dim3(grid_for((uint64_t)kBinRep * kCoarse * cap1, 256, kPersistBlocks)),
                       dim3(256), 0, stream, bin1, cap1, cursor1, tab, make_geo(cap, d3), spill, ctr);
    hipLaunchKernelGGL(k_zero_u32, dim3(4), dim3(256), 0, stream, cursor1, (uint64_t)kBinRep * kCoarse);
    return hipGetLastError();
}

hipError_t launch_insert_records(const uint64_t* keys, const uint32_t* counts, uint64_t n, Slot* tab,
                                 uint64_t cap, SpillBuf spill, unsigned long long* ctr, hipStream_t stream, bool d3,
                                 Frame frame) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_insert_records, dim3(grid_for(n, 256, kPersistBlocks)), dim3(256), 0, stream, keys,
                       counts, n, tab, make_geo(cap, d3, frame), spill, ctr);
    return hipGetLastError();
}

hipError_t launch_rehash(const Slot* from, uint64_t from_cap, Slot* to, uint64_t to_cap, SpillBuf spill,
                         unsigned long long* ctr, hipStream_t stream, bool d3, Frame frame) {
    hipLaunchKernelGGL(k_rehash, dim3(grid_for(from_cap, 256, kPersistBlocks)), dim3(256), 0, stream, from,
                       from_cap, to, make_geo(to_cap, d3, frame), spill, ctr);
    return hipGetLastError();
}

hipError_t launch_key_bbox(const void* pts, int64_t n, int dtype, double scale, uint32_t* out, hipStream_t stream) {
    uint32_t* part = out + 4;
    if (dtype == 1)
        hipLaunchKernelGGL(k_key_bbox<float>, dim3(kBboxBlocks), dim3(256), 0, stream, static_cast<const float*>(pts),
                           n, scale, part);
    else
        hipLaunchKernelGGL(k_key_bbox<double>, dim3(kBboxBlocks), dim3(256), 0, stream,
                           static_cast<const double*>(pts), n, scale, part);
    hipLaunchKernelGGL(k_bbox_merge, dim3(1), dim3(64), 0, stream, part, kBboxBlocks, out);
    return hipGetLastError();
}

hipError_t launch_bin_points_framed(const void* pts, int64_t n, int dtype, double scale, uint32_t* bin1,
                                   uint64_t cap1, uint32_t* cursor1, Slot* tab, uint64_t cap, Frame frame,
                                   SpillBuf spill, unsigned long long* ctr, uint32_t* hll, hipStream_t stream,
                                   const KernelSpan& span) {
    if (n <= 0) return hipSuccess;
    const Geo g = make_geo(cap, false, frame);
    if (!g.framed) return hipErrorInvalidValue;
    const uint32_t tile = BIN_THREADS * kFBinItems1;
    const dim3 grid((unsigned)((n + tile - 1) / tile));
    auto go = [&](auto kernel, const auto* p) {
        launch_k(kernel, grid, dim3(BIN_THREADS), 0u, stream, span, p, n, scale, bin1, cap1, cursor1, tab, g, spill,
                 ctr, hll);
    };
    const float* pf = static_cast<const float*>(pts);
    const double* pd = static_cast<const double*>(pts);
    if (dtype == 1) {
        if (hll) go(k_bin_points_f<float, true, kFBinItems1>, pf);
        else go(k_bin_points_f<float, false, kFBinItems1>, pf);
    } else {
        if (hll) go(k_bin_points_f<double, true, kFBinItems1>, pd);
        else go(k_bin_points_f<double, false, kFBinItems1>, pd);
    }
    return hipGetLastError();
}

hipError_t launch_bin_keys_framed(const uint32_t* bin1, uint64_t cap1, const uint32_t* cursor1, uint32_t* bin2,
                                 uint64_t cap2, uint32_t* cursor2, Slot* tab, uint64_t cap, Frame frame,
                                 SpillBuf spill, unsigned long long* ctr, hipStream_t stream,
                                 const KernelSpan& span) {
    const Geo g = make_geo(cap, false, frame);
    if (!framed_binned_geometry(g)) return hipErrorInvalidValue;
    const uint64_t lists2 = (uint64_t)kBinRep << g.p_log2;
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(lists2, 256, 4096)), dim3(256), 0, stream, cursor2, lists2);
    const uint32_t segs = (uint32_t)((cap1 + kFBinTile - 1) / kFBinTile);
    const dim3 grid(kBinRep * kFrameCoarse * segs);
    launch_k(k_bin_keys_f, grid, dim3(BIN_THREADS), 0u, stream, span, bin1, cap1, cursor1, segs, bin2, cap2, cursor2,
             tab, g, spill, ctr);
    return hipGetLastError();
}

hipError_t launch_aggregate_framed(const uint32_t* bin2, uint64_t cap2, const uint32_t* cursor2, uint32_t* cursor1,
                                  Slot* tab, uint64_t cap, Frame frame, SpillBuf spill, unsigned long long* ctr,
                                  hipStream_t stream, const KernelSpan& span, const AggCensus& census, bool whole,
                                  const AggCount& count) {
    const Geo g = make_geo(cap, false, frame);
    if (!framed_binned_geometry(g)) return hipErrorInvalidValue;
    if (census.rec && g.p_log2 <= kFrameCoarseLog2) return hipErrorInvalidValue;
    if (whole && census.img) return hipErrorInvalidValue;  // the image form does not write the table
    // the counting pass: the 4-byte claim-word update only, and never with a census
    if (count.partials && (census.rec || g.p_log2 <= kFrameCoarseLog2 || count.blk_shift != scan_block_shift(cap)))
        return hipErrorInvalidValue;
    const uint64_t parts = 1ull << g.p_log2;
    hipLaunchKernelGGL(k_snapshot_keys, dim3(1), dim3(64), 0, stream, ctr);
    if (census.rec) (void)launch_zero_u64(reinterpret_cast<uint64_t*>(ctr) + C_DISTINCT, C_SUM - C_DISTINCT + 1, stream);
    if (count.partials)
        hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(kScanBlocks, 256, 64)), dim3(256), 0, stream, count.partials,
                           (uint64_t)kScanBlocks);
    if (g.p_log2 > kFrameCoarseLog2)
        launch_k(k_aggregate_f32, dim3((unsigned)parts), dim3(AGG_THREADS), 0u, stream, span, bin2, cap2, cursor2, tab,
                 g, spill, ctr, census, whole, count);
    else
        launch_k(k_aggregate_f, dim3((unsigned)parts), dim3(AGG_THREADS), 0u, stream, span, bin2, cap2, cursor2, tab, g,
                 spill, ctr, whole);
    hipLaunchKernelGGL(k_zero_u32, dim3(8), dim3(256), 0, stream, cursor1, (uint64_t)kBinRep * kFrameCoarse);
    return hipGetLastError();
}

hipError_t launch_drain_bins_framed(const uint32_t* bin1, uint64_t cap1, uint32_t* cursor1, Slot* tab, uint64_t cap,
                                   Frame frame, SpillBuf spill, unsigned long long* ctr, hipStream_t stream) {
    const Geo g = make_geo(cap, false, frame);
    if (!g.framed) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_drain_bins_f, dim3(grid_for((uint64_t)kBinRep * kFrameCoarse * cap1, 256, kPersistBlocks)),
                       dim3(256), 0, stream, bin1, cap1, cursor1, tab, g, spill, ctr);
    hipLaunchKernelGGL(k_zero_u32, dim3(8), dim3(256), 0, stream, cursor1, (uint64_t)kBinRep * kFrameCoarse);
    return hipGetLastError();
}

hipError_t launch_export_tiles(const Slot* tab, uint64_t tcap, uint64_t* keys, uint32_t* counts, uint64_t cap,
                               uint32_t* partials, unsigned long long* ctr, hipStream_t stream) {
    hipLaunchKernelGGL(k_export_count, dim3(kScanBlocks), dim3(SCAN_THREADS), 0, stream, tab, tcap, partials, ctr);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, stream, partials, ctr + C_DISTINCT);
    hipLaunchKernelGGL(k_export_scatter, dim3(kScanBlocks), dim3(SCAN_THREADS), 0, stream, tab, tcap, partials,
                       keys, counts, cap);
    return hipGetLastError();
}

// Scan block of a partition for tables of 4096 * 2^k slots: block_range gives
// every block max(cap / kScanBlocks, 4096) slots, whole partitions.
uint32_t scan_block_shift(uint64_t cap) {
    const uint64_t parts = std::max<uint64_t>(cap >> kPartLog2, 1);
    uint32_t p_log2 = 0, s_log2 = 0;
    while ((1ull << p_log2) < parts) ++p_log2;
    while ((1ull << s_log2) < (uint64_t)kScanBlocks) ++s_log2;
    return p_log2 > s_log2 ? p_log2 - s_log2 : 0;
}

hipError_t launch_threshold(Slot* tab, const JobView& jv, uint64_t* s_key, uint32_t* s_count, uint32_t* size,
                            uint32_t* partials, unsigned long long* ctr, hipStream_t stream, uint64_t square_cap,
                            bool counted) {
    if (counted && square_cap) return hipErrorInvalidValue;  // the 2x2 marks change significance after the update
    if (square_cap) {
        const int grid = grid_for((square_cap + kPartSlots - 1) >> kPartLog2, 1, 8192);
        hipLaunchKernelGGL(k_square_part, dim3(grid), dim3(SQUARE_THREADS), 0, stream, tab, jv);
        hipLaunchKernelGGL(k_threshold_count<true>, dim3(kScanBlocks), dim3(SCAN_THREADS), 0, stream, tab, jv,
                           partials, ctr);
        hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, stream, partials, ctr + C_SIGNIFICANT);
        hipLaunchKernelGGL((k_threshold_scatter<true, false>), dim3(kScanBlocks), dim3(SCAN_THREADS), 0, stream, tab,
                           jv, partials, s_key, s_count, size, ctr);
    } else {
        if (!counted)
            hipLaunchKernelGGL(k_threshold_count<false>, dim3(kScanBlocks), dim3(SCAN_THREADS), 0, stream, tab, jv,
                               partials, ctr);
        hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, stream, partials, ctr + C_SIGNIFICANT);
        if (counted)
            hipLaunchKernelGGL((k_threshold_scatter<false, true>), dim3(kScanBlocks), dim3(SCAN_THREADS), 0, stream,
                               tab, jv, partials, s_key, s_count, size, ctr);
        else
            hipLaunchKernelGGL((k_threshold_scatter<false, false>), dim3(kScanBlocks), dim3(SCAN_THREADS), 0, stream,
                               tab, jv, partials, s_key, s_count, size, ctr);
    }
    return hipGetLastError();
}

hipError_t launch_agglomerate(const Slot* tab, uint64_t slots_max, const JobView& jv, const uint64_t* s_key,
                              uint32_t* parent, uint32_t* nbr, uint32_t* size, uint64_t s_max,
                              unsigned long long* ctr, hipStream_t stream, const NbrRound* rounds, int nrounds,
                              bool d3, Frame frame) {
    const int grid = (grid_for(s_max, 256, kPersistBlocks) + kXcds - 1) / kXcds * kXcds;
    const int link_grid = grid_for((slots_max + kPartSlots - 1) >> kPartLog2, 1, 8192);
    (void)d3;
    (void)frame;
    if (nrounds <= 0) {
        hipLaunchKernelGGL((k_link_part<false, false>), dim3(link_grid), dim3(LINK_THREADS), 0, stream, tab, jv,
                           parent, nbr, ctr, NbrGroup{});
        hipLaunchKernelGGL(k_jump, dim3(grid), dim3(256), 0, stream, parent, ctr);
        hipLaunchKernelGGL(k_merge, dim3(grid), dim3(256), 0, stream, nbr, 1u, s_key, parent, ctr);
    } else {
        // the first group builds the forest from its offsets; each later group
        // records the edges of up to kLinkGroup rounds more and unites along
        // them
        for (int r0 = 0; r0 < nrounds; r0 += kLinkGroup) {
            NbrGroup grp{};
            grp.nrounds = (uint32_t)std::min(kLinkGroup, nrounds - r0);
            for (uint32_t r = 0; r < grp.nrounds; ++r) grp.r[r] = rounds[r0 + r];
            grp.set_parent = r0 == 0 ? 1u : 0u;
            if (d3)
                hipLaunchKernelGGL((k_link_part<true, true>), dim3(link_grid), dim3(LINK_THREADS), 0, stream, tab, jv,
                                   parent, nbr, ctr, grp);
            else
                hipLaunchKernelGGL((k_link_part<true, false>), dim3(link_grid), dim3(LINK_THREADS), 0, stream, tab, jv,
                                   parent, nbr, ctr, grp);
            if (r0 == 0) hipLaunchKernelGGL(k_jump, dim3(grid), dim3(256), 0, stream, parent, ctr);
            hipLaunchKernelGGL(k_merge, dim3(grid), dim3(256), 0, stream, nbr, grp.nrounds, s_key, parent, ctr);
        }
    }
    // the neighbour lists are dead after the merge pass; their first s words
    // take the final roots
    hipLaunchKernelGGL(k_compress, dim3(grid), dim3(256), 0, stream, jv, parent, nbr, size, ctr);
    return hipGetLastError();
}

bool census_geometry(uint64_t cap, Frame frame) {
    const Geo g = make_geo(cap, false, frame);
    return g.framed && g.cp_log2 == kPartLog2 && g.p_log2 > kFrameCoarseLog2;
}

uint64_t census_words(uint64_t cap) { return (cap >> 5) * 2; }

hipError_t launch_census(Slot* tab, uint64_t cap, Frame frame, const JobView& jv, uint32_t tau, bool square,
                         uint32_t* words, uint32_t* partials, unsigned long long* ctr, hipStream_t stream) {
    const Geo g = make_geo(cap, false, frame);
    uint2* rec = reinterpret_cast<uint2*>(words);
    if (square) {
        const int grid = grid_for((cap + kPartSlots - 1) >> kPartLog2, 1, 8192);
        hipLaunchKernelGGL(k_square_part, dim3(grid), dim3(SQUARE_THREADS), 0, stream, tab, jv);
        hipLaunchKernelGGL(k_census_framed<true>, dim3(kScanBlocks), dim3(CENSUS_THREADS), 0, stream, tab, g, tau,
                           rec, partials, ctr);
    } else {
        hipLaunchKernelGGL(k_census_framed<false>, dim3(kScanBlocks), dim3(CENSUS_THREADS), 0, stream, tab, g, tau,
                           rec, partials, ctr);
    }
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, stream, partials, ctr + C_SIGNIFICANT);
    const uint64_t nrec = cap >> kCensusRecLog2;
    hipLaunchKernelGGL(k_census_offsets, dim3(grid_for(nrec, 256, 4096)), dim3(256), 0, stream, rec, nrec, partials,
                       census_blk_shift(g.p_log2));
    return hipGetLastError();
}

hipError_t launch_census_offsets(uint64_t cap, uint32_t* words, uint32_t* ptotal, unsigned long long* ctr,
                                 hipStream_t stream) {
    const uint64_t parts = cap >> kPartLog2, nrec = cap >> kCensusRecLog2;
    hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, stream, ptotal, (uint32_t)parts, ctr + C_SIGNIFICANT,
                       ptotal + parts, ctr);
    hipLaunchKernelGGL(k_census_offsets, dim3(grid_for(nrec, 256, 4096)), dim3(256), 0, stream,
                       reinterpret_cast<uint2*>(words), nrec, ptotal, 0u);
    return hipGetLastError();
}

hipError_t launch_image_to_table(const uint2* img, Slot* tab, uint64_t cap, Frame frame, hipStream_t stream) {
    hipLaunchKernelGGL(k_image_to_table, dim3(grid_for(cap, 256, 65536)), dim3(256), 0, stream, img, tab,
                       make_geo(cap, false, frame));
    return hipGetLastError();
}

hipError_t launch_link_census(const Slot* tab, const uint2* img, uint64_t cap, Frame frame, uint32_t mu, uint32_t tau,
                              bool square, const uint32_t* words, uint64_t* s_key, uint32_t* s_count,
                              uint32_t* parent, uint32_t* nbr, uint32_t* size, uint64_t s_max,
                              unsigned long long* ctr, hipStream_t stream, bool manhattan) {
    const Geo g = make_geo(cap, false, frame);
    const uint2* rec = reinterpret_cast<const uint2*>(words);
    const int grid = (grid_for(s_max, 256, kPersistBlocks) + kXcds - 1) / kXcds * kXcds;
    const int link_grid = grid_for(cap >> kPartLog2, 1, 8192);
    if (square && img) return hipErrorInvalidValue;  // the 2x2 marks are in the table only
    if (square)
        hipLaunchKernelGGL((k_link_census<true, false>), dim3(link_grid), dim3(LINK_THREADS), 0, stream, tab, img, g,
                           tau, manhattan, rec, s_key, s_count, size, parent, nbr, ctr);
    else if (img)
        hipLaunchKernelGGL((k_link_census<false, true>), dim3(link_grid), dim3(LINK_THREADS), 0, stream, tab, img, g,
                           tau, manhattan, rec, s_key, s_count, size, parent, nbr, ctr);
    else
        hipLaunchKernelGGL((k_link_census<false, false>), dim3(link_grid), dim3(LINK_THREADS), 0, stream, tab, img, g,
                           tau, manhattan, rec, s_key, s_count, size, parent, nbr, ctr);
    hipLaunchKernelGGL(k_jump, dim3(grid), dim3(256), 0, stream, parent, ctr);
    hipLaunchKernelGGL(k_merge, dim3(grid), dim3(256), 0, stream, nbr, 1u, s_key, parent, ctr);
    // the neighbour lists are dead after the merge pass; their first s words
    // take the final roots
    hipLaunchKernelGGL(k_compress_census, dim3(link_grid), dim3(512), 0, stream, rec, cap >> kPartLog2, mu,
                       parent, nbr, size, ctr);
    return hipGetLastError();
}

hipError_t launch_filter_count(const JobView& jv, const uint32_t* root, const uint32_t* size, uint32_t* partials,
                               unsigned long long* ctr, hipStream_t stream) {
    hipLaunchKernelGGL(k_filter_count, dim3(kScanBlocks), dim3(SCAN_THREADS), 0, stream, jv, root, size, partials,
                       ctr);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, stream, partials, ctr + C_TILES);
    return hipGetLastError();
}

hipError_t launch_filter_scatter(const JobView& jv, const uint64_t* s_key, const uint32_t* s_count,
                                 const uint32_t* root, const uint32_t* size, int32_t* out_kx, int32_t* out_ky,
                                 uint32_t* out_count, uint64_t* out_label, uint32_t* out_job,
                                 const uint32_t* partials, const unsigned long long* ctr, hipStream_t stream,
                                 int32_t* out_kz) {
    hipLaunchKernelGGL(k_filter_scatter, dim3(kScanBlocks), dim3(SCAN_THREADS), 0, stream, jv, s_key, s_count, root,
                       size, partials, ctr, out_kx, out_ky, out_kz, out_count, out_label, out_job);
    return hipGetLastError();
}

hipError_t launch_filter(const JobView& jv, const uint64_t* s_key, const uint32_t* s_count, const uint32_t* root,
                         const uint32_t* size, int32_t* out_kx, int32_t* out_ky, uint32_t* out_count,
                         uint64_t* out_label, uint32_t* out_job, uint32_t* partials, unsigned long long* ctr,
                         hipStream_t stream, int32_t* out_kz) {
    hipError_t e = launch_filter_count(jv, root, size, partials, ctr, stream);
    if (e != hipSuccess) return e;
    return launch_filter_scatter(jv, s_key, s_count, root, size, out_kx, out_ky, out_count, out_label, out_job,
                                 partials, ctr, stream, out_kz);
}

hipError_t launch_store_job(const Dims& d, const JobInfo& j, Dims* d_dims, JobInfo* d_job, hipStream_t stream) {
    hipLaunchKernelGGL(k_store_job, dim3(1), dim3(1), 0, stream, d, j, d_dims, d_job);
    return hipGetLastError();
}

hipError_t launch_batch_count(const JobView& jv, const uint32_t* tile_prefix, Slot* tab, const KernelTuning& tu,
                              int max_tiles_grid, hipStream_t stream) {
    int lds_log2 = 0;
    if (tu.preagg_slots > 0)
        while ((1 << lds_log2) < tu.preagg_slots) ++lds_log2;
    const size_t lds = lds_log2 ? (size_t)(1u << lds_log2) * (sizeof(uint64_t) + sizeof(uint32_t)) : 0;
    const dim3 grid((unsigned)max_tiles_grid), block((unsigned)tu.block);
    switch (tu.items) {
        case 1: hipLaunchKernelGGL(k_batch_count<1>, grid, block, lds, stream, jv, tile_prefix, tab, lds_log2); break;
        case 2: hipLaunchKernelGGL(k_batch_count<2>, grid, block, lds, stream, jv, tile_prefix, tab, lds_log2); break;
        case 4: hipLaunchKernelGGL(k_batch_count<4>, grid, block, lds, stream, jv, tile_prefix, tab, lds_log2); break;
        case 8: hipLaunchKernelGGL(k_batch_count<8>, grid, block, lds, stream, jv, tile_prefix, tab, lds_log2); break;
        default: hipLaunchKernelGGL(k_batch_count<16>, grid, block, lds, stream, jv, tile_prefix, tab, lds_log2); break;
    }
    return hipGetLastError();
}

hipError_t launch_batch_binned(const JobView& jv, const uint32_t* tile_prefix, const uint32_t* cjob, uint64_t* bin1,
                               uint32_t* cursor1, uint64_t* bin2, uint32_t* cursor2, Slot* tab, hipStream_t stream) {
    hipLaunchKernelGGL(k_bbin_points, dim3(4096), dim3(BIN_THREADS), 0, stream, jv, tile_prefix, bin1, cursor1, tab);
    hipLaunchKernelGGL(k_bbin_keys, dim3(8192), dim3(BIN_THREADS), 0, stream, jv, cjob, bin1, cursor1, bin2, cursor2,
                       tab);
    hipLaunchKernelGGL(k_bagg, dim3(4096), dim3(AGG_THREADS), 0, stream, jv, bin2, cursor2, tab);
    return hipGetLastError();
}

hipError_t launch_label_table(const int32_t* kx, const int32_t* ky, const uint64_t* label, uint64_t t,
                              uint64_t* tab, uint64_t cap, bool rows, hipStream_t stream, const int32_t* kz) {
    hipLaunchKernelGGL(k_fill_words, dim3(grid_for(2 * cap, 256, kPersistBlocks)), dim3(256), 0, stream, tab,
                       2 * cap, kEmptyKey);
    if (t)
    {
        if (rows)
            hipLaunchKernelGGL(k_label_table<true>, dim3(grid_for(t, 256, kPersistBlocks)), dim3(256), 0, stream, kx,
                               ky, kz, label, t, tab, cap);
        else
            hipLaunchKernelGGL(k_label_table<false>, dim3(grid_for(t, 256, kPersistBlocks)), dim3(256), 0, stream, kx,
                               ky, kz, label, t, tab, cap);
    }
    return hipGetLastError();
}

hipError_t launch_point_labels(const void* pts, int64_t n, int dtype, double scale, const uint64_t* tab,
                               uint64_t cap, uint64_t* out, unsigned long long* err, hipStream_t stream, int dims) {
    if (n <= 0) return hipSuccess;
    const unsigned grid = (unsigned)grid_for((uint64_t)n, 256 * 8, 8192);
    if (dims == 3 && dtype == 1)
        hipLaunchKernelGGL(k_point_labels<Pt3<float>>, dim3(grid), dim3(256), 0, stream,
                           static_cast<const Pt3<float>*>(pts), n, scale, tab, cap, out, err);
    else if (dims == 3)
        hipLaunchKernelGGL(k_point_labels<Pt3<double>>, dim3(grid), dim3(256), 0, stream,
                           static_cast<const Pt3<double>*>(pts), n, scale, tab, cap, out, err);
    else if (dtype == 1)
        hipLaunchKernelGGL(k_point_labels<float>, dim3(grid), dim3(256), 0, stream, static_cast<const float*>(pts), n,
                           scale, tab, cap, out, err);
    else
        hipLaunchKernelGGL(k_point_labels<double>, dim3(grid), dim3(256), 0, stream,
                           static_cast<const double*>(pts), n, scale, tab, cap, out, err);
    return hipGetLastError();
}

hipError_t launch_tile_points_count(const void* pts, int64_t n, int dtype, double scale, const uint64_t* tab,
                                   uint64_t cap, uint32_t* row_of, uint32_t* rank, uint32_t* count, uint64_t t,
                                   uint32_t* partials, unsigned long long* total, uint64_t* start,
                                   unsigned long long* err, hipStream_t stream, int dims) {
    if (n > 0) {
        const unsigned grid = (unsigned)grid_for((uint64_t)n, 256 * 8, 8192);
        if (dims == 3 && dtype == 1)
            hipLaunchKernelGGL(k_point_rows<Pt3<float>>, dim3(grid), dim3(256), 0, stream,
                               static_cast<const Pt3<float>*>(pts), n, scale, tab, cap, row_of, rank, count, err);
        else if (dims == 3)
            hipLaunchKernelGGL(k_point_rows<Pt3<double>>, dim3(grid), dim3(256), 0, stream,
                               static_cast<const Pt3<double>*>(pts), n, scale, tab, cap, row_of, rank, count, err);
        else if (dtype == 1)
            hipLaunchKernelGGL(k_point_rows<float>, dim3(grid), dim3(256), 0, stream, static_cast<const float*>(pts), n,
                               scale, tab, cap, row_of, rank, count, err);
        else
            hipLaunchKernelGGL(k_point_rows<double>, dim3(grid), dim3(256), 0, stream, static_cast<const double*>(pts),
                               n, scale, tab, cap, row_of, rank, count, err);
    }
    hipLaunchKernelGGL(k_rows_sum, dim3(kScanBlocks), dim3(SCAN_THREADS), 0, stream, count, t, partials);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, stream, partials, total);
    hipLaunchKernelGGL(k_rows_start, dim3(kScanBlocks), dim3(SCAN_THREADS), 0, stream, count, t, partials, total,
                       start);
    return hipGetLastError();
}

hipError_t launch_tile_points_scatter(const uint32_t* row_of, const uint32_t* rank, int64_t n,
                                      const uint64_t* start, uint64_t* out, hipStream_t stream) {
    if (n > 0)
        hipLaunchKernelGGL(k_scatter_rows, dim3(grid_for((uint64_t)n, 256 * 8, 8192)), dim3(256), 0, stream, row_of,
                           rank, n, start, out);
    return hipGetLastError();
}

hipError_t launch_points_hll(const void* pts, int64_t n, int dtype, double scale, uint32_t* hll,
                             hipStream_t stream, int dims) {
    if (n <= 0) return hipSuccess;
    const unsigned grid = (unsigned)grid_for((uint64_t)n, 256 * 16, 4096);
    if (dims == 3) {
        if (dtype == 1)
            hipLaunchKernelGGL(k_points_hll<Pt3<float>>, dim3(grid), dim3(256), 0, stream,
                               static_cast<const Pt3<float>*>(pts), n, scale, hll);
        else
            hipLaunchKernelGGL(k_points_hll<Pt3<double>>, dim3(grid), dim3(256), 0, stream,
                               static_cast<const Pt3<double>*>(pts), n, scale, hll);
    } else if (dtype == 1) {
        hipLaunchKernelGGL(k_points_hll<float>, dim3(grid), dim3(256), 0, stream, static_cast<const float*>(pts), n,
                           scale, hll);
    } else {
        hipLaunchKernelGGL(k_points_hll<double>, dim3(grid), dim3(256), 0, stream, static_cast<const double*>(pts), n,
                           scale, hll);
    }
    return hipGetLastError();
}

hipError_t launch_batch_hll(const JobView& jv, const uint32_t* tile_prefix, uint32_t tile, uint32_t* hll,
                            uint32_t njobs, uint32_t tiles, hipStream_t stream) {
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for((uint64_t)njobs << kHllLog2, 256, 256)), dim3(256), 0, stream, hll,
                       (uint64_t)njobs << kHllLog2);
    if (tiles)
        hipLaunchKernelGGL(k_batch_hll, dim3(grid_for(tiles, 1, 8192)), dim3(256), 0, stream, jv, tile_prefix, tile,
                           hll);
    return hipGetLastError();
}

hipError_t launch_fill_dims(Slot* tab, const Dims* dims, hipStream_t stream) {
    hipLaunchKernelGGL(k_fill_dims, dim3(8192), dim3(256), 0, stream, tab, dims);
    return hipGetLastError();
}

hipError_t launch_bounds(const uint32_t* seg_job, const unsigned long long* n, uint32_t* start, uint32_t* end,
                         uint64_t n_max, hipStream_t stream) {
    hipLaunchKernelGGL(k_bounds, dim3(grid_for(n_max, 256, kPersistBlocks)), dim3(256), 0, stream, seg_job, n, start,
                       end);
    return hipGetLastError();
}

hipError_t launch_job_stats(const JobView& jv, const uint32_t* root, const uint32_t* size, const uint32_t* s_start,
                            const uint32_t* s_end, const uint32_t* o_start, const uint32_t* o_end,
                            uint32_t max_jobs, hipStream_t stream) {
    hipLaunchKernelGGL(k_job_stats, dim3(max_jobs * kJobStatSplit), dim3(SCAN_THREADS), 0, stream, jv, root, size,
                       s_start, s_end,
                       o_start, o_end);
    return hipGetLastError();
}

}  // namespace rst
