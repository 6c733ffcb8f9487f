// Internal interface between the host runtime (raster_host.cpp) and the
// gfx950 kernels (raster_kernels.hip).  Not installed; not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rst {

// Empty marker of a table slot.  A valid biased key has a high word of at
// most 2^32 - 2, so it never equals this value.
constexpr uint64_t kEmptyKey = ~0ull;
// aux of a slot whose tile is not significant.
constexpr uint32_t kNotSignificant = 0xFFFFFFFFu;
constexpr uint32_t kSquareKeep = 0xFFFFFFFEu;  // aux of a slot kept by the 2x2 post-step
// Longest probe window of the open-addressing table.  A key lives within this
// many slots of its home slot; an insert that finds the window full of other
// keys spills the key instead, and the table is grown afterwards.
constexpr uint32_t kMaxProbe = 128;

// Table geometry.  The table is cut into partitions of 2^cp_log2 slots
// (4096 once the table is that large); a key's partition is the top p_log2
// bits of its placement hash, its home slot inside the partition the low
// cp_log2 bits of its own hash, and probing wraps inside the partition.  A
// partition is then exactly the slice one workgroup can hold in LDS, and the
// top placement-hash bits name a key's partition whatever the table size.
constexpr uint32_t kPartLog2 = 12;
// A key's partition is chosen by the hash of its super-tile, the square of
// 2^kSuperLog2 x 2^kSuperLog2 tiles that holds it; the slot inside the
// partition by the hash of the key itself.  Tiles that touch usually share a
// partition, so the neighbour lookups and union-find of the agglomeration
// stay inside one 64 KB slice of the table and one short run of the compact
// significant-tile arrays.  A super-tile holds at most 2^(2 kSuperLog2) keys,
// which bounds how unevenly keys spread over partitions.
constexpr uint32_t kSuperLog2 = 3;
constexpr uint64_t kSuperMask = ~((((1ull << kSuperLog2) - 1) << 32) | ((1ull << kSuperLog2) - 1));
// Key frame of a two-dimensional table: a window of 2^kFrameLog2 x
// 2^kFrameLog2 tiles whose smallest biased coordinates are (fx, fy).  A key
// inside the frame is placed by a bijective 34-bit mix h of its super-tile's
// position in the frame: its partition is the top bits of h, its home slot the
// hash of its 32-bit "entry" (the low 26 bits of h and the key's position in
// its super-tile).  The top kFrameCoarseLog2 bits of h pick the key's coarse
// bucket in the binned contraction, so the coarse bucket and the entry give
// the key back exactly, and the binning moves 4-byte entries instead of
// 8-byte keys.  A key outside the frame is placed as in an unframed table.
// on = 0: no frame.
constexpr uint32_t kFrameLog2 = 20;
constexpr uint32_t kFrameStBits = 2 * (kFrameLog2 - 3);  // bits of a super-tile's position (8 x 8 super-tiles)
constexpr uint32_t kFrameCoarseLog2 = 8;
constexpr uint32_t kFrameCoarse = 1u << kFrameCoarseLog2;
constexpr uint32_t kFrameHLow = kFrameStBits - kFrameCoarseLog2;  // h bits held by an entry (26)
struct Frame {
    uint32_t on;
    uint32_t fx, fy;  // biased coordinates of the frame's first tile
};

struct Geo {
    uint64_t cap;      // slots, a power of two
    uint32_t cp_log2;  // log2 slots per partition
    uint32_t p_log2;   // log2 partitions
    uint32_t d3;       // 1: three-dimensional keys (placed by 4x4x4 super-cubes)
    uint32_t framed;   // 1: keys inside the frame (fx, fy) are placed by their frame position
    uint32_t fx, fy;
};
__host__ __device__ inline Geo make_geo(uint64_t cap, bool d3 = false, Frame f = Frame{0, 0, 0}) {
    const uint32_t l = (uint32_t)__builtin_ctzll(cap);  // cap is a power of two
    Geo g;
    g.cap = cap;
    g.cp_log2 = l < kPartLog2 ? l : kPartLog2;
    g.p_log2 = l - g.cp_log2;
    g.d3 = d3 ? 1u : 0u;
    g.framed = (f.on && !d3) ? 1u : 0u;
    g.fx = f.fx;
    g.fy = f.fy;
    return g;
}

// Binned contraction: keys are first binned into 2^kCoarseLog2 buckets by the
// top bits of their hash, then each bucket into its partitions, then every
// partition is updated in LDS by one workgroup.  It needs at least one
// partition per coarse bucket and at most kMaxFine partitions per bucket.
constexpr uint32_t kCoarseLog2 = 7;
constexpr uint32_t kCoarse = 1u << kCoarseLog2;
constexpr uint32_t kMaxFine = 512;
// Every bucket of both binning levels is kept as kBinRep lists, each with its
// own cursor; a workgroup appends to one of them.  Cursor updates from many
// workgroups to one cache line serialise in the memory-side atomic unit, so
// spreading them over kBinRep lines is what lets the binning run at stream
// speed.
constexpr uint32_t kBinRep = 8;

// Distinct-tile sketches: 2^kHllLog2 HyperLogLog registers over a fixed 1/64
// hash sample of the tiles; kHllReps replicas where many workgroups merge.
constexpr uint32_t kHllLog2 = 8;
constexpr uint32_t kHllReps = 64;

inline bool binned_geometry(const Geo& g) {
    return g.cp_log2 == kPartLog2 && g.p_log2 >= kCoarseLog2 && (1ull << (g.p_log2 - kCoarseLog2)) <= kMaxFine;
}
// The same for the framed binning (kFrameCoarse coarse buckets of entries).
inline bool framed_binned_geometry(const Geo& g) {
    return g.framed && g.cp_log2 == kPartLog2 && g.p_log2 >= kFrameCoarseLog2 &&
           (1ull << (g.p_log2 - kFrameCoarseLog2)) <= kMaxFine;
}

// One table slot: 16 bytes, so a probe and the count update touch one line.
struct alignas(16) Slot {
    uint64_t key;    // biased tile key or kEmptyKey
    uint32_t count;  // points on the tile
    uint32_t aux;    // after the significance scan: compact index or kNotSignificant
};
static_assert(sizeof(Slot) == 16, "slot must be 16 bytes");

// Device counter words (unsigned 64-bit), one block per table / job.
enum CounterIndex : int {
    C_INSERTED = 0,  // new keys inserted by counting kernels
    C_SPILLED,       // spill records written (points or rehash entries)
    C_ERROR,         // kErr* bits
    C_DISTINCT,      // occupied slots (m), from the significance scan
    C_SIGNIFICANT,   // s
    C_SUM,           // sum of all counts (equals the points counted)
    C_COMPONENTS,    // roots of the union-find forest
    C_CLUSTERS,      // roots with at least mu tiles
    C_TILES,         // output rows t
    C_TABLE_KEYS,    // keys in the table before a binned update (0: the slices need not be read)
    C_COUNT_
};
constexpr int kCounterWords = 16;  // padded to 128 bytes

constexpr uint64_t kErrRange = 1;
constexpr uint64_t kErrSpillOverflow = 2;
constexpr uint64_t kErrInternal = 4;  // union-find walk hit its bound or an index out of range

// Per-job parameters read by the kernels.  A single table is one job with
// slot_base 0; a batch lays its jobs' tables one after another in one arena,
// each a whole number of 4096-slot partitions.
struct JobInfo {
    const void* pts;      // batched counting: the job's points
    int64_t n;            // batched counting: its point count
    double scale;
    uint64_t slot_base;   // first slot of the job's table
    uint64_t cap;         // slots of the job's table (power of two)
    uint32_t tau, mu;
    int32_t dtype;        // 1 = FP32, 2 = FP64
    uint32_t first_tile;  // batched counting: first point tile of the job
    uint32_t part_base;   // slot_base / 4096: first partition of the job
    uint32_t cbase;       // binned batches: first coarse bucket of the job
    uint32_t cshift;      // binned batches: log2 partitions per coarse bucket
    uint32_t cap2;        // binned batches: keys per partition list of the job
    uint64_t bin2_base;   // binned batches: first key of the job's partition lists
    uint32_t framed;      // single tables: the table's key frame (Geo::framed, fx, fy)
    uint32_t fx, fy;
    uint32_t pad_;
};
__host__ __device__ inline Geo job_geo(const JobInfo& J, bool d3 = false) {
    return make_geo(J.cap, d3, Frame{J.framed, J.fx, J.fy});
}

// One round of the link pass for a neighbourhood other than the eight
// adjacent tiles: up to four backward offsets (the neighbour's key is smaller,
// so each edge is seen once, from its larger-key end).
struct NbrRound {
    int32_t dx[4], dy[4], dz[4];  // dz: 3-D keys only
    uint32_t count;               // offsets in use, 1..4
};
constexpr uint32_t kMaxDelta = 8;

// The rounds one launch of the link pass covers: the partition slice is read
// into LDS once for all of them, and one merge pass unites along all of their
// edges.  The first group also sets every tile's parent to its smallest-key
// neighbour among its offsets; later groups only record edges.
constexpr int kLinkGroup = 4;
struct NbrGroup {
    NbrRound r[kLinkGroup];
    uint32_t nrounds;     // rounds in use, 1..kLinkGroup
    uint32_t set_parent;  // 1 in the first group
};

// Neighbour-list words per significant tile for a neighbourhood of `nrounds`
// rounds (0: the eight adjacent tiles): four per round of one group.
inline uint64_t nbr_words(int nrounds) {
    return 4u * (uint64_t)(nrounds <= 1 ? 1 : nrounds < kLinkGroup ? nrounds : kLinkGroup);
}

// Sizes read from device memory, so that a captured graph can be replayed
// for any batch that fits its buffers.
struct Dims {
    uint64_t slots;    // table slots in use (all jobs)
    uint32_t njobs;
    uint32_t tiles;    // point tiles of the batched counting launch
    uint64_t cap1;     // binned batches: keys per coarse bucket
    uint64_t cap2;     // unused (partition-list capacities are per job)
    uint32_t ncoarse;  // binned batches: coarse buckets in use
    uint32_t segs;     // binned batches: kBinTile segments per coarse bucket
};

// Job-aware views passed to the post-contraction kernels.  part_job maps a
// 4096-slot partition to its job and s_job a compact tile to its job; both
// are null for a single table, and non-null for a batch (even of one job).
struct JobView {
    const Dims* dims;
    const JobInfo* jobs;
    const uint32_t* part_job;
    uint32_t* s_job;
    unsigned long long* job_ctr;  // kCounterWords per job (multi-job only)
};

// Overflow records of the counting kernels.
struct SpillBuf {
    uint64_t* keys;
    uint32_t* counts;
    uint64_t cap;
};

struct KernelTuning {
    int block;         // threads per workgroup of the counting kernel
    int items;         // points per thread per sweep
    int preagg_slots;  // LDS pre-aggregation slots (0 = off)
    int preagg_tiles;  // sweeps a workgroup aggregates before flushing its LDS table
};

// Fixed number of workgroups of the scan passes; the partial-sum array of a
// scan holds this many entries.
constexpr int kScanBlocks = 2048;

// Keys per binning tile (one workgroup pass).
constexpr uint32_t kBinTile = 4096;

// ---- launchers (all enqueue on `stream`, none synchronises) ------------------

hipError_t launch_fill_table(Slot* tab, uint64_t cap, hipStream_t stream);
hipError_t launch_zero_u64(uint64_t* p, uint64_t n, hipStream_t stream);
hipError_t launch_zero_u32(uint32_t* p, uint64_t n, hipStream_t stream);

// Projection + counting of n points into the table (dtype 1 = f32, 2 = f64).
// Events that a timed launch records around its main kernel (taken from
// the kernel's own dispatch, so that timing adds no commands between
// launches); both null: untimed.
struct KernelSpan {
    hipEvent_t a = nullptr, b = nullptr;
};

hipError_t launch_project_count(const void* pts, int64_t n, int dtype, double scale, Slot* tab,
                                 uint64_t cap, SpillBuf spill, unsigned long long* ctr,
                                 const KernelTuning& tu, hipStream_t stream, int dims = 2, Frame frame = Frame{},
                                 const KernelSpan& span = KernelSpan{});

// Tile bounding box of the first n points (two dimensions): out[0..3] =
// smallest and largest biased x, smallest and largest biased y over the
// points with a valid tile (out[0] > out[1] when there is none).  out holds
// kBboxWords words (the rest is scratch).
constexpr int kBboxWords = 4 + 4 * 256;
hipError_t launch_key_bbox(const void* pts, int64_t n, int dtype, double scale, uint32_t* out, hipStream_t stream);

// Framed binned contraction (two dimensions): level 1 appends the entry of
// each point's key to coarse list (replica, h >> kFrameHLow) of bin1
// (kBinRep * kFrameCoarse lists of cap1 entries, counts in cursor1); keys
// outside the frame, and keys past a full list, go straight into the table.
hipError_t launch_bin_points_framed(const void* pts, int64_t n, int dtype, double scale, uint32_t* bin1,
                                   uint64_t cap1, uint32_t* cursor1, Slot* tab, uint64_t cap, Frame frame,
                                   SpillBuf spill, unsigned long long* ctr, uint32_t* hll, hipStream_t stream,
                                   const KernelSpan& span = KernelSpan{});
// Level 2: every coarse list into its partitions' lists (bin2, cap2 entries
// per list; counts in cursor2, cleared here).
hipError_t launch_bin_keys_framed(const uint32_t* bin1, uint64_t cap1, const uint32_t* cursor1, uint32_t* bin2,
                                 uint64_t cap2, uint32_t* cursor2, Slot* tab, uint64_t cap, Frame frame,
                                 SpillBuf spill, unsigned long long* ctr, hipStream_t stream,
                                 const KernelSpan& span = KernelSpan{});
// The final update of an unframed table, or of a framed one of 512+
// partitions without a census, can do the significance scan's counting
// pass: each workgroup adds its partition's slots with count >= tau to
// partials[p >> blk_shift] (the scan block holding the partition: blocks are
// whole partitions for any table of 4096 * 2^k slots; cleared first).
// The scatter pass then totals the occupied slots and their counts.
struct AggCount {
    uint32_t* partials = nullptr;  // kScanBlocks words; null: no counting
    uint32_t tau = 0;
    uint32_t blk_shift = 0;
};
uint32_t scan_block_shift(uint64_t cap);

// Census of the final update (rec null: none): with the table's final
// slices in LDS, the update of a table of 512+ partitions also writes the
// census records of every partition (counts before each 32 slots within the
// partition; rec: 2 words per 32 slots) and, in ptotal (3 words per
// partition), each partition's significant count, then its occupied slots,
// then its count sum.  launch_census_offsets then makes the counts global, as
// launch_census leaves them, and totals the occupied slots and counts in
// ctr[C_DISTINCT] and ctr[C_SUM].
struct AggCensus {
    uint2* rec = nullptr;
    uint32_t* ptotal = nullptr;
    uint32_t tau = 0;
    // non-null: the update writes each slice's image (entry and count per
    // slot, cap pairs) instead of the table; launch_image_to_table writes the
    // keys into the table when it has to grow afterwards
    uint2* img = nullptr;
};
// Update: one workgroup per partition adds its entries to the table in LDS;
// then clears cursor1.  With `whole` (a table not filled yet, holding no key)
// every slot is written, the empty ones too, which fills the table.
hipError_t launch_aggregate_framed(const uint32_t* bin2, uint64_t cap2, const uint32_t* cursor2, uint32_t* cursor1,
                                  Slot* tab, uint64_t cap, Frame frame, SpillBuf spill, unsigned long long* ctr,
                                  hipStream_t stream, const KernelSpan& span = KernelSpan{},
                                  const AggCensus& census = AggCensus{}, bool whole = false,
                                  const AggCount& count = AggCount{});
hipError_t launch_census_offsets(uint64_t cap, uint32_t* words, uint32_t* ptotal, unsigned long long* ctr,
                                 hipStream_t stream);
// Direct insertion of every entry held in the coarse lists (tables outside
// the framed binned geometry).  Clears cursor1.
hipError_t launch_drain_bins_framed(const uint32_t* bin1, uint64_t cap1, uint32_t* cursor1, Slot* tab, uint64_t cap,
                                   Frame frame, SpillBuf spill, unsigned long long* ctr, hipStream_t stream);

// Binned contraction, level 1: project n points and append each key to its
// coarse bucket: bucket b holds keys at bin1[b * cap1 + i], i < cursor1[b].
// Keys past a bucket's capacity go straight into the table, or into the
// spill buffer when tab is null (a table not filled yet); so in level 2.
// hll, if not null, gets the distinct-tile sketch of the keys (kHllReps
// replicas of 2^kHllLog2 registers; merge them by maximum).
hipError_t launch_bin_points(const void* pts, int64_t n, int dtype, double scale, uint64_t* bin1, uint64_t cap1,
                             uint32_t* cursor1, Slot* tab, uint64_t cap, SpillBuf spill, unsigned long long* ctr,
                             uint32_t* hll, hipStream_t stream, int dims = 2, const KernelSpan& span = KernelSpan{});
// Binned contraction, level 2: split every coarse bucket into its partitions
// (bin2, cap2 keys per partition, counts in cursor2, which this clears first).
hipError_t launch_bin_keys(const uint64_t* bin1, uint64_t cap1, const uint32_t* cursor1, uint64_t* bin2,
                           uint64_t cap2, uint32_t* cursor2, Slot* tab, uint64_t cap, SpillBuf spill,
                           unsigned long long* ctr, hipStream_t stream, bool d3 = false,
                           const KernelSpan& span = KernelSpan{});
// Binned contraction, update: one workgroup per partition adds that
// partition's keys to the table in LDS; then clears cursor1 for the next group.
// `whole` as for launch_aggregate_framed.
hipError_t launch_aggregate(const uint64_t* bin2, uint64_t cap2, const uint32_t* cursor2, uint32_t* cursor1,
                            Slot* tab, uint64_t cap, SpillBuf spill, unsigned long long* ctr, hipStream_t stream,
                            const KernelSpan& span = KernelSpan{}, bool whole = false,
                            const AggCount& count = AggCount{});
// Direct insertion of everything held in the coarse buckets (used when the
// table is outside the binned geometry).  Clears cursor1.
hipError_t launch_drain_bins(uint64_t* bin1, uint64_t cap1, uint32_t* cursor1, Slot* tab, uint64_t cap,
                             SpillBuf spill, unsigned long long* ctr, hipStream_t stream, bool d3 = false);

// Insert n (key, count) records (spilled keys, or a rehash source).
hipError_t launch_insert_records(const uint64_t* keys, const uint32_t* counts, uint64_t n,
                                 Slot* tab, uint64_t cap, SpillBuf spill, unsigned long long* ctr,
                                 hipStream_t stream, bool d3 = false, Frame frame = Frame{});

// Move every occupied slot of `from` into `to` (a larger table).
hipError_t launch_rehash(const Slot* from, uint64_t from_cap, Slot* to, uint64_t to_cap,
                         SpillBuf spill, unsigned long long* ctr, hipStream_t stream, bool d3 = false,
                         Frame frame = Frame{});

// Export every occupied (key, count) pair, compacted; writes at most cap rows,
// and the number of occupied slots to ctr[C_DISTINCT].
hipError_t launch_export_tiles(const Slot* tab, uint64_t tcap, uint64_t* keys, uint32_t* counts,
                               uint64_t cap, uint32_t* partials, unsigned long long* ctr,
                               hipStream_t stream);

// Significance scan: flags count >= tau (per job), writes the compact arrays
// S_key, S_count (and S_job for several jobs), sets slot.aux, zeroes size[i],
// and fills ctr[C_DISTINCT], ctr[C_SIGNIFICANT], ctr[C_SUM] (per job too).
// With `counted` (one job, no 2x2 step) the final update has already counted
// the significant slots per scan block into partials (AggCount): the
// counting pass is skipped, and the scatter pass fills ctr[C_DISTINCT] and
// ctr[C_SUM] (cleared by the caller).
hipError_t launch_threshold(Slot* tab, const JobView& jv, uint64_t* s_key, uint32_t* s_count, uint32_t* size,
                            uint32_t* partials, unsigned long long* ctr, hipStream_t stream,
                            uint64_t square_cap = 0, bool counted = false);

// Connected components of the significant tiles (8-adjacency).  On return
// nbr[i] (its first s words) holds the compact index of the smallest tile of
// tile i's component; the component count goes to ctr[C_COMPONENTS] and
// size[root] counts members up to the job's mu (size[root] >= mu exactly when
// the component has at least mu tiles).  parent is scratch; nbr is scratch of
// nbr_words(nrounds) words per significant tile, 16-byte aligned.
hipError_t launch_agglomerate(const Slot* tab, uint64_t slots_max, const JobView& jv, const uint64_t* s_key,
                              uint32_t* parent, uint32_t* nbr, uint32_t* size, uint64_t s_max,
                              unsigned long long* ctr, hipStream_t stream,
                              const NbrRound* rounds = nullptr, int nrounds = 0,
                              bool d3 = false, Frame frame = Frame{});

// Framed single tables of at least 512 partitions (two dimensions, Chebyshev
// or Manhattan distance 1) take the census path instead of launch_threshold and
// launch_agglomerate: launch_census records which slots are significant
// (words: census_words(cap) 32-bit words, 8-byte aligned; partials:
// kScanBlocks words, scanned in place), fills ctr[C_DISTINCT], ctr[C_SUM]
// and ctr[C_SIGNIFICANT], and with `square` runs the 2x2 post-step first.
// launch_link_census then writes S_key, S_count and size[i] = 0 and leaves
// the roots and sizes as launch_agglomerate does (`manhattan`: the two
// edge-sharing neighbours only).
bool census_geometry(uint64_t cap, Frame frame);
uint64_t census_words(uint64_t cap);
hipError_t launch_census(Slot* tab, uint64_t cap, Frame frame, const JobView& jv, uint32_t tau, bool square,
                         uint32_t* words, uint32_t* partials, unsigned long long* ctr, hipStream_t stream);
hipError_t launch_image_to_table(const uint2* img, Slot* tab, uint64_t cap, Frame frame, hipStream_t stream);
// img: the slice image of the final update, or null (read the table).
hipError_t launch_link_census(const Slot* tab, const uint2* img, uint64_t cap, Frame frame, uint32_t mu, uint32_t tau,
                              bool square, const uint32_t* words, uint64_t* s_key, uint32_t* s_count,
                              uint32_t* parent, uint32_t* nbr, uint32_t* size, uint64_t s_max,
                              unsigned long long* ctr, hipStream_t stream, bool manhattan = false);

// mu filter and output compaction: rows of kept components in compact order
// (out_job gets each row's job for several jobs).
hipError_t launch_filter(const JobView& jv, const uint64_t* s_key, const uint32_t* s_count, const uint32_t* root,
                         const uint32_t* size, int32_t* out_kx, int32_t* out_ky, uint32_t* out_count,
                         uint64_t* out_label, uint32_t* out_job, uint32_t* partials, unsigned long long* ctr,
                         hipStream_t stream, int32_t* out_kz = nullptr);

// The two halves of launch_filter: the kept-row count (ctr[C_TILES], and the
// per-block offsets in partials), then the scatter of the rows.
hipError_t launch_filter_count(const JobView& jv, const uint32_t* root, const uint32_t* size, uint32_t* partials,
                               unsigned long long* ctr, hipStream_t stream);
hipError_t launch_filter_scatter(const JobView& jv, const uint64_t* s_key, const uint32_t* s_count,
                                 const uint32_t* root, const uint32_t* size, int32_t* out_kx, int32_t* out_ky,
                                 uint32_t* out_count, uint64_t* out_label, uint32_t* out_job,
                                 const uint32_t* partials, const unsigned long long* ctr, hipStream_t stream,
                                 int32_t* out_kz = nullptr);

// Stores a one-job view's descriptor (d, j) at d_dims / d_job on the device.
hipError_t launch_store_job(const Dims& d, const JobInfo& j, Dims* d_dims, JobInfo* d_job, hipStream_t stream);

// Batched counting: one launch over the point tiles of every job, each point
// added to its job's table with device atomics (LDS pre-aggregation per tile
// when tu.preagg_slots > 0).  A key that finds no room raises its job's
// C_SPILLED count; such a job is redone alone.
hipError_t launch_batch_count(const JobView& jv, const uint32_t* tile_prefix, Slot* tab, const KernelTuning& tu,
                              int max_tiles_grid, hipStream_t stream);

// Binned batched counting: level 1 over job-homogeneous tiles of kBinTile
// points into each job's coarse buckets (cjob maps a coarse bucket to its
// job), level 2 into partition buckets, then the LDS update of every
// partition.  cursor1 (ncoarse) and cursor2 (partitions) must be zero.
// Distinct-tile sketch per job: HyperLogLog registers (2^kHllLog2 per job,
// job-major, zeroed here) over a fixed 1/64 hash sample of each job's tiles.
// Per-point labels: a lookup table {key, label} of t result rows (cap slots,
// a power of two >= 2t; filled here), then the label of every point's tile
// (UINT64_MAX for none; range errors set kErrRange in *err).
hipError_t launch_label_table(const int32_t* kx, const int32_t* ky, const uint64_t* label, uint64_t t,
                              uint64_t* tab, uint64_t cap, bool rows, hipStream_t stream,
                              const int32_t* kz = nullptr);
// Per-tile point lists: rows of the points and their ranks within the rows
// (from the per-row counts), the row offsets (start[0..t]); then the scatter
// of the point indices.
hipError_t launch_tile_points_count(const void* pts, int64_t n, int dtype, double scale, const uint64_t* tab,
                                   uint64_t cap, uint32_t* row_of, uint32_t* rank, uint32_t* count, uint64_t t,
                                   uint32_t* partials, unsigned long long* total, uint64_t* start,
                                   unsigned long long* err, hipStream_t stream, int dims = 2);
hipError_t launch_tile_points_scatter(const uint32_t* row_of, const uint32_t* rank, int64_t n,
                                      const uint64_t* start, uint64_t* out, hipStream_t stream);
hipError_t launch_point_labels(const void* pts, int64_t n, int dtype, double scale, const uint64_t* tab,
                               uint64_t cap, uint64_t* out, unsigned long long* err, hipStream_t stream,
                               int dims = 2);

// Distinct-tile sketch of one point set into hll (kHllReps replicas, not
// zeroed here).
hipError_t launch_points_hll(const void* pts, int64_t n, int dtype, double scale, uint32_t* hll,
                             hipStream_t stream, int dims = 2);
hipError_t launch_batch_hll(const JobView& jv, const uint32_t* tile_prefix, uint32_t tile, uint32_t* hll,
                            uint32_t njobs, uint32_t tiles, hipStream_t stream);

hipError_t launch_batch_binned(const JobView& jv, const uint32_t* tile_prefix, const uint32_t* cjob, uint64_t* bin1,
                               uint32_t* cursor1, uint64_t* bin2, uint32_t* cursor2, Slot* tab, hipStream_t stream);

// Fills table slots [0, dims->slots) with empty slots.
hipError_t launch_fill_dims(Slot* tab, const Dims* dims, hipStream_t stream);

// Per-job boundaries of a job-sorted array seg_job[0, *n): start[j], end[j]
// (both must be zero for jobs without entries beforehand).
hipError_t launch_bounds(const uint32_t* seg_job, const unsigned long long* n, uint32_t* start, uint32_t* end,
                         uint64_t n_max, hipStream_t stream);

// Per-job components, clusters, significant tiles and rows, from the compact
// ranges [s_start, s_end) and row ranges [o_start, o_end).
hipError_t launch_job_stats(const JobView& jv, const uint32_t* root, const uint32_t* size, const uint32_t* s_start,
                            const uint32_t* s_end, const uint32_t* o_start, const uint32_t* o_end,
                            uint32_t max_jobs, hipStream_t stream);

}  // namespace rst
