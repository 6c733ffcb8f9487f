// Host-side runtime pieces shared by the plain, streaming, batched and served
// forms: error reporting, the device memory pool, the table life cycle and the
// result object.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "raster.h"
#include "raster_internal.h"

namespace rst {
class DevicePool;
}

struct raster_result {
    rst::DevicePool* pool = nullptr;  // owner of `block`
    void* block = nullptr;            // one device allocation holding the arrays
    std::shared_ptr<void> shared;     // or: a block shared with other results of one batch
    uint64_t* label = nullptr;
    int32_t* kx = nullptr;
    int32_t* ky = nullptr;
    int32_t* kz = nullptr;  // three-dimensional results only
    int32_t dims = 2;
    uint32_t* count = nullptr;
    int64_t tiles = 0;
    int64_t clusters = 0;
    raster_stats stats{};
    double scale = 0.0;  // the projection the result was computed with
    // per-point labels and per-tile point lists: lookup tables of the rows
    // (tile -> label, tile -> row), built on first use, and a range flag
    std::mutex lt_mu;
    uint64_t* lt = nullptr;
    uint64_t lt_cap = 0;
    uint64_t* rt = nullptr;
    uint64_t rt_cap = 0;
    unsigned long long* lt_err = nullptr;
};

namespace rst {

extern thread_local std::string g_last_error;
raster_status fail(raster_status s, const char* fmt, ...);
raster_status hip_fail(hipError_t e, const char* what);

raster_tuning current_tuning();
KernelTuning kernel_tuning(const raster_tuning& t);
bool scale_for_precision(int32_t p, double* s);
uint64_t next_pow2(uint64_t v);
raster_status check_points(const void* p, int64_t n, raster_dtype dt, uint32_t dims = 2);
raster_status check_params(double scale, uint32_t tau, uint32_t mu);
raster_status check_neighbourhood(int32_t metric, uint32_t delta);
raster_status check_options(const raster_options* o);
uint32_t options_dims(const raster_options* o);  // 3 for three-dimensional points, else 2
// Link rounds of the neighbourhood; empty for Chebyshev 1, which has its own
// fixed-offset pass.
std::vector<NbrRound> neighbourhood_rounds(uint32_t metric, uint32_t delta, uint32_t dims = 2);

class DevicePool {
  public:
    static DevicePool& get(int device);
    hipError_t alloc(void** out, size_t bytes);
    void release(void* p);
    void trim();
    size_t used_bytes();
    size_t cached_bytes();
    size_t block_bytes(void* p);   // size class of a block handed out by alloc
    size_t peak_used(bool reset);  // largest used_bytes() since the last reset

  private:
    std::mutex mu_;
    std::multimap<size_t, void*> free_;
    std::unordered_map<void*, size_t> sizes_;
    size_t cached_ = 0, used_ = 0, peak_ = 0;
    int device_ = 0;
};

struct Buffers {
    DevicePool* pool = nullptr;
    std::vector<void*> blocks;
    ~Buffers();
    hipError_t take(void** out, size_t bytes);
    void give_back(void* p);
    void release_all();
    size_t bytes() const;  // device bytes of the blocks held
};

// Device image of a one-job view.
struct SingleJob {
    Dims dims;
    JobInfo job;
};

// One device tile table and everything needed to fill it and cluster it.
struct TableRun {
    SingleJob single{};
    int device = 0;
    hipStream_t stream = nullptr;
    double scale = 1.0;
    uint32_t tau = 1, mu = 1;
    uint32_t metric = RASTER_CHEBYSHEV, delta = 1;  // neighbourhood of the agglomeration
    bool square = false;                            // the 2x2 post-step before the threshold
    // census of the significant slots taken by the final update (valid while
    // census_cap == cap)
    uint32_t* c_words = nullptr;
    uint32_t* c_ptot = nullptr;
    uint64_t c_words_cap = 0;  // table size the census buffers are sized for
    uint64_t census_cap = 0;
    // an unframed table's final update counted its significant slots per
    // scan block into `partials` (valid while counted_cap == cap)
    uint64_t counted_cap = 0;
    // slice image written by the final update instead of the table (the
    // table is stale while image_cap == cap)
    uint2* img = nullptr;
    uint64_t img_cap = 0, image_cap = 0;
    uint32_t dims = 2;                              // coordinates per point: 2 or 3
    // Occupancy the table is sized for.  Three-dimensional keys are placed
    // in partitions by 4x4x4 blocks, which dense clusters fill completely, so
    // partition loads spread wider than with 8x8 blocks of the plane and the
    // table is kept emptier to avoid overflowing partitions.
    double target_load() const { return dims == 3 ? 0.75 * tuning.load_factor : tuning.load_factor; }
    raster_tuning tuning{};
    Buffers bufs;
    Slot* tab = nullptr;
    uint64_t cap = 0;
    // A new table is filled only when something needs its slots: until then
    // the binning gets no table (keys it would insert directly wait in the
    // spill buffer), the first update writes whole slices, which fills it, and
    // a final update that writes its slice image leaves it untouched.
    bool tab_unfilled = false;
    unsigned long long* ctr = nullptr;    // device counters
    unsigned long long* h_ctr = nullptr;  // pinned host mirror
    uint32_t* partials = nullptr;
    uint64_t* spill_keys[2] = {nullptr, nullptr};
    uint32_t* spill_counts[2] = {nullptr, nullptr};
    uint64_t spill_cap[2] = {0, 0};
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    hipEvent_t ev_chunk = nullptr;
    // device time per kernel kind: 0 = the point-streaming kernel (direct
    // count or level-1 binning), 1 = level-2 binning, 2 = partition update
    struct Span {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Span> spans;
    std::vector<hipEvent_t> ev_free;
    double span_us[3] = {0, 0, 0};
    int64_t span_n[3] = {0, 0, 0};
    // Key frame of the table (two dimensions): decided from the first binned
    // chunk while the table is empty, then fixed for the table's life.
    Frame frame{};
    bool frame_decided = false;
    uint32_t* frame_box = nullptr;  // tile box of the frame sample, while it is being read
    // binned contraction: coarse and partition lists of 8-byte keys, or of
    // 4-byte entries in a framed table
    uint64_t* bin1 = nullptr;
    uint64_t cap1 = 0;
    uint32_t* cursor1 = nullptr;
    uint64_t* bin2 = nullptr;
    uint64_t bin2_slots = 0;
    uint32_t* cursor2 = nullptr;
    uint64_t cursor2_n = 0;
    uint32_t* sketch = nullptr;  // distinct-tile sketch of the binned keys
    uint32_t* h_sketch = nullptr;  // pinned mirror of the registers, read when the table is sized
    uint64_t group_points = 0;  // points binned since the last flush
    uint64_t group_budget = 0;
    uint64_t bin_points = 0;   // keys the coarse buckets are sized for
    bool single_shot = false;  // plain call: all points come in one feed
    int32_t flushes = 0;
    bool chunk_pending = false;
    bool last_binned = false;  // the last chunk was binned whole (no table insert but overflow)
    bool timing_started = false;
    bool hinted = false;  // tile_hint given: the first chunk does not resize the table
    int64_t n_points = 0;
    int64_t grow_events = 0;
    raster_status failed = RASTER_OK;

    ~TableRun();
    raster_status init(double scale, uint32_t tau, uint32_t mu, int64_t tile_hint, hipStream_t stream);
    raster_status feed(const void* pts, int64_t n, raster_dtype dt);
    bool can_bin_unsettled(int64_t n) const;
    raster_status finish(raster_result** out);
    raster_status export_tiles(uint64_t* keys, uint32_t* counts, int64_t cap_rows, int64_t* m);

    raster_status alloc_table(uint64_t c, Slot** t, uint64_t* c_out, bool fill = true);
    raster_status ensure_filled();
    Slot* bin_tab() const { return tab_unfilled ? nullptr : tab; }
    raster_status insert_held(uint64_t* spilled, int* src);
    raster_status decide_frame(const void* pts, int64_t n, raster_dtype dt);
    raster_status frame_begin(const void* pts, int64_t n, raster_dtype dt);
    raster_status frame_end();
    size_t bin_entry_bytes() const { return frame.on ? sizeof(uint32_t) : sizeof(uint64_t); }
    uint32_t coarse_buckets() const { return frame.on ? kFrameCoarse : kCoarse; }
    Geo geo() const { return make_geo(cap, dims == 3, frame); }
    raster_status size_from_sketch(uint64_t points, bool fetched = false);
    raster_status ensure_sketch();
    raster_status ensure_spill(int b, uint64_t need);
    raster_status pull_counters();
    raster_status grow(uint64_t new_cap, uint64_t pending, int src);
    raster_status settle();
    raster_status flush(bool census = false, bool count = false);
    raster_status ensure_census(uint64_t c);
    raster_status ensure_bins(uint64_t want_points);
    raster_status mark_pending();
    raster_status wait_stream();
    raster_status span_events(KernelSpan* sp);
    void span_done(int kind, const KernelSpan& sp);
    void resolve_spans();
};

// Distinct tiles estimated from 2^kHllLog2 sketch registers (HyperLogLog
// with its small-range correction; the sketch holds 1/64 of the tiles).
double hll_estimate(const uint32_t* regs);

}  // namespace rst
