// Host runtime of the RASTER library: argument checks, device memory, the
// table life cycle (size, grow, rehash), the streaming state machine and the
// result objects behind the C ABI of include/raster.h.
//
// Every step of the clustering runs in the kernels of raster_kernels.hip; this
// file only sizes buffers, enqueues launches and reads back a few counters.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <string>
#include <unordered_map>
#include <vector>

#include "raster.h"
#include "raster_internal.h"
#include "raster_runtime.h"

using namespace rst;

// ============================================================ errors =======

namespace rst {

thread_local std::string g_last_error;

raster_status fail(raster_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

raster_status hip_fail(hipError_t e, const char* what) {
    if (e == hipErrorOutOfMemory) return fail(RASTER_E_NOMEM, "%s: out of device memory", what);
    return fail(RASTER_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ========================================================= tuning ==========

static std::mutex g_tuning_mu;
static const raster_tuning kDefaultTuning = {256, 4, 0, 0.6f, 0, 512};
static raster_tuning g_tuning = kDefaultTuning;

raster_tuning current_tuning() {
    std::lock_guard<std::mutex> g(g_tuning_mu);
    return g_tuning;
}

KernelTuning kernel_tuning(const raster_tuning& t) {
    KernelTuning k;
    k.block = t.block;
    k.items = t.items;
    k.preagg_slots = t.preagg_slots;
    k.preagg_tiles = 4;
    return k;
}

// =================================================== device memory pool ====
//
// A caching allocator per device.  Blocks are rounded to size classes and
// returned to a free list on release.  A block may only be released once the
// work that used it is complete (the callers synchronise first), so reuse
// never races with queued kernels.

static size_t size_class(size_t bytes) {
    if (bytes <= 256) return 256;
    if (bytes <= (size_t)2 << 20) {
        size_t c = 256;
        while (c < bytes) c <<= 1;
        return c;
    }
    const size_t g = (size_t)2 << 20;
    return (bytes + g - 1) / g * g;
}

DevicePool& DevicePool::get(int device) {
    static std::mutex mu;
    static std::map<int, DevicePool*> pools;
    std::lock_guard<std::mutex> g(mu);
    auto it = pools.find(device);
    if (it != pools.end()) return *it->second;
    DevicePool* p = new DevicePool();  // lives until process exit
    p->device_ = device;
    pools[device] = p;
    return *p;
}

hipError_t DevicePool::alloc(void** out, size_t bytes) {
    const size_t c = size_class(bytes == 0 ? 1 : bytes);
    {
        std::lock_guard<std::mutex> g(mu_);
        auto it = free_.lower_bound(c);
        // reuse a cached block of the same class, or one at most 2x larger
        if (it != free_.end() && it->first <= c * 2) {
            *out = it->second;
            cached_ -= it->first;
            used_ += it->first;
            peak_ = std::max(peak_, used_);
            free_.erase(it);
            return hipSuccess;
        }
    }
    hipError_t e = hipMalloc(out, c);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        trim();
        e = hipMalloc(out, c);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *out = nullptr;
        return e;
    }
    std::lock_guard<std::mutex> g(mu_);
    sizes_[*out] = c;
    used_ += c;
    peak_ = std::max(peak_, used_);
    return hipSuccess;
}

void DevicePool::release(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> g(mu_);
    auto it = sizes_.find(p);
    if (it == sizes_.end()) return;
    free_.emplace(it->second, p);
    cached_ += it->second;
    used_ -= it->second;
}

void DevicePool::trim() {
    std::multimap<size_t, void*> drop;
    {
        std::lock_guard<std::mutex> g(mu_);
        drop.swap(free_);
        for (auto& kv : drop) sizes_.erase(kv.second);
        cached_ = 0;
    }
    for (auto& kv : drop) (void)hipFree(kv.second);
}

size_t DevicePool::used_bytes() {
    std::lock_guard<std::mutex> g(mu_);
    return used_;
}

size_t DevicePool::cached_bytes() {
    std::lock_guard<std::mutex> g(mu_);
    return cached_;
}

size_t DevicePool::block_bytes(void* p) {
    std::lock_guard<std::mutex> g(mu_);
    auto it = sizes_.find(p);
    return it == sizes_.end() ? 0 : it->second;
}

size_t DevicePool::peak_used(bool reset) {
    std::lock_guard<std::mutex> g(mu_);
    const size_t p = peak_;
    if (reset) peak_ = used_;
    return p;
}

// A set of pool blocks released together.
Buffers::~Buffers() { release_all(); }

void Buffers::release_all() {
    if (!pool) return;
    for (void* p : blocks) pool->release(p);
    blocks.clear();
}

hipError_t Buffers::take(void** out, size_t bytes) {
    hipError_t e = pool->alloc(out, bytes);
    if (e == hipSuccess) blocks.push_back(*out);
    return e;
}

size_t Buffers::bytes() const {
    size_t b = 0;
    if (pool)
        for (void* p : blocks) b += pool->block_bytes(p);
    return b;
}

void Buffers::give_back(void* p) {
    auto it = std::find(blocks.begin(), blocks.end(), p);
    if (it != blocks.end()) {
        blocks.erase(it);
        pool->release(p);
    }
}

// ================================================================ helpers ==

bool scale_for_precision(int32_t p, double* s) {
    if (p < 0 || p > 15) return false;
    double v = 1.0;
    for (int i = 0; i < p; ++i) v *= 10.0;  // every step exact below 2^53
    *s = v;
    return true;
}

uint64_t next_pow2(uint64_t v) {
    uint64_t c = 1;
    while (c < v) c <<= 1;
    return c;
}

const char* range_message(int dims) {
    return dims == 3 ? "a coordinate is not finite or its tile is outside +-(2^20 - 2)"
                     : "a coordinate is not finite or its tile is outside +-(2^31 - 2)";
}

raster_status check_points(const void* p, int64_t n, raster_dtype dt, uint32_t dims) {
    if (dt != RASTER_F32 && dt != RASTER_F64) return fail(RASTER_E_INVAL, "unknown dtype %d", (int)dt);
    if (n < 0) return fail(RASTER_E_INVAL, "negative point count %lld", (long long)n);
    if (n > 0 && !p) return fail(RASTER_E_INVAL, "NULL points with n = %lld", (long long)n);
    const uintptr_t a = (uintptr_t)p;
    // 2-D rows are read as one vector load, 3-D rows one coordinate at a time
    const unsigned align = dims == 3 ? (dt == RASTER_F64 ? 8 : 4) : (dt == RASTER_F64 ? 16 : 8);
    if (n > 0 && (a % align) != 0) return fail(RASTER_E_INVAL, "points must be %u-byte aligned", align);
    return RASTER_OK;
}

raster_status check_params(double scale, uint32_t tau, uint32_t mu) {
    if (tau == 0) return fail(RASTER_E_INVAL, "tau must be >= 1");
    if (mu == 0) return fail(RASTER_E_INVAL, "mu must be >= 1");
    if (!(scale > 0.0) || !std::isfinite(scale)) return fail(RASTER_E_INVAL, "scale must be finite and > 0");
    return RASTER_OK;
}

raster_status check_neighbourhood(int32_t metric, uint32_t delta) {
    if (metric != RASTER_CHEBYSHEV && metric != RASTER_MANHATTAN) return fail(RASTER_E_INVAL, "unknown metric %d", metric);
    if (delta < 1 || delta > kMaxDelta)
        return fail(RASTER_E_INVAL, "delta %u outside [1, %u]", delta, (unsigned)kMaxDelta);
    return RASTER_OK;
}

raster_status check_options(const raster_options* o) {
    if (!o) return RASTER_OK;
    raster_status s = check_neighbourhood((int32_t)o->metric, o->delta);
    if (s != RASTER_OK) return s;
    if (o->square_step > 1) return fail(RASTER_E_INVAL, "square_step must be 0 or 1");
    if (o->dims != 0 && o->dims != 2 && o->dims != 3) return fail(RASTER_E_INVAL, "dims must be 0, 2 or 3");
    if (o->dims == 3 && o->square_step) return fail(RASTER_E_INVAL, "the 2x2 post-step is two-dimensional");
    return RASTER_OK;
}

uint32_t options_dims(const raster_options* o) { return o && o->dims == 3 ? 3u : 2u; }

std::vector<NbrRound> neighbourhood_rounds(uint32_t metric, uint32_t delta, uint32_t dims) {
    std::vector<NbrRound> rounds;
    if (metric == RASTER_CHEBYSHEV && delta == 1 && dims == 2) return rounds;
    // backward offsets (smaller key): each edge is looked up from its
    // larger-key end; keys order tiles lexicographically
    struct Off {
        int32_t dx, dy, dz;
    };
    std::vector<Off> offs;
    const int32_t d = (int32_t)delta;
    const int32_t dzm = dims == 3 ? d : 0;
    for (int32_t dx = -d; dx <= 0; ++dx)
        for (int32_t dy = -d; dy <= d; ++dy)
            for (int32_t dz = -dzm; dz <= dzm; ++dz) {
                if (dx == 0 && (dy > 0 || (dy == 0 && dz >= 0))) continue;
                if (metric == RASTER_MANHATTAN && std::abs(dx) + std::abs(dy) + std::abs(dz) > d) continue;
                offs.push_back({dx, dy, dz});
            }
    // nearest first, so that the first round's parent links cover most edges
    std::stable_sort(offs.begin(), offs.end(), [](const Off& a, const Off& b) {
        return std::abs(a.dx) + std::abs(a.dy) + std::abs(a.dz) < std::abs(b.dx) + std::abs(b.dy) + std::abs(b.dz);
    });
    for (size_t i = 0; i < offs.size(); i += 4) {
        NbrRound r{};
        r.count = (uint32_t)std::min<size_t>(4, offs.size() - i);
        for (uint32_t q = 0; q < r.count; ++q) {
            r.dx[q] = offs[i + q].dx;
            r.dy[q] = offs[i + q].dy;
            r.dz[q] = offs[i + q].dz;
        }
        rounds.push_back(r);
    }
    return rounds;
}

// ============================================================ table run ====

#define HIP_TRY(expr, what)                          \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// ---- process-wide caches of pinned counter mirrors and events ---------------
//
// A stream's begin and end would otherwise pin and free host memory and
// create and destroy events every time, which costs more than a small step's
// kernels.  Events are kept per device (they belong to the device current at
// creation).

namespace {

struct HostCache {
    std::mutex mu;
    std::vector<unsigned long long*> pinned;
    std::vector<uint32_t*> pinned_sketch;  // kHllReps << kHllLog2 registers each
    std::map<std::pair<int, bool>, std::vector<hipEvent_t>> events;  // (device, timing) -> free events

    static HostCache& get() {
        static HostCache* c = new HostCache();  // never destroyed: lives past static teardown
        return *c;
    }
    hipError_t take_pinned(unsigned long long** p) {
        {
            std::lock_guard<std::mutex> g(mu);
            if (!pinned.empty()) {
                *p = pinned.back();
                pinned.pop_back();
                return hipSuccess;
            }
        }
        return hipHostMalloc((void**)p, kCounterWords * sizeof(unsigned long long), hipHostMallocDefault);
    }
    void give_pinned(unsigned long long* p) {
        std::lock_guard<std::mutex> g(mu);
        pinned.push_back(p);
    }
    hipError_t take_pinned_sketch(uint32_t** p) {
        {
            std::lock_guard<std::mutex> g(mu);
            if (!pinned_sketch.empty()) {
                *p = pinned_sketch.back();
                pinned_sketch.pop_back();
                return hipSuccess;
            }
        }
        return hipHostMalloc((void**)p, ((size_t)kHllReps << kHllLog2) * sizeof(uint32_t), hipHostMallocDefault);
    }
    void give_pinned_sketch(uint32_t* p) {
        std::lock_guard<std::mutex> g(mu);
        pinned_sketch.push_back(p);
    }
    hipError_t take_event(int dev, bool timing, hipEvent_t* e) {
        {
            std::lock_guard<std::mutex> g(mu);
            auto& v = events[{dev, timing}];
            if (!v.empty()) {
                *e = v.back();
                v.pop_back();
                return hipSuccess;
            }
        }
        return timing ? hipEventCreate(e) : hipEventCreateWithFlags(e, hipEventDisableTiming);
    }
    void give_event(int dev, bool timing, hipEvent_t e) {
        std::lock_guard<std::mutex> g(mu);
        events[{dev, timing}].push_back(e);
    }
};

}  // namespace

TableRun::~TableRun() {
    HostCache& hc = HostCache::get();
    for (hipEvent_t& e : ev) if (e) hc.give_event(device, true, e);
    if (ev_chunk) hc.give_event(device, false, ev_chunk);
    for (const Span& sp : spans) {
        hc.give_event(device, true, sp.a);
        hc.give_event(device, true, sp.b);
    }
    for (hipEvent_t e : ev_free) hc.give_event(device, true, e);
    if (h_ctr) hc.give_pinned(h_ctr);
    if (h_sketch) hc.give_pinned_sketch(h_sketch);
}

double hll_estimate(const uint32_t* M) {
    constexpr double m = (double)(1u << kHllLog2);
    const double alpha = 0.7213 / (1.0 + 1.079 / m);
    double z = 0.0;
    int zeros = 0;
    for (uint32_t j = 0; j < (1u << kHllLog2); ++j) {
        z += std::ldexp(1.0, -(int)M[j]);
        zeros += M[j] == 0;
    }
    double e = alpha * m * m / z;
    if (e <= 2.5 * m && zeros > 0) e = m * std::log(m / zeros);
    return 64.0 * e;  // the sketch registers 1/64 of the tiles
}

// One-shot calls counted directly take a sketch pass first from this size on;
// below it a wrong guess only costs a cheap table growth.
static constexpr uint64_t kSketchMinPoints = 1u << 16;

// One-shot calls: the table was sized by a guess (n/8 distinct tiles) before
// any key was seen; before the keys are split into partitions, the sketch
// taken while binning sizes it properly.  The table is still empty apart from
// keys that overflowed a bucket, so growing it is cheap.
raster_status TableRun::ensure_sketch() {
    if (sketch) return RASTER_OK;
    const size_t regs = (size_t)kHllReps << kHllLog2;
    HIP_TRY(HostCache::get().take_pinned_sketch(&h_sketch), "hipHostMalloc");
    HIP_TRY(bufs.take((void**)&sketch, regs * sizeof(uint32_t)), "sketch");
    HIP_TRY(launch_zero_u64((uint64_t*)sketch, regs / 2, stream), "zero sketch");
    return RASTER_OK;
}

// Reads the sketch registers (one copy and wait, unless the caller has
// fetched them already) and sizes the table from them.  A single-shot call
// may replace an empty table by one of the estimated size; a stream grows its
// table only when the estimate shows it too full to work in.
raster_status TableRun::size_from_sketch(uint64_t points, bool fetched) {
    const size_t regs = (size_t)kHllReps << kHllLog2;
    if (!fetched) {
        HIP_TRY(hipMemcpyAsync(h_sketch, sketch, regs * sizeof(uint32_t), hipMemcpyDeviceToHost, stream),
                "sketch copy");
        raster_status ws = wait_stream();
        if (ws != RASTER_OK) return ws;
    }
    const uint32_t* h = h_sketch;
    std::vector<uint32_t> M(1u << kHllLog2, 0);
    for (uint32_t r = 0; r < kHllReps; ++r)
        for (uint32_t j = 0; j < (1u << kHllLog2); ++j) M[j] = std::max(M[j], h[((size_t)r << kHllLog2) + j]);
    const double est = hll_estimate(M.data());
    uint64_t want;
    if (single_shot) {
        const double d = std::min<double>(1.25 * est + (double)h_ctr[C_INSERTED], (double)points);
        want = next_pow2((uint64_t)(d / target_load()) + 1);
    } else {
        // a stream's sketch covers every binned point so far, the keys
        // already in the table included.  Its first guess (half a chunk) is
        // kept unless the estimate shows the table too full to work in.
        const double d = std::min<double>(std::max<double>(est, (double)h_ctr[C_INSERTED]), (double)n_points);
        if (d <= 0.85 * (double)cap) return RASTER_OK;
        want = next_pow2((uint64_t)(d / target_load()) + 1);
    }
    if (want <= cap) return RASTER_OK;
    if (h_ctr[C_INSERTED] == 0 && h_ctr[C_SPILLED] == 0) {
        // nothing inserted yet: a fresh table, no rehash
        Slot* nt = nullptr;
        uint64_t nc = 0;
        raster_status st = alloc_table(want, &nt, &nc, !tab_unfilled);
        if (st != RASTER_OK) return st;
        bufs.give_back(tab);
        tab = nt;
        cap = nc;
        return RASTER_OK;
    }
    return grow(want, 0, 0);
}

raster_status TableRun::init(double scale_, uint32_t tau_, uint32_t mu_, int64_t tile_hint,
                             hipStream_t stream_) {
    scale = scale_;
    tau = tau_;
    mu = mu_;
    stream = stream_;
    HIP_TRY(hipGetDevice(&device), "hipGetDevice");
    bufs.pool = &DevicePool::get(device);
    tuning = current_tuning();
    group_budget = (uint64_t)tuning.group_mpoints * 1000000ull;
    HostCache& hc = HostCache::get();
    HIP_TRY(hc.take_pinned(&h_ctr), "hipHostMalloc");
    std::memset(h_ctr, 0, kCounterWords * sizeof(unsigned long long));
    for (hipEvent_t& e : ev) HIP_TRY(hc.take_event(device, true, &e), "hipEventCreate");
    HIP_TRY(hc.take_event(device, false, &ev_chunk), "hipEventCreate");
    HIP_TRY(bufs.take((void**)&ctr, kCounterWords * sizeof(unsigned long long)), "counters");
    HIP_TRY(bufs.take((void**)&partials, kScanBlocks * sizeof(uint32_t)), "scan partials");
    HIP_TRY(launch_zero_u64((uint64_t*)ctr, kCounterWords, stream), "zero counters");
    hinted = tile_hint > 0;
    const double lf = target_load();
    const uint64_t want = (uint64_t)std::max<double>(4096.0, (double)std::max<int64_t>(tile_hint, 1) / lf);
    // not filled here: the binning does without, and the first update fills
    // it by writing whole slices (or leaves it alone when it writes its slice
    // image); anything else calls ensure_filled first
    tab_unfilled = true;
    return alloc_table(next_pow2(want), &tab, &cap, false);
}

raster_status TableRun::alloc_table(uint64_t c, Slot** t, uint64_t* c_out, bool fill) {
    if (c > ((uint64_t)1 << 31)) return fail(RASTER_E_NOMEM, "table of %llu slots is too large", (unsigned long long)c);
    HIP_TRY(bufs.take((void**)t, c * sizeof(Slot)), "tile table");
    if (fill) HIP_TRY(launch_fill_table(*t, c, stream), "fill table");
    *c_out = c;
    return RASTER_OK;
}

// Fills a table left unfilled; called before anything reads or writes its
// slots other than the binning (which then gets no table) and the update
// (which writes whole slices, or only its slice image).
raster_status TableRun::ensure_filled() {
    if (!tab_unfilled) return RASTER_OK;
    HIP_TRY(launch_fill_table(tab, cap, stream), "fill table");
    tab_unfilled = false;
    return RASTER_OK;
}

// Keys held in spill buffer 0 while the table was unfilled (tiles outside the
// key frame, entries past a full list): the table is filled and takes them;
// what does not fit is left in spill buffer 1 (*src = 1) for a growth.  Its
// census and slice image, if any, no longer cover every key.
raster_status TableRun::insert_held(uint64_t* spilled, int* src) {
    raster_status st = ensure_filled();
    if (st != RASTER_OK) return st;
    if (image_cap == cap) {
        HIP_TRY(launch_image_to_table(img, tab, cap, frame, stream), "image to table");
        image_cap = 0;
    }
    census_cap = 0;
    counted_cap = 0;
    if ((st = ensure_spill(1, *spilled)) != RASTER_OK) return st;
    HIP_TRY(launch_zero_u64((uint64_t*)ctr + C_SPILLED, 1, stream), "reset spill counter");
    SpillBuf sp{spill_keys[1], spill_counts[1], spill_cap[1]};
    HIP_TRY(launch_insert_records(spill_keys[0], spill_counts[0], *spilled, tab, cap, sp, ctr, stream, dims == 3,
                                  frame),
            "insert held keys");
    if ((st = pull_counters()) != RASTER_OK) return st;
    if (h_ctr[C_ERROR] & kErrSpillOverflow) return fail(RASTER_E_DEVICE, "spill buffer overflow");
    *spilled = h_ctr[C_SPILLED];
    *src = 1;
    return RASTER_OK;
}

// Points whose tile box decides the key frame: a sample from the start of the
// first chunk (the frame only has to hold most keys; the others go to the
// table directly).
static constexpr int64_t kFrameSample = 1 << 20;

// Chooses the key frame from the tile box of the sample: the frame is centred
// on the box when the box, with a margin of 1/64 of its size plus 64 tiles on
// each side, fits into 2^20 tiles per axis; otherwise the table stays
// unframed.  Tuning mode 3 asks for the unframed binning.
raster_status TableRun::decide_frame(const void* pts, int64_t n, raster_dtype dt) {
    raster_status st = frame_begin(pts, n, dt);
    return st != RASTER_OK ? st : frame_end();
}

// The tile box of the frame sample, copied into the pinned sketch mirror;
// frame_end waits for it, so that host work in between (the table's
// allocation) overlaps the copy.
raster_status TableRun::frame_begin(const void* pts, int64_t n, raster_dtype dt) {
    frame = Frame{0, 0, 0};
    frame_box = nullptr;
    if (dims != 2 || tuning.mode == 3 || n <= 0) return RASTER_OK;
    raster_status st = ensure_sketch();
    if (st != RASTER_OK) return st;
    HIP_TRY(bufs.take((void**)&frame_box, kBboxWords * sizeof(uint32_t)), "frame box");
    HIP_TRY(launch_key_bbox(pts, std::min<int64_t>(n, kFrameSample), (int)dt, scale, frame_box, stream),
            "frame box");
    HIP_TRY(hipMemcpyAsync(h_sketch, frame_box, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, stream),
            "frame box copy");
    HIP_TRY(hipEventRecord(ev_chunk, stream), "hipEventRecord");
    return RASTER_OK;
}

raster_status TableRun::frame_end() {
    if (!frame_box) return RASTER_OK;
    hipError_t e;
    while ((e = hipEventQuery(ev_chunk)) == hipErrorNotReady) std::this_thread::yield();
    if (e != hipSuccess) return hip_fail(e, "hipEventQuery");
    uint32_t bb[4];
    std::memcpy(bb, h_sketch, sizeof bb);
    bufs.give_back(frame_box);
    frame_box = nullptr;
    if (bb[0] > bb[1] || bb[2] > bb[3]) return RASTER_OK;
    const int64_t side = (int64_t)1 << kFrameLog2;
    auto origin = [&](uint32_t lo, uint32_t hi, uint32_t* o) {
        const int64_t w = (int64_t)hi - (int64_t)lo + 1;
        const int64_t margin = w / 64 + 64;
        if (w + 2 * margin > side) return false;
        int64_t f = (int64_t)lo - (side - w) / 2;
        f = std::max<int64_t>(f, 0);
        f = std::min<int64_t>(f, ((int64_t)1 << 32) - side);
        *o = (uint32_t)f;
        return true;
    };
    uint32_t fx = 0, fy = 0;
    if (origin(bb[0], bb[1], &fx) && origin(bb[2], bb[3], &fy)) frame = Frame{1, fx, fy};
    return RASTER_OK;
}

// Makes spill buffer b hold at least `need` records.  Only that buffer is
// replaced, so records still waiting in the other one survive.
raster_status TableRun::ensure_spill(int b, uint64_t need) {
    if (spill_cap[b] >= need) return RASTER_OK;
    const uint64_t c = std::max<uint64_t>(need, 1 << 16);
    if (spill_keys[b]) bufs.give_back(spill_keys[b]);
    if (spill_counts[b]) bufs.give_back(spill_counts[b]);
    spill_keys[b] = nullptr;
    spill_counts[b] = nullptr;
    spill_cap[b] = 0;
    HIP_TRY(bufs.take((void**)&spill_keys[b], c * sizeof(uint64_t)), "spill keys");
    HIP_TRY(bufs.take((void**)&spill_counts[b], c * sizeof(uint32_t)), "spill counts");
    spill_cap[b] = c;
    return RASTER_OK;
}

// Waits for everything enqueued on the stream so far.  The host polls an
// event instead of sleeping in the runtime: the next launches depend on what
// the wait returns, and a sleeping wait adds its wake-up to the time the
// device stands idle.
raster_status TableRun::wait_stream() {
    HIP_TRY(hipEventRecord(ev_chunk, stream), "hipEventRecord");
    hipError_t e;
    while ((e = hipEventQuery(ev_chunk)) == hipErrorNotReady) std::this_thread::yield();
    if (e != hipSuccess) return hip_fail(e, "hipEventQuery");
    return RASTER_OK;
}

raster_status TableRun::pull_counters() {
    HIP_TRY(hipMemcpyAsync(h_ctr, ctr, kCounterWords * sizeof(unsigned long long), hipMemcpyDeviceToHost, stream),
            "counter copy");
    raster_status ws = wait_stream();
    if (ws != RASTER_OK) return ws;
    resolve_spans();
    return RASTER_OK;
}

// ---- per-kernel device timing: events around launches, read after a sync ----

// Two events for a timed launch (recorded by the launch itself).
raster_status TableRun::span_events(KernelSpan* sp) {
    hipEvent_t* e[2] = {&sp->a, &sp->b};
    for (hipEvent_t* x : e) {
        if (!ev_free.empty()) {
            *x = ev_free.back();
            ev_free.pop_back();
        } else {
            HIP_TRY(HostCache::get().take_event(device, true, x), "hipEventCreate");
        }
    }
    return RASTER_OK;
}

// The span's events now follow an enqueued launch: read after the next wait.
void TableRun::span_done(int kind, const KernelSpan& sp) { spans.push_back(Span{kind, sp.a, sp.b}); }

void TableRun::resolve_spans() {
    for (const Span& sp : spans) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, sp.a, sp.b) == hipSuccess) {
            span_us[sp.kind] += 1000.0 * ms;
            span_n[sp.kind] += 1;
        }
        ev_free.push_back(sp.a);
        ev_free.push_back(sp.b);
    }
    spans.clear();
}

// Moves everything into a table of new_cap slots, then re-adds the `pending`
// spilled records held in spill buffer `src`.  Repeats with a larger table
// in the (unlikely) case the new table spills again.  Keys waiting in the
// coarse buckets stay valid: their bucket depends on the key alone.
raster_status TableRun::grow(uint64_t new_cap, uint64_t pending, int src) {
    raster_status fs = ensure_filled();
    if (fs != RASTER_OK) return fs;
    while (true) {
        Slot* nt = nullptr;
        uint64_t nc = 0;
        raster_status st = alloc_table(new_cap, &nt, &nc);
        if (st != RASTER_OK) return st;
        const int dst = src ^ 1;
        // the rehash spills at most `cap` records and the re-insert `pending`
        st = ensure_spill(dst, cap + pending);
        if (st != RASTER_OK) return st;
        HIP_TRY(launch_zero_u64((uint64_t*)ctr + C_INSERTED, 2, stream), "reset counters");
        SpillBuf sp{spill_keys[dst], spill_counts[dst], spill_cap[dst]};
        HIP_TRY(launch_rehash(tab, cap, nt, nc, sp, ctr, stream, dims == 3, frame), "rehash");
        HIP_TRY(launch_insert_records(spill_keys[src], spill_counts[src], pending, nt, nc, sp, ctr, stream, dims == 3,
                                      frame),
                "reinsert");
        raster_status ps = pull_counters();
        if (ps != RASTER_OK) return ps;
        bufs.give_back(tab);
        tab = nt;
        cap = nc;
        grow_events += 1;
        if (h_ctr[C_ERROR] & kErrSpillOverflow) return fail(RASTER_E_DEVICE, "spill buffer overflow while growing");
        pending = h_ctr[C_SPILLED];
        if (pending == 0) return RASTER_OK;
        src = dst;
        new_cap = cap * 2;
    }
}

// Waits for the work enqueued by the last feed or flush, then checks its
// counters: range errors fail the run, spilled records make the table grow.
raster_status TableRun::settle() {
    if (!chunk_pending) return RASTER_OK;
    chunk_pending = false;
    // the counters are copied only now, once for all the work enqueued
    // since the last settle: a copy after every chunk stalls the stream
    HIP_TRY(hipMemcpyAsync(h_ctr, ctr, kCounterWords * sizeof(unsigned long long), hipMemcpyDeviceToHost, stream),
            "counter copy");
    raster_status ws = wait_stream();
    if (ws != RASTER_OK) return ws;
    resolve_spans();
    if (h_ctr[C_ERROR] & kErrRange) {
        failed = RASTER_E_RANGE;
        return fail(RASTER_E_RANGE, "%s", range_message(dims));
    }
    if (h_ctr[C_ERROR] & kErrSpillOverflow) {
        failed = RASTER_E_DEVICE;
        return fail(RASTER_E_DEVICE, "spill buffer overflow");
    }
    uint64_t spilled = h_ctr[C_SPILLED];
    int src = 0;
    if (spilled > 0 && tab_unfilled) {
        raster_status st = insert_held(&spilled, &src);
        if (st != RASTER_OK) {
            failed = st;
            return st;
        }
    }
    if (spilled > 0 && image_cap == cap) {
        // the last update wrote only its slice image: the table takes the
        // keys before it grows
        HIP_TRY(launch_image_to_table(img, tab, cap, frame, stream), "image to table");
        image_cap = 0;
    }
    if (spilled > 0) {
        const double lf = target_load();
        const uint64_t want = next_pow2((uint64_t)((double)(h_ctr[C_INSERTED] + spilled) / lf) + 1);
        raster_status st = grow(std::max<uint64_t>(want, cap * 2), spilled, src);
        if (st != RASTER_OK) {
            failed = st;
            return st;
        }
    }
    return RASTER_OK;
}

// Marks work whose counters the next settle() reads.
raster_status TableRun::mark_pending() {
    chunk_pending = true;
    return RASTER_OK;
}

// Coarse buckets for `want_points` keys per group (at most group_budget).
// They are only re-sized while empty.
raster_status TableRun::ensure_bins(uint64_t want_points) {
    want_points = std::min<uint64_t>(std::max<uint64_t>(want_points, 1u << 20), group_budget);
    if (bin1 && (bin_points >= want_points || group_points > 0)) return RASTER_OK;
    if (bin1) bufs.give_back(bin1);
    bin1 = nullptr;
    // a coarse list receives about want_points / (128 kBinRep) keys; the slack
    // is far beyond the binomial spread, and overflow only costs direct inserts
    const uint64_t lists = (uint64_t)kBinRep * coarse_buckets();
    const uint64_t per = want_points / lists;
    cap1 = (per + per / 50 + 1024 + 255) / 256 * 256;
    HIP_TRY(bufs.take((void**)&bin1, lists * cap1 * bin_entry_bytes()), "coarse buckets");
    if (!cursor1) {
        // room for the framed layout's lists, so that either layout can use it
        const uint64_t n_cursors = (uint64_t)kBinRep * kFrameCoarse;
        HIP_TRY(bufs.take((void**)&cursor1, n_cursors * sizeof(uint32_t)), "coarse cursors");
        HIP_TRY(launch_zero_u64((uint64_t*)cursor1, n_cursors / 2, stream), "zero cursors");
    }
    bin_points = want_points;
    return RASTER_OK;
}

// Applies the keys waiting in the coarse buckets to the table.
// Census buffers for a table of `c` slots (kept across calls when large enough).
raster_status TableRun::ensure_census(uint64_t c) {
    if (c_words && c_words_cap >= c) return RASTER_OK;
    if (c_words) bufs.give_back(c_words);
    if (c_ptot) bufs.give_back(c_ptot);
    c_words = nullptr;
    c_ptot = nullptr;
    c_words_cap = 0;
    HIP_TRY(bufs.take((void**)&c_words, census_words(c) * sizeof(uint32_t)), "census");
    // per partition: significant slots, occupied slots, count sum
    HIP_TRY(bufs.take((void**)&c_ptot, 3 * (c >> kPartLog2) * sizeof(uint32_t)), "census totals");
    c_words_cap = c;
    if (img) bufs.give_back(img);
    img = nullptr;
    img_cap = 0;
    HIP_TRY(bufs.take((void**)&img, c * sizeof(uint2)), "slice image");
    img_cap = c;
    return RASTER_OK;
}

// Updates the table with the binned group.  With `census`, a final update
// of a table of 512+ partitions also takes the census of the significant
// slots (valid while the table keeps its size: census_cap); with `count`, a
// final update without a census does the significance scan's counting pass
// (counted_cap).
raster_status TableRun::flush(bool census, bool count) {
    census_cap = 0;
    counted_cap = 0;
    if (group_points == 0) return RASTER_OK;
    if (image_cap == cap) {
        // an earlier update wrote only its slice image
        raster_status fs = ensure_filled();
        if (fs != RASTER_OK) return fs;
        HIP_TRY(launch_image_to_table(img, tab, cap, frame, stream), "image to table");
        image_cap = 0;
    }
    // the sketch registers come back with the counters, in one wait
    if (sketch) {
        HIP_TRY(hipMemcpyAsync(h_sketch, sketch, ((size_t)kHllReps << kHllLog2) * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, stream),
                "sketch copy");
        chunk_pending = true;
    }
    raster_status st = settle();
    if (st != RASTER_OK) return st;
    if (sketch && (st = size_from_sketch(group_points, true)) != RASTER_OK) return st;
    const Geo g = geo();
    SpillBuf sp{spill_keys[0], spill_counts[0], spill_cap[0]};
    // the drains insert straight into the table
    if (((frame.on && !framed_binned_geometry(g)) || (!frame.on && !binned_geometry(g))) &&
        (st = ensure_filled()) != RASTER_OK)
        return st;
    if (frame.on && !framed_binned_geometry(g)) {
        HIP_TRY(launch_drain_bins_framed(reinterpret_cast<uint32_t*>(bin1), cap1, cursor1, tab, cap, frame, sp, ctr,
                                         stream),
                "drain bins");
    } else if (!frame.on && !binned_geometry(g)) {
        HIP_TRY(launch_drain_bins(bin1, cap1, cursor1, tab, cap, sp, ctr, stream, dims == 3), "drain bins");
    } else {
        const uint64_t lists = (uint64_t)kBinRep << g.p_log2;  // kBinRep lists per partition
        uint64_t c2 = group_points / lists;
        c2 = c2 + c2 / 8 + 4 * (uint64_t)std::sqrt((double)c2 + 1.0) + 64;
        c2 = (c2 + 63) / 64 * 64;
        if (lists * c2 > bin2_slots || lists > cursor2_n) {
            if (bin2) bufs.give_back(bin2);
            if (cursor2) bufs.give_back(cursor2);
            bin2 = nullptr;
            cursor2 = nullptr;
            bin2_slots = lists * c2 + lists * c2 / 4;  // headroom for later groups
            cursor2_n = lists;
            HIP_TRY(bufs.take((void**)&bin2, bin2_slots * bin_entry_bytes()), "partition buckets");
            HIP_TRY(bufs.take((void**)&cursor2, cursor2_n * sizeof(uint32_t)), "partition cursors");
        }
        c2 = bin2_slots / lists;
        KernelSpan t1, t2;
        if ((st = span_events(&t1)) != RASTER_OK || (st = span_events(&t2)) != RASTER_OK) return st;
        if (frame.on)
            HIP_TRY(launch_bin_keys_framed(reinterpret_cast<uint32_t*>(bin1), cap1, cursor1,
                                           reinterpret_cast<uint32_t*>(bin2), c2, cursor2, bin_tab(), cap, frame, sp,
                                           ctr, stream, t1),
                    "bin keys");
        else
            HIP_TRY(launch_bin_keys(bin1, cap1, cursor1, bin2, c2, cursor2, bin_tab(), cap, sp, ctr, stream, dims == 3,
                                    t1),
                    "bin keys");
        span_done(1, t1);
        AggCensus cen;
        if (census && frame.on && census_geometry(cap, frame)) {
            if ((st = ensure_census(cap)) != RASTER_OK) return st;
            cen.rec = reinterpret_cast<uint2*>(c_words);
            cen.ptotal = c_ptot;
            cen.tau = tau;
            cen.img = img;
            census_cap = cap;
            image_cap = cap;
        }
        // an update that writes the table back into a table not filled yet
        // writes whole slices, which fills it
        const bool whole = tab_unfilled && !cen.img;
        // the threshold's counting pass, in an update without a census (the
        // framed one with 4-byte claim words only: 512+ partitions)
        AggCount cnt;
        if (count && !cen.rec && (!frame.on || geo().p_log2 > kFrameCoarseLog2)) {
            cnt.partials = partials;
            cnt.tau = tau;
            cnt.blk_shift = scan_block_shift(cap);
            counted_cap = cap;
        }
        if (frame.on)
            HIP_TRY(launch_aggregate_framed(reinterpret_cast<uint32_t*>(bin2), c2, cursor2, cursor1, tab, cap, frame,
                                            sp, ctr, stream, t2, cen, whole, cnt),
                    "aggregate");
        else
            HIP_TRY(launch_aggregate(bin2, c2, cursor2, cursor1, tab, cap, sp, ctr, stream, t2, whole, cnt),
                    "aggregate");
        if (whole) tab_unfilled = false;
        span_done(2, t2);
    }
    flushes += 1;
    group_points = 0;
    st = mark_pending();
    if (st != RASTER_OK) return st;
    return settle();
}

// Whether a chunk of n points can be binned without first waiting for the
// previous chunk's counters.  Binning writes the table only for keys past a
// full bucket or outside the key frame (or, while the table is unfilled,
// holds them in the spill buffer, which has room for the whole group), so the
// counters can only ask for a flush, a growth or a resize, none of which this
// chunk needs when it fits the group, the bins and the spill buffer as they
// are.  Errors of the earlier chunks are then reported by a later call.
bool TableRun::can_bin_unsettled(int64_t n) const {
    if (!chunk_pending || !last_binned || single_shot || n <= 0 || (uint64_t)n > group_budget) return false;
    const Geo g = geo();
    const bool binned = (tuning.mode >= 2 || (tuning.mode == 0 && (uint64_t)n >= cap / 8)) && binned_geometry(g);
    if (!binned || !bin1 || group_points == 0 || group_points + (uint64_t)n > bin_points) return false;
    return spill_cap[0] >= std::min<uint64_t>(group_budget, group_points + (uint64_t)n);
}

raster_status TableRun::feed(const void* pts, int64_t n, raster_dtype dt) {
    const bool unsettled = can_bin_unsettled(n);
    raster_status st = unsettled ? RASTER_OK : settle();
    if (st != RASTER_OK) return st;
    if (n == 0) return RASTER_OK;
    if ((uint64_t)n_points + (uint64_t)n > 0xFFFFFFFFull)
        return fail(RASTER_E_RANGE, "more than 2^32 - 1 points in one table");
    const double lf = target_load();
    uint64_t want = 0;
    if (unsettled) {
        // the counters are those of an earlier chunk: no growth decision
    } else if (n_points == 0 && !hinted) {
        // no hint and nothing seen yet: size for half the first chunk's points
        // being distinct tiles
        want = next_pow2((uint64_t)((double)n / 2.0 / lf) + 1);
    } else if ((double)h_ctr[C_INSERTED] > lf * (double)cap) {
        // keep the table under its target load: grow before the chunk if the
        // previous chunks already filled it past the target
        want = next_pow2((uint64_t)(2.0 * (double)h_ctr[C_INSERTED] / lf));
    }
    if (want > cap && n_points == 0) {
        // nothing inserted yet: a fresh table (not filled: see tab_unfilled)
        // instead of a rehash and its wait.  The starter table stays held
        // until the run ends.  When the first piece will be binned, its frame
        // box is taken first and read after the allocation.
        const int64_t first = std::min<int64_t>(n, (int64_t)group_budget);
        const bool first_binned = (tuning.mode >= 2 || (tuning.mode == 0 && (uint64_t)first >= next_pow2(want) / 8)) &&
                                  binned_geometry(make_geo(next_pow2(want), dims == 3));
        if (first_binned && !frame_decided && (st = frame_begin(pts, first, dt)) != RASTER_OK) return st;
        Slot* nt = nullptr;
        uint64_t nc = 0;
        if ((st = alloc_table(want, &nt, &nc, false)) != RASTER_OK) return st;
        tab = nt;
        cap = nc;
        tab_unfilled = true;
        if (first_binned && !frame_decided) {
            if ((st = frame_end()) != RASTER_OK) return st;
            frame_decided = true;
        }
    } else if (want > cap) {
        st = grow(want, 0, 0);
        if (st != RASTER_OK) {
            failed = st;
            return st;
        }
    }
    if (!timing_started) {
        HIP_TRY(hipEventRecord(ev[0], stream), "hipEventRecord");
        timing_started = true;
    }
    const size_t point_bytes = (dt == RASTER_F64 ? 8 : 4) * (size_t)dims;
    // Pieces of at most group_budget points, settled in between.  Spill
    // records between two settles come from one piece or one group, so the
    // buffer never needs more than what is binned plus this chunk.
    // A stream sizes the buffer for its whole bin group (which it reaches by
    // the group's end anyway), so that later chunks need no resize and can go
    // in without waiting (can_bin_unsettled).
    // (before a stream's first binned chunk the bins are not sized yet: take
    // the size they will get, so that the next chunk need not wait for this
    // one to resize the buffer)
    const uint64_t bins_expected =
        bin1 ? bin_points : std::min<uint64_t>(group_budget, std::max<uint64_t>(16 * (uint64_t)n, 1u << 20));
    const uint64_t spill_want = group_points + (uint64_t)n + (single_shot ? 0 : bins_expected);
    // a chunk binned without a settle keeps the buffer as it is: it may hold
    // records of the chunks before it (and has room for this one's)
    if (!unsettled && (st = ensure_spill(0, std::min<uint64_t>(group_budget, spill_want))) != RASTER_OK) return st;
    bool all_binned = true;
    for (int64_t off = 0; off < n;) {
        const int64_t piece = std::min<int64_t>(n - off, (int64_t)group_budget);
        const void* p = (const char*)pts + (size_t)off * point_bytes;
        const Geo g = geo();
        const bool binned = (tuning.mode >= 2 || (tuning.mode == 0 && (uint64_t)piece >= cap / 8)) &&
                            binned_geometry(g);
        SpillBuf sp{spill_keys[0], spill_counts[0], spill_cap[0]};
        KernelSpan t0;
        if (binned) {
            // the key frame comes from the first binned chunk of an empty
            // table; a table that already holds keys keeps its placement
            if (!frame_decided) {
                st = n_points == 0 ? decide_frame(p, piece, dt) : RASTER_OK;
                frame_decided = true;
                if (st != RASTER_OK) return st;
            }
            // a one-shot call bins exactly its points; a stream expects more
            // chunks like this one and bins several before updating the table
            st = ensure_bins(single_shot ? (uint64_t)piece : 16 * (uint64_t)piece);
            if (st != RASTER_OK) return st;
            if (group_points + (uint64_t)piece > bin_points) {
                st = flush();
                if (st != RASTER_OK) return st;
                st = ensure_bins(single_shot ? (uint64_t)piece : 16 * (uint64_t)piece);
                if (st != RASTER_OK) return st;
            }
            if ((st = span_events(&t0)) != RASTER_OK) return st;
            // the sketch of the binned keys sizes the table before the flush
            if ((st = ensure_sketch()) != RASTER_OK) return st;
            if (frame.on)
                HIP_TRY(launch_bin_points_framed(p, piece, (int)dt, scale, reinterpret_cast<uint32_t*>(bin1), cap1,
                                                 cursor1, bin_tab(), cap, frame, sp, ctr, sketch, stream, t0),
                        "bin points");
            else
                HIP_TRY(launch_bin_points(p, piece, (int)dt, scale, bin1, cap1, cursor1, bin_tab(), cap, sp, ctr,
                                          sketch, stream, (int)dims, t0),
                        "bin points");
            span_done(0, t0);
            group_points += (uint64_t)piece;
        } else {
            all_binned = false;
            if (single_shot && piece >= (int64_t)kSketchMinPoints && n_points == 0) {
                // one read of the points sizes the table before any insert
                if ((st = ensure_sketch()) != RASTER_OK) return st;
                HIP_TRY(launch_points_hll(p, piece, (int)dt, scale, sketch, stream, (int)dims), "sketch");
                if ((st = size_from_sketch((uint64_t)piece)) != RASTER_OK) return st;
                sp = SpillBuf{spill_keys[0], spill_counts[0], spill_cap[0]};
            }
            if ((st = span_events(&t0)) != RASTER_OK || (st = ensure_filled()) != RASTER_OK) return st;
            HIP_TRY(launch_project_count(p, piece, (int)dt, scale, tab, cap, sp, ctr, kernel_tuning(tuning), stream,
                                         (int)dims, frame, t0),
                    "project_count");
            span_done(0, t0);
        }
        n_points += piece;
        off += piece;
        if ((st = mark_pending()) != RASTER_OK) return st;
        if (off < n && (st = settle()) != RASTER_OK) return st;
    }
    last_binned = all_binned;
    return RASTER_OK;
}

raster_status TableRun::finish(raster_result** out) {
    const std::vector<NbrRound> rounds = neighbourhood_rounds(metric, delta, dims);
    // (Manhattan distance 1 looks up two of the census link pass's four
    // backward neighbours)
    const bool manhattan1 = metric == RASTER_MANHATTAN && delta == 1;
    const bool census_path = dims == 2 && (rounds.empty() || manhattan1);
    // a flush waits for the work before it itself; the final update takes
    // the census with it unless the 2x2 post-step changes significance after
    raster_status st = group_points > 0 ? flush(census_path && !square, !square) : settle();
    if (st != RASTER_OK) return st;
    // a growth after the update (spilled entries) leaves its census stale
    const bool census = census_path && census_geometry(cap, frame);
    const bool fused = census && census_cap == cap;
    // (or, unframed, its counting pass)
    const bool counted = !census && !square && counted_cap == cap;
    if (!timing_started) {
        HIP_TRY(hipEventRecord(ev[0], stream), "hipEventRecord");
        timing_started = true;
    }
    HIP_TRY(hipEventRecord(ev[1], stream), "hipEventRecord");
    const uint64_t m = std::max<uint64_t>(h_ctr[C_INSERTED], 1);
    uint64_t* s_key = nullptr;
    uint32_t *s_count = nullptr, *parent = nullptr, *size = nullptr;
    HIP_TRY(bufs.take((void**)&s_key, m * sizeof(uint64_t)), "S keys");
    HIP_TRY(bufs.take((void**)&s_count, m * sizeof(uint32_t)), "S counts");
    HIP_TRY(bufs.take((void**)&parent, m * sizeof(uint32_t)), "parent");
    HIP_TRY(bufs.take((void**)&size, m * sizeof(uint32_t)), "sizes");
    uint32_t* nbr = nullptr;
    HIP_TRY(bufs.take((void**)&nbr, m * nbr_words((int)rounds.size()) * sizeof(uint32_t)), "neighbour lists");
    // framed tables of 512+ partitions: significant slots found by a census
    // instead of an index written into every significant slot
    if (census && (st = ensure_census(cap)) != RASTER_OK) return st;

    raster_result* r = new raster_result();
    r->pool = bufs.pool;
    r->scale = scale;
    auto drop = [&](raster_status s) {
        raster_result_free(r);
        return s;
    };
    const size_t row_bytes = dims * sizeof(int32_t) + sizeof(uint32_t) + sizeof(uint64_t);
    hipError_t e = r->pool->alloc(&r->block, m * row_bytes + 256);
    if (e != hipSuccess) return drop(hip_fail(e, "result arrays"));
    char* b = (char*)r->block;
    r->label = (uint64_t*)b;
    r->kx = (int32_t*)(b + m * sizeof(uint64_t));
    r->ky = r->kx + m;
    r->count = (uint32_t*)(r->ky + m);
    r->dims = (int32_t)dims;
    if (dims == 3) r->kz = (int32_t*)(r->count + m);

    // one job: the whole table
    single.job.pts = nullptr;
    single.job.n = n_points;
    single.job.scale = scale;
    single.job.slot_base = 0;
    single.job.cap = cap;
    single.job.tau = tau;
    single.job.mu = mu;
    single.job.dtype = 0;
    single.job.first_tile = 0;
    single.job.framed = frame.on;
    single.job.fx = frame.fx;
    single.job.fy = frame.fy;
    single.dims.slots = cap;
    single.dims.njobs = 1;
    single.dims.tiles = 0;
    SingleJob* sj_dev = nullptr;
    HIP_TRY(bufs.take((void**)&sj_dev, sizeof(SingleJob)), "job descriptor");
    // written by a kernel from its arguments: no copy from pageable memory
    HIP_TRY(launch_store_job(single.dims, single.job, &sj_dev->dims, &sj_dev->job, stream), "job descriptor");
    JobView jv{&sj_dev->dims, &sj_dev->job, nullptr, nullptr, nullptr};

    // (the fused census has counted the occupied slots and their sum already)
    e = fused ? launch_zero_u64((uint64_t*)ctr + C_SIGNIFICANT, 1, stream)
              : launch_zero_u64((uint64_t*)ctr + C_DISTINCT, C_COUNT_ - C_DISTINCT, stream);
    if (e == hipSuccess && fused)
        e = launch_zero_u64((uint64_t*)ctr + C_COMPONENTS, C_COUNT_ - C_COMPONENTS, stream);
    // the link pass reads the slice image when the final update wrote one,
    // else the table
    const bool use_img = fused && image_cap == cap;
    if (!use_img && (st = ensure_filled()) != RASTER_OK) return drop(st);
    if (e == hipSuccess)
        e = fused    ? launch_census_offsets(cap, c_words, c_ptot, ctr, stream)
            : census ? launch_census(tab, cap, frame, jv, tau, square, c_words, partials, ctr, stream)
                     : launch_threshold(tab, jv, s_key, s_count, size, partials, ctr, stream, square ? cap : 0, counted);
    if (e == hipSuccess) e = hipEventRecord(ev[2], stream);
    if (e == hipSuccess)
        e = census ? launch_link_census(bin_tab(), use_img ? img : nullptr, cap, frame, mu, tau, square,
                                        c_words, s_key, s_count, parent, nbr,
                                        size, m, ctr, stream, manhattan1)
                   : launch_agglomerate(tab, cap, jv, s_key, parent, nbr, size, m, ctr, stream, rounds.data(),
                                        (int)rounds.size(), dims == 3, frame);
    if (e == hipSuccess) e = hipEventRecord(ev[3], stream);
    if (e == hipSuccess)
        e = launch_filter(jv, s_key, s_count, nbr, size, r->kx, r->ky, r->count, r->label, nullptr, partials, ctr,
                          stream, r->kz);
    if (e == hipSuccess) e = hipEventRecord(ev[4], stream);
    if (e != hipSuccess) return drop(hip_fail(e, "agglomeration launch"));
    raster_status ps = pull_counters();
    if (ps != RASTER_OK) return drop(ps);

    raster_stats& S = r->stats;
    std::memset(&S, 0, sizeof S);
    S.n_points = n_points;
    S.distinct_tiles = (int64_t)h_ctr[C_DISTINCT];
    S.significant_tiles = (int64_t)h_ctr[C_SIGNIFICANT];
    S.components = (int64_t)h_ctr[C_COMPONENTS];
    S.clusters = (int64_t)h_ctr[C_CLUSTERS];
    S.tiles = (int64_t)h_ctr[C_TILES];
    S.table_capacity = (int64_t)cap;
    S.grow_events = grow_events;
    (void)hipEventElapsedTime(&S.us_contract, ev[0], ev[1]);
    (void)hipEventElapsedTime(&S.us_threshold, ev[1], ev[2]);
    (void)hipEventElapsedTime(&S.us_agglomerate, ev[2], ev[3]);
    (void)hipEventElapsedTime(&S.us_filter, ev[3], ev[4]);
    S.us_contract *= 1000.0f;
    S.us_threshold *= 1000.0f;
    S.us_agglomerate *= 1000.0f;
    S.us_filter *= 1000.0f;
    S.count_launches = span_n[0];
    S.us_count_kernel = (float)span_us[0];
    S.us_bin_keys = (float)span_us[1];
    S.us_aggregate = (float)span_us[2];
    S.flushes = flushes;
    S.key_frame = frame.on ? 1 : 0;
    r->tiles = S.tiles;
    r->clusters = S.clusters;
    if (h_ctr[C_ERROR] & kErrInternal) return drop(fail(RASTER_E_DEVICE, "agglomeration state inconsistent"));
    if (h_ctr[C_SUM] != (unsigned long long)n_points || h_ctr[C_DISTINCT] != h_ctr[C_INSERTED])
        return drop(fail(RASTER_E_DEVICE, "table inconsistent: sum %llu vs n %lld, occupied %llu vs inserted %llu",
                         h_ctr[C_SUM], (long long)n_points, h_ctr[C_DISTINCT], h_ctr[C_INSERTED]));
    bufs.give_back(s_key);
    bufs.give_back(s_count);
    bufs.give_back(parent);
    bufs.give_back(size);
    bufs.give_back(nbr);
    bufs.give_back(sj_dev);
    *out = r;
    return RASTER_OK;
}

raster_status TableRun::export_tiles(uint64_t* keys, uint32_t* counts, int64_t cap_rows, int64_t* m) {
    raster_status st = settle();
    if (st != RASTER_OK) return st;
    st = flush();
    if (st != RASTER_OK) return st;
    if (image_cap == cap) {
        // the last update wrote only its slice image
        if ((st = ensure_filled()) != RASTER_OK) return st;
        HIP_TRY(launch_image_to_table(img, tab, cap, frame, stream), "image to table");
        image_cap = 0;
    }
    if ((st = ensure_filled()) != RASTER_OK) return st;
    HIP_TRY(launch_zero_u64((uint64_t*)ctr + C_DISTINCT, 1, stream), "zero counter");
    HIP_TRY(launch_export_tiles(tab, cap, keys, counts, (uint64_t)std::max<int64_t>(cap_rows, 0), partials, ctr,
                                stream),
            "export tiles");
    raster_status ps = pull_counters();
    if (ps != RASTER_OK) return ps;
    *m = (int64_t)h_ctr[C_DISTINCT];
    return RASTER_OK;
}

}  // namespace rst

// ============================================================== C ABI ======

struct raster_stream {
    rst::TableRun run;
    enum State { OPEN, FINISHED, FAILED } state = OPEN;
};

extern "C" {

raster_status raster_cluster_opts(const void* d_points, int64_t n, raster_dtype dt, double scale, uint32_t tau,
                                  uint32_t mu, const raster_options* opts, hipStream_t stream, raster_result** out) {
    if (!out) return fail(RASTER_E_INVAL, "out is NULL");
    *out = nullptr;
    raster_status st = check_params(scale, tau, mu);
    if (st != RASTER_OK) return st;
    st = check_options(opts);
    if (st != RASTER_OK) return st;
    st = check_points(d_points, n, dt, options_dims(opts));
    if (st != RASTER_OK) return st;
    TableRun run;
    run.single_shot = true;
    if (opts) {
        run.metric = (uint32_t)opts->metric;
        run.delta = opts->delta;
        run.square = opts->square_step == 1;
        run.dims = options_dims(opts);
    }
    st = run.init(scale, tau, mu, std::max<int64_t>(n / 8, 1024), stream);
    if (st != RASTER_OK) return st;
    st = run.feed(d_points, n, dt);
    if (st != RASTER_OK) return st;
    return run.finish(out);
}

raster_status raster_cluster_p_opts(const void* d_points, int64_t n, raster_dtype dt, int32_t precision,
                                    uint32_t tau, uint32_t mu, const raster_options* opts, hipStream_t stream,
                                    raster_result** out) {
    double s;
    if (out) *out = nullptr;
    if (!scale_for_precision(precision, &s)) return fail(RASTER_E_INVAL, "precision %d outside [0, 15]", precision);
    return raster_cluster_opts(d_points, n, dt, s, tau, mu, opts, stream, out);
}

raster_status raster_cluster_delta(const void* d_points, int64_t n, raster_dtype dt, double scale, uint32_t tau,
                                   uint32_t mu, raster_metric metric, uint32_t delta, hipStream_t stream,
                                   raster_result** out) {
    const raster_options o{metric, delta, 0, 0};
    return raster_cluster_opts(d_points, n, dt, scale, tau, mu, &o, stream, out);
}

raster_status raster_cluster_scaled(const void* d_points, int64_t n, raster_dtype dt, double scale, uint32_t tau,
                                    uint32_t mu, hipStream_t stream, raster_result** out) {
    return raster_cluster_opts(d_points, n, dt, scale, tau, mu, nullptr, stream, out);
}

raster_status raster_cluster(const void* d_points, int64_t n, raster_dtype dt, int32_t precision, uint32_t tau,
                             uint32_t mu, hipStream_t stream, raster_result** out) {
    double s;
    if (out) *out = nullptr;
    if (!scale_for_precision(precision, &s)) return fail(RASTER_E_INVAL, "precision %d outside [0, 15]", precision);
    return raster_cluster_scaled(d_points, n, dt, s, tau, mu, stream, out);
}

raster_status raster_memory_stats(size_t* used, size_t* cached, size_t* peak_used, int32_t reset_peak) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    DevicePool& p = DevicePool::get(dev);
    if (used) *used = p.used_bytes();
    if (cached) *cached = p.cached_bytes();
    const size_t pk = p.peak_used(reset_peak != 0);
    if (peak_used) *peak_used = pk;
    return RASTER_OK;
}

int64_t raster_result_num_tiles(const raster_result* r) { return r ? r->tiles : -1; }
int64_t raster_result_num_clusters(const raster_result* r) { return r ? r->clusters : -1; }

raster_status raster_result_kz(const raster_result* r, const int32_t** d_kz) {
    if (!r) return fail(RASTER_E_INVAL, "result is NULL");
    if (!d_kz) return fail(RASTER_E_INVAL, "d_kz is NULL");
    *d_kz = r->kz;
    return RASTER_OK;
}

raster_status raster_result_copy_kz(const raster_result* r, int32_t* d_kz, hipStream_t stream) {
    if (!r) return fail(RASTER_E_INVAL, "result is NULL");
    if (!r->kz) return fail(RASTER_E_INVAL, "the result is two-dimensional");
    if (r->tiles == 0) return RASTER_OK;
    if (!d_kz) return fail(RASTER_E_INVAL, "d_kz is NULL");
    HIP_TRY(hipMemcpyAsync(d_kz, r->kz, (size_t)r->tiles * sizeof(int32_t), hipMemcpyDeviceToDevice, stream),
            "kz copy");
    return RASTER_OK;
}

raster_status raster_result_arrays(const raster_result* r, const int32_t** d_kx, const int32_t** d_ky,
                                   const uint32_t** d_count, const uint64_t** d_label) {
    if (!r) return fail(RASTER_E_INVAL, "result is NULL");
    if (d_kx) *d_kx = r->kx;
    if (d_ky) *d_ky = r->ky;
    if (d_count) *d_count = r->count;
    if (d_label) *d_label = r->label;
    return RASTER_OK;
}

raster_status raster_result_copy(const raster_result* r, int32_t* d_kx, int32_t* d_ky, uint32_t* d_count,
                                 uint64_t* d_label, hipStream_t stream) {
    if (!r) return fail(RASTER_E_INVAL, "result is NULL");
    const size_t t = (size_t)r->tiles;
    if (t == 0) return RASTER_OK;
    if (d_kx) HIP_TRY(hipMemcpyAsync(d_kx, r->kx, t * 4, hipMemcpyDeviceToDevice, stream), "copy kx");
    if (d_ky) HIP_TRY(hipMemcpyAsync(d_ky, r->ky, t * 4, hipMemcpyDeviceToDevice, stream), "copy ky");
    if (d_count) HIP_TRY(hipMemcpyAsync(d_count, r->count, t * 4, hipMemcpyDeviceToDevice, stream), "copy count");
    if (d_label) HIP_TRY(hipMemcpyAsync(d_label, r->label, t * 8, hipMemcpyDeviceToDevice, stream), "copy label");
    return RASTER_OK;
}

raster_status raster_result_stats(const raster_result* r, raster_stats* out) {
    if (!r || !out) return fail(RASTER_E_INVAL, "NULL argument");
    *out = r->stats;
    return RASTER_OK;
}

void raster_result_free(raster_result* r) {
    if (!r) return;
    if (r->pool && r->block) r->pool->release(r->block);
    if (r->lt || r->rt || r->lt_err) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        DevicePool& pool = DevicePool::get(dev);
        if (r->lt) pool.release(r->lt);
        if (r->rt) pool.release(r->rt);
        if (r->lt_err) pool.release(r->lt_err);
    }
    delete r;  // a shared block goes back to the pool with its last result
}

// The result's lookup table of one kind (rows = false: tile -> label, true:
// tile -> row), built on first use; the caller holds r->lt_mu.
static raster_status ensure_lookup(raster_result* r, bool rows, DevicePool& pool, hipStream_t stream) {
    if (!r->lt_err) {
        void* e = nullptr;
        HIP_TRY(pool.alloc(&e, sizeof(unsigned long long)), "range flag");
        r->lt_err = (unsigned long long*)e;
    }
    uint64_t*& tab = rows ? r->rt : r->lt;
    uint64_t& tcap = rows ? r->rt_cap : r->lt_cap;
    if (tab) return RASTER_OK;
    // at most half full, so every lookup ends at an empty slot
    const uint64_t cap = next_pow2(std::max<uint64_t>(64, 2 * (uint64_t)r->tiles));
    void* t = nullptr;
    HIP_TRY(pool.alloc(&t, 2 * cap * sizeof(uint64_t)), "lookup table");
    const hipError_t le = launch_label_table(r->kx, r->ky, r->label, (uint64_t)r->tiles, (uint64_t*)t, cap, rows,
                                             stream, r->kz);
    if (le != hipSuccess) {
        pool.release(t);
        return hip_fail(le, "lookup table");
    }
    tab = (uint64_t*)t;
    tcap = cap;
    return RASTER_OK;
}

raster_status raster_result_point_labels(raster_result* r, const void* d_points, int64_t n, raster_dtype dt,
                                         uint64_t* d_labels, hipStream_t stream) {
    if (!r) return fail(RASTER_E_INVAL, "result is NULL");
    raster_status st = check_points(d_points, n, dt, (uint32_t)r->dims);
    if (st != RASTER_OK) return st;
    if (n > 0 && !d_labels) return fail(RASTER_E_INVAL, "labels is NULL with n = %lld", (long long)n);
    if (((uintptr_t)d_labels % 8) != 0) return fail(RASTER_E_INVAL, "labels must be 8-byte aligned");
    if (n == 0) return RASTER_OK;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    DevicePool& pool = DevicePool::get(dev);
    unsigned long long err = 0;
    {
        std::lock_guard<std::mutex> g(r->lt_mu);
        if ((st = ensure_lookup(r, false, pool, stream)) != RASTER_OK) return st;
        HIP_TRY(launch_zero_u64((uint64_t*)r->lt_err, 1, stream), "zero flag");
        HIP_TRY(launch_point_labels(d_points, n, (int)dt, r->scale, r->lt, r->lt_cap, d_labels, r->lt_err, stream,
                                    r->dims),
                "point labels");
        HIP_TRY(hipMemcpyAsync(&err, r->lt_err, sizeof err, hipMemcpyDeviceToHost, stream), "flag copy");
        HIP_TRY(hipStreamSynchronize(stream), "hipStreamSynchronize");
    }
    if (err & kErrRange) return fail(RASTER_E_RANGE, "%s", range_message(r->dims));
    return RASTER_OK;
}

raster_status raster_result_tile_points(raster_result* r, const void* d_points, int64_t n, raster_dtype dt,
                                        uint64_t* d_row_start, uint64_t* d_index, int64_t cap, int64_t* n_kept,
                                        hipStream_t stream) {
    if (n_kept) *n_kept = 0;
    if (!r) return fail(RASTER_E_INVAL, "result is NULL");
    if (!n_kept) return fail(RASTER_E_INVAL, "n_kept is NULL");
    raster_status st = check_points(d_points, n, dt, (uint32_t)r->dims);
    if (st != RASTER_OK) return st;
    if (n >= (int64_t)0xFFFFFFFFll) return fail(RASTER_E_INVAL, "more than 2^32 - 2 points in one call");
    if (!d_row_start || ((uintptr_t)d_row_start % 8) != 0)
        return fail(RASTER_E_INVAL, "row_start must be an 8-byte aligned array of t + 1 words");
    if (cap < 0 || (cap > 0 && (!d_index || ((uintptr_t)d_index % 8) != 0)))
        return fail(RASTER_E_INVAL, "index must be an 8-byte aligned array of cap words");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    DevicePool& pool = DevicePool::get(dev);
    const uint64_t t = (uint64_t)r->tiles;
    // scratch: row and rank of every point, count per row, scan partials and total
    const size_t b_rows = ((size_t)std::max<int64_t>(n, 1) * sizeof(uint32_t) + 255) / 256 * 256;
    const size_t b_count = ((size_t)std::max<uint64_t>(t, 1) * sizeof(uint32_t) + 255) / 256 * 256;
    const size_t b_part = (size_t)kScanBlocks * sizeof(uint32_t);
    void* scratch = nullptr;
    HIP_TRY(pool.alloc(&scratch, 2 * b_rows + b_count + b_part + 256), "tile-point scratch");
    uint32_t* row_of = (uint32_t*)scratch;
    uint32_t* rank = (uint32_t*)((char*)scratch + b_rows);
    uint32_t* count = (uint32_t*)((char*)scratch + 2 * b_rows);
    uint32_t* partials = (uint32_t*)((char*)scratch + 2 * b_rows + b_count);
    unsigned long long* total = (unsigned long long*)((char*)scratch + 2 * b_rows + b_count + b_part);
    // the scratch goes back to the pool only once the stream has passed the
    // work that uses it (every path below has waited, except a failed launch)
    struct Release {
        DevicePool& p;
        void* b;
        hipStream_t s;
        ~Release() {
            (void)hipStreamSynchronize(s);
            p.release(b);
        }
    } rel{pool, scratch, stream};
    unsigned long long h[2] = {0, 0};  // total, range flag
    {
        std::lock_guard<std::mutex> g(r->lt_mu);
        if ((st = ensure_lookup(r, true, pool, stream)) != RASTER_OK) return st;
        HIP_TRY(launch_zero_u64((uint64_t*)r->lt_err, 1, stream), "zero flag");
        HIP_TRY(launch_zero_u32(count, std::max<uint64_t>(t, 1), stream), "zero counts");
        HIP_TRY(launch_tile_points_count(d_points, n, (int)dt, r->scale, r->rt, r->rt_cap, row_of, rank, count, t,
                                         partials, total, d_row_start, r->lt_err, stream, r->dims),
                "tile points");
        HIP_TRY(hipMemcpyAsync(&h[0], total, sizeof h[0], hipMemcpyDeviceToHost, stream), "total copy");
        HIP_TRY(hipMemcpyAsync(&h[1], r->lt_err, sizeof h[1], hipMemcpyDeviceToHost, stream), "flag copy");
        HIP_TRY(hipStreamSynchronize(stream), "hipStreamSynchronize");
        if (h[1] & kErrRange) return fail(RASTER_E_RANGE, "%s", range_message(r->dims));
        *n_kept = (int64_t)h[0];
        if ((int64_t)h[0] > cap)
            return fail(RASTER_E_INVAL, "index holds %lld entries, %lld points lie on kept tiles", (long long)cap,
                        (long long)h[0]);
        HIP_TRY(launch_tile_points_scatter(row_of, rank, n, d_row_start, d_index, stream), "tile points scatter");
        HIP_TRY(hipStreamSynchronize(stream), "hipStreamSynchronize");
    }
    return RASTER_OK;
}

raster_status raster_begin_opts(double scale, uint32_t tau, uint32_t mu, const raster_options* opts,
                                int64_t tile_hint, hipStream_t stream, raster_stream** st) {
    if (!st) return fail(RASTER_E_INVAL, "st is NULL");
    *st = nullptr;
    raster_status s = check_params(scale, tau, mu);
    if (s != RASTER_OK) return s;
    s = check_options(opts);
    if (s != RASTER_OK) return s;
    if (tile_hint < 0) return fail(RASTER_E_INVAL, "negative tile_hint");
    raster_stream* h = new raster_stream();
    if (opts) {
        h->run.metric = (uint32_t)opts->metric;
        h->run.delta = opts->delta;
        h->run.square = opts->square_step == 1;
        h->run.dims = options_dims(opts);
    }
    s = h->run.init(scale, tau, mu, tile_hint, stream);
    if (s != RASTER_OK) {
        delete h;
        return s;
    }
    *st = h;
    return RASTER_OK;
}

raster_status raster_begin_p_opts(int32_t precision, uint32_t tau, uint32_t mu, const raster_options* opts,
                                  int64_t tile_hint, hipStream_t stream, raster_stream** st) {
    double s;
    if (st) *st = nullptr;
    if (!scale_for_precision(precision, &s)) return fail(RASTER_E_INVAL, "precision %d outside [0, 15]", precision);
    return raster_begin_opts(s, tau, mu, opts, tile_hint, stream, st);
}

raster_status raster_begin_delta(double scale, uint32_t tau, uint32_t mu, raster_metric metric, uint32_t delta,
                                 int64_t tile_hint, hipStream_t stream, raster_stream** st) {
    const raster_options o{metric, delta, 0, 0};
    return raster_begin_opts(scale, tau, mu, &o, tile_hint, stream, st);
}

raster_status raster_begin_scaled(double scale, uint32_t tau, uint32_t mu, int64_t tile_hint, hipStream_t stream,
                                  raster_stream** st) {
    return raster_begin_opts(scale, tau, mu, nullptr, tile_hint, stream, st);
}

raster_status raster_begin(int32_t precision, uint32_t tau, uint32_t mu, int64_t tile_hint, hipStream_t stream,
                           raster_stream** st) {
    double s;
    if (st) *st = nullptr;
    if (!scale_for_precision(precision, &s)) return fail(RASTER_E_INVAL, "precision %d outside [0, 15]", precision);
    return raster_begin_scaled(s, tau, mu, tile_hint, stream, st);
}

raster_status raster_feed_chunk(raster_stream* st, const void* d_points, int64_t n, raster_dtype dt) {
    if (!st) return fail(RASTER_E_INVAL, "stream is NULL");
    if (st->state != raster_stream::OPEN) {
        if (st->state == raster_stream::FAILED && st->run.failed != RASTER_OK)
            return fail(st->run.failed, "stream failed earlier: %s", raster_status_string(st->run.failed));
        return fail(RASTER_E_STATE, "stream is not open");
    }
    raster_status s = check_points(d_points, n, dt, st->run.dims);
    if (s != RASTER_OK) return s;
    s = st->run.feed(d_points, n, dt);
    if (s != RASTER_OK && st->run.failed != RASTER_OK) st->state = raster_stream::FAILED;
    return s;
}

raster_status raster_finish(raster_stream* st, raster_result** out) {
    if (!out) return fail(RASTER_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!st) return fail(RASTER_E_INVAL, "stream is NULL");
    if (st->state != raster_stream::OPEN) {
        if (st->state == raster_stream::FAILED && st->run.failed != RASTER_OK)
            return fail(st->run.failed, "stream failed earlier: %s", raster_status_string(st->run.failed));
        return fail(RASTER_E_STATE, "stream is not open");
    }
    raster_status s = st->run.finish(out);
    st->state = (s == RASTER_OK) ? raster_stream::FINISHED : raster_stream::FAILED;
    if (s != RASTER_OK && st->run.failed == RASTER_OK) st->run.failed = s;
    return s;
}

raster_status raster_stream_tiles(raster_stream* st, uint64_t* d_keys, uint32_t* d_counts, int64_t cap,
                                  int64_t* m) {
    if (!st || !m) return fail(RASTER_E_INVAL, "NULL argument");
    if (cap > 0 && (!d_keys || !d_counts)) return fail(RASTER_E_INVAL, "NULL output buffers");
    if (st->state != raster_stream::OPEN) return fail(RASTER_E_STATE, "stream is not open");
    raster_status s = st->run.export_tiles(d_keys, d_counts, cap, m);
    if (s != RASTER_OK && st->run.failed != RASTER_OK) st->state = raster_stream::FAILED;
    return s;
}

void raster_stream_destroy(raster_stream* st) {
    if (!st) return;
    (void)hipStreamSynchronize(st->run.stream);
    delete st;
}

raster_status raster_set_tuning(const raster_tuning* t) {
    raster_tuning v = kDefaultTuning;
    if (t) {
        v = *t;
        if (v.block < 64 || v.block > 1024 || v.block % 64) return fail(RASTER_E_INVAL, "block must be 64..1024, x64");
        if (!(v.items == 1 || v.items == 2 || v.items == 4 || v.items == 8 || v.items == 16))
            return fail(RASTER_E_INVAL, "items must be 1, 2, 4, 8 or 16");
        if (v.preagg_slots != 0 &&
            (v.preagg_slots < 256 || v.preagg_slots > 4096 || (v.preagg_slots & (v.preagg_slots - 1))))
            return fail(RASTER_E_INVAL, "preagg_slots must be 0 or a power of two in [256, 4096]");
        if (!(v.load_factor > 0.05f && v.load_factor <= 0.9f)) return fail(RASTER_E_INVAL, "load_factor in (0.05, 0.9]");
        if (v.mode < 0 || v.mode > 3) return fail(RASTER_E_INVAL, "mode must be 0, 1, 2 or 3");
        if (v.group_mpoints < 1 || v.group_mpoints > 4096) return fail(RASTER_E_INVAL, "group_mpoints in [1, 4096]");
    }
    std::lock_guard<std::mutex> g(g_tuning_mu);
    g_tuning = v;
    return RASTER_OK;
}

raster_status raster_get_tuning(raster_tuning* t) {
    if (!t) return fail(RASTER_E_INVAL, "NULL argument");
    *t = current_tuning();
    return RASTER_OK;
}

const char* raster_status_string(raster_status s) {
    switch (s) {
        case RASTER_OK: return "RASTER_OK";
        case RASTER_E_INVAL: return "RASTER_E_INVAL";
        case RASTER_E_RANGE: return "RASTER_E_RANGE";
        case RASTER_E_NOMEM: return "RASTER_E_NOMEM";
        case RASTER_E_DEVICE: return "RASTER_E_DEVICE";
        case RASTER_E_STATE: return "RASTER_E_STATE";
        case RASTER_E_BUDGET: return "RASTER_E_BUDGET";
    }
    return "RASTER_E_UNKNOWN";
}

const char* raster_last_error(void) { return g_last_error.c_str(); }

const char* raster_version(void) { return "raster-mi355x 0.1 (gfx950)"; }

}  // extern "C"
