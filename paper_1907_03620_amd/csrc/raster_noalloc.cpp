// raster_cluster_noalloc: the plain clustering call (Algorithm 1, eight
// neighbours) for callers that cannot allocate device memory.  Every scratch
// buffer -- tile table, compact arrays, union-find words, counters, scan
// partials, the job descriptor -- is carved out of one file-scope device
// array; the caller passes the points and the output rows.
//
// The array is one per device and process, allocated when the code object is
// loaded and held until the process ends.  Its device address is looked up
// once per device (hipGetSymbolAddress) and only that address is handed to
// kernels and copies: the array's name in host code is a host-side stand-in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "raster.h"
#include "raster_internal.h"
#include "raster_runtime.h"

namespace {

using namespace rst;

constexpr int64_t kMaxPoints = RASTER_NOALLOC_MAX_POINTS;
// table: a power of two of at least 4 slots per point, so that the table is
// at most a quarter full
constexpr uint64_t kMaxSlots = (uint64_t)4 * kMaxPoints;
static_assert((kMaxSlots & (kMaxSlots - 1)) == 0, "slot bound must be a power of two");
constexpr uint64_t kSpillRecords = 1u << 14;

constexpr size_t up256(size_t v) { return (v + 255) & ~(size_t)255; }
constexpr size_t kOffTable = 0;
constexpr size_t kOffSKey = up256(kOffTable + kMaxSlots * sizeof(Slot));
constexpr size_t kOffSCount = up256(kOffSKey + kMaxPoints * sizeof(uint64_t));
constexpr size_t kOffParent = up256(kOffSCount + kMaxPoints * sizeof(uint32_t));
constexpr size_t kOffSize = up256(kOffParent + kMaxPoints * sizeof(uint32_t));
constexpr size_t kOffNbr = up256(kOffSize + kMaxPoints * sizeof(uint32_t));
// four neighbour-list words per tile for the eight-neighbour pass
constexpr size_t kOffSpillKeys = up256(kOffNbr + kMaxPoints * 4 * sizeof(uint32_t));
constexpr size_t kOffSpillCounts = up256(kOffSpillKeys + kSpillRecords * sizeof(uint64_t));
constexpr size_t kOffCtr = up256(kOffSpillCounts + kSpillRecords * sizeof(uint32_t));
constexpr size_t kOffPartials = up256(kOffCtr + kCounterWords * sizeof(unsigned long long));
constexpr size_t kOffDims = up256(kOffPartials + kScanBlocks * sizeof(uint32_t));
constexpr size_t kOffJob = up256(kOffDims + sizeof(Dims));
constexpr size_t kScratchBytes = up256(kOffJob + sizeof(JobInfo));
static_assert(kScratchBytes == RASTER_NOALLOC_SCRATCH_BYTES, "header states the scratch size");

}  // namespace

// The scratch array.  Host code never passes its name to a kernel or a copy:
// it uses the device address looked up below.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_setup_mu;
unsigned char* g_scratch[kMaxDevices] = {};
// one call at a time per device: the calls share the device's array
std::mutex g_call_mu[kMaxDevices];

// Device address of this device's array (the device must be current).
raster_status scratch_of(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(RASTER_E_DEVICE, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> g(g_setup_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(RASTER_E_DEVICE, "hipGetSymbolAddress(scratch) gave NULL");
        g_scratch[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch[dev];
    return RASTER_OK;
}

#define NA_TRY(expr, what)                               \
    do {                                                 \
        const hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// Counters after the work enqueued so far (pageable copy, then a wait).
raster_status read_counters(const unsigned long long* d_ctr, unsigned long long* h, hipStream_t stream) {
    NA_TRY(hipMemcpyAsync(h, d_ctr, kCounterWords * sizeof(unsigned long long), hipMemcpyDeviceToHost, stream),
           "counter copy");
    NA_TRY(hipStreamSynchronize(stream), "hipStreamSynchronize");
    return RASTER_OK;
}

}  // namespace

extern "C" raster_status raster_cluster_noalloc(const void* d_points, int64_t n, raster_dtype dt, int32_t precision,
                                                uint32_t tau, uint32_t mu, hipStream_t stream, int32_t* d_kx,
                                                int32_t* d_ky, uint32_t* d_count, uint64_t* d_label,
                                                int64_t max_rows, int64_t* rows, raster_stats* stats) {
    if (!rows) return fail(RASTER_E_INVAL, "rows is NULL");
    *rows = 0;
    double scale;
    if (!scale_for_precision(precision, &scale)) return fail(RASTER_E_INVAL, "precision %d outside [0, 15]", precision);
    raster_status st = check_params(scale, tau, mu);
    if (st != RASTER_OK) return st;
    st = check_points(d_points, n, dt, 2);
    if (st != RASTER_OK) return st;
    if (n > kMaxPoints)
        return fail(RASTER_E_INVAL, "%lld points exceed the fixed scratch of raster_cluster_noalloc (at most %lld)",
                    (long long)n, (long long)kMaxPoints);
    if (max_rows < 0) return fail(RASTER_E_INVAL, "negative max_rows");
    if (max_rows > 0 && (!d_kx || !d_ky || !d_count || !d_label))
        return fail(RASTER_E_INVAL, "NULL output array with max_rows = %lld", (long long)max_rows);

    int dev = 0;
    NA_TRY(hipGetDevice(&dev), "hipGetDevice");
    unsigned char* base = nullptr;
    if ((st = scratch_of(dev, &base)) != RASTER_OK) return st;
    std::lock_guard<std::mutex> call(g_call_mu[dev]);

    Slot* tab = reinterpret_cast<Slot*>(base + kOffTable);
    uint64_t* s_key = reinterpret_cast<uint64_t*>(base + kOffSKey);
    uint32_t* s_count = reinterpret_cast<uint32_t*>(base + kOffSCount);
    uint32_t* parent = reinterpret_cast<uint32_t*>(base + kOffParent);
    uint32_t* size = reinterpret_cast<uint32_t*>(base + kOffSize);
    uint32_t* nbr = reinterpret_cast<uint32_t*>(base + kOffNbr);
    unsigned long long* ctr = reinterpret_cast<unsigned long long*>(base + kOffCtr);
    uint32_t* partials = reinterpret_cast<uint32_t*>(base + kOffPartials);
    Dims* d_dims = reinterpret_cast<Dims*>(base + kOffDims);
    JobInfo* d_job = reinterpret_cast<JobInfo*>(base + kOffJob);
    const SpillBuf sp{reinterpret_cast<uint64_t*>(base + kOffSpillKeys),
                      reinterpret_cast<uint32_t*>(base + kOffSpillCounts), kSpillRecords};

    // the array keeps the previous call's contents: clear what starts empty
    const uint64_t cap = next_pow2(std::max<uint64_t>(4096, 4 * (uint64_t)n));
    NA_TRY(launch_fill_table(tab, cap, stream), "fill table");
    NA_TRY(launch_zero_u64(reinterpret_cast<uint64_t*>(ctr), kCounterWords, stream), "zero counters");
    NA_TRY(launch_project_count(d_points, n, (int)dt, scale, tab, cap, sp, ctr, kernel_tuning(current_tuning()),
                                stream, 2),
           "project_count");

    Dims dims{};
    dims.slots = cap;
    dims.njobs = 1;
    JobInfo job{};
    job.n = n;
    job.scale = scale;
    job.cap = cap;
    job.tau = tau;
    job.mu = mu;
    NA_TRY(launch_store_job(dims, job, d_dims, d_job, stream), "job descriptor");
    const JobView jv{d_dims, d_job, nullptr, nullptr, nullptr};
    const uint64_t m_max = std::max<int64_t>(n, 1);
    NA_TRY(launch_threshold(tab, jv, s_key, s_count, size, partials, ctr, stream), "threshold");
    NA_TRY(launch_agglomerate(tab, cap, jv, s_key, parent, nbr, size, m_max, ctr, stream), "agglomerate");
    // the component root of every significant tile is now in nbr
    NA_TRY(launch_filter_count(jv, nbr, size, partials, ctr, stream), "filter count");
    unsigned long long h[kCounterWords];
    if ((st = read_counters(ctr, h, stream)) != RASTER_OK) return st;
    if (h[C_ERROR] & kErrRange)
        return fail(RASTER_E_RANGE, "a coordinate is not finite or its tile is outside +-(2^31 - 2)");
    if (h[C_SPILLED] || (h[C_ERROR] & kErrSpillOverflow))
        return fail(RASTER_E_NOMEM, "the fixed table of raster_cluster_noalloc overflowed (%llu keys spilled); "
                    "use raster_cluster", h[C_SPILLED]);
    if (h[C_ERROR] & kErrInternal) return fail(RASTER_E_DEVICE, "agglomeration state inconsistent");
    if (h[C_SUM] != (unsigned long long)n || h[C_DISTINCT] != h[C_INSERTED])
        return fail(RASTER_E_DEVICE, "table inconsistent: sum %llu vs n %lld, occupied %llu vs inserted %llu",
                    h[C_SUM], (long long)n, h[C_DISTINCT], h[C_INSERTED]);
    const int64_t t = (int64_t)h[C_TILES];
    *rows = t;
    if (t > max_rows)
        return fail(RASTER_E_INVAL, "the result has %lld rows, the output arrays hold %lld", (long long)t,
                    (long long)max_rows);
    if (t > 0) {
        NA_TRY(launch_filter_scatter(jv, s_key, s_count, nbr, size, d_kx, d_ky, d_count, d_label, nullptr, partials,
                                     ctr, stream),
               "filter scatter");
        NA_TRY(hipStreamSynchronize(stream), "hipStreamSynchronize");
    }
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        stats->n_points = n;
        stats->distinct_tiles = (int64_t)h[C_DISTINCT];
        stats->significant_tiles = (int64_t)h[C_SIGNIFICANT];
        stats->components = (int64_t)h[C_COMPONENTS];
        stats->clusters = (int64_t)h[C_CLUSTERS];
        stats->tiles = t;
        stats->table_capacity = (int64_t)cap;
        stats->count_launches = n > 0 ? 1 : 0;
    }
    return RASTER_OK;
}
