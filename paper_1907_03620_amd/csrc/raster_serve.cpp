// Batched and served forms of the RASTER library.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <vector>
#include <string>
#include <thread>
#include <unordered_map>

#include "raster.h"
#include "raster_runtime.h"

using namespace rst;

#define HIP_TRY_S(expr, what)                              \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return hip_fail(e_, what);   \
    } while (0)

// ----------------------------------------------------------------- batch ---
//
// A batch is clustered by one pipeline over all its jobs: one fused counting
// launch over every job's point tiles, then the job-aware significance scan,
// agglomeration and mu filter over one arena holding every job's table.  All
// sizes the kernels need are read from device memory, so the pipeline is
// captured once into a HIP graph and replayed for every batch that fits the
// engine's buffers; a batch that does not fit grows the buffers and
// re-captures.  A job whose table turns out too small (a key found its probe
// window full) is redone alone with the growable single-table path.

namespace rst {

struct BatchEngine {
    int device = 0;
    hipStream_t bs = nullptr;  // capture and replay stream
    hipEvent_t ev_in = nullptr;
    Buffers bufs;
    uint64_t arena_cap = 0, parts_cap = 0, s_cap = 0;
    uint32_t jobs_cap = 0;
    Slot* arena = nullptr;
    JobInfo* jobs_dev = nullptr;
    Dims* dims_dev = nullptr;
    uint32_t* tile_prefix = nullptr;
    uint32_t* part_job = nullptr;
    unsigned long long* ctr = nullptr;
    unsigned long long* job_ctr = nullptr;
    uint64_t* s_key = nullptr;
    uint32_t *s_count = nullptr, *s_job = nullptr, *parent = nullptr, *nbr = nullptr, *size = nullptr;
    int32_t *o_kx = nullptr, *o_ky = nullptr;
    uint32_t *o_count = nullptr, *o_job = nullptr;
    uint64_t* o_label = nullptr;
    uint32_t* bounds = nullptr;  // s_start, s_end, o_start, o_end: jobs_cap each
    uint32_t* partials = nullptr;
    // binned counting
    uint64_t coarse_cap = 0, bin1_cap = 0, bin2_cap = 0;  // coarse buckets, keys
    uint32_t* cjob = nullptr;
    uint32_t* cursor1 = nullptr;
    uint32_t* cursor2 = nullptr;
    uint64_t* bin1 = nullptr;
    uint64_t* bin2 = nullptr;
    uint32_t* h_cjob = nullptr;
    bool graph_binned = false;
    // pinned host mirrors
    JobInfo* h_jobs = nullptr;
    Dims* h_dims = nullptr;
    uint32_t* h_tile_prefix = nullptr;
    uint32_t* h_part_job = nullptr;
    unsigned long long* h_job_ctr = nullptr;
    unsigned long long* h_ctr = nullptr;
    uint32_t* h_bounds = nullptr;
    // distinct-tile sketch pass (before the tables are sized)
    uint32_t sk_cap = 0;
    JobInfo* sk_jobs = nullptr;
    Dims* sk_dims = nullptr;
    uint32_t* sk_prefix = nullptr;
    uint32_t* sk_hll = nullptr;
    JobInfo* h_sk_jobs = nullptr;
    Dims* h_sk_dims = nullptr;
    uint32_t* h_sk_prefix = nullptr;
    uint32_t* h_sk_hll = nullptr;
    Buffers sk_bufs;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    raster_tuning graph_tuning{};
    bool graph_valid = false;
    // neighbourhood of the agglomeration (Section 3.2): that of the current
    // run and that the captured graph was recorded with (its link launches
    // carry the offsets as arguments)
    uint32_t metric = RASTER_CHEBYSHEV, delta = 1;
    uint32_t graph_metric = RASTER_CHEBYSHEV, graph_delta = 1;
    bool square = false, graph_square = false;  // the 2x2 post-step (Section 3.6)
    std::vector<NbrRound> rounds;
    uint64_t nbr_cap_words = 4;  // neighbour-list words per tile the buffer holds
    std::mutex mu;
    float last_us = 0.f;  // device time of the last replay

    ~BatchEngine() { release(); }
    void release_host() {
        if (h_jobs) (void)hipHostFree(h_jobs);
        if (h_dims) (void)hipHostFree(h_dims);
        if (h_tile_prefix) (void)hipHostFree(h_tile_prefix);
        if (h_part_job) (void)hipHostFree(h_part_job);
        if (h_job_ctr) (void)hipHostFree(h_job_ctr);
        if (h_ctr) (void)hipHostFree(h_ctr);
        if (h_bounds) (void)hipHostFree(h_bounds);
        if (h_cjob) (void)hipHostFree(h_cjob);
        h_cjob = nullptr;
        h_jobs = nullptr;
        h_dims = nullptr;
        h_tile_prefix = nullptr;
        h_part_job = nullptr;
        h_job_ctr = nullptr;
        h_ctr = nullptr;
        h_bounds = nullptr;
    }
    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        graph_valid = false;
    }
    void release_sketch() {
        sk_bufs.release_all();
        if (h_sk_jobs) (void)hipHostFree(h_sk_jobs);
        if (h_sk_dims) (void)hipHostFree(h_sk_dims);
        if (h_sk_prefix) (void)hipHostFree(h_sk_prefix);
        if (h_sk_hll) (void)hipHostFree(h_sk_hll);
        h_sk_jobs = nullptr;
        h_sk_dims = nullptr;
        h_sk_prefix = nullptr;
        h_sk_hll = nullptr;
        sk_jobs = nullptr;
        sk_dims = nullptr;
        sk_prefix = nullptr;
        sk_hll = nullptr;
        sk_cap = 0;
    }
    void release() {
        if (bs) (void)hipStreamSynchronize(bs);
        drop_graph();
        bufs.release_all();
        release_host();
        release_sketch();
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (bs) (void)hipStreamDestroy(bs);
        ev_in = nullptr;
        bs = nullptr;
        arena_cap = parts_cap = s_cap = 0;
        coarse_cap = bin1_cap = bin2_cap = 0;
        jobs_cap = 0;
    }

    raster_status init() {
        if (bs) return RASTER_OK;
        hipError_t e = hipGetDevice(&device);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&bs, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_in, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "batch engine");
        bufs.pool = &DevicePool::get(device);
        sk_bufs.pool = bufs.pool;
        return RASTER_OK;
    }

    // Distinct tiles per job, estimated from one pass over the points (see
    // k_batch_hll); tile_prefix and tile as for the counting launch.
    raster_status estimate_distinct(const raster_job* jobs, int32_t n_jobs, const std::vector<uint32_t>& prefix,
                                    uint32_t tile, std::vector<double>* est) {
        if ((uint32_t)n_jobs > sk_cap) {
            (void)hipStreamSynchronize(bs);
            release_sketch();
            sk_cap = (uint32_t)n_jobs + (uint32_t)n_jobs / 4 + 8;
            hipError_t e = sk_bufs.take((void**)&sk_jobs, sk_cap * sizeof(JobInfo));
            if (e == hipSuccess) e = sk_bufs.take((void**)&sk_dims, sizeof(Dims));
            if (e == hipSuccess) e = sk_bufs.take((void**)&sk_prefix, (sk_cap + 1) * sizeof(uint32_t));
            if (e == hipSuccess) e = sk_bufs.take((void**)&sk_hll, ((size_t)sk_cap << kHllLog2) * sizeof(uint32_t));
            if (e == hipSuccess) e = hipHostMalloc((void**)&h_sk_jobs, sk_cap * sizeof(JobInfo), 0);
            if (e == hipSuccess) e = hipHostMalloc((void**)&h_sk_dims, sizeof(Dims), 0);
            if (e == hipSuccess) e = hipHostMalloc((void**)&h_sk_prefix, (sk_cap + 1) * sizeof(uint32_t), 0);
            if (e == hipSuccess)
                e = hipHostMalloc((void**)&h_sk_hll, ((size_t)sk_cap << kHllLog2) * sizeof(uint32_t), 0);
            if (e != hipSuccess) {
                release_sketch();
                return hip_fail(e, "distinct-tile sketch buffers");
            }
        }
        std::memset(h_sk_jobs, 0, n_jobs * sizeof(JobInfo));
        for (int32_t i = 0; i < n_jobs; ++i) {
            double sc = jobs[i].scale;
            if (!(sc > 0.0)) scale_for_precision(jobs[i].precision, &sc);
            JobInfo& J = h_sk_jobs[i];
            J.pts = jobs[i].d_points;
            J.n = jobs[i].n;
            J.scale = sc;
            J.dtype = (int32_t)jobs[i].dt;
            J.first_tile = prefix[i];
            h_sk_prefix[i] = prefix[i];
        }
        h_sk_prefix[n_jobs] = prefix[n_jobs];
        std::memset(h_sk_dims, 0, sizeof(Dims));
        h_sk_dims->njobs = (uint32_t)n_jobs;
        h_sk_dims->tiles = prefix[n_jobs];
        hipError_t e = hipMemcpyAsync(sk_jobs, h_sk_jobs, n_jobs * sizeof(JobInfo), hipMemcpyHostToDevice, bs);
        if (e == hipSuccess) e = hipMemcpyAsync(sk_dims, h_sk_dims, sizeof(Dims), hipMemcpyHostToDevice, bs);
        if (e == hipSuccess)
            e = hipMemcpyAsync(sk_prefix, h_sk_prefix, (n_jobs + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, bs);
        const JobView jv{sk_dims, sk_jobs, nullptr, nullptr, nullptr};
        if (e == hipSuccess)
            e = launch_batch_hll(jv, sk_prefix, tile, sk_hll, (uint32_t)n_jobs, prefix[n_jobs], bs);
        const size_t regs = (size_t)n_jobs << kHllLog2;
        if (e == hipSuccess)
            e = hipMemcpyAsync(h_sk_hll, sk_hll, regs * sizeof(uint32_t), hipMemcpyDeviceToHost, bs);
        if (e == hipSuccess) e = hipStreamSynchronize(bs);
        if (e != hipSuccess) return hip_fail(e, "distinct-tile sketch");
        est->assign(n_jobs, 0.0);
        for (int32_t i = 0; i < n_jobs; ++i) (*est)[i] = hll_estimate(h_sk_hll + ((size_t)i << kHllLog2));
        return RASTER_OK;
    }

    // Grows every buffer to hold the given totals (with headroom), dropping
    // the captured graph when anything moves.
    raster_status reserve(uint64_t slots, uint64_t s_need, uint32_t njobs, uint64_t ncoarse, uint64_t b1, uint64_t b2,
                          uint64_t words) {
        const bool ok = slots <= arena_cap && s_need <= s_cap && njobs <= jobs_cap && ncoarse <= coarse_cap &&
                        b1 <= bin1_cap && b2 <= bin2_cap && words <= nbr_cap_words;
        if (ok) return RASTER_OK;
        (void)hipStreamSynchronize(bs);
        drop_graph();
        bufs.release_all();
        release_host();
        arena_cap = std::max<uint64_t>(slots + slots / 4, arena_cap);
        arena_cap = (arena_cap + 2 * kPartSlotsHost - 1) / (2 * kPartSlotsHost) * (2 * kPartSlotsHost);
        parts_cap = arena_cap / kPartSlotsHost;
        s_cap = std::max<uint64_t>(s_need + s_need / 4 + 1024, s_cap);
        jobs_cap = std::max<uint32_t>(njobs + njobs / 4 + 8, jobs_cap);
        coarse_cap = std::max<uint64_t>((ncoarse + ncoarse / 4 + 9) & ~1ull, coarse_cap);
        bin1_cap = std::max<uint64_t>(b1 + b1 / 4, bin1_cap);
        bin2_cap = std::max<uint64_t>(b2 + b2 / 4, bin2_cap);
        nbr_cap_words = std::max<uint64_t>(words, nbr_cap_words);
        auto take = [&](void** p, size_t bytes, const char* what) -> raster_status {
            hipError_t e = bufs.take(p, bytes);
            return e == hipSuccess ? RASTER_OK : hip_fail(e, what);
        };
        raster_status st;
#define TAKE(ptr, bytes, what) \
    if ((st = take((void**)&(ptr), (bytes), (what))) != RASTER_OK) return st
        TAKE(arena, arena_cap * sizeof(Slot), "batch arena");
        TAKE(jobs_dev, jobs_cap * sizeof(JobInfo), "job table");
        TAKE(dims_dev, sizeof(Dims), "dims");
        TAKE(tile_prefix, (jobs_cap + 1) * sizeof(uint32_t), "tile prefix");
        TAKE(part_job, parts_cap * sizeof(uint32_t), "partition map");
        TAKE(ctr, kCounterWords * sizeof(unsigned long long), "counters");
        TAKE(job_ctr, (size_t)jobs_cap * kCounterWords * sizeof(unsigned long long), "job counters");
        TAKE(s_key, s_cap * sizeof(uint64_t), "S keys");
        TAKE(s_count, s_cap * sizeof(uint32_t), "S counts");
        TAKE(s_job, s_cap * sizeof(uint32_t), "S jobs");
        TAKE(parent, s_cap * sizeof(uint32_t), "parents");
        TAKE(nbr, s_cap * nbr_cap_words * sizeof(uint32_t), "neighbour lists");
        TAKE(size, s_cap * sizeof(uint32_t), "sizes");
        TAKE(o_kx, s_cap * sizeof(int32_t), "rows");
        TAKE(o_ky, s_cap * sizeof(int32_t), "rows");
        TAKE(o_count, s_cap * sizeof(uint32_t), "rows");
        TAKE(o_label, s_cap * sizeof(uint64_t), "rows");
        TAKE(o_job, s_cap * sizeof(uint32_t), "rows");
        TAKE(bounds, (size_t)4 * jobs_cap * sizeof(uint32_t), "job bounds");
        TAKE(partials, kScanBlocks * sizeof(uint32_t), "scan partials");
        TAKE(cjob, coarse_cap * sizeof(uint32_t), "coarse map");
        TAKE(cursor1, coarse_cap * sizeof(uint32_t), "coarse cursors");
        TAKE(cursor2, parts_cap * sizeof(uint32_t), "partition cursors");
        if (bin1_cap) TAKE(bin1, bin1_cap * sizeof(uint64_t), "coarse buckets");
        if (bin2_cap) TAKE(bin2, bin2_cap * sizeof(uint64_t), "partition buckets");
#undef TAKE
        hipError_t e = hipHostMalloc((void**)&h_jobs, jobs_cap * sizeof(JobInfo), hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void**)&h_dims, sizeof(Dims), hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void**)&h_tile_prefix, (jobs_cap + 1) * sizeof(uint32_t), 0);
        if (e == hipSuccess) e = hipHostMalloc((void**)&h_part_job, parts_cap * sizeof(uint32_t), 0);
        if (e == hipSuccess)
            e = hipHostMalloc((void**)&h_job_ctr, (size_t)jobs_cap * kCounterWords * sizeof(unsigned long long), 0);
        if (e == hipSuccess) e = hipHostMalloc((void**)&h_ctr, kCounterWords * sizeof(unsigned long long), 0);
        if (e == hipSuccess) e = hipHostMalloc((void**)&h_bounds, (size_t)4 * jobs_cap * sizeof(uint32_t), 0);
        if (e == hipSuccess) e = hipHostMalloc((void**)&h_cjob, coarse_cap * sizeof(uint32_t), 0);
        if (e != hipSuccess) return hip_fail(e, "pinned batch mirrors");
        return RASTER_OK;
    }

    JobView view() const {
        return JobView{dims_dev, jobs_dev, part_job, s_job, job_ctr};
    }

    // The pipeline; enqueued on bs, directly or under capture.
    hipError_t enqueue(const raster_tuning& tu, bool binned) {
        const JobView jv = view();
        hipError_t e = launch_zero_u64((uint64_t*)ctr, kCounterWords, bs);
        if (e == hipSuccess) e = launch_zero_u64((uint64_t*)job_ctr, (uint64_t)jobs_cap * kCounterWords, bs);
        if (e == hipSuccess) e = launch_zero_u64((uint64_t*)bounds, (uint64_t)2 * jobs_cap, bs);
        if (e == hipSuccess) e = launch_fill_dims(arena, dims_dev, bs);
        if (binned) {
            if (e == hipSuccess) e = launch_zero_u64((uint64_t*)cursor1, coarse_cap / 2, bs);
            if (e == hipSuccess) e = launch_zero_u64((uint64_t*)cursor2, parts_cap / 2, bs);
            if (e == hipSuccess)
                e = launch_batch_binned(jv, tile_prefix, cjob, bin1, cursor1, bin2, cursor2, arena, bs);
        } else {
            if (e == hipSuccess) e = launch_batch_count(jv, tile_prefix, arena, kernel_tuning(tu), 4096, bs);
        }
        if (e == hipSuccess)
            e = launch_threshold(arena, jv, s_key, s_count, size, partials, ctr, bs, square ? arena_cap : 0);
        if (e == hipSuccess)
            e = launch_agglomerate(arena, arena_cap, jv, s_key, parent, nbr, size, s_cap, ctr, bs, rounds.data(),
                                   (int)rounds.size());
        if (e == hipSuccess)
            e = launch_filter(jv, s_key, s_count, nbr, size, o_kx, o_ky, o_count, o_label, o_job, partials, ctr, bs);
        uint32_t* s_start = bounds;
        uint32_t* s_end = bounds + jobs_cap;
        uint32_t* o_start = bounds + 2 * jobs_cap;
        uint32_t* o_end = bounds + 3 * jobs_cap;
        if (e == hipSuccess) e = launch_bounds(s_job, ctr + C_SIGNIFICANT, s_start, s_end, s_cap, bs);
        if (e == hipSuccess) e = launch_bounds(o_job, ctr + C_TILES, o_start, o_end, s_cap, bs);
        if (e == hipSuccess) e = launch_job_stats(jv, nbr, size, s_start, s_end, o_start, o_end, jobs_cap, bs);
        return e;
    }

    raster_status run(const raster_job* jobs, int32_t n_jobs, hipStream_t user, raster_result** outs,
                      std::vector<int32_t>* redo, uint32_t metric_ = RASTER_CHEBYSHEV, uint32_t delta_ = 1,
                      bool square_ = false);

    static constexpr uint64_t kPartSlotsHost = 4096;
};

raster_status BatchEngine::run(const raster_job* jobs, int32_t n_jobs, hipStream_t user, raster_result** outs,
                               std::vector<int32_t>* redo, uint32_t metric_, uint32_t delta_, bool square_) {
    raster_status st = init();
    if (st != RASTER_OK) return st;
    metric = metric_;
    delta = delta_;
    square = square_;
    rounds = neighbourhood_rounds(metric, delta);
    const raster_tuning tu = current_tuning();
    // every job's table sized from its estimated distinct tiles (a job that
    // still overflows is redone alone); the sketch reads the points in tiles
    // of its own size
    constexpr uint64_t sk_tile = 4096;
    std::vector<uint32_t> sk_prefix(n_jobs + 1);
    uint64_t sk_tiles = 0;
    for (int32_t i = 0; i < n_jobs; ++i) {
        sk_prefix[i] = (uint32_t)sk_tiles;
        sk_tiles += ((uint64_t)jobs[i].n + sk_tile - 1) / sk_tile;
        if (sk_tiles > 0xFFFFFFF0ull) return fail(RASTER_E_NOMEM, "batch too large for one launch");
    }
    sk_prefix[n_jobs] = (uint32_t)sk_tiles;
    hipError_t e = hipEventRecord(ev_in, user);
    if (e == hipSuccess) e = hipStreamWaitEvent(bs, ev_in, 0);
    if (e != hipSuccess) return hip_fail(e, "batch stream order");
    std::vector<double> distinct;
    st = estimate_distinct(jobs, n_jobs, sk_prefix, (uint32_t)sk_tile, &distinct);
    if (st != RASTER_OK) return st;
    std::vector<uint64_t> caps(n_jobs);
    bool binned = tu.mode != 1;
    for (int32_t i = 0; i < n_jobs; ++i) {
        const uint64_t n = (uint64_t)jobs[i].n;
        const double d = std::min<double>(1.25 * distinct[i], (double)n);
        // at least one partition per coarse bucket of about 32K keys (at most
        // 128), which bounds the coarse-bucket capacity
        const uint64_t nc = std::min<uint64_t>(next_pow2(std::max<uint64_t>(1, (n + 32767) / 32768)), 128);
        caps[i] = next_pow2(std::max<uint64_t>(nc * kPartSlotsHost, (uint64_t)(d / tu.load_factor) + 1));
        // level 2 splits a coarse bucket into at most kMaxFine partitions
        if (caps[i] / kPartSlotsHost > 128ull * kMaxFine) binned = false;
    }
    const uint64_t tile = binned ? (uint64_t)kBinTile : (uint64_t)tu.block * (uint64_t)tu.items;
    // work tiles of every job
    std::vector<uint32_t> tiles(n_jobs);
    uint64_t tiles_total = 0;
    for (int32_t i = 0; i < n_jobs; ++i) {
        tiles[i] = (uint32_t)(((uint64_t)jobs[i].n + tile - 1) / tile);
        tiles_total += tiles[i];
        if (tiles_total > 0xFFFFFFF0ull) return fail(RASTER_E_NOMEM, "batch too large for one launch");
    }
    // layout of the tables and coarse buckets
    std::vector<uint64_t> bases(n_jobs), b2base(n_jobs);
    std::vector<uint32_t> ncs(n_jobs), shifts(n_jobs), cbases(n_jobs), cap2s(n_jobs);
    uint64_t slots = 0, pts_total = 0, ncoarse = 0, per1 = 1, b2_total = 0;
    for (int32_t i = 0; i < n_jobs; ++i) {
        const uint64_t n = (uint64_t)jobs[i].n;
        bases[i] = slots;
        slots += caps[i];
        pts_total += n;
        // about 32K keys per coarse bucket, at most 128 buckets per job
        const uint64_t parts = caps[i] / kPartSlotsHost;
        uint64_t nc = next_pow2(std::max<uint64_t>(1, (n + 32767) / 32768));
        nc = std::min<uint64_t>(nc, std::min<uint64_t>(parts, 128));
        ncs[i] = (uint32_t)nc;
        shifts[i] = (uint32_t)(__builtin_ctzll(parts) - __builtin_ctzll(nc));
        cbases[i] = (uint32_t)ncoarse;
        ncoarse += nc;
        per1 = std::max<uint64_t>(per1, (n + nc - 1) / nc);
        // partition-list capacity: the expected share plus slack far beyond
        // the binomial spread; a key past it is added directly instead
        const uint64_t per2 = (n + parts - 1) / parts;
        uint64_t c2 = per2 + per2 / 8 + 4 * (uint64_t)std::sqrt((double)per2) + 256;
        c2 = (c2 + 63) / 64 * 64;
        cap2s[i] = (uint32_t)c2;
        b2base[i] = b2_total;
        b2_total += parts * c2;
    }
    if (slots > (1ull << 33)) return fail(RASTER_E_NOMEM, "batch too large for one launch");
    // coarse-bucket capacity: the expected share plus slack far beyond the
    // binomial spread; a key past it is added directly instead
    uint64_t cap1 = per1 + per1 / 16 + 4 * (uint64_t)std::sqrt((double)per1) + 1024;
    cap1 = (cap1 + 255) / 256 * 256;
    const uint64_t s_need = std::max<uint64_t>(1, std::min<uint64_t>(slots, pts_total));
    st = reserve(slots, s_need, (uint32_t)n_jobs, binned ? ncoarse : 0, binned ? ncoarse * cap1 : 0,
                 binned ? b2_total : 0, nbr_words((int)rounds.size()));
    if (st != RASTER_OK) return st;
    // host mirrors
    uint32_t tp = 0;
    for (int32_t i = 0; i < n_jobs; ++i) {
        double sc = jobs[i].scale;
        if (!(sc > 0.0)) scale_for_precision(jobs[i].precision, &sc);
        JobInfo& J = h_jobs[i];
        J.pts = jobs[i].d_points;
        J.n = jobs[i].n;
        J.scale = sc;
        J.slot_base = bases[i];
        J.cap = caps[i];
        J.tau = jobs[i].tau;
        J.mu = jobs[i].mu;
        J.dtype = (int32_t)jobs[i].dt;
        J.first_tile = tp;
        J.part_base = (uint32_t)(bases[i] / kPartSlotsHost);
        J.cbase = cbases[i];
        J.cshift = shifts[i];
        J.cap2 = cap2s[i];
        J.bin2_base = b2base[i];
        J.framed = 0;  // batch tables are unframed
        J.fx = 0;
        J.fy = 0;
        h_tile_prefix[i] = tp;
        tp += tiles[i];
        for (uint64_t p = bases[i] / kPartSlotsHost; p < (bases[i] + caps[i]) / kPartSlotsHost; ++p)
            h_part_job[p] = (uint32_t)i;
        if (binned)
            for (uint32_t c = 0; c < ncs[i]; ++c) h_cjob[cbases[i] + c] = (uint32_t)i;
    }
    h_tile_prefix[n_jobs] = tp;
    h_dims->slots = slots;
    h_dims->njobs = (uint32_t)n_jobs;
    h_dims->tiles = tp;
    h_dims->cap1 = cap1;
    h_dims->cap2 = 0;
    h_dims->ncoarse = binned ? (uint32_t)ncoarse : 0;
    h_dims->segs = (uint32_t)((cap1 + kBinTile - 1) / kBinTile);
    e = hipMemcpyAsync(jobs_dev, h_jobs, n_jobs * sizeof(JobInfo), hipMemcpyHostToDevice, bs);
    if (e == hipSuccess) e = hipMemcpyAsync(dims_dev, h_dims, sizeof(Dims), hipMemcpyHostToDevice, bs);
    if (e == hipSuccess)
        e = hipMemcpyAsync(tile_prefix, h_tile_prefix, (n_jobs + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, bs);
    if (e == hipSuccess)
        e = hipMemcpyAsync(part_job, h_part_job, (slots / kPartSlotsHost) * sizeof(uint32_t), hipMemcpyHostToDevice,
                           bs);
    if (e == hipSuccess && binned)
        e = hipMemcpyAsync(cjob, h_cjob, ncoarse * sizeof(uint32_t), hipMemcpyHostToDevice, bs);
    if (e != hipSuccess) return hip_fail(e, "batch upload");
    const bool same_tuning = graph_tuning.block == tu.block && graph_tuning.items == tu.items &&
                             graph_tuning.preagg_slots == tu.preagg_slots && graph_binned == binned &&
                             graph_metric == metric && graph_delta == delta && graph_square == square;
    if (!graph_valid || !same_tuning) {
        drop_graph();
        e = hipStreamBeginCapture(bs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t le = enqueue(tu, binned);
            e = hipStreamEndCapture(bs, &graph);
            if (le != hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph();
            (void)hipGetLastError();
            return hip_fail(e, "batch graph capture");
        }
        graph_valid = true;
        graph_tuning = tu;
        graph_binned = binned;
        graph_metric = metric;
        graph_delta = delta;
        graph_square = square;
    }
    hipEvent_t t0 = nullptr, t1 = nullptr;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    (void)hipEventRecord(t0, bs);
    e = hipGraphLaunch(exec, bs);
    (void)hipEventRecord(t1, bs);
    if (e == hipSuccess) e = hipMemcpyAsync(h_ctr, ctr, kCounterWords * sizeof(unsigned long long), hipMemcpyDeviceToHost, bs);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h_job_ctr, job_ctr, (size_t)n_jobs * kCounterWords * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, bs);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h_bounds, bounds, (size_t)4 * jobs_cap * sizeof(uint32_t), hipMemcpyDeviceToHost, bs);
    if (e == hipSuccess) e = hipStreamSynchronize(bs);
    if (e == hipSuccess) (void)hipEventElapsedTime(&last_us, t0, t1);
    last_us *= 1000.f;
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (e != hipSuccess) return hip_fail(e, "batch run");
    if (h_ctr[C_ERROR] & kErrInternal) return fail(RASTER_E_DEVICE, "agglomeration state inconsistent");
    for (int32_t i = 0; i < n_jobs; ++i)
        if (h_job_ctr[(size_t)i * kCounterWords + C_ERROR] & kErrRange)
            return fail(RASTER_E_RANGE, "job %d: a coordinate is not finite or its tile is out of range", i);
    // copy the rows out of the reusable buffers into one block the results share
    const uint64_t t = h_ctr[C_TILES];
    const size_t row_bytes = 2 * sizeof(int32_t) + sizeof(uint32_t) + sizeof(uint64_t);
    void* block = nullptr;
    e = bufs.pool->alloc(&block, t * row_bytes + 256);
    if (e != hipSuccess) return hip_fail(e, "batch result block");
    DevicePool* pool = bufs.pool;
    std::shared_ptr<void> owner(block, [pool](void* p) { pool->release(p); });
    char* b = (char*)block;
    uint64_t* lab = (uint64_t*)b;
    int32_t* kx = (int32_t*)(b + t * sizeof(uint64_t));
    int32_t* ky = kx + t;
    uint32_t* cnt = (uint32_t*)(ky + t);
    if (t) {
        e = hipMemcpyAsync(lab, o_label, t * 8, hipMemcpyDeviceToDevice, bs);
        if (e == hipSuccess) e = hipMemcpyAsync(kx, o_kx, t * 4, hipMemcpyDeviceToDevice, bs);
        if (e == hipSuccess) e = hipMemcpyAsync(ky, o_ky, t * 4, hipMemcpyDeviceToDevice, bs);
        if (e == hipSuccess) e = hipMemcpyAsync(cnt, o_count, t * 4, hipMemcpyDeviceToDevice, bs);
        if (e == hipSuccess) e = hipStreamSynchronize(bs);
        if (e != hipSuccess) return hip_fail(e, "batch result copy");
    }
    const uint32_t* o_start = h_bounds + 2 * jobs_cap;
    for (int32_t i = 0; i < n_jobs; ++i) {
        const unsigned long long* c = h_job_ctr + (size_t)i * kCounterWords;
        if (c[C_SPILLED] > 0) {
            redo->push_back(i);
            continue;
        }
        if (c[C_SUM] != (unsigned long long)jobs[i].n)
            return fail(RASTER_E_DEVICE, "job %d: counts sum to %llu, not %lld", i, c[C_SUM], (long long)jobs[i].n);
        raster_result* r = new raster_result();
        r->shared = owner;
        r->scale = h_jobs[i].scale;
        const uint64_t off = c[C_TILES] ? o_start[i] : 0;
        r->label = lab + off;
        r->kx = kx + off;
        r->ky = ky + off;
        r->count = cnt + off;
        raster_stats& S = r->stats;
        std::memset(&S, 0, sizeof S);
        S.n_points = jobs[i].n;
        S.distinct_tiles = (int64_t)c[C_DISTINCT];
        S.significant_tiles = (int64_t)c[C_SIGNIFICANT];
        S.components = (int64_t)c[C_COMPONENTS];
        S.clusters = (int64_t)c[C_CLUSTERS];
        S.tiles = (int64_t)c[C_TILES];
        S.table_capacity = (int64_t)caps[i];
        S.us_contract = last_us;  // the whole batch's device time
        r->tiles = S.tiles;
        r->clusters = S.clusters;
        outs[i] = r;
    }
    return RASTER_OK;
}

static std::mutex g_engines_mu;
static std::map<int, BatchEngine*> g_engines;

BatchEngine& default_engine() {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> g(g_engines_mu);
    auto it = g_engines.find(dev);
    if (it != g_engines.end()) return *it->second;
    BatchEngine* e = new BatchEngine();  // lives until process exit
    g_engines[dev] = e;
    return *e;
}

raster_status validate_job(const raster_job& j, int32_t i) {
    raster_status st = check_points(j.d_points, j.n, j.dt);
    double sc = j.scale;
    if (st == RASTER_OK && !(sc > 0.0) && !scale_for_precision(j.precision, &sc))
        st = fail(RASTER_E_INVAL, "job %d: precision %d outside [0, 15]", i, j.precision);
    if (st == RASTER_OK) st = check_params(sc, j.tau, j.mu);
    if (st == RASTER_OK && (uint64_t)j.n > 0xFFFFFFFFull) st = fail(RASTER_E_RANGE, "job %d: too many points", i);
    return st;
}

// One batch of jobs that share their options; a job that spilled is redone
// alone through the plain path with the same options.
static raster_status run_group(BatchEngine& eng, const raster_job* jobs, int32_t n_jobs, hipStream_t stream,
                               raster_result** outs, const raster_options& o) {
    std::vector<int32_t> redo;
    raster_status st;
    {
        std::lock_guard<std::mutex> g(eng.mu);
        st = eng.run(jobs, n_jobs, stream, outs, &redo, (uint32_t)o.metric, o.delta, o.square_step != 0);
    }
    for (size_t k = 0; st == RASTER_OK && k < redo.size(); ++k) {
        const raster_job& j = jobs[redo[k]];
        double sc = j.scale;
        if (!(sc > 0.0)) scale_for_precision(j.precision, &sc);
        st = raster_cluster_opts(j.d_points, j.n, j.dt, sc, j.tau, j.mu, &o, stream, &outs[redo[k]]);
        if (st == RASTER_OK) outs[redo[k]]->stats.redone = 1;
    }
    return st;
}

raster_status run_batch(BatchEngine& eng, const raster_job* jobs, int32_t n_jobs, hipStream_t stream,
                        raster_result** outs, const raster_options* opts) {
    for (int32_t i = 0; i < n_jobs; ++i) outs[i] = nullptr;
    for (int32_t i = 0; i < n_jobs; ++i) {
        raster_status st = validate_job(jobs[i], i);
        if (st == RASTER_OK && opts) st = check_options(&opts[i]);
        if (st == RASTER_OK && opts && opts[i].dims == 3)
            st = fail(RASTER_E_INVAL, "job %d: batches take two-dimensional points only", i);
        if (st != RASTER_OK) return st;
    }
    if (n_jobs == 0) return RASTER_OK;
    // jobs grouped by options, each group one batch, in first-seen order
    auto same = [](const raster_options& a, const raster_options& b) {
        return a.metric == b.metric && a.delta == b.delta && (a.square_step != 0) == (b.square_step != 0);
    };
    std::vector<raster_options> keys;
    std::vector<std::vector<int32_t>> members;
    for (int32_t i = 0; i < n_jobs; ++i) {
        const raster_options k = opts ? raster_options{opts[i].metric, opts[i].delta, opts[i].square_step ? 1u : 0u, 2u}
                                      : raster_options{RASTER_CHEBYSHEV, 1u, 0u, 2u};
        size_t g = 0;
        while (g < keys.size() && !same(keys[g], k)) ++g;
        if (g == keys.size()) {
            keys.push_back(k);
            members.emplace_back();
        }
        members[g].push_back(i);
    }
    raster_status st = RASTER_OK;
    if (keys.size() == 1) {
        st = run_group(eng, jobs, n_jobs, stream, outs, keys[0]);
    } else {
        for (size_t g = 0; st == RASTER_OK && g < keys.size(); ++g) {
            std::vector<raster_job> sub;
            for (int32_t i : members[g]) sub.push_back(jobs[i]);
            std::vector<raster_result*> res(sub.size(), nullptr);
            st = run_group(eng, sub.data(), (int32_t)sub.size(), stream, res.data(), keys[g]);
            for (size_t k = 0; k < sub.size(); ++k) outs[members[g][k]] = res[k];
        }
    }
    if (st != RASTER_OK) {
        for (int32_t k = 0; k < n_jobs; ++k) {
            raster_result_free(outs[k]);
            outs[k] = nullptr;
        }
    }
    return st;
}

}  // namespace rst

extern "C" raster_status raster_cluster_batch(const raster_job* jobs, int32_t n_jobs, hipStream_t stream,
                                              raster_result** outs) {
    if (n_jobs < 0 || (n_jobs > 0 && (!jobs || !outs))) return fail(RASTER_E_INVAL, "bad batch arguments");
    return run_batch(default_engine(), jobs, n_jobs, stream, outs, nullptr);
}

extern "C" raster_status raster_cluster_batch_opts(const raster_job* jobs, const raster_options* opts, int32_t n_jobs,
                                                   hipStream_t stream, raster_result** outs) {
    if (n_jobs < 0 || (n_jobs > 0 && (!jobs || !outs))) return fail(RASTER_E_INVAL, "bad batch arguments");
    return run_batch(default_engine(), jobs, n_jobs, stream, outs, opts);
}

// ---------------------------------------------------------------- server ---
//
// Continuous batching: max_slots worker threads, each owning a batch engine
// (its own HIP stream and resident device buffers).  A free worker takes the
// queued jobs, in arrival order, that fit the memory budget left by the
// batches already running, runs them as one batch, and hands out the results.
// Jobs arriving while batches are on the GPU are picked up by the next free
// worker, so their work overlaps the running batches.
//
// Ordering: a job's points may still be in production on the submitter's
// stream.  Submission records an event there; the job's sketch and its run
// wait for that event on the device.
//
// Admission: at submission a distinct-tile sketch of the job's points is
// enqueued on the server's sketch stream (one read of the points).  When the
// job reaches the head of the queue its device footprint is computed from
// that estimate: the table the run will size from it (with one growth step
// in reserve), the binning and spill scratch its point count needs, the
// compact arrays and its rows.  A worker admits jobs while the footprints of
// the running batches, plus the buffers other idle engines keep, plus the new
// jobs fit the budget; a worker that cannot admit the head job releases its
// own engine's buffers first.  The library's in-use device bytes therefore
// stay within the budget while the server runs.

struct SketchBuf {
    uint32_t* dev = nullptr;   // kHllReps << kHllLog2 registers
    uint32_t* host = nullptr;  // pinned copy
};

struct ServerJob {
    uint64_t ticket = 0;
    raster_job job{};
    raster_options opts{RASTER_CHEBYSHEV, 1u, 0u, 2u};  // the job's neighbourhood
    size_t bytes = 0;        // device footprint, once charged
    bool charged = false;
    hipEvent_t ready = nullptr;     // recorded on the submitter's stream
    hipEvent_t sketched = nullptr;  // recorded after the sketch's copy
    SketchBuf sk;
    std::chrono::steady_clock::time_point submitted;
    bool done = false;
    raster_status status = RASTER_OK;
    raster_result* result = nullptr;
    double latency = 0.0;
    std::string error;
};

struct raster_server {
    size_t budget = 0;
    int slots = 1;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<ServerJob*> queue;
    std::unordered_map<uint64_t, ServerJob*> jobs;
    uint64_t next_ticket = 1;
    size_t in_flight = 0;         // footprints of running batches
    std::vector<size_t> resident; // buffers each idle engine keeps
    size_t peak_charged = 0;      // largest in_flight + resident seen
    bool stop = false;
    std::vector<std::thread> workers;
    std::vector<BatchEngine*> engines;
    hipStream_t sk_stream = nullptr;  // sketches of submitted jobs
    std::vector<hipEvent_t> free_events;
    std::vector<SketchBuf> free_sketches;
    Buffers sk_bufs;
};

static size_t table_bytes(double distinct, double lf) {
    return (size_t)next_pow2(std::max<uint64_t>(4096, (uint64_t)(distinct / lf) + 1)) * sizeof(Slot);
}

// Device footprint of one job of n points with about d distinct tiles, as
// the larger of what a plain run takes (first table from the n/8 guess, the
// sketch-sized table and a growth step, binning and spill scratch, compact
// arrays, neighbour lists and rows) and what the job adds to a batch engine
// (arena share, coarse and partition buckets, per-slot compact arrays, rows;
// the engine keeps a quarter of headroom on each).
static size_t job_footprint(int64_t n_, double est) {
    const raster_tuning tu = current_tuning();
    const double lf = tu.load_factor;
    const double n = (double)std::max<int64_t>(n_, 1);
    const double d = std::min(1.25 * est + 1024.0, n);
    const size_t t0 = table_bytes(std::max(n / 8.0, 1024.0), lf);
    const size_t t1 = table_bytes(d, lf);
    // binned counting (tables of at least 2^19 slots) adds two levels of key
    // buckets, at least 8 MiB for the first; the direct path a 64 KiB sketch
    const bool binned = t0 / sizeof(Slot) >= (1u << 19) || tu.mode == 2;
    const double bins = binned ? 19.5 * n + (double)(10u << 20) : (double)(64u << 10);
    const double solo = (double)t0 + 3.0 * (double)t1 + bins + 12.0 * n + 56.0 * d + (double)(1u << 20);
    const double cap = (double)t1 / sizeof(Slot);
    const double batch = 1.25 * ((double)t1 + 18.0 * n + 100.0 * std::min(cap, n)) + (double)(1u << 20);
    return (size_t)std::max(solo, batch);
}

static constexpr size_t kMaxBatchJobs = 128;
static constexpr uint64_t kMaxBatchPoints = 256ull * 1000 * 1000;
// Jobs of at least this many points run alone: their passes already fill the
// GPU, and fusing them would hold small jobs queued behind them.
static constexpr uint64_t kSoloPoints = 2ull * 1000 * 1000;

// Turns the job's sketch into its footprint (waits for the sketch if it is
// still running) and returns the sketch buffers.  Called with s->mu held.
static void charge(raster_server* s, ServerJob* j) {
    if (j->charged) return;
    double est = (double)j->job.n;
    if (j->sketched && hipEventSynchronize(j->sketched) == hipSuccess) {
        std::vector<uint32_t> M(1u << kHllLog2, 0);
        for (uint32_t r = 0; r < kHllReps; ++r)
            for (uint32_t k = 0; k < (1u << kHllLog2); ++k)
                M[k] = std::max(M[k], j->sk.host[((size_t)r << kHllLog2) + k]);
        est = hll_estimate(M.data());
    }
    j->bytes = job_footprint(j->job.n, est);
    j->charged = true;
    if (j->sk.dev) s->free_sketches.push_back(j->sk);
    j->sk = SketchBuf{};
    if (j->sketched) s->free_events.push_back(j->sketched);
    j->sketched = nullptr;
}

static size_t others_resident(const raster_server* s, int slot) {
    size_t r = 0;
    for (int k = 0; k < (int)s->resident.size(); ++k)
        if (k != slot) r += s->resident[k];
    return r;
}

static void server_worker(raster_server* s, int slot) {
    (void)hipSetDevice(s->device);
    BatchEngine& eng = *s->engines[slot];
    while (true) {
        std::vector<ServerJob*> batch;
        size_t bytes = 0;
        bool release_own = false;
        {
            std::unique_lock<std::mutex> g(s->mu);
            s->cv_work.wait(g, [&] { return !s->queue.empty() || s->stop; });
            if (s->queue.empty()) return;  // stopping and drained
            ServerJob* head = s->queue.front();
            charge(s, head);
            if (head->bytes > s->budget) {
                s->queue.pop_front();
                head->status = RASTER_E_BUDGET;
                head->error = "the job's device footprint (" + std::to_string(head->bytes) +
                              " bytes) exceeds the server's budget";
                head->latency = std::chrono::duration<double>(std::chrono::steady_clock::now() - head->submitted).count();
                head->done = true;
                if (head->ready) s->free_events.push_back(head->ready);
                head->ready = nullptr;
                g.unlock();
                s->cv_done.notify_all();
                continue;
            }
            // this engine's own buffers are reused by its next batch
            const size_t avail_all = s->budget - std::min(s->budget, s->in_flight + others_resident(s, slot));
            if (head->bytes > avail_all) {
                if (s->resident[slot] > 0) {
                    release_own = true;  // make room: drop this idle engine's buffers
                    s->resident[slot] = 0;
                } else {
                    s->cv_work.wait(g);  // a batch ending or an engine releasing its buffers wakes us
                    continue;
                }
            } else {
                // a large job runs alone; small jobs waiting together share
                // one fused batch
                uint64_t pts = 0;
                while (!s->queue.empty() && batch.size() < kMaxBatchJobs) {
                    ServerJob* j = s->queue.front();
                    charge(s, j);
                    if (j->bytes > avail_all - bytes) break;
                    const bool large = (uint64_t)j->job.n >= kSoloPoints;
                    if (!batch.empty() && (large || pts + (uint64_t)j->job.n > kMaxBatchPoints)) break;
                    batch.push_back(j);
                    bytes += j->bytes;
                    pts += (uint64_t)j->job.n;
                    s->queue.pop_front();
                    if (large) break;
                }
                // the engine keeps its buffers while it runs: a fused batch
                // reuses them (it is charged at least what they hold); a job
                // alone takes the plain path, which allocates beside them
                bytes = batch.size() == 1 ? bytes + s->resident[slot] : std::max(bytes, s->resident[slot]);
                s->resident[slot] = 0;
                s->in_flight += bytes;
                s->peak_charged = std::max(s->peak_charged, s->in_flight + others_resident(s, slot));
            }
        }
        if (release_own) {
            eng.release();
            s->cv_work.notify_all();
            continue;
        }
        s->cv_work.notify_all();  // another worker may take what is left
        std::vector<raster_job> jv(batch.size());
        std::vector<raster_options> ov(batch.size());
        std::vector<raster_result*> outs(batch.size(), nullptr);
        raster_status st = eng.init();
        for (size_t i = 0; i < batch.size(); ++i) {
            jv[i] = batch[i]->job;
            ov[i] = batch[i]->opts;
            // the points are ready once the submitter's stream has passed
            // the event recorded at submission
            if (st == RASTER_OK && batch[i]->ready && hipStreamWaitEvent(eng.bs, batch[i]->ready, 0) != hipSuccess)
                st = fail(RASTER_E_DEVICE, "stream order of a served job");
        }
        if (st != RASTER_OK) {
            // nothing ran
        } else if (batch.size() == 1) {
            // nothing to fuse with: the plain path has the least fixed cost
            const raster_job& j = jv[0];
            double sc = j.scale;
            if (!(sc > 0.0)) scale_for_precision(j.precision, &sc);
            st = raster_cluster_opts(j.d_points, j.n, j.dt, sc, j.tau, j.mu, &ov[0], eng.bs, &outs[0]);
        } else {
            st = run_batch(eng, jv.data(), (int32_t)jv.size(), eng.bs, outs.data(), ov.data());
        }
        std::string err = st == RASTER_OK ? std::string() : g_last_error;
        if (st != RASTER_OK && batch.size() > 1) {
            // isolate the failing job(s): redo each job alone
            st = RASTER_OK;
            for (size_t i = 0; i < batch.size(); ++i) {
                raster_status si = run_batch(eng, &jv[i], 1, eng.bs, &outs[i], &ov[i]);
                if (si != RASTER_OK) batch[i]->error = g_last_error;
                batch[i]->status = si;
            }
        } else {
            for (size_t i = 0; i < batch.size(); ++i) {
                batch[i]->status = st;
                batch[i]->error = err;
            }
        }
        // cached pool blocks beyond the budget go back to the device
        DevicePool& pool = DevicePool::get(s->device);
        if (pool.used_bytes() + pool.cached_bytes() > s->budget) pool.trim();
        const size_t kept = eng.bufs.bytes() + eng.sk_bufs.bytes();
        const auto t1 = std::chrono::steady_clock::now();
        {
            std::lock_guard<std::mutex> g(s->mu);
            for (size_t i = 0; i < batch.size(); ++i) {
                batch[i]->result = outs[i];
                batch[i]->latency = std::chrono::duration<double>(t1 - batch[i]->submitted).count();
                batch[i]->done = true;
                if (batch[i]->ready) s->free_events.push_back(batch[i]->ready);
                batch[i]->ready = nullptr;
            }
            s->in_flight -= bytes;
            s->resident[slot] = kept;
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
}

extern "C" raster_status raster_server_create(size_t budget_bytes, int32_t max_slots, raster_server** srv) {
    if (!srv) return fail(RASTER_E_INVAL, "srv is NULL");
    *srv = nullptr;
    if (budget_bytes == 0 || max_slots < 1 || max_slots > 16)
        return fail(RASTER_E_INVAL, "budget must be positive and slots in [1, 16]");
    raster_server* s = new raster_server();
    s->budget = budget_bytes;
    s->slots = max_slots;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->sk_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "server setup");
    }
    s->sk_bufs.pool = &DevicePool::get(s->device);
    s->resident.assign(max_slots, 0);
    for (int i = 0; i < max_slots; ++i) {
        s->engines.push_back(new BatchEngine());
        raster_status st = s->engines.back()->init();
        if (st != RASTER_OK) {
            for (BatchEngine* b : s->engines) delete b;
            (void)hipStreamDestroy(s->sk_stream);
            delete s;
            return st;
        }
    }
    for (int i = 0; i < max_slots; ++i) s->workers.emplace_back(server_worker, s, i);
    *srv = s;
    return RASTER_OK;
}

extern "C" raster_status raster_server_submit(raster_server* s, const raster_job* job, uint64_t* ticket) {
    return raster_server_submit_stream(s, job, nullptr, nullptr, ticket);
}

extern "C" raster_status raster_server_submit_opts(raster_server* s, const raster_job* job,
                                                   const raster_options* opts, uint64_t* ticket) {
    return raster_server_submit_stream(s, job, opts, nullptr, ticket);
}

// An event and a sketch buffer from the server's free lists (or new ones).
static raster_status take_submit_resources(raster_server* s, hipEvent_t* ready, hipEvent_t* sketched,
                                           SketchBuf* sk) {
    {
        std::lock_guard<std::mutex> g(s->mu);
        for (hipEvent_t* e : {ready, sketched}) {
            if (!s->free_events.empty()) {
                *e = s->free_events.back();
                s->free_events.pop_back();
            }
        }
        if (!s->free_sketches.empty()) {
            *sk = s->free_sketches.back();
            s->free_sketches.pop_back();
        }
    }
    for (hipEvent_t* e : {ready, sketched})
        if (!*e) HIP_TRY_S(hipEventCreateWithFlags(e, hipEventDisableTiming), "server event");
    if (!sk->dev) {
        const size_t regs = (size_t)kHllReps << kHllLog2;
        std::lock_guard<std::mutex> g(s->mu);
        HIP_TRY_S(s->sk_bufs.take((void**)&sk->dev, regs * sizeof(uint32_t)), "server sketch");
        HIP_TRY_S(hipHostMalloc((void**)&sk->host, regs * sizeof(uint32_t), hipHostMallocDefault), "server sketch");
    }
    return RASTER_OK;
}

extern "C" raster_status raster_server_submit_stream(raster_server* s, const raster_job* job,
                                                     const raster_options* opts, hipStream_t stream,
                                                     uint64_t* ticket) {
    if (!s || !job || !ticket) return fail(RASTER_E_INVAL, "NULL argument");
    raster_status st = validate_job(*job, 0);
    if (st == RASTER_OK) st = check_options(opts);
    if (st == RASTER_OK && opts && opts->dims == 3)
        st = fail(RASTER_E_INVAL, "server jobs take two-dimensional points only");
    if (st != RASTER_OK) return st;
    // the smallest footprint the job can have (a single distinct tile)
    const size_t least = job_footprint(job->n, 1.0);
    if (least > s->budget)
        return fail(RASTER_E_BUDGET, "job needs at least %zu bytes of device memory, more than the budget %zu", least,
                    s->budget);
    ServerJob* j = new ServerJob();
    j->job = *job;
    if (opts) j->opts = raster_options{opts->metric, opts->delta, opts->square_step ? 1u : 0u, 2u};
    st = take_submit_resources(s, &j->ready, &j->sketched, &j->sk);
    if (st != RASTER_OK) {
        delete j;
        return st;
    }
    double sc = job->scale;
    if (!(sc > 0.0)) scale_for_precision(job->precision, &sc);
    hipError_t e = hipEventRecord(j->ready, stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(s->sk_stream, j->ready, 0);
    if (e == hipSuccess) e = launch_zero_u64((uint64_t*)j->sk.dev, ((size_t)kHllReps << kHllLog2) / 2, s->sk_stream);
    if (e == hipSuccess && job->n > 0)
        e = launch_points_hll(job->d_points, job->n, (int)job->dt, sc, j->sk.dev, s->sk_stream, 2);
    if (e == hipSuccess)
        e = hipMemcpyAsync(j->sk.host, j->sk.dev, ((size_t)kHllReps << kHllLog2) * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, s->sk_stream);
    if (e == hipSuccess) e = hipEventRecord(j->sketched, s->sk_stream);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s->sk_stream);
        std::lock_guard<std::mutex> g(s->mu);
        s->free_events.push_back(j->ready);
        s->free_events.push_back(j->sketched);
        s->free_sketches.push_back(j->sk);
        delete j;
        return hip_fail(e, "served job sketch");
    }
    j->submitted = std::chrono::steady_clock::now();
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) {
            (void)hipEventSynchronize(j->sketched);
            s->free_events.push_back(j->ready);
            s->free_events.push_back(j->sketched);
            s->free_sketches.push_back(j->sk);
            delete j;
            return fail(RASTER_E_STATE, "server is stopping");
        }
        j->ticket = s->next_ticket++;
        s->jobs[j->ticket] = j;
        s->queue.push_back(j);
    }
    s->cv_work.notify_one();
    *ticket = j->ticket;
    return RASTER_OK;
}

extern "C" raster_status raster_server_wait(raster_server* s, uint64_t ticket, raster_result** out,
                                           double* latency_s) {
    if (!s || !out) return fail(RASTER_E_INVAL, "NULL argument");
    *out = nullptr;
    ServerJob* j = nullptr;
    {
        std::unique_lock<std::mutex> g(s->mu);
        auto it = s->jobs.find(ticket);
        if (it == s->jobs.end()) return fail(RASTER_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
        j = it->second;
        s->cv_done.wait(g, [&] { return j->done; });
        s->jobs.erase(ticket);
    }
    raster_status st = j->status;
    *out = j->result;
    if (latency_s) *latency_s = j->latency;
    std::string err = j->error;
    delete j;
    if (st != RASTER_OK) return fail(st, "job failed: %s", err.c_str());
    return RASTER_OK;
}

extern "C" raster_status raster_server_memory(raster_server* s, size_t* budget, size_t* peak_charged) {
    if (!s) return fail(RASTER_E_INVAL, "server is NULL");
    std::lock_guard<std::mutex> g(s->mu);
    if (budget) *budget = s->budget;
    if (peak_charged) *peak_charged = s->peak_charged;
    return RASTER_OK;
}

extern "C" void raster_server_destroy(raster_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (std::thread& t : s->workers)
        if (t.joinable()) t.join();
    if (s->sk_stream) (void)hipStreamSynchronize(s->sk_stream);
    for (auto& kv : s->jobs) {
        raster_result_free(kv.second->result);
        if (kv.second->ready) s->free_events.push_back(kv.second->ready);
        if (kv.second->sketched) s->free_events.push_back(kv.second->sketched);
        if (kv.second->sk.dev) s->free_sketches.push_back(kv.second->sk);
        delete kv.second;
    }
    for (BatchEngine* b : s->engines) delete b;
    for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);
    for (SketchBuf& b : s->free_sketches)
        if (b.host) (void)hipHostFree(b.host);
    s->sk_bufs.release_all();
    if (s->sk_stream) (void)hipStreamDestroy(s->sk_stream);
    delete s;
}
