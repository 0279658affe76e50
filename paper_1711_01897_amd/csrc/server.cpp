// Device request server: continuous batching of entry requests.
//
// The paper lets each H-matrix block's CPU thread launch its own small
// kernels and relies on hardware work queues to overlap them (Section 4).
// Here every host thread submits requests to one server instead:
//
//  * admission: a request is taken into the next batch when a batch slot is
//    free and the slot's share of the device arena still has room for the
//    request's inputs, outputs, partial sums and block tables (admission by
//    memory);
//  * fusion: all admitted requests of one kernel variant run in one launch,
//    one 256-lane workgroup per (request, fixed item, lane chunk), whatever
//    request the workgroup belongs to and whichever side is fixed; the block
//    tables are written on the host while the batch is staged;
//  * overlap: several slots rotate, each with its own stream; dispatcher
//    threads stage and enqueue the next batches while earlier ones run or are
//    being consumed, so consecutive batches overlap on the device and
//    requests that arrive meanwhile wait only for the next free slot;
//  * staging: each slot has pinned host staging and a device arena; the
//    inputs are copied to the arena in one copy, and the kernels store
//    results and near-field flags straight into the staging (host-coherent,
//    uncached on the device), so a batch is one copy and its launches;
//  * completion: completion threads wait for each batch's event, check the
//    near-field flags, copy results to the callers' buffers (or lend the
//    caller a pointer into the pinned staging until it releases it), wake
//    the waiters and record submit-to-completion latency.
// Each request's result is computed by the same workgroups with the same
// summation order whichever batch it lands in.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <map>
#include <new>
#include <thread>

#include <immintrin.h>

#include "bem_internal.hpp"

namespace bem {

namespace {

constexpr int kMaxSlots = 16;
constexpr int kMaxThreads = 4;
constexpr int kTimedEvery = 8;
constexpr int kKeys = 64;   // launch groups: (kernel op 0..7, space, prec, rule)

int env_int(const char *name, int dflt, int lo, int hi)
{
    const char *e = std::getenv(name);
    if (!e) return dflt;
    return std::max(lo, std::min(hi, std::atoi(e)));
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Streaming (non-temporal) copy of `bytes` (a multiple of 16) to 16-byte
// aligned staging: the records go to memory without first reading their
// cache lines into this core's cache.  Ordered before later stores by an
// sfence (issued once per submission group).
void stream_copy(void *dst, const void *src, size_t bytes)
{
    __m128i *d = static_cast<__m128i *>(dst);
    const __m128i *p = static_cast<const __m128i *>(src);
    for (size_t i = 0; i < bytes / 16; ++i) _mm_stream_si128(d + i, _mm_loadu_si128(p + i));
}


struct Launch {
    Variant v{};
    int key = 0;                 // member list of the group
    size_t off_tab = 0;          // EntryBlock table
    int64_t count = 0;           // workgroups
    int64_t entries = 0, evals = 0, loads = 0;
};

struct KStat {
    int64_t launches = 0, workgroups = 0, entries = 0, evals = 0, loads = 0, blocks = 0;
    double seconds = 0.0, seconds_events = 0.0;
};

// A submitter's requests inside a batch filled through the fast path: they
// complete with one callback.
struct FastGroup {
    int first = 0, n = 0;              // positions in Batch::reqs
    void (*cb)(Request **, size_t, void *) = nullptr;
    void *ctx = nullptr;
    bem_mesh *mesh = nullptr;
    double t_submit = 0.0;
};

struct Batch {
    int slot = 0;
    std::vector<Request *> reqs;
    // fast path (submitters write their records into the slot themselves)
    bool fast = false;
    std::vector<FastGroup> groups;
    char *hb = nullptr;                // the slot's host staging
    hipError_t error = hipSuccess;     // set before the callbacks run
    double t_done = 0.0;
    bool persist = false;              // published to a persistent launch (completion word, no event)
    uint64_t pseq = 0;                 // its sequence number there
    std::vector<Launch> launches;
    std::vector<hipEvent_t> ev;   // start/stop per launch (timed batches)
    hipEvent_t ev_done = nullptr;
    hipError_t enqueue_error = hipSuccess;
    double t_launch = 0.0;
    double t_hip = 0.0;           // host seconds inside the enqueue calls
    double t_take = 0.0, t_enq = 0.0, q_sum = 0.0;   // latency legs (q_sum: summed queue waits)
    size_t off_clock = 0;         // timed batches: per-launch {start, end} device clock records
    int64_t entries = 0, evals = 0;
    std::atomic<int> refs{1};     // completion thread + borrowed results
    bool timed = false;           // per-launch events recorded

    // Back to a fresh batch, keeping the vectors' capacity.
    void reset()
    {
        std::vector<Request *> r;
        std::vector<FastGroup> g;
        std::vector<Launch> l;
        std::vector<hipEvent_t> e;
        r.swap(reqs);
        g.swap(groups);
        l.swap(launches);
        e.swap(ev);
        this->~Batch();
        new (this) Batch();
        r.clear();
        g.clear();
        l.clear();
        e.clear();
        reqs.swap(r);
        groups.swap(g);
        launches.swap(l);
        ev.swap(e);
    }
};

// Per dispatcher thread: group member lists, reused across batches.
struct Scratch {
    std::vector<int> members[kKeys];
};

class Server;
void persist_register_exit(Server *s);

class Server {
public:
    size_t arena_bytes = size_t(1) << 30;
    int max_batch = 16384;
    int nslots = 16;    // BEM_SERVER_SLOTS; by default one per MiB of arena, 2 to kMaxSlots
    int nstreams = 4;   // BEM_SERVER_STREAMS (slot s uses stream s % nstreams), default one per hardware queue
    int ndisp = 1;      // BEM_SERVER_DISPATCHERS
    int ncomp = 1;      // BEM_SERVER_COMPLETERS
    bool spin = false;       // BEM_SERVER_SPIN: completion threads poll batch events instead of blocking
    // BEM_SERVER_MIN_BATCH / BEM_SERVER_MAX_WAIT_US: a batch is taken once
    // this many requests are pending or the oldest has waited this long
    // (defaults 1 and 0: take whatever is pending)
    int min_batch = 1;
    double max_wait_s = 0.0;
    bool log_launches = false;   // BEM_DEBUG_LAUNCHES: print each timed launch (grid, duration) to stderr
    // BEM_SERVER_DIRECT (default 1): batches with no inputs of their own and
    // no singular pairs (the rows and columns of resident lane sets) skip the
    // staging copy; the entry kernels read descriptors and block records
    // from the host-coherent staging itself (a few host-link reads per
    // workgroup instead of a copy kernel and its launch gap per batch:
    // about 4% more throughput on the 1M-triangle cylinder)
    bool direct = true;
    bool time_phases = false;    // BEM_DEBUG_TIMING: per-phase host seconds of dispatch and completion
    // dispatch: group, layout, blocks, inputs+descriptors, enqueue; completion: wait, statistics, statuses,
    // callbacks, release
    double ph_disp[5] = {}, ph_comp[5] = {};
    int64_t ph_nd = 0, ph_nc = 0;

    std::mutex mu;
    std::condition_variable cv;    // dispatchers: pending requests, free slots
    std::condition_variable cvc;   // completers: batches in flight
    // pending requests with their slot bytes, so taking a batch reads no
    // request memory while the lock is held
    struct Pending {
        Request *r;
        size_t bytes;
    };
    std::deque<Pending> pending;
    uint64_t generation = 0;   // bumped by reconfigure (guarded by mu)

    // Fast path.  Requests whose lane side is resident on the device, with a
    // completion callback, borrowed results and no singular pairs (the rows
    // and columns ACA workers ask for) skip the pending queue: a submitting
    // thread reserves room in the open batch (request positions, block
    // records, output bytes; under mu, O(1) per request), then writes its
    // descriptors, block records and status words straight into the slot's
    // host-coherent staging without the lock.  The dispatcher closes the
    // open batch, waits until every reservation is written and launches it;
    // the kernels read the records from the staging.  No other thread
    // touches these requests until their submitter's callback.
    struct Open {
        Batch *b = nullptr;
        int key = -1;
        int nreq = 0, writers = 0;
        int64_t nblk = 0;
        size_t out = 0;                 // output bytes reserved (from off_out0)
        int64_t entries = 0, evals = 0, loads = 0;
        double t_first = 0.0;
        bool closed = false;            // taken by the dispatcher; the last writer launches it
        double t_close = 0.0;
    };
    Open *open = nullptr;              // guarded by mu
    bool fast_enabled = true;          // BEM_SERVER_FAST (default 1)
    int fast_min = 256;                // BEM_SERVER_FAST_MIN: close at this many requests ...
    double fast_wait_s = 30e-6;        // BEM_SERVER_FAST_WAIT_US: ... or when the first has waited this long
    // slot layout of a fast batch: descriptors | status words | block records | clock records | outputs
    int fmaxreq = 0;
    int64_t fmaxblk = 0;
    size_t f_status = 0, f_blk = 0, f_clock = 0, f_out0 = 0;
    // Persistent launches (BEM_SERVER_PERSIST; switched off, see start()).
    // Closed fast batches are published to one resident launch of their kernel variant
    // (entries.hip, kp_*), which claims their blocks as they appear and
    // stores a completion word per batch into host memory: no launch and no
    // event per batch.  One launch runs at a time; it ends after
    // BEM_SERVER_PERSIST_IDLE_US without a batch or when a batch of another
    // variant finds it idle (that batch and any until it has ended are
    // launched on their own).  BEM_SERVER_PERSIST_WGS: workgroups per compute
    // unit (default one less than fit, so launches of other kernels keep
    // room).
    struct PRun {
        uint64_t id = 0;
        int key = -1;
        Variant v{};
        int groups = 0;
        uint64_t seq0 = 0;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        int64_t entries = 0, evals = 0, loads = 0, blocks = 0;
    };
    bool persist_enabled = true;
    int persist_wgs = 0;
    double persist_idle_s = 1e-3;
    int n_cu = 0;
    std::mutex pmu;                    // everything below; taken before stat_mu and ev_mu
    PersistHost *ph = nullptr, *ph_dev = nullptr;
    PersistCtl *pctl = nullptr;
    hipStream_t pstream = nullptr;
    bool p_running = false, p_stopping = false;
    PRun p_cur;
    std::vector<PRun> p_ended;         // ended, not yet in the statistics
    uint64_t p_next_seq = 0, p_next_id = 1;
    int p_occ[kKeys] = {};             // resident workgroups per compute unit (-1: none)

    std::deque<Batch *> inflight;
    std::mutex pool_mu;
    std::vector<Batch *> batch_pool;   // reset batch records for reuse
    bool slot_busy[kMaxSlots] = {};
    bool started = false, stop = false;
    int device = 0;
    hipStream_t streams[kMaxSlots] = {};
    char *d_arena = nullptr, *h_stage = nullptr;
    char *h_stage_dev = nullptr;   // device address of h_stage
    size_t slot_bytes = 0;
    std::vector<std::thread> threads;
    std::mutex ev_mu;
    std::vector<hipEvent_t> event_pool;
    std::atomic<int64_t> batch_counter{0};
    double clock_hz = 1e8;   // device constant-rate clock

    // statistics
    std::mutex stat_mu;
    int64_t n_requests = 0, n_entries = 0, n_batches = 0, n_evals = 0, n_launches = 0, n_timed = 0;
    double busy = 0.0, last_done = 0.0, kernel_s = 0.0;
    double dispatch_s = 0.0, complete_s = 0.0, wait_s = 0.0, dispatch_hip_s = 0.0;
    double leg_queue = 0.0, leg_stage = 0.0, leg_device = 0.0, leg_complete = 0.0;   // request-weighted sums
    std::vector<float> latencies;
    std::map<Variant, KStat> kstats;

    int start()
    {
        if (started) return BEM_OK;
        // Persistent launches are switched off: they served the tests and
        // benchmarks of one build correctly (at 0.55x the throughput of
        // launched batches), and the two variants after it stalled a served
        // ACA run on the level-4 icosphere (a batch never completed) with the
        // cause not found.  Asking for them is an error until that is resolved.
        if (env_int("BEM_SERVER_PERSIST", 0, 0, 1) != 0)
            return fail(BEM_E_ARG, "BEM_SERVER_PERSIST=1: persistent launches are switched off in this build");
        // a slot stays busy until the workers hand back the results they
        // borrowed from it, so more slots keep more batches moving; small
        // arenas keep slots of at least 1 MiB
        const int def_slots = (int)std::min<size_t>(kMaxSlots, std::max<size_t>(2, arena_bytes >> 20));
        nslots = env_int("BEM_SERVER_SLOTS", def_slots, 2, kMaxSlots);
        // one stream per hardware queue: streams that share a queue run
        // their packets in one order, so more streams than queues only
        // serialise batches behind each other
        const int hwq = env_int("GPU_MAX_HW_QUEUES", 4, 1, kMaxSlots);
        nstreams = env_int("BEM_SERVER_STREAMS", std::min(nslots, hwq), 1, nslots);
        ndisp = env_int("BEM_SERVER_DISPATCHERS", ndisp, 1, kMaxThreads);
        ncomp = env_int("BEM_SERVER_COMPLETERS", ncomp, 1, kMaxThreads);
        spin = env_int("BEM_SERVER_SPIN", spin ? 1 : 0, 0, 1) != 0;
        min_batch = env_int("BEM_SERVER_MIN_BATCH", 1, 1, 1 << 20);
        max_wait_s = 1e-6 * env_int("BEM_SERVER_MAX_WAIT_US", 0, 0, 1000000);
        log_launches = env_int("BEM_DEBUG_LAUNCHES", 0, 0, 1) != 0;
        direct = env_int("BEM_SERVER_DIRECT", 1, 0, 1) != 0;
        time_phases = std::getenv("BEM_DEBUG_TIMING") != nullptr;
        hipError_t e = hipGetDevice(&device);
        int khz = 0;
        if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device);
        clock_hz = khz > 0 ? 1e3 * khz : 1e8;
        for (int i = 0; i < nstreams && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&streams[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipMalloc(&d_arena, arena_bytes);
        // inputs are staged here and copied to the device arena; the kernels
        // store results and flags straight into it, uncached (coherent), so
        // they are in host memory once the batch event completes
        if (e == hipSuccess) e = hipHostMalloc(&h_stage, arena_bytes, hipHostMallocCoherent);
        if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&h_stage_dev, h_stage, 0);
        if (e != hipSuccess) {
            if (d_arena) (void)hipFree(d_arena);
            d_arena = nullptr;
            return fail(e == hipErrorOutOfMemory ? BEM_E_OOM : BEM_E_DEVICE,
                        std::string("server start: ") + hipGetErrorString(e));
        }
        slot_bytes = (arena_bytes / nslots) & ~(size_t)255;
        fast_enabled = env_int("BEM_SERVER_FAST", 1, 0, 1) != 0;
        fast_min = env_int("BEM_SERVER_FAST_MIN", 256, 1, 1 << 20);
        fast_wait_s = 1e-6 * env_int("BEM_SERVER_FAST_WAIT_US", 30, 0, 1000000);
        fmaxreq = (int)std::min<size_t>({(size_t)8192, (size_t)max_batch, std::max<size_t>(16, slot_bytes / 4096)});
        fmaxblk = 4 * (int64_t)fmaxreq;
        f_status = align256(sizeof(ReqDev) * (size_t)fmaxreq);
        f_blk = align256(f_status + sizeof(int32_t) * (size_t)fmaxreq);
        f_clock = align256(f_blk + sizeof(EntryBlock) * (size_t)fmaxblk);
        f_out0 = align256(f_clock + 16 * (size_t)fmaxblk);
        if (f_out0 + (size_t(1) << 16) > slot_bytes) fast_enabled = false;
        persist_enabled = false;   // switched off (above)
        persist_wgs = env_int("BEM_SERVER_PERSIST_WGS", 0, 0, 64);
        persist_idle_s = 1e-6 * env_int("BEM_SERVER_PERSIST_IDLE_US", 1000, 10, 10000000);
        if (persist_enabled && persist_start() != hipSuccess) persist_enabled = false;
        started = true;
        for (int i = 0; i < ndisp; ++i) threads.emplace_back([this] { dispatch_loop(); });
        for (int i = 0; i < ncomp; ++i) threads.emplace_back([this] { complete_loop(); });
        return BEM_OK;
    }

    hipError_t persist_start()
    {
        hipError_t e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
        if (e == hipSuccess && !ph) e = hipHostMalloc((void **)&ph, sizeof(PersistHost), hipHostMallocCoherent);
        if (e == hipSuccess) {
            std::memset(ph, 0, sizeof(PersistHost));
            e = hipHostGetDevicePointer((void **)&ph_dev, ph, 0);
        }
        if (e == hipSuccess && !pctl) e = hipMalloc((void **)&pctl, sizeof(PersistCtl));
        if (e == hipSuccess && !pstream) e = hipStreamCreateWithFlags(&pstream, hipStreamNonBlocking);
        for (int &o : p_occ) o = 0;
        p_running = p_stopping = false;
        p_next_seq = 0;
        if (e == hipSuccess) persist_register_exit(this);
        return e;
    }

    // The current launch has stored its exit word (it has left or is leaving).
    bool persist_exited_locked() const
    {
        const uint64_t w = *reinterpret_cast<const volatile uint64_t *>(&ph->exit_word);
        return (w >> 40) == p_cur.id;
    }
    uint64_t persist_exit_seq_locked() const
    {
        const uint64_t w = *reinterpret_cast<const volatile uint64_t *>(&ph->exit_word);
        return (w & ((uint64_t(1) << 40) - 1)) - 1;
    }

    void persist_end_locked()
    {
        p_ended.push_back(p_cur);
        p_running = p_stopping = false;
    }

    bool persist_launch_locked(int key, uint64_t seq0)
    {
        const Variant v{key >> 3, (key >> 2) & 1, (key >> 1) & 1, (key & 1) ? 6 : 4};
        if (p_occ[key] == 0) {
            const int occ = persistent_occupancy(v);
            p_occ[key] = occ > 0 ? occ : -1;
        }
        if (p_occ[key] < 0) return false;
        const int wpc = persist_wgs > 0 ? std::min(persist_wgs, p_occ[key]) : std::max(1, p_occ[key] - 1);
        PRun r;
        r.id = p_next_id++;
        r.key = key;
        r.v = v;
        r.v.persist = 1;
        r.groups = 1 + n_cu * wpc;
        r.seq0 = seq0;
        r.e0 = get_event();
        r.e1 = get_event();
        PersistArgs a;
        a.host = ph_dev;
        a.done = &ph_dev->done[0][0];
        a.exit_word = &ph_dev->exit_word;
        a.ctl = pctl;
        a.seq0 = seq0;
        a.id = r.id;
        a.idle_ticks = (long long)(persist_idle_s * clock_hz);
        if (launch_persistent(v, a, r.groups, pstream, r.e0, r.e1) != hipSuccess) {
            std::lock_guard<std::mutex> g(ev_mu);
            event_pool.push_back(r.e0);
            event_pool.push_back(r.e1);
            return false;
        }
        p_cur = r;
        p_running = true;
        p_stopping = false;
        return true;
    }

    // A launch that has ended leaves batches it did not take to a new launch
    // of the same variant (an idle end racing with a publication, or a stop).
    void persist_check_locked()
    {
        if (!p_running || !persist_exited_locked()) return;
        const uint64_t first = persist_exit_seq_locked();
        const int key = p_cur.key;
        persist_end_locked();
        if (first < p_next_seq) persist_launch_locked(key, first);
    }

    // Publishes a closed fast batch to the persistent launch of its variant,
    // starting one if none runs.  False: it is launched on its own.
    bool persist_publish(Open *o)
    {
        if (o->nblk > kPersistMaxBlocks) return false;
        Batch *b = o->b;
        std::lock_guard<std::mutex> g(pmu);
        persist_check_locked();
        if (p_running && p_stopping) return false;   // until it has left
        if (p_running && p_cur.key != o->key) {
            // another variant's launch: ask it to end once it has nothing in flight
            if (!p_stopping) {
                bool idle = true;
                for (uint64_t q = p_next_seq > (uint64_t)kPersistRing ? p_next_seq - kPersistRing : 0; q < p_next_seq; ++q)
                    idle = idle && *reinterpret_cast<volatile uint64_t *>(&ph->done[q % kPersistRing][0]) == q + 1;
                if (idle) {
                    *reinterpret_cast<volatile uint64_t *>(&ph->stop) = p_cur.id;
                    p_stopping = true;
                }
            }
            return false;
        }
        if (!p_running && !persist_launch_locked(o->key, p_next_seq)) return false;
        const uint64_t seq = p_next_seq;
        PersistEntry &e = ph->ring[seq % kPersistRing];
        // the entry's previous batch has completed (normally long ago: at most
        // one batch per slot is in flight)
        if (seq >= (uint64_t)kPersistRing) {
            const volatile uint64_t *pw = &ph->done[seq % kPersistRing][0];
            for (int64_t spin = 0; *pw != seq - kPersistRing + 1; ++spin) {
                _mm_pause();
                if ((spin & 1023) == 1023) {
                    persist_check_locked();
                    if (!p_running || p_cur.key != o->key) return false;
                }
            }
        }
        char *hd = h_stage_dev + (size_t)b->slot * slot_bytes;
        e.reqs = reinterpret_cast<const ReqDev *>(hd);
        e.blocks = reinterpret_cast<const EntryBlock *>(hd + f_blk);
        e.clock = b->timed ? reinterpret_cast<unsigned long long *>(hd + f_clock) : nullptr;
        e.nblk = o->nblk;
        __atomic_store_n(&e.seq1, seq + 1, __ATOMIC_RELEASE);
        p_next_seq = seq + 1;
        p_cur.entries += o->entries;
        p_cur.evals += o->evals;
        p_cur.loads += o->loads;
        p_cur.blocks += o->nblk;
        b->persist = true;
        b->pseq = seq;
        return true;
    }

    // Waits for the completion word of a published batch.
    void persist_wait(Batch *b)
    {
        const volatile uint64_t *w = &ph->done[b->pseq % kPersistRing][0];
        for (int64_t spin = 0; *w != b->pseq + 1; ++spin) {
            _mm_pause();
            if ((spin & 4095) == 4095) {
                std::lock_guard<std::mutex> g(pmu);
                persist_check_locked();
            }
            if (spin > (int64_t(1) << 16)) std::this_thread::yield();
        }
        std::atomic_thread_fence(std::memory_order_acquire);
    }

    // Ends the running launch (waits up to `limit` seconds for it to leave)
    // and moves ended launches into the statistics.
    void persist_quiesce(double limit)
    {
        if (!ph) return;
        std::lock_guard<std::mutex> g(pmu);
        if (p_running) {
            *reinterpret_cast<volatile uint64_t *>(&ph->stop) = p_cur.id;
            p_stopping = true;
            const double t0 = now_seconds();
            while (!persist_exited_locked() && now_seconds() - t0 < limit) std::this_thread::yield();
            persist_check_locked();
        }
        for (PRun &r : p_ended) {
            float ms = 0.f;
            if (hipEventSynchronize(r.e1) == hipSuccess && hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
                std::lock_guard<std::mutex> gs(stat_mu);
                KStat &k = kstats[r.v];
                k.launches += 1;
                k.workgroups += r.groups;
                k.blocks += r.blocks;
                k.entries += r.entries;
                k.evals += r.evals;
                k.loads += r.loads;
                k.seconds += 1e-3 * ms;
                k.seconds_events += 1e-3 * ms;
            }
            std::lock_guard<std::mutex> ge(ev_mu);
            event_pool.push_back(r.e0);
            event_pool.push_back(r.e1);
        }
        p_ended.clear();
    }

    // Events skip the system-scope fence (a device cache writeback and
    // invalidation per event): results are stored into host-coherent
    // (fine-grained) staging, which the device keeps coherent with the host
    // without that flush once the storing kernel has completed, and timing
    // events must not charge such cache work to the timed kernel.
    hipEvent_t get_event()
    {
        std::lock_guard<std::mutex> g(ev_mu);
        if (!event_pool.empty()) {
            hipEvent_t e = event_pool.back();
            event_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
        return e;
    }

    void finish(Request *r, int status)
    {
        r->t_done = now_seconds();
        r->mesh->inflight.fetch_sub(1);
        {
            std::lock_guard<std::mutex> g(r->mu);
            r->status = status;
            r->done = true;
        }
        r->cv.notify_all();
    }

    // Completes the requests of one batch: statuses are final, callback
    // requests are handed over in one call per (callback, context).
    void finish_all(std::vector<Request *> &rs, const std::vector<int> &st)
    {
        const double t = now_seconds();
        std::vector<std::pair<std::pair<void *, void *>, std::vector<Request *>>> groups;
        size_t last = 0;
        for (size_t i = 0; i < rs.size(); ++i) {
            Request *r = rs[i];
            if (!r->on_done) {
                finish(r, st[i]);
                continue;
            }
            r->t_done = t;
            r->status = st[i];
            r->done = true;
            dec_inflight(r->mesh);
            const std::pair<void *, void *> key{(void *)r->on_done, r->cb_ctx};
            // a submitter's requests sit together in the batch: try the last group first
            size_t g = last;
            if (g >= groups.size() || groups[g].first != key) {
                g = 0;
                while (g < groups.size() && groups[g].first != key) ++g;
                if (g == groups.size()) groups.push_back({key, {}});
                last = g;
            }
            groups[g].second.push_back(r);
        }
        dec_inflight(nullptr);
        for (auto &g : groups) {
            auto cb = reinterpret_cast<void (*)(Request **, size_t, void *)>(g.first.first);
            cb(g.second.data(), g.second.size(), g.first.second);
        }
    }

    // Mesh in-flight counts drop once per run of requests on the same mesh
    // (nullptr flushes the run); completion threads keep their own run.
    void dec_inflight(bem_mesh *m)
    {
        thread_local bem_mesh *cur = nullptr;
        thread_local int64_t cnt = 0;
        if (m == cur) {
            ++cnt;
            return;
        }
        if (cur && cnt) cur->inflight.fetch_sub(cnt);
        cur = m;
        cnt = m ? 1 : 0;
    }

    // batch-level slack: alignment of sections and tables
    static constexpr size_t kSlack = size_t(1) << 17;
    bool fits(const Request *r) const { return r->batch_bytes + kSlack <= slot_bytes; }

    int submit_many(Request *const *rs, size_t n)
    {
        // block records and descriptors are built here, on the submitting
        // thread, while its request data is in its own cache
        uint64_t gen = 0;
        {
            std::lock_guard<std::mutex> g(mu);
            if (stop) return fail(BEM_E_BUSY, "server is being reconfigured");
            if (!started) {
                int rc = start();
                if (rc != BEM_OK) return rc;
            }
            gen = generation;
        }
        // slot_bytes is fixed while the server runs (reconfiguration needs an
        // idle server and bumps the generation, checked below)
        if (fast_enabled && n > 0 && fast_eligible(rs, n) && submit_fast(rs, n, gen)) return BEM_OK;
        for (size_t i = 0; i < n; ++i) {
            rs[i]->fast = false;
            prebuild_staging(*rs[i]);
        }
        for (size_t i = 0; i < n; ++i)
            if (!fits(rs[i])) return fail(BEM_E_OOM, "request larger than a server batch slot; raise the arena size");
        thread_local std::vector<Pending> items;
        items.resize(n);
        const double t = now_seconds();
        for (size_t i = 0; i < n; ++i) {
            Request *r = rs[i];
            r->t_submit = t;
            r->done = false;
            r->result = nullptr;
            r->batch = nullptr;
            items[i] = Pending{r, r->batch_bytes};
        }
        // in-flight counts per run of requests on one mesh, before the
        // requests become visible to the dispatcher
        auto count = [&](int sign) {
            bem_mesh *cur = nullptr;
            int64_t cnt = 0;
            for (size_t i = 0; i < n; ++i) {
                if (rs[i]->mesh != cur) {
                    if (cur) cur->inflight.fetch_add(sign * cnt);
                    cur = rs[i]->mesh;
                    cnt = 0;
                }
                ++cnt;
            }
            if (cur) cur->inflight.fetch_add(sign * cnt);
        };
        count(1);
        {
            std::lock_guard<std::mutex> g(mu);
            if (stop || generation != gen || !started) {
                count(-1);
                return fail(BEM_E_BUSY, "server is being reconfigured");
            }
            pending.insert(pending.end(), items.begin(), items.end());
        }
        cv.notify_one();
        return BEM_OK;
    }

    // Requests that can go through the fast path together: one submitter
    // (callback, context), one mesh and one launch group, borrowed results,
    // a device-resident lane side, no singular pairs, no inputs to stage.
    bool fast_eligible(Request *const *rs, size_t n) const
    {
        const Request &a = *rs[0];
        if (!a.on_done || !a.mesh) return false;
        const int key = request_key(a);
        for (size_t i = 0; i < n; ++i) {
            const Request &r = *rs[i];
            if (r.on_done != a.on_done || r.cb_ctx != a.cb_ctx || r.mesh != a.mesh || !r.borrow || !r.ext ||
                !r.near_items.empty() || r.in_bytes != 0 || r.nblocks <= 0 || r.nblocks > fmaxblk ||
                request_key(r) != key)
                return false;
        }
        return true;
    }

    // Reserves room for rs[0..n) in the open batch and writes their records
    // into its staging; false when there is no open batch, it holds another
    // launch group, or it has no room (the caller queues them instead).
    bool submit_fast(Request *const *rs, size_t n, uint64_t gen)
    {
        const int key = request_key(*rs[0]);
        int64_t blk = 0, ent = 0, ev = 0, ld = 0;
        size_t outb = 0;
        for (size_t i = 0; i < n; ++i) {
            const Request &r = *rs[i];
            blk += r.nblocks;
            outb += r.out_bytes;
            ent += r.entries();
            ev += r.evals;
            ld += r.nfix * r.nlane;
        }
        Open *o = nullptr;
        Batch *b = nullptr;
        int i0 = 0;
        int64_t b0 = 0;
        size_t o0 = 0;
        const double t = now_seconds();
        bool wake = false;
        {
            std::lock_guard<std::mutex> g(mu);
            if (stop || generation != gen || !started || !open) return false;
            o = open;
            if (o->nreq > 0 && o->key != key) return false;
            if (o->nreq + (int64_t)n > fmaxreq || o->nblk + blk > fmaxblk || f_out0 + o->out + outb > slot_bytes)
                return false;
            if (o->nreq == 0) {
                o->key = key;
                o->t_first = t;
            }
            i0 = o->nreq;
            b0 = o->nblk;
            o0 = o->out;
            o->nreq += (int)n;
            o->nblk += blk;
            o->out += outb;
            o->entries += ent;
            o->evals += ev;
            o->loads += ld;
            o->writers += 1;
            b = o->b;
            FastGroup fg;
            fg.first = i0;
            fg.n = (int)n;
            fg.cb = rs[0]->on_done;
            fg.ctx = rs[0]->cb_ctx;
            fg.mesh = rs[0]->mesh;
            fg.t_submit = t;
            b->groups.push_back(fg);
            b->reqs.insert(b->reqs.end(), rs, rs + n);
            wake = i0 == 0 || o->nreq >= fast_min;
        }
        // the records, without the lock (the dispatcher launches the batch
        // only after every reservation is written)
        char *hd = h_stage_dev + (size_t)b->slot * slot_bytes;
        ReqDev *desc = reinterpret_cast<ReqDev *>(b->hb);
        int32_t *stw = reinterpret_cast<int32_t *>(b->hb + f_status);
        EntryBlock *blocks = reinterpret_cast<EntryBlock *>(b->hb + f_blk);
        size_t oo = f_out0 + o0;
        int64_t bb = b0;
        static_assert(sizeof(ReqDev) % 16 == 0 && sizeof(EntryBlock) % 16 == 0, "records are 16-byte multiples");
        thread_local std::vector<EntryBlock> tb;
        for (size_t k = 0; k < n; ++k) {
            Request *r = rs[k];
            const int i = i0 + (int)k;
            ReqDev d;
            describe_request(*r, d);
            finish_descriptor(*r, hd, oo, f_status + sizeof(int32_t) * (size_t)i, d);
            stream_copy(desc + i, &d, sizeof(ReqDev));
            _mm_stream_si32(reinterpret_cast<int *>(stw + i), 0);
            tb.resize((size_t)r->nblocks);
            const int64_t nb = write_blocks(*r, i, tb.data());
            stream_copy(blocks + bb, tb.data(), sizeof(EntryBlock) * (size_t)nb);
            bb += nb;
            r->t_submit = t;
            r->done = false;
            r->fast = true;
            r->batch = b;
            r->result = b->hb + oo;
            r->off_out = oo;
            r->off_status = f_status + sizeof(int32_t) * (size_t)i;
            oo += r->out_bytes;
        }
        rs[0]->mesh->inflight.fetch_add((int64_t)n);
        _mm_sfence();   // the streamed records are in memory before the batch can be launched
        bool last = false;
        {
            std::lock_guard<std::mutex> g(mu);
            last = --o->writers == 0 && o->closed;
        }
        // a batch closed while its reservations were being written is
        // launched by the writer that finishes last
        if (last) launch_closed(o);
        if (wake) cv.notify_one();
        return true;
    }

    // Closes the open batch o (mu held): the next submissions go to a new
    // open batch if a slot is free and nothing is queued; if reservations of
    // o are still being written, the last writer launches it.
    void close_open_locked(Open *o, double t)
    {
        open = nullptr;
        o->t_close = t;
        o->closed = true;
        const int fs = free_slot();
        if (fs >= 0 && pending.empty()) {
            open = new Open();
            open->b = new_fast_batch(fs);
            slot_busy[fs] = true;
        }
    }

    // Launches a closed fast batch whose reservations are all written and
    // hands it to the completion thread.
    void launch_closed(Open *fo)
    {
        launch_fast(fo);
        Batch *b = fo->b;
        const double t1 = now_seconds();
        double qs = 0.0;
        for (const FastGroup &g : b->groups) qs += g.n * (fo->t_close - g.t_submit);
        b->t_take = fo->t_close;
        b->t_enq = t1;
        b->q_sum = qs;
        delete fo;
        {
            std::lock_guard<std::mutex> g(stat_mu);
            dispatch_s += t1 - b->t_take;
            dispatch_hip_s += b->t_hip;
        }
        {
            std::lock_guard<std::mutex> g(mu);
            inflight.push_back(b);
        }
        cvc.notify_one();
    }

    // Batch records are reused.  A fast batch reserves room for up to 8,192
    // request pointers; allocating that per batch and freeing it on another
    // thread made the allocator grow and shrink its heaps with mprotect and
    // munmap, system calls that interrupt every core the process runs on.
    Batch *take_batch()
    {
        {
            std::lock_guard<std::mutex> g(pool_mu);
            if (!batch_pool.empty()) {
                Batch *b = batch_pool.back();
                batch_pool.pop_back();
                return b;
            }
        }
        return new Batch();
    }

    void give_batch(Batch *b)
    {
        b->reset();
        std::lock_guard<std::mutex> g(pool_mu);
        batch_pool.push_back(b);
    }

    Batch *new_fast_batch(int slot)
    {
        Batch *b = take_batch();
        b->slot = slot;
        b->fast = true;
        b->hb = h_stage + (size_t)slot * slot_bytes;
        b->reqs.reserve((size_t)fmaxreq);
        return b;
    }

    // Launches a closed open batch (every reservation written).
    void launch_fast(Open *o)
    {
        Batch *b = o->b;
        hipStream_t stream = streams[b->slot % nstreams];
        char *hd = h_stage_dev + (size_t)b->slot * slot_bytes;
        Launch L;
        L.key = o->key;
        L.v = Variant{o->key >> 3, (o->key >> 2) & 1, (o->key >> 1) & 1, (o->key & 1) ? 6 : 4};
        L.off_tab = f_blk;
        L.count = o->nblk;
        L.entries = o->entries;
        L.evals = o->evals;
        L.loads = o->loads;
        b->entries = o->entries;
        b->evals = o->evals;
        b->timed = (batch_counter.fetch_add(1) % kTimedEvery) == 0;
        b->off_clock = f_clock;
        b->launches.push_back(L);
        b->t_launch = now_seconds();
        b->t_hip = b->t_launch;
        if (persist_enabled && persist_publish(o)) {
            b->t_hip = now_seconds() - b->t_hip;
            return;
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        unsigned long long *ck = nullptr;
        if (b->timed) {
            e0 = get_event();
            e1 = get_event();
            b->ev.push_back(e0);
            b->ev.push_back(e1);
            ck = reinterpret_cast<unsigned long long *>(hd + f_clock);
        }
        hipError_t e = launch_entries(L.v, reinterpret_cast<const ReqDev *>(hd),
                                      reinterpret_cast<const EntryBlock *>(hd + f_blk), L.count, stream, ck, e0, e1);
        if (e != hipSuccess) b->enqueue_error = e;
        b->ev_done = get_event();
        e = hipEventRecord(b->ev_done, stream);
        if (e != hipSuccess && b->enqueue_error == hipSuccess) b->enqueue_error = e;
        b->t_hip = now_seconds() - b->t_hip;
    }

    int free_slot() const
    {
        for (int s = 0; s < nslots; ++s)
            if (!slot_busy[s]) return s;
        return -1;
    }

    void dispatch_loop()
    {
        (void)hipSetDevice(device);
        Scratch sc;
        for (;;) {
            std::vector<Request *> take;
            int slot = -1;
            bool more = false;
            Open *fo = nullptr;   // a fast batch to close and launch
            {
                std::unique_lock<std::mutex> lk(mu);
                for (;;) {
                    if (stop) break;
                    if (open && open->nreq > 0) {
                        const double waited = now_seconds() - open->t_first;
                        if (open->nreq >= fast_min || waited >= fast_wait_s) {
                            fo = open;
                            open = nullptr;
                            break;
                        }
                        if (!pending.empty() && free_slot() >= 0) break;
                        cv.wait_for(lk, std::chrono::duration<double>(fast_wait_s - waited));
                        continue;
                    }
                    // queued requests take a free slot before a new open batch does
                    if (!pending.empty() && free_slot() >= 0) break;
                    if (fast_enabled && !open) {
                        // keep one batch open for fast submissions
                        const int fs = free_slot();
                        if (fs >= 0) {
                            open = new Open();
                            open->b = new_fast_batch(fs);
                            slot_busy[fs] = true;
                            continue;
                        }
                    }
                    cv.wait(lk);
                }
                if (fo && !stop) {
                    // the next open batch, if a slot is free and nothing is queued
                    close_open_locked(fo, now_seconds());
                    const bool ready = fo->writers == 0;
                    lk.unlock();
                    // reservations still being written: their last writer launches the batch
                    if (ready) launch_closed(fo);
                    continue;
                }
                while (!stop && min_batch > 1 && (int)pending.size() < min_batch) {
                    const double waited = now_seconds() - pending.front().r->t_submit;
                    if (waited >= max_wait_s) break;
                    cv.wait_for(lk, std::chrono::duration<double>(max_wait_s - waited));
                    if (pending.empty() || free_slot() < 0)
                        cv.wait(lk, [&] { return stop || (!pending.empty() && free_slot() >= 0); });
                }
                if (stop) {
                    std::vector<Request *> left;
                    for (const Pending &p : pending) left.push_back(p.r);
                    pending.clear();
                    lk.unlock();
                    finish_all(left, std::vector<int>(left.size(), BEM_E_CANCELLED));
                    return;
                }
                slot = free_slot();
                size_t bytes = kSlack;
                while (!pending.empty() && (int)take.size() < max_batch) {
                    const Pending &p = pending.front();
                    if (!take.empty() && bytes + p.bytes > slot_bytes) break;
                    take.push_back(p.r);
                    bytes += p.bytes;
                    pending.pop_front();
                }
                slot_busy[slot] = true;
                more = !pending.empty() && free_slot() >= 0;
            }
            if (more) cv.notify_one();   // another dispatcher can take the rest meanwhile
            const double t0 = now_seconds();
            double qs = 0.0;
            for (Request *r : take) qs += t0 - r->t_submit;
            Batch *b = build_and_launch(slot, take, sc);
            const double t1 = now_seconds();
            b->t_take = t0;
            b->t_enq = t1;
            b->q_sum = qs;
            {
                std::lock_guard<std::mutex> g(stat_mu);
                dispatch_s += t1 - t0;
                dispatch_hip_s += b->t_hip;
            }
            {
                std::lock_guard<std::mutex> g(mu);
                inflight.push_back(b);
            }
            cvc.notify_one();
        }
    }

    Batch *build_and_launch(int slot, std::vector<Request *> &take, Scratch &sc)
    {
        Batch *b = take_batch();
        b->slot = slot;
        b->reqs = take;
        char *hb = h_stage + (size_t)slot * slot_bytes;
        char *hd = h_stage_dev + (size_t)slot * slot_bytes;   // the slot's staging, device address
        char *db = d_arena + (size_t)slot * slot_bytes;
        hipStream_t stream = streams[slot % nstreams];
        const int n = (int)take.size();
        double tp[6] = {};
        if (time_phases) tp[0] = now_seconds();

        // launch groups by (op, space, prec, rule)
        for (auto &g : sc.members) g.clear();
        for (int i = 0; i < n; ++i) {
            Request &r = *take[i];
            if (r.nblocks > 0) sc.members[r.key].push_back(i);
            b->entries += r.entries();
            b->evals += r.evals;
        }
        std::vector<Launch> launches;
        for (int key = 0; key < kKeys; ++key) {
            if (sc.members[key].empty()) continue;
            Launch L;
            L.key = key;
            L.v = Variant{key >> 3, (key >> 2) & 1, (key >> 1) & 1, (key & 1) ? 6 : 4};
            for (int i : sc.members[key]) {
                const Request &r = *take[i];
                L.entries += r.entries();
                L.count += r.nblocks;
                L.evals += r.evals;
                L.loads += r.nfix * r.nlane;
            }
            launches.push_back(L);
        }

        if (time_phases) tp[1] = now_seconds();
        // layout: descriptors | block tables | inputs  (copied to the device
        // arena by a kernel) || clock records | status | outputs  (stored by
        // the kernels into the staging)
        // (offsets first, checked against the slot, then the staging writes)
        size_t off = align256(sizeof(ReqDev) * n);
        for (Launch &L : launches) {
            L.off_tab = off;
            off = align256(off + sizeof(EntryBlock) * (size_t)L.count);
        }
        // singular pairs of BEM_NEAR_SINGULAR requests (few requests carry
        // any), one contiguous run and one launch per (kernel, precision)
        struct NearRun {
            size_t off = 0;
            int64_t count = 0;
            std::vector<int> members;
        };
        NearRun near_runs[8];
        auto near_group = [&](const Request &r) { return 2 * kernel_op(r.op) + (r.prec == BEM_FP32 ? 1 : 0); };
        // P1 singular pairs: one region (pairs | gather records | sources |
        // local matrices) and one pair launch + one gather per (kernel, precision)
        struct P1Run {
            std::vector<int> members;
            int64_t items = 0, recs = 0, src = 0;
            size_t off = 0;
            NearP1Layout L{};
        };
        P1Run p1_runs[12];
        for (int i = 0; i < n; ++i)
            if (!take[i]->near_items.empty() && take[i]->space != BEM_P0) {
                P1Run &g = p1_runs[near_p1_group(*take[i])];
                g.members.push_back(i);
                g.items += (int64_t)take[i]->near_items.size();
                g.recs += (int64_t)take[i]->near_recs.size();
                g.src += (int64_t)take[i]->near_src.size();
            } else if (!take[i]->near_items.empty()) {
                NearRun &g = near_runs[near_group(*take[i])];
                g.members.push_back(i);
                g.count += (int64_t)take[i]->near_items.size();
            }
        for (NearRun &g : near_runs)
            if (g.count) {
                g.off = off;
                off = align256(off + sizeof(NearItem) * (size_t)g.count);
            }
        // group 2 g + fp32 -> layout mode and kernel operator
        auto p1_mode = [](int gi) {
            const int g = gi >> 1;
            return g == 2 ? 1 : (g == 5 ? 3 : (g >= 3 ? 2 : 0));
        };
        auto p1_op = [](int gi) {
            const int g = gi >> 1;
            return g == 2 ? (int)BEM_LAPLACE_HYPS : (g == 5 ? (int)BEM_HELMHOLTZ_HYPS : (g >= 3 ? g - 1 : g));
        };
        for (int gi = 0; gi < 12; ++gi)
            if (P1Run &g = p1_runs[gi]; g.items) {
                g.off = off;
                g.L = near_p1_layout(p1_mode(gi), g.items, g.recs, g.src);
                off = align256(off + g.L.bytes);
            }
        const size_t off_in = off;
        for (int i = 0; i < n; ++i) off += take[i]->in_bytes;
        bool has_near = false;
        for (const NearRun &g : near_runs) has_near = has_near || g.count > 0;
        for (const P1Run &g : p1_runs) has_near = has_near || g.items > 0;
        const bool direct_batch = direct && off == off_in && !has_near;
        // descriptors and block tables: the device arena (after the staging
        // copy) or, for a direct batch, the staging itself
        char *src = direct_batch ? hd : db;
        const size_t h2d_end = align256(off);
        // every kTimedEvery-th batch times its launches: per workgroup a
        // {start, end} device-clock record, read back after the launches
        b->timed = (batch_counter.fetch_add(1) % kTimedEvery) == 0;
        const size_t off_clock = h2d_end;
        int64_t nblk = 0;
        for (const Launch &L : launches) nblk += L.count;
        off = off_clock + (b->timed ? 16 * (size_t)nblk : 0);
        const size_t off_status = align256(off);
        off = align256(off_status + sizeof(int32_t) * n);
        std::vector<size_t> out_off(n);
        for (int i = 0; i < n; ++i) {
            out_off[i] = off;
            off += take[i]->out_bytes;
        }
        if (off > slot_bytes) {
            // admission keeps this from happening; fail the batch rather than overrun the slot
            b->t_launch = now_seconds();
            b->ev_done = get_event();
            (void)hipEventRecord(b->ev_done, stream);
            for (Request *r : take) r->off_status = SIZE_MAX;
            return b;
        }

        // staging writes
        if (time_phases) tp[2] = now_seconds();
        static_assert(sizeof(EntryBlock) == 64, "block records are 64 bytes");
        for (const Launch &L : launches) {
            EntryBlock *p = reinterpret_cast<EntryBlock *>(hb + L.off_tab);
            int64_t k = 0;
            for (int i : sc.members[L.key]) {
                const Request &r = *take[i];
                const int64_t nb = (int64_t)r.pre_blocks.size();
                std::memcpy(p + k, r.pre_blocks.data(), sizeof(EntryBlock) * (size_t)nb);
                for (int64_t j = 0; j < nb; ++j) p[k + j].req |= i << 1;
                k += nb;
            }
        }
        if (time_phases) tp[3] = now_seconds();
        ReqDev *hreq = reinterpret_cast<ReqDev *>(hb);
        size_t in = off_in;
        for (int i = 0; i < n; ++i) {
            hreq[i] = take[i]->pre_dev;
            in += stage_own_inputs(*take[i], hb, db, in, hreq[i]);
        }
        std::memset(hb + off_status, 0, sizeof(int32_t) * n);
        for (const NearRun &g : near_runs) {
            NearItem *q = reinterpret_cast<NearItem *>(hb + g.off);
            for (int i : g.members) {
                const Request &r = *take[i];
                std::memcpy(q, r.near_items.data(), sizeof(NearItem) * r.near_items.size());
                for (size_t j = 0; j < r.near_items.size(); ++j)
                    q[j].out = hd + out_off[i] + (size_t)r.near_index[j] * r.elem_bytes;
                q += r.near_items.size();
            }
        }
        for (const P1Run &g : p1_runs) {
            int64_t pb = 0, rb = 0, sb = 0;
            for (int i : g.members) {
                const Request &r = *take[i];
                stage_near_p1(r, g.L, hb + g.off, db + g.off, hd + out_off[i], pb, rb, sb);
                pb += (int64_t)r.near_items.size();
                rb += (int64_t)r.near_recs.size();
                sb += (int64_t)r.near_src.size();
            }
        }
        b->off_clock = off_clock;
        for (int i = 0; i < n; ++i) {
            Request &r = *take[i];
            finish_descriptor(r, hd, out_off[i], off_status + sizeof(int32_t) * i, hreq[i]);
            r.off_out = out_off[i];
            r.off_status = off_status + sizeof(int32_t) * i;
        }
        b->launches = std::move(launches);

        // enqueue: the input copy, the launches (timed ones also with HIP
        // events around each launch), the batch event
        b->t_launch = now_seconds();
        b->t_hip = b->t_launch;
        auto note = [&](hipError_t e) {
            if (e != hipSuccess && b->enqueue_error == hipSuccess) b->enqueue_error = e;
        };
        if (!direct_batch) note(launch_stage_copy(hd, db, h2d_end, stream));
        const ReqDev *dreq = reinterpret_cast<const ReqDev *>(src);
        int64_t blk0 = 0;
        for (const Launch &L : b->launches) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            unsigned long long *ck = nullptr;
            if (b->timed) {
                e0 = get_event();
                e1 = get_event();
                b->ev.push_back(e0);
                b->ev.push_back(e1);
                ck = reinterpret_cast<unsigned long long *>(hd + off_clock) + 2 * blk0;
            }
            note(launch_entries(L.v, dreq, reinterpret_cast<const EntryBlock *>(src + L.off_tab), L.count, stream, ck,
                                e0, e1));
            blk0 += L.count;
        }
        // singular pairs after the entry kernels, on the same stream
        for (int gi = 0; gi < 8; ++gi)
            if (near_runs[gi].count)
                note(launch_near(gi >> 1, gi & 1, reinterpret_cast<const NearItem *>(db + near_runs[gi].off),
                                 near_runs[gi].count, stream));
        for (int gi = 0; gi < 12; ++gi)
            if (p1_runs[gi].items)
                note(launch_near_p1_region(p1_op(gi), gi & 1, p1_runs[gi].L, db + p1_runs[gi].off, p1_runs[gi].items,
                                           p1_runs[gi].recs, stream));
        b->ev_done = get_event();
        note(hipEventRecord(b->ev_done, stream));
        b->t_hip = now_seconds() - b->t_hip;
        if (time_phases) {
            tp[4] = b->t_launch;
            tp[5] = now_seconds();
            std::lock_guard<std::mutex> g(stat_mu);
            for (int i = 0; i < 5; ++i) ph_disp[i] += tp[i + 1] - tp[i];
            ph_nd += 1;
        }
        return b;
    }

    void release_batch(Batch *b, int n = 1)
    {
        if (b->refs.fetch_sub(n) != n) return;
        {
            std::lock_guard<std::mutex> g(ev_mu);
            for (hipEvent_t ev : b->ev) event_pool.push_back(ev);
            if (b->ev_done) event_pool.push_back(b->ev_done);
        }
        {
            std::lock_guard<std::mutex> g(mu);
            slot_busy[b->slot] = false;
        }
        cv.notify_one();
        give_batch(b);
    }

    void complete_loop()
    {
        (void)hipSetDevice(device);
        for (;;) {
            Batch *b = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cvc.wait(lk, [&] { return !inflight.empty() || (stop && pending.empty()); });
                if (inflight.empty()) return;
                b = inflight.front();
                inflight.pop_front();
            }
            const double tw0 = now_seconds();
            hipError_t e = hipSuccess;
            if (b->persist) {
                persist_wait(b);
            } else if (spin) {
                while ((e = hipEventQuery(b->ev_done)) == hipErrorNotReady) __builtin_ia32_pause();
            } else {
                e = hipEventSynchronize(b->ev_done);
            }
            if (e == hipSuccess) e = b->enqueue_error;
            const double t_done = now_seconds();
            double tc[6] = {tw0, t_done, 0, 0, 0, 0};
            double ks = 0.0;
            std::vector<double> dur(b->launches.size(), 0.0), dev(b->launches.size(), 0.0);
            if (b->timed && e == hipSuccess) {
                const unsigned long long *ck =
                    reinterpret_cast<const unsigned long long *>(h_stage + (size_t)b->slot * slot_bytes + b->off_clock);
                for (size_t i = 0; i < b->launches.size(); ++i) {
                    float ms = 0.f;
                    if (!b->persist && hipEventElapsedTime(&ms, b->ev[2 * i], b->ev[2 * i + 1]) == hipSuccess)
                        dur[i] = ms * 1e-3;
                    // kernel execution: earliest workgroup start to latest workgroup end
                    unsigned long long t0 = ~0ull, t1 = 0;
                    for (int64_t w = 0; w < b->launches[i].count; ++w) {
                        t0 = std::min(t0, ck[2 * w]);
                        t1 = std::max(t1, ck[2 * w + 1]);
                    }
                    if (t1 > t0) dev[i] = (double)(t1 - t0) / clock_hz;
                    ks += dev[i];
                    if (log_launches) {
                        // workgroup durations and start offsets (median, max), device clock
                        const int64_t nw = b->launches[i].count;
                        std::vector<double> wd(nw), ws(nw);
                        for (int64_t w = 0; w < nw; ++w) {
                            wd[w] = 1e6 * (double)(ck[2 * w + 1] - ck[2 * w]) / clock_hz;
                            ws[w] = 1e6 * (double)(ck[2 * w] - t0) / clock_hz;
                        }
                        std::sort(wd.begin(), wd.end());
                        std::sort(ws.begin(), ws.end());
                        fprintf(stderr,
                                "[bem-launch] slot %d grid %lld events_us %.2f clock_us %.2f wg_us med %.2f max %.2f "
                                "start_us med %.2f max %.2f\n",
                                b->slot, (long long)nw, 1e6 * dur[i], 1e6 * dev[i], wd[nw / 2], wd[nw - 1], ws[nw / 2],
                                ws[nw - 1]);
                    }
                    ck += 2 * b->launches[i].count;
                }
            }
            {
                std::lock_guard<std::mutex> g(stat_mu);
                n_batches += 1;
                n_requests += (int64_t)b->reqs.size();
                n_entries += b->entries;
                n_evals += b->evals;
                if (b->timed) {
                    n_timed += 1;
                    n_launches += (int64_t)b->launches.size();
                    kernel_s += ks;
                }
                busy += std::max(0.0, t_done - std::max(b->t_launch, last_done));
                last_done = std::max(last_done, t_done);
                if (b->fast) {
                    for (const FastGroup &g : b->groups)
                        for (int i = 0; i < g.n && latencies.size() < (size_t(1) << 24); ++i)
                            latencies.push_back((float)(t_done - g.t_submit));
                } else {
                    for (Request *r : b->reqs)
                        if (latencies.size() < (size_t(1) << 24)) latencies.push_back((float)(t_done - r->t_submit));
                }
                // a persistent launch's statistics are its own (persist_quiesce)
                for (size_t i = 0; b->timed && !b->persist && i < b->launches.size(); ++i) {
                    const Launch &L = b->launches[i];
                    KStat &k = kstats[L.v];
                    k.launches += 1;
                    k.workgroups += L.count;
                    k.blocks += L.count;
                    k.entries += L.entries;
                    k.evals += L.evals;
                    k.loads += L.loads;
                    k.seconds += dev[i];
                    k.seconds_events += dur[i];
                }
            }
            if (time_phases) tc[2] = now_seconds();
            if (b->fast) {
                // statuses stay in the staging (server_request_status); one
                // callback per submitter group, no request is touched here
                b->error = e;
                b->t_done = t_done;
                const double nreq = (double)b->reqs.size();
                b->refs.fetch_add((int)b->reqs.size());   // each request holds its result until released
                if (time_phases) tc[3] = now_seconds();
                for (const FastGroup &g : b->groups) {
                    g.mesh->inflight.fetch_sub(g.n);
                    g.cb(b->reqs.data() + g.first, (size_t)g.n, g.ctx);
                }
                if (time_phases) tc[4] = now_seconds();
                const double leg_q = b->q_sum, leg_s = nreq * (b->t_enq - b->t_take), leg_d = nreq * (t_done - b->t_enq);
                release_batch(b);   // b may be gone from here on
                const double t_fin = now_seconds();
                std::lock_guard<std::mutex> g(stat_mu);
                if (time_phases) {
                    tc[5] = t_fin;
                    for (int i = 0; i < 5; ++i) ph_comp[i] += tc[i + 1] - tc[i];
                    ph_nc += 1;
                }
                wait_s += t_done - tw0;
                complete_s += t_fin - t_done;
                leg_queue += leg_q;
                leg_stage += leg_s;
                leg_device += leg_d;
                leg_complete += nreq * (t_fin - t_done);
                continue;
            }
            char *hb = h_stage + (size_t)b->slot * slot_bytes;
            std::vector<Request *> reqs;
            reqs.swap(b->reqs);
            std::vector<int> sts(reqs.size(), BEM_OK);
            int lent = 0;
            for (size_t i = 0; i < reqs.size(); ++i) {
                Request *r = reqs[i];
                int st = BEM_OK;
                if (r->off_status == SIZE_MAX) {
                    st = fail(BEM_E_INTERNAL, "batch layout exceeded its slot");
                } else if (e != hipSuccess) {
                    st = fail(BEM_E_DEVICE, std::string("batch failed: ") + hipGetErrorString(e));
                } else if (*reinterpret_cast<int32_t *>(hb + r->off_status) != 0) {
                    st = BEM_E_NEARFIELD;
                } else if (r->borrow) {
                    ++lent;
                    r->result = hb + r->off_out;
                    r->batch = b;
                } else if (r->out_host) {
                    std::memcpy(r->out_host, hb + r->off_out, (size_t)r->entries() * r->elem_bytes);
                }
                sts[i] = st;
            }
            b->refs.fetch_add(lent);  // before any borrower can release
            const double nreq = (double)reqs.size();
            const double leg_q = b->q_sum, leg_s = nreq * (b->t_enq - b->t_take), leg_d = nreq * (t_done - b->t_enq);
            if (time_phases) tc[3] = now_seconds();
            finish_all(reqs, sts);
            if (time_phases) tc[4] = now_seconds();
            release_batch(b);   // b may be gone from here on
            {
                const double t_fin = now_seconds();
                if (time_phases) {
                    tc[5] = t_fin;
                    std::lock_guard<std::mutex> g(stat_mu);
                    for (int i = 0; i < 5; ++i) ph_comp[i] += tc[i + 1] - tc[i];
                    ph_nc += 1;
                }
                std::lock_guard<std::mutex> g(stat_mu);
                wait_s += t_done - tw0;
                complete_s += t_fin - t_done;
                leg_queue += leg_q;
                leg_stage += leg_s;
                leg_device += leg_d;
                leg_complete += nreq * (t_fin - t_done);
            }
        }
    }

    // New arena size and batch bound.  A running server is drained first: it
    // must be idle (nothing pending or in flight, no result still lent); its
    // threads, streams and arena are released and the next submission starts
    // it again with the new sizes.
    int reconfigure(size_t arena, int mb)
    {
        bool running;
        {
            std::lock_guard<std::mutex> g(mu);
            running = started;
            if (running) {
                bool busy = !pending.empty() || !inflight.empty() || (open && (open->nreq > 0 || open->writers > 0));
                for (int i = 0; i < nslots; ++i) busy = busy || (slot_busy[i] && !(open && open->b->slot == i));
                if (busy) return fail(BEM_E_BUSY, "server has requests in flight or results still lent");
                stop = true;
            }
        }
        if (running) {
            cv.notify_all();
            cvc.notify_all();
            for (std::thread &t : threads) t.join();
            threads.clear();
            // the persistent launch reads the staging: it ends before the staging goes
            persist_quiesce(10.0);
            if (pstream) (void)hipStreamSynchronize(pstream);
            for (int i = 0; i < nstreams; ++i)
                if (streams[i]) (void)hipStreamDestroy(streams[i]);
            for (int i = 0; i < kMaxSlots; ++i) streams[i] = nullptr;
            if (open) {   // empty (checked above)
                give_batch(open->b);
                delete open;
                open = nullptr;
            }
            for (int i = 0; i < kMaxSlots; ++i) slot_busy[i] = false;
            (void)hipFree(d_arena);
            (void)hipHostFree(h_stage);
            d_arena = h_stage = h_stage_dev = nullptr;
        }
        std::lock_guard<std::mutex> g(mu);
        started = false;
        stop = false;
        ++generation;
        arena_bytes = arena;
        max_batch = mb;
        return BEM_OK;
    }

    void kernel_stats(bem_kernel_stats_t *out, int max, int *count, int reset)
    {
        if (started) persist_quiesce(2.0);
        std::lock_guard<std::mutex> g(stat_mu);
        int i = 0;
        for (auto &kv : kstats) {
            if (i < max && out) {
                bem_kernel_stats_t &o = out[i];
                const Variant &v = kv.first;
                o.op = v.op;
                o.space = v.space;
                o.prec = v.prec;
                o.quad_points = v.q;
                o.persistent = v.persist;
                o.reserved = 0;
                o.launches = kv.second.launches;
                o.workgroups = kv.second.workgroups;
                o.entries = kv.second.entries;
                o.pair_evals = kv.second.evals;
                o.triangle_loads = kv.second.loads;
                o.seconds = kv.second.seconds;
                o.seconds_events = kv.second.seconds_events;
                o.blocks = kv.second.blocks;
            }
            ++i;
        }
        if (count) *count = i;
        if (reset) kstats.clear();
    }

    void stats(bem_server_stats_t *s, int reset)
    {
        std::lock_guard<std::mutex> g(stat_mu);
        s->requests = n_requests;
        s->entries = n_entries;
        s->batches = n_batches;
        s->kernel_evals = n_evals;
        s->busy_seconds = busy;
        // timed batches are a sample: scale to all batches
        const double scale = n_timed ? (double)n_batches / (double)n_timed : 0.0;
        s->kernel_seconds = kernel_s * scale;
        s->kernel_launches = n_launches;
        s->dispatch_seconds = dispatch_s;
        s->complete_seconds = complete_s;
        s->wait_seconds = wait_s;
        s->dispatch_hip_seconds = dispatch_hip_s;
        const double nr = n_requests ? (double)n_requests : 1.0;
        s->mean_queue_seconds = leg_queue / nr;
        s->mean_stage_seconds = leg_stage / nr;
        s->mean_device_seconds = leg_device / nr;
        s->mean_complete_seconds = leg_complete / nr;
        s->latency_p50 = s->latency_p99 = s->latency_max = 0.0;
        if (!latencies.empty()) {
            std::vector<float> v(latencies);
            auto pct = [&](double q) {
                size_t k = (size_t)std::min<double>(v.size() - 1, std::floor(q * (v.size() - 1) + 0.5));
                std::nth_element(v.begin(), v.begin() + k, v.end());
                return (double)v[k];
            };
            s->latency_p50 = pct(0.50);
            s->latency_p99 = pct(0.99);
            s->latency_max = *std::max_element(latencies.begin(), latencies.end());
        }
        if (reset) {
            n_requests = n_entries = n_batches = n_evals = n_launches = n_timed = 0;
            busy = kernel_s = 0.0;
            dispatch_s = complete_s = wait_s = dispatch_hip_s = 0.0;
            leg_queue = leg_stage = leg_device = leg_complete = 0.0;
            latencies.clear();
        }
    }
};

Server &server()
{
    static Server *s = new Server();  // lives until process exit
    return *s;
}

// At process exit a persistent launch still waiting for batches is asked to
// end, and given a moment to do so, with plain host stores and loads (the
// runtime may already be going away, so no HIP call).
Server *g_exit_server = nullptr;

void persist_at_exit()
{
    Server *s = g_exit_server;
    if (!s || !s->ph) return;
    volatile uint64_t *stop = &s->ph->stop;
    *stop = ~uint64_t(0) >> 1;
    const volatile uint64_t *w = &s->ph->exit_word;
    const uint64_t id = s->p_cur.id;
    const double t0 = now_seconds();
    while (s->p_running && (*w >> 40) != id && now_seconds() - t0 < 0.5) std::this_thread::yield();
}

void persist_register_exit(Server *s)
{
    if (g_exit_server) return;
    g_exit_server = s;
    std::atexit(persist_at_exit);
}

}  // namespace

int server_configure(size_t arena_bytes, int max_batch)
{
    if (arena_bytes < (size_t(4) << 20)) return fail(BEM_E_ARG, "arena must be at least 4 MiB");
    if (max_batch < 1) return fail(BEM_E_ARG, "max_batch_requests must be >= 1");
    return server().reconfigure(arena_bytes, max_batch);
}

int server_submit(Request *r) { return server().submit_many(&r, 1); }

int server_submit_many(Request *const *rs, size_t n) { return server().submit_many(rs, n); }

void server_print_phases()
{
    Server &S = server();
    std::lock_guard<std::mutex> g(S.stat_mu);
    if (!S.time_phases || S.ph_nd == 0 || S.ph_nc == 0) return;
    const double d = 1e6 / (double)S.ph_nd, c = 1e6 / (double)S.ph_nc;
    fprintf(stderr, "[bem] dispatch us/batch: group %.2f layout %.2f blocks %.2f inputs %.2f enqueue %.2f (%lld batches)\n",
            S.ph_disp[0] * d, S.ph_disp[1] * d, S.ph_disp[2] * d, S.ph_disp[3] * d, S.ph_disp[4] * d,
            (long long)S.ph_nd);
    fprintf(stderr, "[bem] completion us/batch: wait %.2f stats %.2f statuses %.2f callbacks %.2f release %.2f\n",
            S.ph_comp[0] * c, S.ph_comp[1] * c, S.ph_comp[2] * c, S.ph_comp[3] * c, S.ph_comp[4] * c);
    for (double &x : S.ph_disp) x = 0.0;
    for (double &x : S.ph_comp) x = 0.0;
    S.ph_nd = S.ph_nc = 0;
}

int server_wait(Request *r, double timeout_s)
{
    std::unique_lock<std::mutex> lk(r->mu);
    if (timeout_s < 0) {
        r->cv.wait(lk, [&] { return r->done; });
    } else if (!r->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return r->done; })) {
        return BEM_E_TIMEOUT;
    }
    return r->status;
}

int server_request_status(const Request *r)
{
    if (!r->fast) return r->status;
    const Batch *b = static_cast<const Batch *>(r->batch);
    if (b->error != hipSuccess) return BEM_E_DEVICE;
    return *reinterpret_cast<const volatile int32_t *>(b->hb + r->off_status) != 0 ? BEM_E_NEARFIELD : BEM_OK;
}

double server_request_done_time(const Request *r)
{
    return r->fast ? static_cast<const Batch *>(r->batch)->t_done : r->t_done;
}

void server_release(Request *r)
{
    if (!r->batch) return;
    Batch *b = static_cast<Batch *>(r->batch);
    r->batch = nullptr;
    r->result = nullptr;
    server().release_batch(b);
}

void server_release_batch(void *batch, int n)
{
    if (batch && n > 0) server().release_batch(static_cast<Batch *>(batch), n);
}

int server_stats(bem_server_stats_t *s, int reset)
{
    server().stats(s, reset);
    return BEM_OK;
}

int server_kernel_stats(bem_kernel_stats_t *out, int max, int *count, int reset)
{
    server().kernel_stats(out, max, count, reset);
    return BEM_OK;
}

int server_ensure_started()
{
    Server &s = server();
    std::lock_guard<std::mutex> g(s.mu);
    return s.start();
}

bool server_running() { return server().started; }

}  // namespace bem
