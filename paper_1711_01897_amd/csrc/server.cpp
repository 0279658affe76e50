// Device request server: continuous batching of entry requests.
//
// The paper lets each H-matrix block's CPU thread launch its own small
// kernels and relies on hardware work queues to overlap them (Section 4).
// Here every host thread submits requests to one server instead:
//
//  * admission: a request is taken into the next batch when a batch slot is
//    free and the slot's share of the device arena still has room for the
//    request's inputs, outputs, partial sums and tile tables (admission by
//    memory);
//  * fusion: all admitted requests of one kernel variant run in one launch,
//    one wavefront per tile, whatever request the tile belongs to; the tile
//    tables are built on the device from per-request tile counts;
//  * overlap: several slots rotate, each with its own stream, so the
//    dispatcher stages and enqueues the next batches while earlier ones run
//    or are being consumed, and consecutive batches overlap on the device;
//    requests that arrive meanwhile wait only for the next free slot;
//  * completion: a second thread waits for each batch's event, checks the
//    near-field flags, copies results to the callers' buffers (or lends the
//    caller a pointer into the pinned staging until it releases it), wakes
//    the waiters and records submit-to-completion latency.
// Each request's result is computed by the same tiles with the same
// summation order whichever batch it lands in.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <deque>
#include <map>
#include <thread>

#include "bem_internal.hpp"

namespace bem {

namespace {

constexpr int kMaxSlots = 16;
constexpr int kTimedEvery = 4;

int env_int(const char *name, int dflt, int lo, int hi)
{
    const char *e = std::getenv(name);
    if (!e) return dflt;
    return std::max(lo, std::min(hi, std::atoi(e)));
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Launch {
    Variant v{};
    bool reduce = false;
    int ng = 0;                  // requests in the group
    size_t off_greq = 0, off_gpre = 0, off_tiles = 0;
    int64_t ntiles = 0;
    int64_t entries = 0, evals = 0, loads = 0;
};

struct KStat {
    int64_t launches = 0, entries = 0, evals = 0, loads = 0;
    double seconds = 0.0;
};

struct Batch {
    int slot = 0;
    std::vector<Request *> reqs;
    std::vector<Launch> launches;
    std::vector<hipEvent_t> ev;   // start/stop per entry or reduction launch
    hipEvent_t ev_done = nullptr;
    double t_launch = 0.0;
    int64_t entries = 0, evals = 0;
    std::atomic<int> refs{1};     // completion thread + borrowed results
    bool timed = false;           // per-launch events recorded
};

class Server {
public:
    size_t arena_bytes = size_t(1) << 30;
    int max_batch = 16384;
    int nslots = 8;     // BEM_SERVER_SLOTS
    int nstreams = 8;   // BEM_SERVER_STREAMS (slot s uses stream s % nstreams), default one per slot

    std::mutex mu;
    std::condition_variable cv;    // dispatcher: pending requests, free slots
    std::condition_variable cvc;   // completer: batches in flight
    std::deque<Request *> pending;
    std::deque<Batch *> inflight;
    bool slot_busy[kMaxSlots] = {};
    bool started = false, stop = false;
    int device = 0;
    hipStream_t streams[kMaxSlots] = {};
    char *d_arena = nullptr, *h_stage = nullptr;
    size_t slot_bytes = 0;
    std::thread dispatcher, completer;
    std::mutex ev_mu;
    std::vector<hipEvent_t> event_pool;

    // statistics
    std::mutex stat_mu;
    int64_t n_requests = 0, n_entries = 0, n_batches = 0, n_evals = 0, n_launches = 0, n_timed = 0;
    double busy = 0.0, last_done = 0.0, kernel_s = 0.0, reduce_s = 0.0;
    double dispatch_s = 0.0, complete_s = 0.0, wait_s = 0.0;
    std::vector<float> latencies;
    std::map<std::pair<Variant, int>, KStat> kstats;
    std::vector<int> group_members[64], rgroup_members[4];   // dispatcher scratch
    int64_t batch_counter = 0;

    int start()
    {
        if (started) return BEM_OK;
        nslots = env_int("BEM_SERVER_SLOTS", nslots, 2, kMaxSlots);
        nstreams = env_int("BEM_SERVER_STREAMS", nslots, 1, nslots);
        hipError_t e = hipGetDevice(&device);
        for (int i = 0; i < nstreams && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&streams[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipMalloc(&d_arena, arena_bytes);
        if (e == hipSuccess) e = hipHostMalloc(&h_stage, arena_bytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            if (d_arena) (void)hipFree(d_arena);
            d_arena = nullptr;
            return fail(e == hipErrorOutOfMemory ? BEM_E_OOM : BEM_E_DEVICE,
                        std::string("server start: ") + hipGetErrorString(e));
        }
        slot_bytes = (arena_bytes / nslots) & ~(size_t)255;
        started = true;
        dispatcher = std::thread([this] { dispatch_loop(); });
        completer = std::thread([this] { complete_loop(); });
        return BEM_OK;
    }

    hipEvent_t get_event()
    {
        std::lock_guard<std::mutex> g(ev_mu);
        if (!event_pool.empty()) {
            hipEvent_t e = event_pool.back();
            event_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
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
        for (size_t i = 0; i < rs.size(); ++i) {
            Request *r = rs[i];
            if (!r->on_done) {
                finish(r, st[i]);
                continue;
            }
            r->t_done = t;
            r->status = st[i];
            r->done = true;
            r->mesh->inflight.fetch_sub(1);
            const std::pair<void *, void *> key{(void *)r->on_done, r->cb_ctx};
            size_t g = 0;
            while (g < groups.size() && groups[g].first != key) ++g;
            if (g == groups.size()) groups.push_back({key, {}});
            groups[g].second.push_back(r);
        }
        for (auto &g : groups) {
            auto cb = reinterpret_cast<void (*)(Request **, size_t, void *)>(g.first.first);
            cb(g.second.data(), g.second.size(), g.first.second);
        }
    }

    // batch-level slack: alignment of sections and group tables
    static constexpr size_t kSlack = size_t(1) << 17;
    bool fits(const Request *r) const { return r->batch_bytes + kSlack <= slot_bytes; }

    int submit_many(Request *const *rs, size_t n)
    {
        {
            std::lock_guard<std::mutex> g(mu);
            if (!started) {
                int rc = start();
                if (rc != BEM_OK) return rc;
            }
            for (size_t i = 0; i < n; ++i)
                if (!fits(rs[i])) return fail(BEM_E_OOM, "request larger than a server batch slot; raise the arena size");
            const double t = now_seconds();
            for (size_t i = 0; i < n; ++i) {
                Request *r = rs[i];
                r->t_submit = t;
                r->done = false;
                r->result = nullptr;
                r->batch = nullptr;
                r->mesh->inflight.fetch_add(1);
                pending.push_back(r);
            }
        }
        cv.notify_one();
        return BEM_OK;
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
        for (;;) {
            std::vector<Request *> take;
            int slot = -1;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stop || (!pending.empty() && free_slot() >= 0); });
                if (stop) {
                    std::vector<Request *> left(pending.begin(), pending.end());
                    pending.clear();
                    lk.unlock();
                    finish_all(left, std::vector<int>(left.size(), BEM_E_CANCELLED));
                    return;
                }
                slot = free_slot();
                size_t bytes = kSlack;
                while (!pending.empty() && (int)take.size() < max_batch) {
                    Request *r = pending.front();
                    const size_t rb = r->batch_bytes;
                    if (!take.empty() && bytes + rb > slot_bytes) break;
                    take.push_back(r);
                    bytes += rb;
                    pending.pop_front();
                }
                slot_busy[slot] = true;
            }
            const double t0 = now_seconds();
            Batch *b = build_and_launch(slot, take);
            const double t1 = now_seconds();
            {
                std::lock_guard<std::mutex> g(stat_mu);
                dispatch_s += t1 - t0;
            }
            {
                std::lock_guard<std::mutex> g(mu);
                inflight.push_back(b);
            }
            cvc.notify_one();
        }
    }

    Batch *build_and_launch(int slot, std::vector<Request *> &take)
    {
        Batch *b = new Batch();
        b->slot = slot;
        b->reqs = take;
        char *hb = h_stage + (size_t)slot * slot_bytes;
        char *db = d_arena + (size_t)slot * slot_bytes;
        hipStream_t stream = streams[slot % nstreams];
        const int n = (int)take.size();

        // kernel variant groups (entry launches) and reduction groups, indexed
        // by (op, space, prec, rule, fixed side) and (prec, complex)
        for (auto &g : group_members) g.clear();
        for (auto &g : rgroup_members) g.clear();
        for (int i = 0; i < n; ++i) {
            Request &r = *take[i];
            if (r.ntiles > 0)
                group_members[(((r.op * 2 + r.space) * 2 + r.prec) * 2 + (r.mesh->q == 6 ? 1 : 0)) * 2 + r.rowfix]
                    .push_back(i);
            if (r.nrtiles > 0) rgroup_members[r.prec * 2 + (is_complex_op(r.op) ? 1 : 0)].push_back(i);
            b->entries += r.entries();
            b->evals += r.evals;
        }
        std::vector<std::pair<Variant, const std::vector<int> *>> groups;
        for (int key = 0; key < 64; ++key) {
            if (group_members[key].empty()) continue;
            const int rowfix = key & 1, q = (key >> 1) & 1 ? 6 : 4, prec = (key >> 2) & 1, space = (key >> 3) & 1,
                      op = key >> 4;
            groups.push_back({Variant{op, space, prec, q, rowfix}, &group_members[key]});
        }
        std::vector<std::pair<std::pair<int, int>, const std::vector<int> *>> rgroups;
        for (int key = 0; key < 4; ++key)
            if (!rgroup_members[key].empty()) rgroups.push_back({{key >> 1, key & 1}, &rgroup_members[key]});

        // layout: descriptors | group tables | inputs | status | outputs || partials | tiles
        // (offsets first, checked against the slot, then the staging writes)
        std::vector<Launch> launches;
        for (auto &g : groups) {
            Launch L;
            L.v = g.first;
            L.reduce = false;
            L.ng = (int)g.second->size();
            launches.push_back(L);
        }
        for (auto &g : rgroups) {
            Launch L;
            L.v = Variant{g.first.second ? BEM_HELMHOLTZ_SLP : BEM_LAPLACE_SLP, BEM_P1, g.first.first, 0, 0};
            L.reduce = true;
            L.ng = (int)g.second->size();
            launches.push_back(L);
        }
        std::vector<const std::vector<int> *> members;
        for (auto &g : groups) members.push_back(g.second);
        for (auto &g : rgroups) members.push_back(g.second);
        size_t off = 0;
        const size_t off_reqs = off;
        off = align256(off + sizeof(ReqDev) * n);
        for (size_t gi = 0; gi < launches.size(); ++gi) {
            Launch &L = launches[gi];
            L.off_greq = off;
            off = align256(off + 4 * (size_t)L.ng);
            L.off_gpre = off;
            off = align256(off + 8 * ((size_t)L.ng + 1));
            for (int i : *members[gi]) {
                const Request &r = *take[i];
                L.ntiles += L.reduce ? r.nrtiles : r.ntiles;
                L.entries += r.entries();
                if (!L.reduce) {
                    L.evals += r.evals;
                    L.loads += r.nfix * r.nlane;
                }
            }
        }
        const size_t off_groups = off;
        off = align256(off + sizeof(GroupDesc) * launches.size());
        const size_t off_in = off;
        for (int i = 0; i < n; ++i) off += take[i]->in_bytes;
        const size_t off_status = align256(off);
        off = align256(off_status + 2 * sizeof(int32_t) * n);
        const size_t h2d_end = off;
        std::vector<size_t> out_off(n), part_off(n);
        for (int i = 0; i < n; ++i) {
            out_off[i] = off;
            off += take[i]->out_bytes;
        }
        const size_t d2h_end = off;
        off = align256(off);
        for (int i = 0; i < n; ++i) {
            part_off[i] = off;
            off += take[i]->part_bytes;
        }
        off = align256(off);
        for (Launch &L : launches) {
            L.off_tiles = off;
            off = align256(off + (L.reduce ? sizeof(RTile) : sizeof(Tile)) * (size_t)L.ntiles);
        }
        if (off > slot_bytes) {
            // admission keeps this from happening; fail the batch rather than overrun the slot
            b->launches.clear();
            b->t_launch = now_seconds();
            b->ev_done = get_event();
            (void)hipEventRecord(b->ev_done, stream);
            for (Request *r : take) r->off_status = SIZE_MAX;
            return b;
        }

        // staging writes
        ReqDev *hreq = reinterpret_cast<ReqDev *>(hb + off_reqs);
        for (size_t gi = 0; gi < launches.size(); ++gi) {
            const Launch &L = launches[gi];
            int32_t *greq = reinterpret_cast<int32_t *>(hb + L.off_greq);
            int64_t *gpre = reinterpret_cast<int64_t *>(hb + L.off_gpre);
            int64_t acc = 0;
            size_t k = 0;
            for (int i : *members[gi]) {
                greq[k] = i;
                gpre[k] = acc;
                acc += L.reduce ? take[i]->nrtiles : take[i]->ntiles;
                ++k;
            }
            gpre[k] = acc;
        }
        size_t in = off_in;
        for (int i = 0; i < n; ++i) in += stage_request_inputs(*take[i], hb, db, in, hreq[i]);
        std::memset(hb + off_status, 0, 2 * sizeof(int32_t) * n);
        for (int i = 0; i < n; ++i) {
            Request &r = *take[i];
            finish_descriptor(r, db, out_off[i], part_off[i], off_status + 8 * i, hreq[i]);
            r.off_out = out_off[i];
            r.off_status = off_status + 8 * i;
        }
        b->launches = launches;
        GroupDesc *gd = reinterpret_cast<GroupDesc *>(hb + off_groups);
        int64_t tile_total = 0;
        for (size_t gi = 0; gi < launches.size(); ++gi) {
            const Launch &L = launches[gi];
            gd[gi].tile0 = tile_total;
            gd[gi].ntiles = L.ntiles;
            gd[gi].greq = reinterpret_cast<const int32_t *>(db + L.off_greq);
            gd[gi].gpre = reinterpret_cast<const int64_t *>(db + L.off_gpre);
            gd[gi].tiles = db + L.off_tiles;
            gd[gi].ng = L.ng;
            gd[gi].kind = L.reduce ? 1 : 0;
            tile_total += L.ntiles;
        }

        b->t_launch = now_seconds();
        (void)hipMemcpyAsync(db, hb, h2d_end, hipMemcpyHostToDevice, stream);
        const ReqDev *dreq = reinterpret_cast<const ReqDev *>(db + off_reqs);
        (void)launch_build_all(dreq, reinterpret_cast<const GroupDesc *>(db + off_groups), (int)b->launches.size(),
                               tile_total, stream);
        // n + 1 events bracket n consecutive launches, on every kTimedEvery-th
        // batch (launch durations are sampled; the batch event is always kept)
        b->timed = (batch_counter++ % kTimedEvery) == 0;
        if (b->timed && !b->launches.empty()) {
            hipEvent_t e = get_event();
            (void)hipEventRecord(e, stream);
            b->ev.push_back(e);
        }
        for (const Launch &L : b->launches) {
            if (L.reduce)
                (void)launch_p1_reduce(L.v.prec, is_complex_op(L.v.op), dreq,
                                       reinterpret_cast<const RTile *>(db + L.off_tiles), L.ntiles, stream);
            else
                (void)launch_entries(L.v, dreq, reinterpret_cast<const Tile *>(db + L.off_tiles), L.ntiles, stream);
            if (b->timed) {
                hipEvent_t e = get_event();
                (void)hipEventRecord(e, stream);
                b->ev.push_back(e);
            }
        }
        (void)hipMemcpyAsync(hb + off_status, db + off_status, d2h_end - off_status, hipMemcpyDeviceToHost, stream);
        b->ev_done = get_event();
        (void)hipEventRecord(b->ev_done, stream);
        return b;
    }

    void release_batch(Batch *b)
    {
        if (b->refs.fetch_sub(1) != 1) return;
        {
            std::lock_guard<std::mutex> g(ev_mu);
            for (hipEvent_t ev : b->ev) event_pool.push_back(ev);
            event_pool.push_back(b->ev_done);
        }
        {
            std::lock_guard<std::mutex> g(mu);
            slot_busy[b->slot] = false;
        }
        cv.notify_one();
        delete b;
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
            hipError_t e = hipEventSynchronize(b->ev_done);
            const double t_done = now_seconds();
            double ks = 0.0, rs = 0.0;
            std::vector<double> dur(b->launches.size(), 0.0);
            if (b->timed)
                for (size_t i = 0; i < b->launches.size(); ++i) {
                    float ms = 0.f;
                    if (hipEventElapsedTime(&ms, b->ev[i], b->ev[i + 1]) == hipSuccess) {
                        dur[i] = ms * 1e-3;
                        (b->launches[i].reduce ? rs : ks) += ms * 1e-3;
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
                    reduce_s += rs;
                }
                busy += t_done - std::max(b->t_launch, last_done);
                last_done = t_done;
                for (Request *r : b->reqs)
                    if (latencies.size() < (size_t(1) << 24)) latencies.push_back((float)(t_done - r->t_submit));
                for (size_t i = 0; b->timed && i < b->launches.size(); ++i) {
                    const Launch &L = b->launches[i];
                    KStat &k = kstats[{L.v, L.reduce ? 1 : 0}];
                    k.launches += 1;
                    k.entries += L.entries;
                    k.evals += L.evals;
                    k.loads += L.loads;
                    k.seconds += dur[i];
                }
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
            finish_all(reqs, sts);
            release_batch(b);
            {
                std::lock_guard<std::mutex> g(stat_mu);
                wait_s += t_done - tw0;
                complete_s += now_seconds() - t_done;
            }
        }
    }

    void kernel_stats(bem_kernel_stats_t *out, int max, int *count, int reset)
    {
        std::lock_guard<std::mutex> g(stat_mu);
        int i = 0;
        for (auto &kv : kstats) {
            if (i < max && out) {
                bem_kernel_stats_t &o = out[i];
                const Variant &v = kv.first.first;
                o.op = v.op;
                o.space = v.space;
                o.prec = v.prec;
                o.quad_points = v.q;
                o.rowfix = v.rowfix;
                o.reduce = kv.first.second;
                o.launches = kv.second.launches;
                o.entries = kv.second.entries;
                o.pair_evals = kv.second.evals;
                o.triangle_loads = kv.second.loads;
                o.seconds = kv.second.seconds;
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
        s->kernel_seconds_p1_reduce = reduce_s * scale;
        s->kernel_launches = n_launches;
        s->dispatch_seconds = dispatch_s;
        s->complete_seconds = complete_s;
        s->wait_seconds = wait_s;
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
            busy = kernel_s = reduce_s = 0.0;
            dispatch_s = complete_s = wait_s = 0.0;
            latencies.clear();
        }
    }
};

Server &server()
{
    static Server *s = new Server();  // lives until process exit
    return *s;
}

}  // namespace

int server_configure(size_t arena_bytes, int max_batch)
{
    Server &s = server();
    std::lock_guard<std::mutex> g(s.mu);
    if (s.started) return fail(BEM_E_BUSY, "server already running");
    if (arena_bytes < (size_t(4) << 20)) return fail(BEM_E_ARG, "arena must be at least 4 MiB");
    if (max_batch < 1) return fail(BEM_E_ARG, "max_batch_requests must be >= 1");
    s.arena_bytes = arena_bytes;
    s.max_batch = max_batch;
    return BEM_OK;
}

int server_submit(Request *r) { return server().submit_many(&r, 1); }

int server_submit_many(Request *const *rs, size_t n) { return server().submit_many(rs, n); }

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

void server_release(Request *r)
{
    if (!r->batch) return;
    Batch *b = static_cast<Batch *>(r->batch);
    r->batch = nullptr;
    r->result = nullptr;
    server().release_batch(b);
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
