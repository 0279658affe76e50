// Device request server: continuous batching of entry requests.
//
// The paper lets each H-matrix block's CPU thread launch its own small
// kernels and relies on hardware work queues to overlap them (Section 4).
// Here every host thread submits requests to one server instead:
//
//  * admission: a request is taken into the next batch when a batch slot is
//    free and the slot's share of the device arena still has room for the
//    request's inputs, outputs and partial sums (admission by memory);
//  * fusion: all admitted requests of one kernel variant run in one launch,
//    one wavefront per tile, whatever request the tile belongs to;
//  * overlap: two slots alternate, so the dispatcher stages batch b+1 (and
//    enqueues it behind batch b on the same stream) while batch b runs, and
//    requests that arrive meanwhile wait only for the next free slot;
//  * completion: a second thread waits for each batch's event, checks the
//    near-field flags, copies results to the callers' buffers, wakes the
//    waiters and records submit-to-completion latency.
// Each request's result is computed by the same tiles with the same
// summation order whichever batch it lands in.
#include <algorithm>
#include <deque>
#include <map>
#include <thread>

#include "bem_internal.hpp"

namespace bem {

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Launch {
    Variant v;
    int first, count;  // tile range
    bool reduce;       // P1 reduction launch (v.prec and cplx from v.op)
};

struct Batch {
    int slot = 0;
    std::vector<Request *> reqs;
    std::vector<Launch> launches;
    std::vector<hipEvent_t> ev;   // start/stop per launch
    hipEvent_t ev_done = nullptr;
    double t_launch = 0.0;
    int64_t entries = 0, evals = 0;
};

class Server {
public:
    size_t arena_bytes = size_t(512) << 20;
    int max_batch = 8192;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request *> pending;
    std::deque<Batch *> inflight;
    bool slot_busy[2] = {false, false};
    bool started = false, stop = false;
    int device = 0;
    hipStream_t stream = nullptr;
    char *d_arena = nullptr, *h_stage = nullptr;
    size_t half = 0;
    std::thread dispatcher, completer;
    std::vector<hipEvent_t> event_pool;

    // statistics
    std::mutex stat_mu;
    int64_t n_requests = 0, n_entries = 0, n_batches = 0, n_evals = 0, n_launches = 0;
    double busy = 0.0, last_done = 0.0, kernel_s = 0.0, reduce_s = 0.0;
    std::vector<float> latencies;

    int start()
    {
        if (started) return BEM_OK;
        hipError_t e = hipGetDevice(&device);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipMalloc(&d_arena, arena_bytes);
        if (e == hipSuccess) e = hipHostMalloc(&h_stage, arena_bytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            if (d_arena) (void)hipFree(d_arena);
            d_arena = nullptr;
            return fail(e == hipErrorOutOfMemory ? BEM_E_OOM : BEM_E_DEVICE,
                        std::string("server start: ") + hipGetErrorString(e));
        }
        half = arena_bytes / 2;
        started = true;
        dispatcher = std::thread([this] { dispatch_loop(); });
        completer = std::thread([this] { complete_loop(); });
        return BEM_OK;
    }

    hipEvent_t get_event()
    {
        if (!event_pool.empty()) {
            hipEvent_t e = event_pool.back();
            event_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }

    void put_event(hipEvent_t e) { event_pool.push_back(e); }

    void finish(Request *r, int status)
    {
        r->t_done = now_seconds();
        r->mesh->inflight.fetch_sub(1);
        void (*cb)(Request *, void *) = r->on_done;
        void *ctx = r->cb_ctx;
        {
            std::lock_guard<std::mutex> g(r->mu);
            r->status = status;
            r->done = true;
        }
        r->cv.notify_all();
        if (cb) cb(r, ctx);
    }

    int submit(Request *r)
    {
        {
            std::lock_guard<std::mutex> g(mu);
            if (!started) {
                int rc = start();
                if (rc != BEM_OK) return rc;
            }
            if (request_bytes(*r) + 4096 > half)
                return fail(BEM_E_OOM, "request larger than a server batch slot; raise the arena size");
            r->t_submit = now_seconds();
            r->done = false;
            r->mesh->inflight.fetch_add(1);
            pending.push_back(r);
        }
        cv.notify_all();
        return BEM_OK;
    }

    void dispatch_loop()
    {
        (void)hipSetDevice(device);
        for (;;) {
            std::vector<Request *> take;
            int slot = -1;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stop || (!pending.empty() && (!slot_busy[0] || !slot_busy[1])); });
                if (stop) {
                    for (Request *r : pending) {
                        lk.unlock();
                        finish(r, BEM_E_CANCELLED);
                        lk.lock();
                    }
                    pending.clear();
                    return;
                }
                slot = !slot_busy[0] ? 0 : 1;
                size_t bytes = 4096;
                while (!pending.empty() && (int)take.size() < max_batch) {
                    Request *r = pending.front();
                    const size_t rb = request_bytes(*r);
                    if (!take.empty() && bytes + rb > half) break;
                    take.push_back(r);
                    bytes += rb;
                    pending.pop_front();
                }
                slot_busy[slot] = true;
            }
            Batch *b = build_and_launch(slot, take);
            {
                std::lock_guard<std::mutex> g(mu);
                inflight.push_back(b);
            }
            cv.notify_all();
        }
    }

    Batch *build_and_launch(int slot, std::vector<Request *> &take)
    {
        Batch *b = new Batch();
        b->slot = slot;
        b->reqs = take;
        char *hb = h_stage + (size_t)slot * half;
        char *db = d_arena + (size_t)slot * half;
        const int n = (int)take.size();

        // tiles grouped by kernel variant, reductions by (precision, complex)
        std::map<Variant, std::vector<Tile>> groups;
        std::map<std::pair<int, int>, std::vector<RTile>> rgroups;
        for (int i = 0; i < n; ++i) {
            Request &r = *take[i];
            Variant v{r.op, r.space, r.prec, r.mesh->q, r.rowfix};
            std::vector<RTile> rt;
            make_tiles(r, i, groups[v], rt);
            if (!rt.empty()) {
                auto &dst = rgroups[{r.prec, is_complex_op(r.op) ? 1 : 0}];
                dst.insert(dst.end(), rt.begin(), rt.end());
            }
            b->entries += r.entries();
            b->evals += r.evals;
        }
        size_t ntiles = 0, nrt = 0;
        for (auto &g : groups) ntiles += g.second.size();
        for (auto &g : rgroups) nrt += g.second.size();

        size_t off = 0;
        const size_t off_reqs = off;
        off = align256(off + sizeof(ReqDev) * n);
        const size_t off_tiles = off;
        off = align256(off + sizeof(Tile) * ntiles);
        const size_t off_rtiles = off;
        off = align256(off + sizeof(RTile) * nrt);
        std::vector<size_t> in_off(n);
        for (int i = 0; i < n; ++i) {
            in_off[i] = off;
            off += take[i]->in_bytes;
        }
        const size_t in_end = off;
        const size_t off_status = align256(off);
        off = align256(off_status + sizeof(int32_t) * n);
        std::vector<size_t> out_off(n);
        for (int i = 0; i < n; ++i) {
            out_off[i] = off;
            off += take[i]->out_bytes;
        }
        const size_t out_end = off;
        std::vector<size_t> part_off(n);
        for (int i = 0; i < n; ++i) {
            part_off[i] = off;
            off += take[i]->part_bytes;
        }

        ReqDev *hreq = reinterpret_cast<ReqDev *>(hb + off_reqs);
        for (int i = 0; i < n; ++i)
            place_request(*take[i], hb, db, in_off[i], out_off[i], part_off[i], off_status + 4 * i, hreq[i]);
        std::memset(hb + off_status, 0, sizeof(int32_t) * n);
        Tile *ht = reinterpret_cast<Tile *>(hb + off_tiles);
        size_t pos = 0;
        for (auto &g : groups) {
            std::memcpy(ht + pos, g.second.data(), sizeof(Tile) * g.second.size());
            b->launches.push_back(Launch{g.first, (int)pos, (int)g.second.size(), false});
            pos += g.second.size();
        }
        RTile *hrt = reinterpret_cast<RTile *>(hb + off_rtiles);
        pos = 0;
        for (auto &g : rgroups) {
            std::memcpy(hrt + pos, g.second.data(), sizeof(RTile) * g.second.size());
            Variant v{g.first.second ? BEM_HELMHOLTZ_SLP : BEM_LAPLACE_SLP, BEM_P1, g.first.first, 0, 0};
            b->launches.push_back(Launch{v, (int)pos, (int)g.second.size(), true});
            pos += g.second.size();
        }

        b->t_launch = now_seconds();
        // inputs and zeroed status words in one copy
        (void)hipMemcpyAsync(db, hb, off_status + sizeof(int32_t) * n, hipMemcpyHostToDevice, stream);
        const ReqDev *dreq = reinterpret_cast<const ReqDev *>(db + off_reqs);
        const Tile *dt = reinterpret_cast<const Tile *>(db + off_tiles);
        const RTile *drt = reinterpret_cast<const RTile *>(db + off_rtiles);
        for (const Launch &L : b->launches) {
            hipEvent_t e0 = get_event(), e1 = get_event();
            (void)hipEventRecord(e0, stream);
            if (L.reduce)
                (void)launch_p1_reduce(L.v.prec, is_complex_op(L.v.op), dreq, drt + L.first, L.count, stream);
            else
                (void)launch_entries(L.v, dreq, dt + L.first, L.count, stream);
            (void)hipEventRecord(e1, stream);
            b->ev.push_back(e0);
            b->ev.push_back(e1);
        }
        (void)hipMemcpyAsync(hb + off_status, db + off_status, out_end - off_status, hipMemcpyDeviceToHost, stream);
        b->ev_done = get_event();
        (void)hipEventRecord(b->ev_done, stream);
        (void)in_end;
        return b;
    }

    void complete_loop()
    {
        (void)hipSetDevice(device);
        for (;;) {
            Batch *b = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return !inflight.empty() || (stop && pending.empty()); });
                if (inflight.empty()) return;
                b = inflight.front();
            }
            hipError_t e = hipEventSynchronize(b->ev_done);
            const double t_done = now_seconds();
            double ks = 0.0, rs = 0.0;
            for (size_t i = 0; i < b->launches.size(); ++i) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, b->ev[2 * i], b->ev[2 * i + 1]) == hipSuccess) {
                    if (b->launches[i].reduce)
                        rs += ms * 1e-3;
                    else
                        ks += ms * 1e-3;
                }
            }
            char *hb = h_stage + (size_t)b->slot * half;
            for (Request *r : b->reqs) {
                int st = BEM_OK;
                if (e != hipSuccess) {
                    st = fail(BEM_E_DEVICE, std::string("batch failed: ") + hipGetErrorString(e));
                } else if (*reinterpret_cast<int32_t *>(hb + r->off_status) != 0) {
                    st = BEM_E_NEARFIELD;
                } else if (r->out_host) {
                    std::memcpy(r->out_host, hb + r->off_out, (size_t)r->entries() * r->elem_bytes);
                }
                finish(r, st);
            }
            {
                std::lock_guard<std::mutex> g(stat_mu);
                n_batches += 1;
                n_requests += (int64_t)b->reqs.size();
                n_entries += b->entries;
                n_evals += b->evals;
                n_launches += (int64_t)b->launches.size();
                kernel_s += ks;
                reduce_s += rs;
                busy += t_done - std::max(b->t_launch, last_done);
                last_done = t_done;
                for (Request *r : b->reqs)
                    if (latencies.size() < (size_t(1) << 24)) latencies.push_back((float)(r->t_done - r->t_submit));
            }
            {
                std::lock_guard<std::mutex> g(mu);
                for (hipEvent_t ev : b->ev) put_event(ev);
                put_event(b->ev_done);
                inflight.pop_front();
                slot_busy[b->slot] = false;
            }
            cv.notify_all();
            delete b;
        }
    }

    void stats(bem_server_stats_t *s, int reset)
    {
        std::lock_guard<std::mutex> g(stat_mu);
        s->requests = n_requests;
        s->entries = n_entries;
        s->batches = n_batches;
        s->kernel_evals = n_evals;
        s->busy_seconds = busy;
        s->kernel_seconds = kernel_s;
        s->kernel_seconds_p1_reduce = reduce_s;
        s->kernel_launches = n_launches;
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
            n_requests = n_entries = n_batches = n_evals = n_launches = 0;
            busy = kernel_s = reduce_s = 0.0;
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
    if (arena_bytes < (size_t(1) << 20)) return fail(BEM_E_ARG, "arena must be at least 1 MiB");
    if (max_batch < 1) return fail(BEM_E_ARG, "max_batch_requests must be >= 1");
    s.arena_bytes = arena_bytes;
    s.max_batch = max_batch;
    return BEM_OK;
}

int server_submit(Request *r) { return server().submit(r); }

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

int server_stats(bem_server_stats_t *s, int reset)
{
    server().stats(s, reset);
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
