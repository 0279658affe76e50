// ACA on device-evaluated rows and columns, and H-matrix assembly.
//
// Section 4 of the paper gives every admissible block to one CPU thread that
// runs ACA and sends each row and column it needs to the GPU.  Here a small
// pool of worker threads each keeps several blocks in flight as resumable
// ACA state machines: a worker submits the next row or column request of
// every block it holds to the request server, and while those requests run
// (fused with the other workers' requests) it consumes finished ones, so
// the device sees large batches of uneven requests while pivoting and
// residual updates stay on the host in FP64.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <complex>
#include <chrono>
#include <deque>
#include <type_traits>
#include <thread>
#include <memory>
#include <mutex>
#include <new>
#include <sys/mman.h>
#include <unistd.h>

#include "aca.hpp"
#include <unordered_map>
#include "bem_internal.hpp"
#include "tree.hpp"

using cd = std::complex<double>;

namespace bem {

// Factor and dense-block values live in large blocks bump-allocated per
// worker instead of three heap vectors per leaf: assembly makes no
// allocator call per block, and destroying an H-matrix (or running a plan
// again) hands its blocks back to a process-wide pool, which keeps them up
// to an eighth of physical memory (at least 1 GiB): repeated assemblies and
// plan runs then reuse memory that is already mapped instead of faulting in
// and zeroing new pages (a run over a quarter of the 1M-triangle cylinder's
// blocks holds ~6 GB of FP64 factors).
constexpr size_t kPoolDoubles = size_t(1) << 19;   // 4 MiB per block

size_t pool_keep_blocks()
{
    static const size_t keep = [] {
        const long pages = sysconf(_SC_PHYS_PAGES), psz = sysconf(_SC_PAGE_SIZE);
        const double eighth = pages > 0 && psz > 0 ? (double)pages * (double)psz / 8.0 : 0.0;
        return std::max<size_t>(256, (size_t)(eighth / (double)(kPoolDoubles * sizeof(double))));
    }();
    return keep;
}

struct ValueBlock {
    double *p = nullptr;
    size_t n = 0;   // doubles; kPoolDoubles for pooled blocks
};

class ValuePool {
public:
    ValueBlock take(size_t n)
    {
        if (n <= kPoolDoubles) {
            {
                std::lock_guard<std::mutex> g(mu_);
                if (!free_.empty()) {
                    double *p = free_.back();
                    free_.pop_back();
                    return {p, kPoolDoubles};
                }
            }
            void *p = std::aligned_alloc(size_t(1) << 21, kPoolDoubles * sizeof(double));
            if (!p) throw std::bad_alloc();
            (void)madvise(p, kPoolDoubles * sizeof(double), MADV_HUGEPAGE);
            return {static_cast<double *>(p), kPoolDoubles};
        }
        return {new double[n], n};
    }
    void give(std::vector<ValueBlock> &v)
    {
        std::lock_guard<std::mutex> g(mu_);
        for (const ValueBlock &b : v) {
            if (b.n == kPoolDoubles && free_.size() < pool_keep_blocks())
                free_.push_back(b.p);
            else if (b.n == kPoolDoubles)
                std::free(b.p);
            else
                delete[] b.p;
        }
        v.clear();
    }

private:
    std::mutex mu_;
    std::vector<double *> free_;
};

ValuePool &value_pool()
{
    static ValuePool *pool = new ValuePool();   // never destroyed: outlives every H-matrix
    return *pool;
}

// One worker's bump allocator over pool blocks.
struct ValueArena {
    std::vector<ValueBlock> blocks;
    double *cur = nullptr;
    size_t left = 0;
    double *take(size_t n)
    {
        if (n > left || !cur) {   // a block always exists, so pointers are never null
            const ValueBlock b = value_pool().take(n);
            blocks.push_back(b);
            cur = b.p;
            left = b.n;
        }
        double *p = cur;
        cur += n;
        left -= n;
        return p;
    }
};

}  // namespace bem

struct bem_hmat {
    int op = 0, space = 0;
    bool cplx = false;
    int64_t ndof = 0;
    bem::Partition part;
    struct Leaf {
        int adm = 0;
        int rank = 0;
        int64_t r0 = 0, m = 0, c0 = 0, n = 0;   // rows part.perm[r0, r0 + m), columns part.perm[c0, c0 + n)
        const double *U = nullptr, *V = nullptr, *D = nullptr;   // complex values interleaved
    };
    std::vector<Leaf> leaves;
    std::vector<bem::ValueBlock> store;   // owns the values the leaves point to
    bem_hmat_stats st{};
    // Hypersingular operator through the single layer on DP1 (Eq.
    // hyp_via_slp): `inner` is that single layer's H-matrix; per triangle t
    // the curls of its three hat functions (curl[9 t + 3 a + j]) and its unit
    // normal (normal[3 t + j]) give the sparse factors Q_j and P_j.
    bem_hmat *inner = nullptr;
    std::vector<int32_t> tri;
    std::vector<double> curl, normal;
    double k = 0.0;
    const int32_t *rows(const Leaf &L) const { return part.perm.data() + L.r0; }
    const int32_t *cols(const Leaf &L) const { return part.perm.data() + L.c0; }
    ~bem_hmat()
    {
        bem::value_pool().give(store);
        delete inner;
    }
};

namespace bem {

namespace {

double vanish_scale(const bem_mesh &m, int op, int space, double k, double dist)
{
    const double d = dist > 0.0 ? dist : m.mean_edge;
    // (integral of a basis function)^2 ~ J^2 times (1/2)^2 for P0 (a triangle),
    // 1 for P1 (a star of ~6 triangles, 1/3 each), (1/6)^2 for DP1
    const double J2 = m.mean_J * m.mean_J * (space == BEM_P0 ? 0.25 : (space == BEM_P1 ? 1.0 : 1.0 / 36.0));
    const double inv4pi = 0.0795774715459476678844418816862571;
    if (op == BEM_LAPLACE_SLP || op == BEM_HELMHOLTZ_SLP) return J2 * inv4pi / d;
    if (op == BEM_LAPLACE_HYPS || op == BEM_HELMHOLTZ_HYPS)   // second derivatives of g, plus the k^2 term
        return J2 * inv4pi * (1.0 / (d * d * d) + k * k / d);
    const bool helm_dl = op == BEM_HELMHOLTZ_DLP || op == BEM_HELMHOLTZ_ADLP;
    return J2 * inv4pi * (1.0 + (helm_dl ? k * d : 0.0)) / (d * d);
}

double default_zero_abs(const bem_mesh &m, int op, int space, double k, int prec, double dist)
{
    return (prec == BEM_FP32 ? 1e-6 : 1e-12) * vanish_scale(m, op, space, k, dist);
}

// support box of a dof list
void support_box(const bem_mesh &m, int space, const int32_t *dofs, int64_t n, double *lo, double *hi)
{
    for (int d = 0; d < 3; ++d) {
        lo[d] = INFINITY;
        hi[d] = -INFINITY;
    }
    auto add_tri = [&](int64_t t) {
        for (int k = 0; k < 3; ++k)
            for (int d = 0; d < 3; ++d) {
                const double x = m.xyz[3 * m.tri[3 * t + k] + d];
                lo[d] = std::min(lo[d], x);
                hi[d] = std::max(hi[d], x);
            }
    };
    for (int64_t i = 0; i < n; ++i) {
        if (space == BEM_P0) {
            add_tri(dofs[i]);
        } else if (space == BEM_DP1) {
            add_tri(dofs[i] / 3);
        } else {
            for (int64_t s = m.star_ptr[dofs[i]]; s < m.star_ptr[dofs[i] + 1]; ++s) add_tri(m.star[s] >> 2);
        }
    }
}

double box_distance(const double *alo, const double *ahi, const double *blo, const double *bhi)
{
    double g[3];
    for (int k = 0; k < 3; ++k) g[k] = std::max(0.0, std::max(alo[k] - bhi[k], blo[k] - ahi[k]));
    return std::sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
}

template <typename T>
void to_scalar(const void *src, int prec, int64_t n, T *dst);

template <>
void to_scalar<double>(const void *src, int prec, int64_t n, double *dst)
{
    if (prec == BEM_FP32) {
        const float *s = (const float *)src;
        for (int64_t i = 0; i < n; ++i) dst[i] = s[i];
    } else {
        std::memcpy(dst, src, sizeof(double) * n);
    }
}

template <>
void to_scalar<cd>(const void *src, int prec, int64_t n, cd *dst)
{
    if (prec == BEM_FP32) {
        const float *s = (const float *)src;
        for (int64_t i = 0; i < n; ++i) dst[i] = cd(s[2 * i], s[2 * i + 1]);
    } else {
        const double *s = (const double *)src;
        for (int64_t i = 0; i < n; ++i) dst[i] = cd(s[2 * i], s[2 * i + 1]);
    }
}

template <typename T>
void store_cols(const AcaBuf<T> &src, int k, int64_t len, int64_t cap, void *dst);

template <>
void store_cols<double>(const AcaBuf<double> &src, int k, int64_t len, int64_t cap, void *dst)
{
    (void)cap;
    std::memcpy(dst, src.data(), sizeof(double) * len * k);
}

template <>
void store_cols<cd>(const AcaBuf<cd> &src, int k, int64_t len, int64_t cap, void *dst)
{
    (void)cap;
    std::memcpy(dst, src.data(), sizeof(cd) * len * k);
}

// Feeds a device result (FP32 or FP64 entries, real or complex) to the ACA
// state machine without an intermediate FP64 copy.
template <typename T>
void aca_consume(AcaCore<T> &core, const void *p, int prec)
{
    const bool row = core.phase == AcaCore<T>::NEED_ROW;
    if constexpr (std::is_same<T, double>::value) {
        if (prec == BEM_FP32) {
            if (row) core.consume_row(static_cast<const float *>(p));
            else core.consume_col(static_cast<const float *>(p));
        } else {
            if (row) core.consume_row(static_cast<const double *>(p));
            else core.consume_col(static_cast<const double *>(p));
        }
    } else {
        if (prec == BEM_FP32) {
            if (row) core.consume_row(static_cast<const std::complex<float> *>(p));
            else core.consume_col(static_cast<const std::complex<float> *>(p));
        } else {
            if (row) core.consume_row(static_cast<const cd *>(p));
            else core.consume_col(static_cast<const cd *>(p));
        }
    }
}

// Lane sets of several dof lists, expanded on the host (in parallel) and
// uploaded to the device in one buffer.
struct ResidentLanes {
    int32_t *dev = nullptr;
    float *geo = nullptr;              // FP32 records gathered per lane position, all sets
    int4 *meta = nullptr;              // their vertex ids
    std::vector<LaneRef> refs;
    std::vector<int32_t> chunk_host;   // chunk tables of all sets, host copies
    ResidentLanes() = default;
    ResidentLanes(const ResidentLanes &) = delete;
    ~ResidentLanes()
    {
        if (dev) (void)hipFree(dev);
        if (geo) (void)hipFree(geo);
        if (meta) (void)hipFree(meta);
    }
};

int make_resident(const bem_mesh &m, int space, const std::vector<std::pair<const int32_t *, int64_t>> &lists,
                  ResidentLanes &out)
{
    const size_t n = lists.size();
    std::vector<LaneSet> sets(n);
    const unsigned nth = std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nth; ++t)
        th.emplace_back([&, t] {
            for (size_t i = t; i < n; i += nth)
                if (lists[i].first) build_lane_set(m, space, lists[i].first, lists[i].second, sets[i]);
        });
    for (auto &x : th) x.join();
    // one int32 buffer: per set, the chunk table (16-byte aligned int4
    // records), lanes, segment pointers and segments
    auto pad4 = [](size_t x) { return (x + 3) & ~(size_t)3; };
    size_t total = 0;
    for (auto &ls : sets) total += pad4(ls.ints());
    std::vector<int32_t> host(std::max<size_t>(total, 4));
    out.refs.assign(n, LaneRef());
    std::vector<size_t> at(n);
    size_t pos = 0;
    for (size_t i = 0; i < n; ++i) {
        at[i] = pos;
        const LaneSet &ls = sets[i];
        for (const std::vector<int32_t> *v : {&ls.chunk, &ls.lane, &ls.seg_ptr, &ls.seg}) {
            std::copy(v->begin(), v->end(), host.begin() + pos);
            pos += v->size();
        }
        pos = pad4(pos);
    }
    std::vector<size_t> ch_at(n);
    size_t nch = 0;
    for (size_t i = 0; i < n; ++i) {
        ch_at[i] = nch;
        nch += sets[i].chunk.size();
    }
    out.chunk_host.resize(std::max<size_t>(nch, 1));
    for (size_t i = 0; i < n; ++i) std::copy(sets[i].chunk.begin(), sets[i].chunk.end(), out.chunk_host.begin() + ch_at[i]);
    BEM_HIP_TRY(hipMalloc(&out.dev, sizeof(int32_t) * host.size()));
    BEM_HIP_TRY(hipMemcpy(out.dev, host.data(), sizeof(int32_t) * host.size(), hipMemcpyHostToDevice));
    // lane records gathered once, so the entry kernels read a lane's
    // geometry without going through its triangle index
    std::vector<size_t> lane_at(n);
    size_t nl = 0;
    for (size_t i = 0; i < n; ++i) {
        lane_at[i] = nl;
        nl += sets[i].lane.size();
    }
    if (nl > 0) {
        std::vector<int32_t> idx(nl);
        for (size_t i = 0; i < n; ++i) std::copy(sets[i].lane.begin(), sets[i].lane.end(), idx.begin() + lane_at[i]);
        int32_t *d_idx = nullptr;
        BEM_HIP_TRY(hipMalloc(&d_idx, sizeof(int32_t) * nl));
        hipError_t e = hipMemcpy(d_idx, idx.data(), sizeof(int32_t) * nl, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMalloc(&out.geo, sizeof(float) * kGeo32Stride * nl);
        if (e == hipSuccess) e = hipMalloc(&out.meta, sizeof(int4) * nl);
        if (e == hipSuccess) e = launch_gather(m.d_g32, m.d_vtx, d_idx, 0, (int64_t)nl, out.geo, out.meta, 0);
        if (e == hipSuccess) e = hipStreamSynchronize(0);
        (void)hipFree(d_idx);
        if (e != hipSuccess)
            return fail(e == hipErrorOutOfMemory ? BEM_E_OOM : BEM_E_DEVICE,
                        std::string("lane records: ") + hipGetErrorString(e));
    }
    for (size_t i = 0; i < n; ++i) {
        const LaneSet &ls = sets[i];
        LaneRef &r = out.refs[i];
        const int32_t *base = out.dev + at[i];
        r.ndof = ls.ndof;
        r.nlane = (int64_t)ls.lane.size();
        r.nseg = (int64_t)ls.seg.size();
        r.nchunk = ls.nchunk();
        r.ndistinct = ls.ndistinct;
        r.chunk = ls.chunk.empty() ? nullptr : reinterpret_cast<const int4 *>(base);
        r.chunk_host = out.chunk_host.data() + ch_at[i];
        const bool has = out.geo && !ls.lane.empty();
        r.geo = has ? out.geo + kGeo32Stride * lane_at[i] : nullptr;
        r.meta = has ? out.meta + lane_at[i] : nullptr;
        base += ls.chunk.size();
        r.lane = ls.lane.empty() ? nullptr : base;
        base += ls.lane.size();
        r.seg_ptr = ls.seg_ptr.empty() ? nullptr : base;
        base += ls.seg_ptr.size();
        r.seg = ls.seg.empty() ? nullptr : base;
    }
    return BEM_OK;
}

// Completion queue of one worker.  The worker spins briefly before it
// sleeps, so a completion that arrives within the spin window costs the
// completion thread no wake-up call.
struct DoneQueue {
    std::mutex mu;
    std::condition_variable cv;
    std::vector<Request *> q;
    std::atomic<int> ready{0};
    bool sleeping = false;   // guarded by mu
    double spin_s = 0.0;
    static void push(Request **rs, size_t n, void *ctx)
    {
        DoneQueue *d = (DoneQueue *)ctx;
        bool wake;
        {
            std::lock_guard<std::mutex> g(d->mu);
            d->q.insert(d->q.end(), rs, rs + n);
            d->ready.store(1, std::memory_order_release);
            wake = d->sleeping;
        }
        if (wake) d->cv.notify_one();
    }
    // Up to `most` finished requests, oldest first.
    void pop_some(std::vector<Request *> &out, size_t most)
    {
        if (spin_s > 0.0 && !ready.load(std::memory_order_acquire)) {
            const double t0 = now_seconds();
            int it = 0;
            while (!ready.load(std::memory_order_acquire)) {
                __builtin_ia32_pause();
                if ((++it & 63) == 0 && now_seconds() - t0 > spin_s) break;
            }
        }
        std::unique_lock<std::mutex> lk(mu);
        sleeping = true;
        cv.wait(lk, [&] { return !q.empty(); });
        sleeping = false;
        if (q.size() <= most) {
            out.swap(q);
            q.clear();
        } else {
            out.assign(q.begin(), q.begin() + most);
            q.erase(q.begin(), q.begin() + most);
        }
        ready.store(q.empty() ? 0 : 1, std::memory_order_relaxed);
    }
};

struct AssemblyCtx;

struct Job {
    int64_t leaf;
    int adm;
    AssemblyCtx *plan = nullptr;   // the block's plan context (null: the run's own context)
};

template <typename T>
struct Slot {
    int64_t leaf = -1;
    bool adm = false;
    AssemblyCtx *P = nullptr;   // context of the block's plan (operator, mesh, H-matrix, lane sets)
    int arena = 0;              // the worker's value arena for that plan
    double t_start = 0.0;
    AcaCore<T> core;
    Request req;
    std::vector<T> buf;
    bool busy = false;
};

struct AssemblyCtx {
    bem_mesh *mesh;
    int op, space, prec;
    double k, tol;
    int max_rank;
    bem_hmat *h;
    const std::vector<LaneRef> *lanes;  // per cluster id
    int dense_near = BEM_NEAR_SKIP;      // near-field policy of the dense leaves
    std::vector<Job> jobs;
    const double *arrival = nullptr;     // per job: earliest start, seconds after t0 (null: all at t0)
    double t0 = 0.0;
    std::atomic<int64_t> next{0};
    std::atomic<int> error{0};
    std::mutex err_mu;
    std::string err_msg;
    std::atomic<int64_t> aca_entries{0}, dense_entries{0}, requests{0};
    std::mutex busy_mu;
    double busy = 0.0;
    double qdelay = 0.0, proc = 0.0;   // completion -> pickup, pickup -> resubmit (summed over requests)
    int64_t nproc = 0;
    double t_conv = 0.0, t_aca = 0.0, t_rel = 0.0, t_prep = 0.0, t_flush = 0.0;   // worker phases (summed)
    double start_delay = 0.0, block_time = 0.0;   // arrival -> start, start -> done (summed over blocks)
    int64_t blocks_done = 0;

    void set_error(int code, const std::string &msg)
    {
        std::lock_guard<std::mutex> g(err_mu);
        if (!error.load()) {
            error = code;
            err_msg = msg;
        }
    }
};

// Spin window of an idle worker before it sleeps (BEM_WORKER_SPIN_US,
// microseconds; default 0: sleep at once).
double worker_spin_seconds()
{
    static const double v = [] {
        const char *e = std::getenv("BEM_WORKER_SPIN_US");
        return 1e-6 * (e ? std::max(0.0, std::atof(e)) : 0.0);
    }();
    return v;
}

// Finished requests a worker takes at once (BEM_WORKER_POP, default 128) and
// the number of follow-up requests after which it submits them without
// waiting for the rest of what it took (BEM_WORKER_FLUSH, default 128).
// Smaller flushes shorten a block's wait between requests but hand the
// dispatcher smaller batches and reserve room in the open batch more often;
// on the icosphere assemblies they were slower, and on the served cylinder
// 64/64 against 128/128 held batches longer between their closing and their
// launch (55-68 against 35 µs) with p50 0.16-0.18 against 0.13 ms.
int worker_env(const char *name, int def)
{
    const char *e = std::getenv(name);
    return e ? std::max(1, std::atoi(e)) : def;
}

// Per-worker tallies, added to the assembly's totals when the worker ends.
struct WorkerTally {
    int64_t aca_entries = 0, dense_entries = 0, requests = 0;
};

template <typename T>
int prepare_slot(AssemblyCtx &C, Slot<T> &s, DoneQueue &dq, int64_t tag, WorkerTally &w)
{
    bem_hmat::Leaf &L = C.h->leaves[s.leaf];
    Request &r = s.req;
    r.mesh = C.mesh;
    r.op = C.op;
    r.space = C.space;
    r.prec = C.prec;
    r.k = C.k;
    r.borrow = true;
    r.out_host = nullptr;
    r.on_done = &DoneQueue::push;
    r.cb_ctx = &dq;
    r.tag = tag;
    if (!s.adm) {
        r.near = C.dense_near;
        r.separated = false;
        r.rows.assign(C.h->rows(L), C.h->rows(L) + L.m);
        r.cols.assign(C.h->cols(L), C.h->cols(L) + L.n);
        r.nrows = (int64_t)r.rows.size();
        r.ncols = (int64_t)r.cols.size();
        if (r.near == BEM_NEAR_SINGULAR) {
            // triangles sharing a vertex both contain it, so leaves whose support
            // boxes are apart have no singular pairs: skip the search for them
            double alo[3], ahi[3], blo[3], bhi[3];
            support_box(*C.mesh, C.space, r.rows.data(), r.nrows, alo, ahi);
            support_box(*C.mesh, C.space, r.cols.data(), r.ncols, blo, bhi);
            if (box_distance(alo, ahi, blo, bhi) > 0.0) r.near = BEM_NEAR_SKIP;
        }
        const int rc = expand_request(r);
        if (rc != BEM_OK) return rc;
        w.dense_entries += r.entries();
    } else {
        r.near = BEM_NEAR_ERROR;
        // admissible: the support boxes of the two clusters are apart, so no
        // triangle of one shares a vertex with a triangle of the other
        r.separated = true;
        const Block &bk = C.h->part.blocks[s.leaf];
        if (s.core.phase == AcaCore<T>::NEED_ROW)
            expand_single_fixed(r, C.h->rows(L)[s.core.i], 1, &(*C.lanes)[bk.sigma]);
        else
            expand_single_fixed(r, C.h->cols(L)[s.core.j], 0, &(*C.lanes)[bk.tau]);
        w.aca_entries += r.entries();
    }
    w.requests += 1;
    return BEM_OK;
}

template <typename T>
void worker(AssemblyCtx &C, int per_worker)
{
    DoneQueue dq;
    dq.spin_s = worker_spin_seconds();
    static const int pop_most = worker_env("BEM_WORKER_POP", 128);
    static const int flush_every = worker_env("BEM_WORKER_FLUSH", 128);
    // per-request phase timers (a clock read costs tens of nanoseconds, a
    // noticeable share of a request's host work): only with BEM_DEBUG_TIMING
    static const bool fine = std::getenv("BEM_DEBUG_TIMING") != nullptr;
    WorkerTally tally;
    // values of the blocks this worker finishes, one arena per plan (a run
    // over several plans hands each plan's values to its own H-matrix)
    std::vector<std::pair<AssemblyCtx *, ValueArena>> arenas;
    auto arena_of = [&](AssemblyCtx *P) -> int {
        for (size_t i = 0; i < arenas.size(); ++i)
            if (arenas[i].first == P) return (int)i;
        arenas.emplace_back(P, ValueArena());
        return (int)arenas.size() - 1;
    };
    std::vector<Slot<T>> slots(per_worker);
    std::vector<Request *> submit, done;
    int active = 0;
    // borrowed results go back once per run of requests from the same batch
    void *rel_batch = nullptr;
    int rel_n = 0;
    auto release_run = [&]() {
        server_release_batch(rel_batch, rel_n);
        rel_batch = nullptr;
        rel_n = 0;
    };
    bool exhausted = false;
    double start_delay = 0.0, block_time = 0.0;
    int64_t blocks_done = 0;
    const int64_t njobs = (int64_t)C.jobs.size();
    // Takes the next job into slot si if it has arrived: 1 started, 0 the next
    // job has not arrived yet, -1 none left (or an error).
    auto start_job = [&](int64_t si) -> int {
        Slot<T> &s = slots[si];
        if (exhausted || C.error.load()) return -1;
        int64_t j = C.next.load(std::memory_order_relaxed);
        double t = 0.0;
        for (;;) {
            if (j >= njobs) {
                exhausted = true;
                return -1;
            }
            if (C.arrival) {
                t = now_seconds();
                if (C.t0 + C.arrival[j] > t) return 0;
            }
            if (C.next.compare_exchange_weak(j, j + 1)) break;
        }
        if (C.arrival) start_delay += t - (C.t0 + C.arrival[j]);
        s.leaf = C.jobs[j].leaf;
        s.adm = C.jobs[j].adm != 0;
        s.P = C.jobs[j].plan ? C.jobs[j].plan : &C;
        s.arena = arena_of(s.P);
        s.t_start = now_seconds();
        if (s.adm) {
            const AssemblyCtx &P = *s.P;
            const bem_hmat::Leaf &L = P.h->leaves[s.leaf];
            const Block &bk = P.h->part.blocks[s.leaf];
            const Cluster &a = P.h->part.nodes[bk.tau];
            const Cluster &b = P.h->part.nodes[bk.sigma];
            s.core.init(L.m, L.n, P.tol, P.max_rank,
                        default_zero_abs(*P.mesh, P.op, P.space, P.k, P.prec, support_distance(a, b)));
        }
        const int rc = prepare_slot(*s.P, s, dq, si, tally);
        if (rc != BEM_OK) {
            C.set_error(rc, std::string("request: ") + bem_last_error());
            return -1;
        }
        s.busy = true;
        ++active;
        submit.push_back(&s.req);
        return 1;
    };
    // free slots, lowest index on top
    std::vector<int64_t> free_slots;
    for (int64_t si = per_worker - 1; si >= 0; --si) free_slots.push_back(si);
    auto fill = [&]() {
        while (!free_slots.empty()) {
            if (start_job(free_slots.back()) <= 0) break;
            free_slots.pop_back();
        }
    };
    auto flush = [&]() {
        if (submit.empty()) return;
        const int rc = server_submit_many(submit.data(), submit.size());
        if (rc != BEM_OK) {
            C.set_error(rc, std::string("submit: ") + bem_last_error());
            // nothing was queued: these requests will never complete
            for (Request *r : submit) {
                slots[r->tag].busy = false;
                --active;
                free_slots.push_back(r->tag);
            }
        }
        submit.clear();
    };
    double busy = 0.0, qd = 0.0, pr = 0.0;
    double tc = 0.0, ta = 0.0, tr = 0.0, tp = 0.0, tf = 0.0;
    int64_t np = 0;
    double tb = now_seconds();
    fill();
    flush();
    for (;;) {
        if (active == 0) {
            if (exhausted || C.error.load()) break;
            // nothing in flight and the next block has not arrived: sleep until
            // it does (in short steps, so an error elsewhere is seen soon)
            const int64_t j = C.next.load();
            if (j < njobs && C.arrival) {
                const double wait = C.t0 + C.arrival[j] - now_seconds();
                if (wait > 0.0) {
                    busy += now_seconds() - tb;
                    std::this_thread::sleep_for(std::chrono::duration<double>(std::min(wait, 2e-4)));
                    tb = now_seconds();
                }
            }
            fill();
            flush();
            continue;
        }
        busy += now_seconds() - tb;
        dq.pop_some(done, (size_t)pop_most);
        tb = now_seconds();
        if (fine)
            for (Request *r : done) qd += tb - server_request_done_time(r);
        np += (int64_t)done.size();
        for (size_t di = 0; di < done.size(); ++di) {
            Request *r = done[di];
            if (di + 2 < done.size()) {
                // the entries of a request two ahead were written by the device
                // and are not in this core's cache: start their loads now
                const Request *nx = done[di + 2];
                if (const char *res = static_cast<const char *>(nx->result)) {
                    __builtin_prefetch(res);
                    __builtin_prefetch(res + 64);
                    __builtin_prefetch(res + 128);
                    __builtin_prefetch(res + 192);
                }
                __builtin_prefetch(&slots[nx->tag]);
            }
            if ((int)submit.size() >= flush_every) {
                const double f0 = fine ? now_seconds() : 0.0;
                flush();
                if (fine) tf += now_seconds() - f0;
            }
            Slot<T> &s = slots[r->tag];
            bool finished = false;
            const int rst = server_request_status(r);
            if (rst != BEM_OK) {
                C.set_error(rst, rst == BEM_E_NEARFIELD ? "admissible block met a vertex-sharing pair"
                                                        : "device request failed");
                finished = true;
            } else {
                AssemblyCtx &P = *s.P;
                ValueArena &arena = arenas[s.arena].second;
                bem_hmat::Leaf &L = P.h->leaves[s.leaf];
                const int64_t cnt = r->entries();
                if (!s.adm) {
                    const double c0 = fine ? now_seconds() : 0.0;
                    s.buf.resize(cnt);
                    to_scalar<T>(r->result, P.prec, cnt, s.buf.data());
                    if (fine) tc += now_seconds() - c0;
                    double *D = arena.take((size_t)cnt * (sizeof(T) / sizeof(double)));
                    std::memcpy(D, s.buf.data(), sizeof(T) * cnt);
                    L.D = D;
                    finished = true;
                } else {
                    const double a0 = fine ? now_seconds() : 0.0;
                    aca_consume(s.core, r->result, P.prec);
                    if (fine) ta += now_seconds() - a0;
                    if (s.core.phase == AcaCore<T>::DONE) {
                        L.rank = s.core.k;
                        const size_t f = sizeof(T) / sizeof(double);
                        double *U = arena.take(s.core.U.size() * f);
                        double *V = arena.take(s.core.V.size() * f);
                        std::memcpy(U, s.core.U.data(), sizeof(T) * s.core.U.size());
                        std::memcpy(V, s.core.V.data(), sizeof(T) * s.core.V.size());
                        L.U = U;
                        L.V = V;
                        finished = true;
                    }
                }
            }
            if (r->batch) {
                const double c1 = fine ? now_seconds() : 0.0;
                if (r->batch != rel_batch) {
                    release_run();
                    rel_batch = r->batch;
                }
                ++rel_n;
                r->batch = nullptr;
                r->result = nullptr;
                if (fine) tr += now_seconds() - c1;
            }
            if (finished || C.error.load()) {
                s.busy = false;
                --active;
                block_time += now_seconds() - s.t_start;
                ++blocks_done;
                free_slots.push_back(r->tag);
                if (!C.error.load()) fill();
                continue;
            }
            const double p0 = fine ? now_seconds() : 0.0;
            const int rc = prepare_slot(*s.P, s, dq, r->tag, tally);
            if (fine) tp += now_seconds() - p0;
            if (rc != BEM_OK) {
                C.set_error(rc, std::string("request: ") + bem_last_error());
                s.busy = false;
                --active;
                free_slots.push_back(r->tag);
                continue;
            }
            submit.push_back(&s.req);
        }
        release_run();
        const size_t nd = done.size();
        done.clear();
        fill();   // blocks that arrived meanwhile
        const double f0 = fine ? now_seconds() : 0.0;
        flush();
        if (fine) {
            const double f1 = now_seconds();
            tf += f1 - f0;
            pr += (f1 - tb) * (double)nd;
        }
    }
    busy += now_seconds() - tb;
    release_run();
    C.aca_entries.fetch_add(tally.aca_entries);
    C.dense_entries.fetch_add(tally.dense_entries);
    C.requests.fetch_add(tally.requests);
    std::lock_guard<std::mutex> g(C.busy_mu);
    for (auto &pa : arenas) pa.first->h->store.insert(pa.first->h->store.end(), pa.second.blocks.begin(),
                                                      pa.second.blocks.end());
    C.busy += busy;
    C.qdelay += qd;
    C.proc += pr;
    C.nproc += np;
    C.t_conv += tc;
    C.t_aca += ta;
    C.t_rel += tr;
    C.t_prep += tp;
    C.t_flush += tf;
    C.start_delay += start_delay;
    C.block_time += block_time;
    C.blocks_done += blocks_done;
}

template <typename T>
int aca_block_impl(bem_mesh *mesh, int op, int space, double k, const int32_t *rows, int64_t m, const int32_t *cols,
                   int64_t n, const bem_aca_params *p, int prec, void *U, void *V, int32_t *rank, int64_t *entries)
{
    {
        Request probe;
        probe.mesh = mesh;
        probe.op = op;
        probe.space = space;
        probe.prec = prec;
        probe.k = k;
        probe.near = BEM_NEAR_ERROR;
        probe.rows.assign(rows, rows + m);
        probe.cols.assign(cols, cols + n);
        probe.nrows = 0;
        probe.ncols = 0;
        const int rc = expand_request(probe);  // validates indices, op, k
        if (rc != BEM_OK) return rc;
    }
    double zero_abs = p->zero_abs;
    if (zero_abs < 0) {
        double alo[3], ahi[3], blo[3], bhi[3];
        support_box(*mesh, space, rows, m, alo, ahi);
        support_box(*mesh, space, cols, n, blo, bhi);
        zero_abs = default_zero_abs(*mesh, op, space, k, prec, box_distance(alo, ahi, blo, bhi));
    }
    ResidentLanes lanes;
    int rc = make_resident(*mesh, space, {{rows, m}, {cols, n}}, lanes);
    if (rc != BEM_OK) return rc;
    AcaCore<T> core;
    core.init(m, n, p->tol, p->max_rank, zero_abs);
    Request r;
    std::vector<char> out;
    std::vector<T> buf;
    int64_t count = 0;
    while (core.phase != AcaCore<T>::DONE) {
        r.mesh = mesh;
        r.op = op;
        r.space = space;
        r.prec = prec;
        r.k = k;
        r.near = BEM_NEAR_ERROR;
        if (core.phase == AcaCore<T>::NEED_ROW)
            expand_single_fixed(r, rows[core.i], 1, &lanes.refs[1]);
        else
            expand_single_fixed(r, cols[core.j], 0, &lanes.refs[0]);
        out.resize((size_t)r.entries() * r.elem_bytes);
        r.out_host = out.data();
        r.on_done = nullptr;
        rc = server_submit(&r);
        if (rc != BEM_OK) return rc;
        rc = server_wait(&r, -1.0);
        if (rc != BEM_OK) return rc == BEM_E_NEARFIELD ? fail(rc, "block contains a vertex-sharing pair") : rc;
        count += r.entries();
        aca_consume(core, out.data(), prec);
    }
    store_cols<T>(core.U, core.k, m, p->max_rank, U);
    store_cols<T>(core.V, core.k, n, p->max_rank, V);
    *rank = core.k;
    if (entries) *entries = count;
    return BEM_OK;
}

}  // namespace

int aca_block(bem_mesh *mesh, int op, int space, double k, const int32_t *rows, int64_t m, const int32_t *cols,
              int64_t n, const bem_aca_params *p, int prec, void *U, void *V, int32_t *rank, int64_t *entries)
{
    if (!mesh || !p || !U || !V || !rank) return fail(BEM_E_ARG, "null argument");
    if (m <= 0 || n <= 0 || (m > 0 && !rows) || (n > 0 && !cols)) return fail(BEM_E_ARG, "empty block");
    if (p->max_rank < 1 || !(p->tol >= 0.0)) return fail(BEM_E_ARG, "bad ACA parameters");
    if (is_complex_op(op))
        return aca_block_impl<cd>(mesh, op, space, k, rows, m, cols, n, p, prec, U, V, rank, entries);
    return aca_block_impl<double>(mesh, op, space, k, rows, m, cols, n, p, prec, U, V, rank, entries);
}

int aca_callback(int64_t m, int64_t n, int is_complex, bem_row_fn get_row, bem_col_fn get_col, void *ctx,
                 const bem_aca_params *p, void *U, void *V, int32_t *rank)
{
    if (!get_row || !get_col || !p || !U || !V || !rank || m <= 0 || n <= 0 || p->max_rank < 1)
        return fail(BEM_E_ARG, "bad ACA arguments");
    const double zero_abs = p->zero_abs < 0 ? 0.0 : p->zero_abs;
    if (is_complex) {
        AcaCore<cd> core;
        core.init(m, n, p->tol, p->max_rank, zero_abs);
        std::vector<cd> buf;
        while (core.phase != AcaCore<cd>::DONE) {
            if (core.phase == AcaCore<cd>::NEED_ROW) {
                buf.assign(n, cd(0));
                get_row(ctx, core.i, reinterpret_cast<double *>(buf.data()));
                core.consume_row(buf.data());
            } else {
                buf.assign(m, cd(0));
                get_col(ctx, core.j, reinterpret_cast<double *>(buf.data()));
                core.consume_col(buf.data());
            }
        }
        store_cols<cd>(core.U, core.k, m, p->max_rank, U);
        store_cols<cd>(core.V, core.k, n, p->max_rank, V);
        *rank = core.k;
    } else {
        AcaCore<double> core;
        core.init(m, n, p->tol, p->max_rank, zero_abs);
        std::vector<double> buf;
        while (core.phase != AcaCore<double>::DONE) {
            if (core.phase == AcaCore<double>::NEED_ROW) {
                buf.assign(n, 0.0);
                get_row(ctx, core.i, buf.data());
                core.consume_row(buf.data());
            } else {
                buf.assign(m, 0.0);
                get_col(ctx, core.j, buf.data());
                core.consume_col(buf.data());
            }
        }
        store_cols<double>(core.U, core.k, m, p->max_rank, U);
        store_cols<double>(core.V, core.k, n, p->max_rank, V);
        *rank = core.k;
    }
    return BEM_OK;
}

int hmat_assemble(bem_mesh *mesh, int op, int space, double k, const bem_hmat_params *p, bem_hmat **out);

// Eq. hyp_via_slp: D = sum_j Q_j^T S Q_j - k^2 sum_j P_j^T S P_j, S the
// single layer (Laplace or Helmholtz) on DP1 assembled as an H-matrix with
// the same parameters, Q_j the j-th curl component of the hat functions
// (constant on a triangle, the same value on its three DP1 functions), P_j
// the hat functions times the j-th normal component.  On a flat triangle
// curl lambda_a = n x grad lambda_a = (v_{a+1} - v_{a+2}) / J.
int hmat_assemble_hyps_via_slp(bem_mesh *mesh, int op, double k, const bem_hmat_params *p, bem_hmat **out)
{
    bem_hmat_params q = *p;
    q.hyps_via_slp = 0;
    bem_hmat *S = nullptr;
    const int slp = op == BEM_LAPLACE_HYPS ? BEM_LAPLACE_SLP : BEM_HELMHOLTZ_SLP;
    const int rc = hmat_assemble(mesh, slp, BEM_DP1, k, &q, &S);
    if (rc != BEM_OK) return rc;
    bem_hmat *h = new bem_hmat();
    h->op = op;
    h->space = BEM_P1;
    h->cplx = is_complex_op(op);
    h->ndof = mesh->nv;
    h->inner = S;
    h->k = op == BEM_LAPLACE_HYPS ? 0.0 : k;
    h->tri = mesh->tri;
    const int64_t nt = mesh->nt;
    h->curl.resize(9 * (size_t)nt);
    h->normal.resize(3 * (size_t)nt);
    for (int64_t t = 0; t < nt; ++t) {
        const double *v[3];
        for (int a = 0; a < 3; ++a) v[a] = &mesh->xyz[3 * (size_t)mesh->tri[3 * t + a]];
        double e1[3], e2[3];
        for (int d = 0; d < 3; ++d) {
            e1[d] = v[1][d] - v[0][d];
            e2[d] = v[2][d] - v[0][d];
        }
        const double N[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        const double J = std::sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
        for (int d = 0; d < 3; ++d) h->normal[3 * t + d] = N[d] / J;
        for (int a = 0; a < 3; ++a)
            for (int d = 0; d < 3; ++d) h->curl[9 * t + 3 * a + d] = (v[(a + 1) % 3][d] - v[(a + 2) % 3][d]) / J;
    }
    h->st = S->st;
    h->st.ndof = mesh->nv;
    *out = h;
    return BEM_OK;
}

int hmat_assemble(bem_mesh *mesh, int op, int space, double k, const bem_hmat_params *p, bem_hmat **out)
{
    if (!mesh || !p || !out) return fail(BEM_E_ARG, "null argument");
    if (p->leaf_size < 1 || !(p->eta > 0) || p->max_rank < 1 || !(p->aca_tol >= 0) || p->dense_mode < 0 ||
        p->dense_mode > 2 || p->max_block < 0 || p->hyps_via_slp < 0 || p->hyps_via_slp > 1)
        return fail(BEM_E_ARG, "bad H-matrix parameters");
    if (p->hyps_via_slp && (op == BEM_LAPLACE_HYPS || op == BEM_HELMHOLTZ_HYPS)) {
        if (space != BEM_P1) return fail(BEM_E_ARG, "the hypersingular operator needs continuous (P1) functions");
        return hmat_assemble_hyps_via_slp(mesh, op, k, p, out);
    }
    {
        // validate op/k/space/prec once with an empty request
        Request probe;
        probe.mesh = mesh;
        probe.op = op;
        probe.space = space;
        probe.prec = p->prec;
        probe.k = k;
        probe.near = p->dense_mode == 2 ? BEM_NEAR_SINGULAR : BEM_NEAR_SKIP;
        const int rc = expand_request(probe);
        if (rc != BEM_OK) return rc;
    }
    const double t0 = now_seconds();
    bem_hmat *h = new bem_hmat();
    h->op = op;
    h->space = space;
    h->cplx = is_complex_op(op);
    h->ndof = space_ndof(*mesh, space);
    std::vector<double> pts, slo, shi;
    dof_geometry(*mesh, space, pts, slo, shi);
    build_partition(pts, slo, shi, p->leaf_size, p->eta, p->max_block, h->part);
    const double t_part = now_seconds();
    const auto &P = h->part;
    h->leaves.resize(P.blocks.size());
    AssemblyCtx C;
    C.mesh = mesh;
    C.op = op;
    C.space = space;
    C.prec = p->prec;
    C.k = k;
    C.tol = p->aca_tol;
    C.dense_near = p->dense_mode == 2 ? BEM_NEAR_SINGULAR : BEM_NEAR_SKIP;
    C.max_rank = p->max_rank;
    C.h = h;
    std::vector<std::pair<const int32_t *, int64_t>> lists(P.nodes.size(), {nullptr, 0});
    for (const Block &bk : P.blocks)
        if (bk.admissible)
            for (int cid : {bk.tau, bk.sigma}) {
                const Cluster &cl = P.nodes[cid];
                lists[cid] = {P.perm.data() + cl.begin, cl.end - cl.begin};
            }
    ResidentLanes lanes;
    {
        const int rc = make_resident(*mesh, space, lists, lanes);
        if (rc != BEM_OK) {
            delete h;
            return rc;
        }
    }
    C.lanes = &lanes.refs;
    for (size_t b = 0; b < P.blocks.size(); ++b) {
        const Cluster &a = P.nodes[P.blocks[b].tau], &c = P.nodes[P.blocks[b].sigma];
        auto &L = h->leaves[b];
        L.adm = P.blocks[b].admissible;
        L.r0 = a.begin;
        L.m = a.end - a.begin;
        L.c0 = c.begin;
        L.n = c.end - c.begin;
        if (L.adm || p->dense_mode >= 1) C.jobs.push_back(Job{(int64_t)b, L.adm});
    }
    // largest blocks first
    std::stable_sort(C.jobs.begin(), C.jobs.end(), [&](const Job &x, const Job &y) {
        const auto &a = h->leaves[x.leaf], &b = h->leaves[y.leaf];
        const int64_t cx = x.adm ? (a.m + a.n) * 16 : a.m * a.n;
        const int64_t cy = y.adm ? (b.m + b.n) * 16 : b.m * b.n;
        return cx > cy;
    });
    const double t_setup = now_seconds();
    const int nw = std::max(1, p->n_workers);
    const int per = std::max(1, p->blocks_per_worker);
    std::vector<std::thread> th;
    for (int w = 0; w < nw; ++w) {
        if (h->cplx)
            th.emplace_back([&] { worker<cd>(C, per); });
        else
            th.emplace_back([&] { worker<double>(C, per); });
    }
    for (auto &t : th) t.join();
    const double t_aca = now_seconds();
    if (C.error.load() != 0) {
        const int code = C.error.load();
        std::string msg = C.err_msg;
        delete h;
        return fail(code, "H-matrix assembly: " + msg);
    }
    bem_hmat_stats &s = h->st;
    s.ndof = h->ndof;
    s.aca_entries = C.aca_entries.load();
    s.dense_entries = C.dense_entries.load();
    s.aca_requests = C.requests.load();
    size_t bytes = 0;
    for (auto &L : h->leaves) {
        if (L.adm) {
            s.admissible_blocks++;
            s.rank_sum += L.rank;
            s.rank_max = std::max(s.rank_max, L.rank);
        } else {
            s.dense_blocks++;
        }
        const size_t f = h->cplx ? 2 : 1;
        if (L.adm)
            bytes += sizeof(double) * f * (size_t)L.rank * (size_t)(L.m + L.n);
        else if (L.D)
            bytes += sizeof(double) * f * (size_t)(L.m * L.n);
    }
    s.bytes = bytes;
    s.seconds = now_seconds() - t0;
    s.partition_seconds = t_part - t0;
    s.setup_seconds = t_setup - t_part;
    s.aca_seconds = t_aca - t_setup;
    s.worker_busy_seconds = C.busy;
    if (std::getenv("BEM_DEBUG_TIMING")) {
        const double np = (double)std::max<int64_t>(1, C.nproc);
        fprintf(stderr, "[bem] assembly %.3fs: partition %.3f setup %.3f aca %.3f; %lld completions, mean pickup delay %.1f us, mean batch-processing span %.1f us\n",
                s.seconds, s.partition_seconds, s.setup_seconds, s.aca_seconds, (long long)C.nproc,
                1e6 * C.qdelay / np, 1e6 * C.proc / np);
        fprintf(stderr, "[bem] worker us/request: busy %.3f convert %.3f aca %.3f release %.3f prepare %.3f submit %.3f\n",
                1e6 * C.busy / np, 1e6 * C.t_conv / np, 1e6 * C.t_aca / np, 1e6 * C.t_rel / np, 1e6 * C.t_prep / np,
                1e6 * C.t_flush / np);
        server_print_phases();
    }
    *out = h;
    return BEM_OK;
}

}  // namespace bem

// An ACA plan: the partition and resident lane sets of one operator on one
// mesh, kept between runs; the H-matrix object holds the leaves, whose
// factors are those of the last run.
struct bem_aca_plan {
    bem_mesh *mesh = nullptr;
    int op = 0, space = 0;
    double k = 0.0;
    bem_hmat_params p{};
    bem_hmat *h = nullptr;
    bem::ResidentLanes lanes;
    std::vector<int64_t> adm;       // leaf index of each plan block
    std::vector<int64_t> last;      // leaves of the last run
    double setup_seconds = 0.0;
    std::mutex run_mu;              // one run at a time
    ~bem_aca_plan() { delete h; }
};

namespace bem {

int plan_create(bem_mesh *mesh, int op, int space, double k, const bem_hmat_params *p, bem_aca_plan **out)
{
    if (!mesh || !p || !out) return fail(BEM_E_ARG, "null argument");
    if (p->leaf_size < 1 || !(p->eta > 0) || p->max_rank < 1 || !(p->aca_tol >= 0) || p->max_block < 0 ||
        p->n_workers < 1 || p->blocks_per_worker < 1)
        return fail(BEM_E_ARG, "bad plan parameters");
    {
        Request probe;
        probe.mesh = mesh;
        probe.op = op;
        probe.space = space;
        probe.prec = p->prec;
        probe.k = k;
        probe.near = BEM_NEAR_ERROR;
        const int rc = expand_request(probe);
        if (rc != BEM_OK) return rc;
    }
    const double t0 = now_seconds();
    bem_aca_plan *pl = new bem_aca_plan();
    pl->mesh = mesh;
    pl->op = op;
    pl->space = space;
    pl->k = k;
    pl->p = *p;
    pl->h = new bem_hmat();
    bem_hmat *h = pl->h;
    h->op = op;
    h->space = space;
    h->cplx = is_complex_op(op);
    h->ndof = space_ndof(*mesh, space);
    std::vector<double> pts, slo, shi;
    dof_geometry(*mesh, space, pts, slo, shi);
    build_partition(pts, slo, shi, p->leaf_size, p->eta, p->max_block, h->part);
    const auto &P = h->part;
    h->leaves.resize(P.blocks.size());
    std::vector<std::pair<const int32_t *, int64_t>> lists(P.nodes.size(), {nullptr, 0});
    for (size_t b = 0; b < P.blocks.size(); ++b) {
        const Block &bk = P.blocks[b];
        const Cluster &a = P.nodes[bk.tau], &c = P.nodes[bk.sigma];
        auto &L = h->leaves[b];
        L.adm = bk.admissible;
        L.r0 = a.begin;
        L.m = a.end - a.begin;
        L.c0 = c.begin;
        L.n = c.end - c.begin;
        if (!bk.admissible) continue;
        pl->adm.push_back((int64_t)b);
        for (int cid : {bk.tau, bk.sigma}) {
            const Cluster &cl = P.nodes[cid];
            lists[cid] = {P.perm.data() + cl.begin, cl.end - cl.begin};
        }
    }
    const int rc = make_resident(*mesh, space, lists, pl->lanes);
    if (rc != BEM_OK) {
        delete pl;
        return rc;
    }
    pl->setup_seconds = now_seconds() - t0;
    *out = pl;
    return BEM_OK;
}

int plan_info(const bem_aca_plan *pl, int64_t *nb, int64_t *ndof, double *setup)
{
    if (!pl) return fail(BEM_E_ARG, "null plan");
    if (nb) *nb = (int64_t)pl->adm.size();
    if (ndof) *ndof = pl->h->ndof;
    if (setup) *setup = pl->setup_seconds;
    return BEM_OK;
}

int plan_block(const bem_aca_plan *pl, int64_t b, int64_t *m, int64_t *n, const int32_t **rows, const int32_t **cols)
{
    if (!pl || b < 0 || b >= (int64_t)pl->adm.size()) return fail(BEM_E_ARG, "plan block out of range");
    const auto &L = pl->h->leaves[pl->adm[b]];
    if (m) *m = L.m;
    if (n) *n = L.n;
    if (rows) *rows = pl->h->rows(L);
    if (cols) *cols = pl->h->cols(L);
    return BEM_OK;
}

int plan_run(bem_aca_plan *pl, const int64_t *blocks, const double *arrival, int64_t n, int prec,
             bem_aca_run_stats *st)
{
    if (!pl || (n > 0 && !blocks) || n < 0) return fail(BEM_E_ARG, "bad run arguments");
    if (prec != BEM_FP32 && prec != BEM_FP64) return fail(BEM_E_ARG, "unknown precision");
    const int64_t nb = (int64_t)pl->adm.size();
    for (int64_t i = 0; i < n; ++i) {
        if (blocks[i] < 0 || blocks[i] >= nb) return fail(BEM_E_ARG, "plan block out of range");
        if (arrival && (!std::isfinite(arrival[i]) || arrival[i] < 0.0 || (i > 0 && arrival[i] < arrival[i - 1])))
            return fail(BEM_E_ARG, "arrival times must be finite, >= 0 and non-decreasing");
    }
    std::lock_guard<std::mutex> run_guard(pl->run_mu);
    bem_hmat *h = pl->h;
    // the previous run's factors go back to the pool
    for (int64_t leaf : pl->last) {
        auto &L = h->leaves[leaf];
        L.rank = 0;
        L.U = L.V = nullptr;
    }
    pl->last.clear();
    value_pool().give(h->store);
    AssemblyCtx C;
    C.mesh = pl->mesh;
    C.op = pl->op;
    C.space = pl->space;
    C.prec = prec;
    C.k = pl->k;
    C.tol = pl->p.aca_tol;
    C.max_rank = pl->p.max_rank;
    C.h = h;
    C.lanes = &pl->lanes.refs;
    C.jobs.reserve((size_t)n);
    for (int64_t i = 0; i < n; ++i) C.jobs.push_back(Job{pl->adm[blocks[i]], 1});
    C.arrival = arrival;
    const int nw = std::max(1, pl->p.n_workers);
    const int per = std::max(1, pl->p.blocks_per_worker);
    C.t0 = now_seconds();
    std::vector<std::thread> th;
    for (int w = 0; w < nw; ++w) {
        if (h->cplx)
            th.emplace_back([&] { worker<cd>(C, per); });
        else
            th.emplace_back([&] { worker<double>(C, per); });
    }
    for (auto &t : th) t.join();
    const double t1 = now_seconds();
    for (const Job &j : C.jobs) pl->last.push_back(j.leaf);
    if (C.error.load() != 0) return fail(C.error.load(), "ACA run: " + C.err_msg);
    if (st) {
        *st = bem_aca_run_stats{};
        st->blocks = n;
        st->entries = C.aca_entries.load();
        st->requests = C.requests.load();
        for (const Job &j : C.jobs) {
            const auto &L = h->leaves[j.leaf];
            st->rank_sum += L.rank;
            st->rank_max = std::max(st->rank_max, (int32_t)L.rank);
        }
        st->seconds = t1 - C.t0;
        const double nd = (double)std::max<int64_t>(1, C.blocks_done);
        st->mean_start_delay = C.start_delay / nd;
        st->mean_block_seconds = C.block_time / nd;
    }
    if (std::getenv("BEM_DEBUG_TIMING")) {
        const double np = (double)std::max<int64_t>(1, C.nproc);
        fprintf(stderr, "[bem] run %.3fs: %lld completions, mean pickup delay %.1f us, mean batch-processing span %.1f us\n",
                t1 - C.t0, (long long)C.nproc, 1e6 * C.qdelay / np, 1e6 * C.proc / np);
        fprintf(stderr, "[bem] worker us/request: busy %.3f convert %.3f aca %.3f release %.3f prepare %.3f submit %.3f\n",
                1e6 * C.busy / np, 1e6 * C.t_conv / np, 1e6 * C.t_aca / np, 1e6 * C.t_rel / np, 1e6 * C.t_prep / np,
                1e6 * C.t_flush / np);
        server_print_phases();
    }
    return BEM_OK;
}

// One served stream over the blocks of several plans (the served mixed
// workload): one pool of workers takes the blocks in arrival order whatever
// plan they belong to, each block with its own plan's operator, mesh,
// wavenumber, H-matrix and lane sets.
int plans_run(bem_aca_plan *const *plans, int64_t np, const int64_t *pidx, const int64_t *blocks,
              const double *arrival, int64_t n, int prec, int n_workers, int per_worker, bem_aca_run_stats *st)
{
    if (!plans || np < 1 || n < 0 || (n > 0 && (!pidx || !blocks)) || n_workers < 1 || per_worker < 1)
        return fail(BEM_E_ARG, "bad run arguments");
    if (prec != BEM_FP32 && prec != BEM_FP64) return fail(BEM_E_ARG, "unknown precision");
    for (int64_t p = 0; p < np; ++p)
        if (!plans[p]) return fail(BEM_E_ARG, "null plan");
    const bool cplx = plans[0]->h->cplx;
    for (int64_t p = 0; p < np; ++p)
        if (plans[p]->h->cplx != cplx) return fail(BEM_E_ARG, "the plans of one run must share the value type");
    for (int64_t i = 0; i < n; ++i) {
        if (pidx[i] < 0 || pidx[i] >= np) return fail(BEM_E_ARG, "plan index out of range");
        if (blocks[i] < 0 || blocks[i] >= (int64_t)plans[pidx[i]]->adm.size())
            return fail(BEM_E_ARG, "plan block out of range");
        if (arrival && (!std::isfinite(arrival[i]) || arrival[i] < 0.0 || (i > 0 && arrival[i] < arrival[i - 1])))
            return fail(BEM_E_ARG, "arrival times must be finite, >= 0 and non-decreasing");
    }
    // every distinct plan, locked in address order (one run per plan at a time)
    std::vector<bem_aca_plan *> distinct(plans, plans + np);
    std::sort(distinct.begin(), distinct.end());
    distinct.erase(std::unique(distinct.begin(), distinct.end()), distinct.end());
    std::vector<std::unique_lock<std::mutex>> locks;
    for (bem_aca_plan *pl : distinct) locks.emplace_back(pl->run_mu);
    std::vector<std::unique_ptr<AssemblyCtx>> ctx(distinct.size());
    for (size_t d = 0; d < distinct.size(); ++d) {
        bem_aca_plan *pl = distinct[d];
        bem_hmat *h = pl->h;
        for (int64_t leaf : pl->last) {   // the previous run's factors go back to the pool
            auto &L = h->leaves[leaf];
            L.rank = 0;
            L.U = L.V = nullptr;
        }
        pl->last.clear();
        value_pool().give(h->store);
        ctx[d].reset(new AssemblyCtx());
        AssemblyCtx &c = *ctx[d];
        c.mesh = pl->mesh;
        c.op = pl->op;
        c.space = pl->space;
        c.prec = prec;
        c.k = pl->k;
        c.tol = pl->p.aca_tol;
        c.max_rank = pl->p.max_rank;
        c.h = h;
        c.lanes = &pl->lanes.refs;
    }
    auto ctx_of = [&](bem_aca_plan *pl) {
        return ctx[std::lower_bound(distinct.begin(), distinct.end(), pl) - distinct.begin()].get();
    };
    AssemblyCtx M;   // the run: jobs, arrivals, counters; per-block fields come from the jobs' plans
    M.mesh = plans[0]->mesh;
    M.prec = prec;
    M.jobs.reserve((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        bem_aca_plan *pl = plans[pidx[i]];
        Job j{pl->adm[blocks[i]], 1};
        j.plan = ctx_of(pl);
        M.jobs.push_back(j);
    }
    M.arrival = arrival;
    M.t0 = now_seconds();
    std::vector<std::thread> th;
    for (int w = 0; w < n_workers; ++w) {
        if (cplx)
            th.emplace_back([&] { worker<cd>(M, per_worker); });
        else
            th.emplace_back([&] { worker<double>(M, per_worker); });
    }
    for (auto &t : th) t.join();
    const double t1 = now_seconds();
    for (const Job &j : M.jobs)
        for (bem_aca_plan *pl : distinct)
            if (ctx_of(pl) == j.plan) {
                pl->last.push_back(j.leaf);
                break;
            }
    if (M.error.load() != 0) return fail(M.error.load(), "ACA run: " + M.err_msg);
    if (st) {
        *st = bem_aca_run_stats{};
        st->blocks = n;
        st->entries = M.aca_entries.load();
        st->requests = M.requests.load();
        for (const Job &j : M.jobs) {
            const auto &L = j.plan->h->leaves[j.leaf];
            st->rank_sum += L.rank;
            st->rank_max = std::max(st->rank_max, (int32_t)L.rank);
        }
        st->seconds = t1 - M.t0;
        const double nd = (double)std::max<int64_t>(1, M.blocks_done);
        st->mean_start_delay = M.start_delay / nd;
        st->mean_block_seconds = M.block_time / nd;
    }
    return BEM_OK;
}

int plan_factors(const bem_aca_plan *pl, int64_t b, int32_t *rank, void *U, void *V)
{
    if (!pl || !rank || b < 0 || b >= (int64_t)pl->adm.size()) return fail(BEM_E_ARG, "plan block out of range");
    const int64_t leaf = pl->adm[b];
    if (std::find(pl->last.begin(), pl->last.end(), leaf) == pl->last.end())
        return fail(BEM_E_ARG, "block was not approximated by the last run");
    const auto &L = pl->h->leaves[leaf];
    *rank = L.rank;
    const size_t f = pl->h->cplx ? 2 : 1;
    if (U && L.U) std::memcpy(U, L.U, sizeof(double) * f * (size_t)L.m * (size_t)L.rank);
    if (V && L.V) std::memcpy(V, L.V, sizeof(double) * f * (size_t)L.n * (size_t)L.rank);
    return BEM_OK;
}

int plan_destroy(bem_aca_plan *pl)
{
    if (!pl) return fail(BEM_E_ARG, "null plan");
    {
        std::lock_guard<std::mutex> g(pl->run_mu);
    }
    delete pl;
    return BEM_OK;
}

int hmat_matvec(const bem_hmat *h, const void *xv, void *yv);

// D x by Eq. hyp_via_slp: per component j, z = Q_j x on DP1, w = S z, y +=
// Q_j^T w; for Helmholtz also y -= k^2 P_j^T S P_j x.
int hyps_via_slp_matvec(const bem_hmat *h, const void *xv, void *yv)
{
    const int64_t nv = h->ndof, nt = (int64_t)h->tri.size() / 3;
    const int f = h->cplx ? 2 : 1;
    const double *x = (const double *)xv;
    std::vector<double> y((size_t)nv * f, 0.0), z((size_t)3 * nt * f), w((size_t)3 * nt * f);
    for (int pass = 0; pass < (h->k != 0.0 ? 2 : 1); ++pass)
        for (int j = 0; j < 3; ++j) {
            for (int64_t t = 0; t < nt; ++t)
                for (int c = 0; c < f; ++c) {
                    if (pass == 0) {
                        double v = 0.0;
                        for (int a = 0; a < 3; ++a) v += h->curl[9 * t + 3 * a + j] * x[f * h->tri[3 * t + a] + c];
                        for (int a = 0; a < 3; ++a) z[f * (3 * t + a) + c] = v;
                    } else {
                        for (int a = 0; a < 3; ++a)
                            z[f * (3 * t + a) + c] = h->normal[3 * t + j] * x[f * h->tri[3 * t + a] + c];
                    }
                }
            const int rc = hmat_matvec(h->inner, z.data(), w.data());
            if (rc != BEM_OK) return rc;
            const double s = pass == 0 ? 1.0 : -h->k * h->k;
            for (int64_t t = 0; t < nt; ++t)
                for (int c = 0; c < f; ++c) {
                    if (pass == 0) {
                        const double sum = (w[f * (3 * t) + c] + w[f * (3 * t + 1) + c]) + w[f * (3 * t + 2) + c];
                        for (int a = 0; a < 3; ++a) y[f * h->tri[3 * t + a] + c] += h->curl[9 * t + 3 * a + j] * sum;
                    } else {
                        for (int a = 0; a < 3; ++a)
                            y[f * h->tri[3 * t + a] + c] += s * h->normal[3 * t + j] * w[f * (3 * t + a) + c];
                    }
                }
        }
    std::memcpy(yv, y.data(), sizeof(double) * y.size());
    return BEM_OK;
}

int hmat_matvec(const bem_hmat *h, const void *xv, void *yv)
{
    if (!h || !xv || !yv) return fail(BEM_E_ARG, "null argument");
    if (h->inner) return hyps_via_slp_matvec(h, xv, yv);
    const int64_t n = h->ndof;
    const int f = h->cplx ? 2 : 1;
    const double *x = (const double *)xv;
    const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::vector<double>> acc(nth, std::vector<double>((size_t)n * f, 0.0));
    auto run = [&](int tid) {
        std::vector<double> &y = acc[tid];
        std::vector<cd> tmp;
        for (size_t b = tid; b < h->leaves.size(); b += nth) {
            const auto &L = h->leaves[b];
            const int64_t m = L.m, nc = L.n;
            const int32_t *rows = h->rows(L), *cols = h->cols(L);
            if (h->cplx) {
                const cd *X = reinterpret_cast<const cd *>(x);
                cd *Y = reinterpret_cast<cd *>(y.data());
                if (L.adm) {
                    const cd *U = reinterpret_cast<const cd *>(L.U);
                    const cd *V = reinterpret_cast<const cd *>(L.V);
                    tmp.assign(L.rank, cd(0));
                    for (int l = 0; l < L.rank; ++l)
                        for (int64_t c = 0; c < nc; ++c) tmp[l] += V[(size_t)l * nc + c] * X[cols[c]];
                    for (int l = 0; l < L.rank; ++l)
                        for (int64_t r = 0; r < m; ++r) Y[rows[r]] += U[(size_t)l * m + r] * tmp[l];
                } else if (L.D) {
                    const cd *D = reinterpret_cast<const cd *>(L.D);
                    for (int64_t r = 0; r < m; ++r) {
                        cd s = 0;
                        for (int64_t c = 0; c < nc; ++c) s += D[r * nc + c] * X[cols[c]];
                        Y[rows[r]] += s;
                    }
                }
            } else {
                if (L.adm) {
                    std::vector<double> t(L.rank, 0.0);
                    for (int l = 0; l < L.rank; ++l)
                        for (int64_t c = 0; c < nc; ++c) t[l] += L.V[(size_t)l * nc + c] * x[cols[c]];
                    for (int l = 0; l < L.rank; ++l)
                        for (int64_t r = 0; r < m; ++r) y[rows[r]] += L.U[(size_t)l * m + r] * t[l];
                } else if (L.D) {
                    for (int64_t r = 0; r < m; ++r) {
                        double s = 0;
                        for (int64_t c = 0; c < nc; ++c) s += L.D[r * nc + c] * x[cols[c]];
                        y[rows[r]] += s;
                    }
                }
            }
        }
    };
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t) th.emplace_back(run, t);
    for (auto &t : th) t.join();
    double *y = (double *)yv;
    for (int64_t i = 0; i < n * f; ++i) {
        double s = 0.0;
        for (int t = 0; t < nth; ++t) s += acc[t][i];
        y[i] = s;
    }
    return BEM_OK;
}

int hmat_block_info(const bem_hmat *h, int64_t b, int32_t *adm, int64_t *m, int64_t *n, int32_t *rank,
                    const int32_t **rows, const int32_t **cols)
{
    if (h && h->inner) h = h->inner;   // the blocks of the single layer on DP1
    if (!h || b < 0 || b >= (int64_t)h->leaves.size()) return fail(BEM_E_ARG, "block index out of range");
    const auto &L = h->leaves[b];
    if (adm) *adm = L.adm;
    if (m) *m = L.m;
    if (n) *n = L.n;
    if (rank) *rank = L.rank;
    if (rows) *rows = h->rows(L);
    if (cols) *cols = h->cols(L);
    return BEM_OK;
}

int hmat_block_dense(const bem_hmat *h, int64_t b, void *outv)
{
    if (h && h->inner) h = h->inner;
    if (!h || !outv || b < 0 || b >= (int64_t)h->leaves.size()) return fail(BEM_E_ARG, "bad block");
    const auto &L = h->leaves[b];
    const int64_t m = L.m, n = L.n;
    if (h->cplx) {
        cd *out = (cd *)outv;
        if (L.adm) {
            const cd *U = reinterpret_cast<const cd *>(L.U);
            const cd *V = reinterpret_cast<const cd *>(L.V);
            for (int64_t r = 0; r < m; ++r)
                for (int64_t c = 0; c < n; ++c) {
                    cd s = 0;
                    for (int l = 0; l < L.rank; ++l) s += U[(size_t)l * m + r] * V[(size_t)l * n + c];
                    out[r * n + c] = s;
                }
        } else if (L.D) {
            std::memcpy(out, L.D, sizeof(cd) * m * n);
        } else {
            std::fill(out, out + m * n, cd(0));
        }
    } else {
        double *out = (double *)outv;
        if (L.adm) {
            for (int64_t r = 0; r < m; ++r)
                for (int64_t c = 0; c < n; ++c) {
                    double s = 0;
                    for (int l = 0; l < L.rank; ++l) s += L.U[(size_t)l * m + r] * L.V[(size_t)l * n + c];
                    out[r * n + c] = s;
                }
        } else if (L.D) {
            std::memcpy(out, L.D, sizeof(double) * m * n);
        } else {
            std::fill(out, out + m * n, 0.0);
        }
    }
    return BEM_OK;
}

int hmat_stats(const bem_hmat *h, bem_hmat_stats *s)
{
    if (!h || !s) return fail(BEM_E_ARG, "null argument");
    *s = h->st;
    return BEM_OK;
}

int hmat_destroy(bem_hmat *h)
{
    delete h;
    return BEM_OK;
}

}  // namespace bem
