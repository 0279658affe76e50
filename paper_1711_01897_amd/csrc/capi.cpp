// extern "C" entry points of libbem (declared in include/bem.h).
#include <algorithm>
#include <cmath>
#include <new>

#include "bem_internal.hpp"
#include "tree.hpp"

namespace bem {
const char *last_error();
int mesh_create_impl(const double *, int64_t, const int32_t *, int64_t, int, bem_mesh **);
int mesh_destroy_impl(bem_mesh *);
int server_configure(size_t, int);
int server_stats(bem_server_stats_t *, int);
int server_kernel_stats(bem_kernel_stats_t *, int, int *, int);
int aca_block(bem_mesh *, int, int, double, const int32_t *, int64_t, const int32_t *, int64_t, const bem_aca_params *,
              int, void *, void *, int32_t *, int64_t *);
int aca_callback(int64_t, int64_t, int, bem_row_fn, bem_col_fn, void *, const bem_aca_params *, void *, void *,
                 int32_t *);
int hmat_assemble(bem_mesh *, int, int, double, const bem_hmat_params *, bem_hmat **);
int hmat_matvec(const bem_hmat *, const void *, void *);
int hmat_block_info(const bem_hmat *, int64_t, int32_t *, int64_t *, int64_t *, int32_t *, const int32_t **,
                    const int32_t **);
int hmat_block_dense(const bem_hmat *, int64_t, void *);
int hmat_stats(const bem_hmat *, bem_hmat_stats *);
int hmat_destroy(bem_hmat *);
int plan_create(bem_mesh *, int, int, double, const bem_hmat_params *, bem_aca_plan **);
int plan_info(const bem_aca_plan *, int64_t *, int64_t *, double *);
int plan_block(const bem_aca_plan *, int64_t, int64_t *, int64_t *, const int32_t **, const int32_t **);
int plan_run(bem_aca_plan *, const int64_t *, const double *, int64_t, int, bem_aca_run_stats *);
int plans_run(bem_aca_plan *const *, int64_t, const int64_t *, const int64_t *, const double *, int64_t, int, int,
              int, bem_aca_run_stats *);
int plan_factors(const bem_aca_plan *, int64_t, int32_t *, void *, void *);
int plan_destroy(bem_aca_plan *);
int eval_dense(bem_mesh *, int, int, double, const int32_t *, int64_t, const int32_t *, int64_t, int, int, void *,
               bem_dense_stats *);
}  // namespace bem

using namespace bem;

struct bem_ticket {
    Request req;
};

namespace {

int fill_request(Request &r, bem_mesh *mesh, bem_op op, bem_space space, double k, const int32_t *rows, int64_t nrows,
                 const int32_t *cols, int64_t ncols, bem_prec prec, bem_near near)
{
    if (!mesh) return fail(BEM_E_ARG, "null mesh");
    if (nrows < 0 || ncols < 0) return fail(BEM_E_ARG, "negative request size");
    if ((nrows > 0 && !rows) || (ncols > 0 && !cols)) return fail(BEM_E_ARG, "null index array");
    r.mesh = mesh;
    r.op = op;
    r.space = space;
    r.prec = prec;
    r.near = near;
    r.k = k;
    r.nrows = nrows;
    r.ncols = ncols;
    r.rows.assign(rows, rows + nrows);
    r.cols.assign(cols, cols + ncols);
    return expand_request(r);
}

// Pinned staging buffers of the async path.  A buffer is freed once the
// event recorded after its copy has completed; completed buffers are
// reclaimed on later calls (or immediately when no event could be recorded).
std::mutex g_stage_mu;
std::vector<std::pair<hipEvent_t, char *>> g_stage_pending;

void reclaim_stages(bool all)
{
    std::lock_guard<std::mutex> g(g_stage_mu);
    auto it = g_stage_pending.begin();
    while (it != g_stage_pending.end()) {
        if (all ? hipEventSynchronize(it->first) == hipSuccess : hipEventQuery(it->first) == hipSuccess) {
            (void)hipEventDestroy(it->first);
            (void)hipHostFree(it->second);
            it = g_stage_pending.erase(it);
        } else {
            ++it;
        }
    }
}

char *pinned_stage(size_t bytes)
{
    reclaim_stages(false);
    char *p = nullptr;
    if (hipHostMalloc((void **)&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
    return p;
}

void pinned_release(char *p, hipEvent_t after)
{
    if (!after) {
        // nothing was enqueued that reads p
        (void)hipHostFree(p);
        return;
    }
    std::lock_guard<std::mutex> g(g_stage_mu);
    g_stage_pending.push_back({after, p});
}

// Enqueues an expanded request on `s` with its result in device memory
// dev_out.  Workspace layout: descriptor | block table | singular pairs |
// inputs | status word, copied to the device in one piece before the
// launches.  With fixed == nullptr the workspace comes from the
// stream-ordered allocator and the host image from pinned staging released
// once its copy has completed; otherwise both live in fixed memory: the
// workspace is `fixed` (fixed_bytes long; larger requests fail), the host
// image a per-thread pageable buffer whose copy completes before the call
// returns (a pageable host-to-device copy is synchronous with the host).
int enqueue_device_request(Request &r, void *dev_out, hipStream_t s, char *fixed, size_t fixed_bytes)
{
    bem_mesh *mesh = r.mesh;
    if (r.near == BEM_NEAR_ERROR) {
        // host-side check: nothing may be enqueued for a failing request
        if (r.space == BEM_P0) {
            for (int32_t a : r.rows)
                for (int32_t b : r.cols)
                    if (mesh->adjacent(a, b)) return fail(BEM_E_NEARFIELD, "a contributing triangle pair shares a vertex");
        } else {
            for (size_t f = 0; 2 * f + 1 < r.fix.size(); ++f)
                for (int32_t st = r.fix[2 * f]; st < r.fix[2 * f + 1]; ++st)
                    for (int32_t t : r.own.lane)
                        if (mesh->adjacent(mesh->star[st] >> 2, t))
                            return fail(BEM_E_NEARFIELD, "a contributing triangle pair shares a vertex");
        }
    }
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t off = 0;
    const size_t off_req = off;
    off = al(off + sizeof(ReqDev));
    const size_t off_b = off;
    off = al(off + sizeof(EntryBlock) * (size_t)r.nblocks);
    const size_t off_near = off;
    const bool p1_near = r.space != BEM_P0 && !r.near_items.empty();
    off = al(off + (p1_near ? near_p1_layout(r).bytes : sizeof(NearItem) * r.near_items.size()));
    const size_t off_in = off;
    off = al(off + r.in_bytes);
    const size_t off_status = off;
    off = al(off + 8);
    const size_t in_total = off;
    if (fixed && in_total > fixed_bytes)
        return fail(BEM_E_OOM, "request needs " + std::to_string(in_total) + " bytes of workspace, more than the " +
                                   std::to_string(fixed_bytes) + "-byte static workspace of the no-allocation entry point");
    char *host = nullptr;
    thread_local std::vector<char> pageable;
    if (fixed) {
        pageable.assign(in_total, 0);
        host = pageable.data();
    } else {
        // descriptors go through pinned staging that is released once the
        // copy has completed (checked on later calls), so nothing here waits
        host = pinned_stage(in_total);
        if (!host) return fail(BEM_E_OOM, "pinned staging allocation failed");
        std::memset(host, 0, in_total);
    }
    char *ws = fixed;
    if (!fixed) {
        hipError_t e = hipMallocAsync((void **)&ws, in_total, s);
        if (e != hipSuccess) {
            pinned_release(host, nullptr);
            return fail(BEM_E_DEVICE, std::string("hipMallocAsync: ") + hipGetErrorString(e));
        }
    }
    ReqDev d;
    stage_request_inputs(r, host, ws, off_in, d);
    finish_descriptor(r, ws, 0, off_status, d);
    d.out = dev_out;
    std::memcpy(host + off_req, &d, sizeof(ReqDev));
    write_blocks(r, 0, reinterpret_cast<EntryBlock *>(host + off_b));
    if (p1_near) {
        stage_near_p1(r, near_p1_layout(r), host + off_near, ws + off_near, static_cast<char *>(dev_out), 0, 0, 0);
    } else {
        NearItem *q = reinterpret_cast<NearItem *>(host + off_near);
        for (size_t j = 0; j < r.near_items.size(); ++j) {
            q[j] = r.near_items[j];
            q[j].out = static_cast<char *>(dev_out) + (size_t)r.near_index[j] * r.elem_bytes;
        }
    }
    hipError_t e = hipMemcpyAsync(ws, host, in_total, hipMemcpyHostToDevice, s);
    if (!fixed) {
        hipEvent_t ev = nullptr;
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(ev, s);
        pinned_release(host, e == hipSuccess ? ev : nullptr);
    }
    if (e != hipSuccess) return fail(BEM_E_DEVICE, std::string("staging copy: ") + hipGetErrorString(e));
    const ReqDev *dreq = (const ReqDev *)(ws + off_req);
    Variant v{kernel_op(r.op), r.space, r.prec, mesh->q};
    BEM_HIP_TRY(launch_entries(v, dreq, (const EntryBlock *)(ws + off_b), r.nblocks, s));
    if (p1_near)
        BEM_HIP_TRY(launch_near_p1_region(r.op == BEM_LAPLACE_HYPS || r.op == BEM_HELMHOLTZ_HYPS ? (int)r.op
                                                                                                : kernel_op(r.op),
                                          r.prec == BEM_FP32, near_p1_layout(r), ws + off_near,
                                          (int64_t)r.near_items.size(), (int64_t)r.near_recs.size(), s));
    else
        BEM_HIP_TRY(launch_near(kernel_op(r.op), r.prec == BEM_FP32, (const NearItem *)(ws + off_near),
                                (int64_t)r.near_items.size(), s));
    if (!fixed) BEM_HIP_TRY(hipFreeAsync(ws, s));
    return BEM_OK;
}

// Workspace of bem_eval_entries_async_noalloc: one request's descriptor,
// block table, singular-pair records, inputs and status word.  Each device
// the library runs on holds its own copy for the life of the process; host
// code reaches it only through the address hipGetSymbolAddress returns for
// that device.
constexpr size_t kNoAllocBytes = size_t(32) << 20;
__device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device`, looked up once per device
// with that device current (the previous current device is restored).
int noalloc_workspace(int device, char **out)
{
    if (device < 0 || device >= kMaxDevices) return fail(BEM_E_ARG, "device ordinal out of range");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = 0;
        BEM_HIP_TRY(hipGetDevice(&cur));
        if (cur != device) BEM_HIP_TRY(hipSetDevice(device));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return fail(BEM_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[device] = static_cast<char *>(p);
    }
    *out = g_scratch_ptr[device];
    return BEM_OK;
}

}  // namespace

extern "C" {

const char *bem_last_error(void) { return bem::last_error(); }

int bem_mesh_create(const double *xyz, int64_t nv, const int32_t *tri, int64_t nt, int quad_points, bem_mesh **out)
{
    return mesh_create_impl(xyz, nv, tri, nt, quad_points, out);
}

int bem_mesh_destroy(bem_mesh *mesh) { return mesh_destroy_impl(mesh); }

int bem_mesh_info(const bem_mesh *m, bem_mesh_info_t *info)
{
    if (!m || !info) return fail(BEM_E_ARG, "null argument");
    info->nv = m->nv;
    info->nt = m->nt;
    info->quad_points = m->q;
    info->max_star = m->max_star;
    info->mean_jacobian = m->mean_J;
    info->mean_edge = m->mean_edge;
    info->device_bytes = m->dev_bytes;
    return BEM_OK;
}

int bem_eval_entries(bem_mesh *mesh, bem_op op, bem_space space, double k, const int32_t *rows, int64_t nrows,
                     const int32_t *cols, int64_t ncols, bem_prec prec, bem_near near, void *out)
{
    Request *r = new (std::nothrow) Request();
    if (!r) return fail(BEM_E_OOM, "host allocation failed");
    int rc = fill_request(*r, mesh, op, space, k, rows, nrows, cols, ncols, prec, near);
    if (rc == BEM_OK && r->entries() > 0) {
        if (!out) {
            rc = fail(BEM_E_ARG, "null output");
        } else {
            r->out_host = out;
            rc = server_submit(r);
            if (rc == BEM_OK) {
                rc = server_wait(r, -1.0);
                if (rc == BEM_E_NEARFIELD) fail(rc, "a contributing triangle pair shares a vertex");
            }
        }
    }
    delete r;
    return rc;
}

int bem_submit(bem_mesh *mesh, bem_op op, bem_space space, double k, const int32_t *rows, int64_t nrows,
               const int32_t *cols, int64_t ncols, bem_prec prec, bem_near near, void *out, bem_ticket **ticket)
{
    if (!ticket) return fail(BEM_E_ARG, "null ticket");
    bem_ticket *t = new (std::nothrow) bem_ticket();
    if (!t) return fail(BEM_E_OOM, "host allocation failed");
    Request &r = t->req;
    int rc = fill_request(r, mesh, op, space, k, rows, nrows, cols, ncols, prec, near);
    if (rc == BEM_OK) {
        if (r.entries() == 0) {
            r.done = true;
            r.status = BEM_OK;
            r.t_submit = r.t_done = now_seconds();
        } else if (!out) {
            rc = fail(BEM_E_ARG, "null output");
        } else {
            r.out_host = out;
            rc = server_submit(&r);
        }
    }
    if (rc != BEM_OK) {
        delete t;
        return rc;
    }
    *ticket = t;
    return BEM_OK;
}

int bem_ticket_wait(bem_ticket *t, double timeout_s)
{
    if (!t) return fail(BEM_E_ARG, "null ticket");
    const int rc = server_wait(&t->req, timeout_s);
    if (rc == BEM_E_NEARFIELD) fail(rc, "a contributing triangle pair shares a vertex");
    return rc;
}

int bem_ticket_times(const bem_ticket *t, double *t_submit, double *t_done)
{
    if (!t) return fail(BEM_E_ARG, "null ticket");
    if (t_submit) *t_submit = t->req.t_submit;
    if (t_done) *t_done = t->req.t_done;
    return BEM_OK;
}

int bem_ticket_free(bem_ticket *t)
{
    if (!t) return BEM_OK;
    (void)server_wait(&t->req, -1.0);
    delete t;
    return BEM_OK;
}

int bem_eval_entries_async(bem_mesh *mesh, bem_op op, bem_space space, double k, const int32_t *rows, int64_t nrows,
                           const int32_t *cols, int64_t ncols, bem_prec prec, bem_near near, void *dev_out,
                           void *stream)
{
    Request r;
    int rc = fill_request(r, mesh, op, space, k, rows, nrows, cols, ncols, prec, near);
    if (rc != BEM_OK) return rc;
    if (r.entries() == 0) return BEM_OK;
    if (!dev_out) return fail(BEM_E_ARG, "null output");
    return enqueue_device_request(r, dev_out, (hipStream_t)stream, nullptr, 0);
}

int bem_eval_entries_async_noalloc(bem_mesh *mesh, bem_op op, bem_space space, double k, const int32_t *rows,
                                   int64_t nrows, const int32_t *cols, int64_t ncols, bem_prec prec, bem_near near,
                                   void *dev_out, void *stream)
{
    Request r;
    int rc = fill_request(r, mesh, op, space, k, rows, nrows, cols, ncols, prec, near);
    if (rc != BEM_OK) return rc;
    if (r.entries() == 0) return BEM_OK;
    if (!dev_out) return fail(BEM_E_ARG, "null output");
    char *ws = nullptr;
    rc = noalloc_workspace(mesh->device, &ws);
    if (rc != BEM_OK) return rc;
    return enqueue_device_request(r, dev_out, (hipStream_t)stream, ws, kNoAllocBytes);
}

int bem_server_config(size_t arena_bytes, int max_batch_requests)
{
    return server_configure(arena_bytes, max_batch_requests);
}

int bem_server_stats(bem_server_stats_t *stats, int reset)
{
    if (!stats) return fail(BEM_E_ARG, "null argument");
    return server_stats(stats, reset);
}

int bem_server_kernel_stats(bem_kernel_stats_t *out, int max_entries, int *count, int reset)
{
    if (max_entries < 0 || !count) return fail(BEM_E_ARG, "bad arguments");
    return server_kernel_stats(out, max_entries, count, reset);
}

int bem_aca_block(bem_mesh *mesh, bem_op op, bem_space space, double k, const int32_t *rows, int64_t m,
                  const int32_t *cols, int64_t n, const bem_aca_params *params, bem_prec prec, void *U, void *V,
                  int32_t *rank, int64_t *entries_evaluated)
{
    return aca_block(mesh, op, space, k, rows, m, cols, n, params, prec, U, V, rank, entries_evaluated);
}

int bem_aca_callback(int64_t m, int64_t n, int is_complex, bem_row_fn get_row, bem_col_fn get_col, void *ctx,
                     const bem_aca_params *params, void *U, void *V, int32_t *rank)
{
    return aca_callback(m, n, is_complex, get_row, get_col, ctx, params, U, V, rank);
}

int bem_partition(const double *xyz, int64_t nv, const int32_t *tri, int64_t nt, bem_space space, int32_t leaf_size,
                  double eta, int32_t max_block, int32_t *perm, int32_t *cl_begin, int32_t *cl_end, int64_t max_clusters, int32_t *blocks,
                  int64_t max_blocks, int64_t *nclusters, int64_t *nblocks)
{
    if (!xyz || !tri || nv < 1 || nt < 1 || leaf_size < 1 || !(eta > 0) || max_block < 0 || !nclusters || !nblocks)
        return fail(BEM_E_ARG, "bad partition arguments");
    if (space != BEM_P0 && space != BEM_P1 && space != BEM_DP1) return fail(BEM_E_ARG, "unknown space");
    for (int64_t i = 0; i < 3 * nt; ++i)
        if (tri[i] < 0 || tri[i] >= nv) return fail(BEM_E_ARG, "triangle vertex index out of range");
    bem_mesh m;
    m.nv = nv;
    m.nt = nt;
    m.xyz.assign(xyz, xyz + 3 * nv);
    m.tri.assign(tri, tri + 3 * nt);
    std::vector<double> pts, slo, shi;
    dof_geometry(m, space, pts, slo, shi);
    Partition P;
    build_partition(pts, slo, shi, leaf_size, eta, max_block, P);
    *nclusters = (int64_t)P.nodes.size();
    *nblocks = (int64_t)P.blocks.size();
    if ((int64_t)P.nodes.size() > max_clusters || (int64_t)P.blocks.size() > max_blocks)
        return fail(BEM_E_ARG, "capacity too small");
    if (perm) std::copy(P.perm.begin(), P.perm.end(), perm);
    for (size_t c = 0; c < P.nodes.size(); ++c) {
        if (cl_begin) cl_begin[c] = (int32_t)P.nodes[c].begin;
        if (cl_end) cl_end[c] = (int32_t)P.nodes[c].end;
    }
    if (blocks)
        for (size_t b = 0; b < P.blocks.size(); ++b) {
            blocks[3 * b] = P.blocks[b].tau;
            blocks[3 * b + 1] = P.blocks[b].sigma;
            blocks[3 * b + 2] = P.blocks[b].admissible;
        }
    return BEM_OK;
}

int bem_hmat_assemble(bem_mesh *mesh, bem_op op, bem_space space, double k, const bem_hmat_params *params,
                      bem_hmat **out)
{
    return hmat_assemble(mesh, op, space, k, params, out);
}

int bem_hmat_matvec(const bem_hmat *h, const void *x, void *y) { return hmat_matvec(h, x, y); }

int bem_hmat_stats_get(const bem_hmat *h, bem_hmat_stats *stats) { return hmat_stats(h, stats); }

int bem_hmat_block_info(const bem_hmat *h, int64_t b, int32_t *admissible, int64_t *m, int64_t *n, int32_t *rank,
                        const int32_t **rows, const int32_t **cols)
{
    return hmat_block_info(h, b, admissible, m, n, rank, rows, cols);
}

int bem_hmat_block_dense(const bem_hmat *h, int64_t b, void *out) { return hmat_block_dense(h, b, out); }

int bem_hmat_destroy(bem_hmat *h) { return hmat_destroy(h); }

int bem_aca_plan_create(bem_mesh *mesh, bem_op op, bem_space space, double k, const bem_hmat_params *params,
                        bem_aca_plan **out)
{
    return plan_create(mesh, op, space, k, params, out);
}

int bem_aca_plan_info(const bem_aca_plan *plan, int64_t *n_blocks, int64_t *ndof, double *setup_seconds)
{
    return plan_info(plan, n_blocks, ndof, setup_seconds);
}

int bem_aca_plan_block(const bem_aca_plan *plan, int64_t b, int64_t *m, int64_t *n, const int32_t **rows,
                       const int32_t **cols)
{
    return plan_block(plan, b, m, n, rows, cols);
}

int bem_aca_plan_run(bem_aca_plan *plan, const int64_t *blocks, const double *arrival, int64_t n, bem_prec prec,
                     bem_aca_run_stats *stats)
{
    return plan_run(plan, blocks, arrival, n, prec, stats);
}

int bem_aca_plans_run(bem_aca_plan *const *plans, int64_t nplans, const int64_t *plan_index, const int64_t *blocks,
                      const double *arrival, int64_t n, bem_prec prec, int32_t n_workers, int32_t blocks_per_worker,
                      bem_aca_run_stats *stats)
{
    return plans_run(plans, nplans, plan_index, blocks, arrival, n, prec, n_workers, blocks_per_worker, stats);
}

int bem_aca_plan_factors(const bem_aca_plan *plan, int64_t b, int32_t *rank, void *U, void *V)
{
    return plan_factors(plan, b, rank, U, V);
}

int bem_aca_plan_destroy(bem_aca_plan *plan) { return plan_destroy(plan); }

int bem_eval_dense(bem_mesh *mesh, bem_op op, bem_space space, double k, const int32_t *rows, int64_t nrows,
                   const int32_t *cols, int64_t ncols, bem_prec prec, bem_near near, void *out, bem_dense_stats *stats)
{
    if (nrows > 0 && ncols > 0 && !out) return fail(BEM_E_ARG, "null output");
    return eval_dense(mesh, op, space, k, rows, nrows, cols, ncols, prec, near, out, stats);
}

}  // extern "C"
