// Pair-based evaluation of P1 blocks (the dense weak-form assembly of
// Section 3): every regular triangle pair of star(rows) x star(cols) is
// integrated once into its 3 x 3 local matrix on the device, then each entry
// adds its pairs' local values in a fixed order (entries.hip: k_local_*,
// k_gather_dense_*).  Rows go in panels whose local matrices fit a device
// budget; the panels run on a compute stream while a copy stream moves the
// previous panel's entries to pinned host memory and the calling thread
// copies the one before into `out`, so assembly and transfer overlap
// (Section 3's chunked assembly with overlapped transfers).
#include <algorithm>
#include <cstdlib>

#include "bem_internal.hpp"

namespace bem {

hipError_t launch_dense_local(int op, bool fp32, const bem_mesh &m, const int32_t *test, int ntest,
                              const int32_t *trial, int ntrial, void *Lr, void *Li, double k, hipStream_t s);
hipError_t launch_dense_gather(bool fp32, bool cplx, const void *Lr, const void *Li, int ntrial, const int32_t *rptr,
                               const int32_t *rsrc, int nrows, const int32_t *cptr, const int32_t *csrc, int ncols,
                               void *out, hipStream_t s);

namespace {

// Sorted distinct triangles of the stars of `dofs`, and per dof its star as
// (index in that list << 2 | local vertex), ascending triangles.
void star_lists(const bem_mesh &m, const int32_t *dofs, int64_t n, std::vector<int32_t> &tris,
                std::vector<int32_t> &ptr, std::vector<int32_t> &src)
{
    tris.clear();
    for (int64_t i = 0; i < n; ++i)
        for (int64_t s = m.star_ptr[dofs[i]]; s < m.star_ptr[dofs[i] + 1]; ++s) tris.push_back(m.star[s] >> 2);
    std::sort(tris.begin(), tris.end());
    tris.erase(std::unique(tris.begin(), tris.end()), tris.end());
    ptr.assign(1, 0);
    src.clear();
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t s = m.star_ptr[dofs[i]]; s < m.star_ptr[dofs[i] + 1]; ++s) {
            const int32_t t = m.star[s] >> 2;
            const int32_t idx = (int32_t)(std::lower_bound(tris.begin(), tris.end(), t) - tris.begin());
            src.push_back((idx << 2) | (m.star[s] & 3));
        }
        ptr.push_back((int32_t)src.size());
    }
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

struct Panel {
    int64_t r0 = 0, nr = 0;
    std::vector<int32_t> tris, ptr, src;
    size_t off_tris = 0, off_ptr = 0, off_src = 0;   // in the index buffer, int32 units
};

}  // namespace

int eval_dense(bem_mesh *m, int op, int space, double k, const int32_t *rows, int64_t nrows, const int32_t *cols,
               int64_t ncols, int prec, int near, void *out, bem_dense_stats *st)
{
    if (!m) return fail(BEM_E_ARG, "null mesh");
    if (nrows < 0 || ncols < 0 || (nrows > 0 && !rows) || (ncols > 0 && !cols)) return fail(BEM_E_ARG, "bad indices");
    {
        Request probe;   // validates operator, space, k, precision and policy
        probe.mesh = m;
        probe.op = op;
        probe.space = space;
        probe.prec = prec;
        probe.k = k;
        probe.near = near;
        const int rc = expand_request(probe);
        if (rc != BEM_OK) return rc;
    }
    if (space != BEM_P1) return fail(BEM_E_ARG, "pair-based blocks are P1 only");
    if (op != BEM_LAPLACE_SLP && op != BEM_LAPLACE_DLP && op != BEM_HELMHOLTZ_SLP && op != BEM_HELMHOLTZ_DLP)
        return fail(BEM_E_ARG, "pair-based blocks: single and double layer only");
    if (near == BEM_NEAR_SINGULAR) return fail(BEM_E_ARG, "pair-based blocks: BEM_NEAR_ERROR or BEM_NEAR_SKIP");
    for (int64_t i = 0; i < nrows; ++i)
        if (rows[i] < 0 || rows[i] >= m->nv) return fail(BEM_E_ARG, "row index out of range");
    for (int64_t i = 0; i < ncols; ++i)
        if (cols[i] < 0 || cols[i] >= m->nv) return fail(BEM_E_ARG, "column index out of range");
    if (st) *st = bem_dense_stats{};
    if (nrows == 0 || ncols == 0) return BEM_OK;
    if (ncols > INT32_MAX / 4) return fail(BEM_E_ARG, "too many columns");
    const double t0 = now_seconds();
    const bool fp32 = prec == BEM_FP32, cplx = is_complex_op(op);
    const size_t real = fp32 ? 4 : 8, elem = out_elem_bytes(op, prec);

    std::vector<int32_t> ctris, cptr, csrc;
    star_lists(*m, cols, ncols, ctris, cptr, csrc);
    const int64_t ntrial = (int64_t)ctris.size();
    if (ntrial > INT32_MAX / 4) return fail(BEM_E_ARG, "too many trial triangles");
    if (near == BEM_NEAR_ERROR) {
        // nothing is launched for a failing request: every vertex-sharing pair
        // between the row stars and the column stars is an error
        std::vector<char> mark(m->nv, 0);
        for (int32_t t : ctris)
            for (int a = 0; a < 3; ++a) mark[m->tri[3 * (size_t)t + a]] = 1;
        for (int64_t i = 0; i < nrows; ++i)
            for (int64_t s = m->star_ptr[rows[i]]; s < m->star_ptr[rows[i] + 1]; ++s) {
                const int32_t t = m->star[s] >> 2;
                for (int a = 0; a < 3; ++a)
                    if (mark[m->tri[3 * (size_t)t + a]]) return fail(BEM_E_NEARFIELD, "a contributing triangle pair shares a vertex");
            }
    }
    // panels: at most 65,535 rows (the gather's grid) and local matrices of at
    // most BEM_DENSE_BUDGET_MB (default 1024) MiB
    const char *env = std::getenv("BEM_DENSE_BUDGET_MB");
    const size_t budget = (size_t)std::max(16, env ? std::atoi(env) : 1024) << 20;
    const size_t per_test = 9 * real * (cplx ? 2 : 1) * (size_t)ntrial;   // local values of one test triangle
    std::vector<Panel> panels;
    size_t max_test = 0;
    {
        int64_t r = 0;
        while (r < nrows) {
            // grow the panel while its row stars fit the budget (about 2 test
            // triangles per row: start from that estimate and shrink)
            int64_t nr = std::min<int64_t>({nrows - r, 65535, std::max<int64_t>(1, (int64_t)(budget / per_test) / 2)});
            Panel P;
            for (;;) {
                star_lists(*m, rows + r, nr, P.tris, P.ptr, P.src);
                if (P.tris.size() * per_test <= budget || nr == 1) break;
                nr = std::max<int64_t>(1, nr / 2);
            }
            if (P.tris.size() * per_test > budget)
                return fail(BEM_E_OOM, "one row's local matrices exceed the dense budget (BEM_DENSE_BUDGET_MB)");
            P.r0 = r;
            P.nr = nr;
            max_test = std::max(max_test, P.tris.size());
            panels.push_back(std::move(P));
            r += nr;
        }
    }
    int64_t max_rows = 0;
    for (const Panel &P : panels) max_rows = std::max(max_rows, P.nr);
    // one int32 buffer for every index list
    std::vector<int32_t> idx;
    auto put = [&](const std::vector<int32_t> &v) {
        const size_t at = idx.size();
        idx.insert(idx.end(), v.begin(), v.end());
        while (idx.size() % 4) idx.push_back(0);
        return at;
    };
    const size_t off_ctris = put(ctris), off_cptr = put(cptr), off_csrc = put(csrc);
    for (Panel &P : panels) {
        P.off_tris = put(P.tris);
        P.off_ptr = put(P.ptr);
        P.off_src = put(P.src);
    }
    const size_t panel_out = (size_t)max_rows * (size_t)ncols * elem;
    DevBuf d_idx, d_L, d_out;
    char *h_stage = nullptr;
    hipStream_t sc = nullptr, sx = nullptr;
    hipEvent_t ev[8] = {};
    int rc = BEM_OK;
    auto cleanup = [&]() {
        if (sc) (void)hipStreamSynchronize(sc);
        if (sx) (void)hipStreamSynchronize(sx);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (sc) (void)hipStreamDestroy(sc);
        if (sx) (void)hipStreamDestroy(sx);
        if (h_stage) (void)hipHostFree(h_stage);
    };
    hipError_t e = hipMalloc(&d_idx.p, 4 * idx.size());
    if (e == hipSuccess) e = hipMalloc(&d_L.p, max_test * per_test);
    if (e == hipSuccess) e = hipMalloc(&d_out.p, 2 * panel_out);
    if (e == hipSuccess) e = hipHostMalloc((void **)&h_stage, 2 * panel_out, hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sc, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sx, hipStreamNonBlocking);
    for (int i = 0; i < 8 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&ev[i], i < 4 ? hipEventDisableTiming : 0);
    if (e == hipSuccess) e = hipMemcpy(d_idx.p, idx.data(), 4 * idx.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        cleanup();
        return fail(e == hipErrorOutOfMemory ? BEM_E_OOM : BEM_E_DEVICE, std::string("dense set-up: ") + hipGetErrorString(e));
    }
    const int32_t *D = static_cast<const int32_t *>(d_idx.p);
    hipEvent_t *computed = ev, *copied = ev + 2;   // per output buffer
    hipEvent_t t_start = ev[4], t_local = ev[5], t_end = ev[6];
    char *L = static_cast<char *>(d_L.p);
    void *Li = cplx ? L + max_test * per_test / 2 : nullptr;
    double local_s = 0.0;
    int64_t pairs = 0;
    auto finish = [&](size_t p) {
        const Panel &P = panels[p];
        const int b = (int)(p % 2);
        hipError_t x = hipEventSynchronize(copied[b]);
        if (x != hipSuccess) return x;
        std::memcpy(static_cast<char *>(out) + (size_t)P.r0 * ncols * elem, h_stage + b * panel_out,
                    (size_t)P.nr * ncols * elem);
        return hipSuccess;
    };
    for (size_t p = 0; p < panels.size() && e == hipSuccess; ++p) {
        const Panel &P = panels[p];
        const int b = (int)(p % 2);
        char *dout = static_cast<char *>(d_out.p) + b * panel_out;
        if (p >= 2) e = hipStreamWaitEvent(sc, copied[b], 0);
        const bool timed = p == 0;
        if (e == hipSuccess && timed) e = hipEventRecord(t_start, sc);
        if (e == hipSuccess)
            e = launch_dense_local(op, fp32, *m, D + P.off_tris, (int)P.tris.size(), D + off_ctris, (int)ntrial, L, Li,
                                   k, sc);
        if (e == hipSuccess && timed) e = hipEventRecord(t_local, sc);
        if (e == hipSuccess)
            e = launch_dense_gather(fp32, cplx, L, Li, (int)ntrial, D + P.off_ptr, D + P.off_src, (int)P.nr,
                                    D + off_cptr, D + off_csrc, (int)ncols, dout, sc);
        if (e == hipSuccess && timed) e = hipEventRecord(t_end, sc);
        if (e == hipSuccess) e = hipEventRecord(computed[b], sc);
        pairs += (int64_t)P.tris.size() * ntrial;
        if (e == hipSuccess && p >= 1) e = finish(p - 1);
        if (e == hipSuccess) e = hipStreamWaitEvent(sx, computed[b], 0);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h_stage + b * panel_out, dout, (size_t)P.nr * ncols * elem, hipMemcpyDeviceToHost, sx);
        if (e == hipSuccess) e = hipEventRecord(copied[b], sx);
        if (e == hipSuccess && timed) {
            float ms0 = 0.f;
            // the first panel's kernel times (one synchronisation, at the end of the first panel)
            if (hipEventSynchronize(t_end) == hipSuccess && hipEventElapsedTime(&ms0, t_start, t_local) == hipSuccess)
                local_s = 1e-3 * ms0;
            if (st) {
                float ms1 = 0.f;
                if (hipEventElapsedTime(&ms1, t_local, t_end) == hipSuccess) st->first_gather_seconds = 1e-3 * ms1;
                st->first_local_seconds = local_s;
                st->first_pairs = (int64_t)P.tris.size() * ntrial;
            }
        }
    }
    if (e == hipSuccess) e = finish(panels.size() - 1);
    if (e != hipSuccess) rc = fail(BEM_E_DEVICE, std::string("dense block: ") + hipGetErrorString(e));
    cleanup();
    if (st && rc == BEM_OK) {
        st->pairs = pairs;
        st->panels = (int64_t)panels.size();
        st->seconds = now_seconds() - t0;
    }
    return rc;
}

}  // namespace bem
