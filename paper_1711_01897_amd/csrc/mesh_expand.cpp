// Mesh residency and request expansion (host side).
//
// A request A[rows, cols] becomes work for the entry kernels:
//  * P0 (dof = triangle): entry (i, j) is the single triangle pair (T_i, T_j).
//    The longer of the two index lists runs across the lanes of a workgroup
//    (in chunks of 256), the other one is the workgroup's fixed side.
//  * P1 (dof = vertex, hat functions, Section 2): entry (I, J) sums over the
//    triangles m around I and n around J.  With the column side on the lanes,
//    the requested columns are cut into runs whose stars together hold at
//    most 256 triangles; each run's triangles form one chunk of lanes, every
//    lane triangle serving each of its requested vertices in the run, and the
//    fixed side of a workgroup is the star of one row vertex.  A segment list
//    maps every requested column to its (lane triangle, local vertex) partial
//    sums in ascending triangle order, which fixes the order of the final
//    per-entry sum.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <string>

#include "bem_internal.hpp"

namespace bem {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

const char *last_error() { return g_last_error.c_str(); }

double now_seconds()
{
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

bool is_complex_op(int op)
{
    return op == BEM_HELMHOLTZ_SLP || op == BEM_HELMHOLTZ_DLP || op == BEM_HELMHOLTZ_ADLP || op == BEM_HELMHOLTZ_HYPS;
}

bool is_adjoint_op(int op) { return op == BEM_LAPLACE_ADLP || op == BEM_HELMHOLTZ_ADLP; }

int64_t space_ndof(const bem_mesh &m, int space)
{
    return space == BEM_P0 ? m.nt : (space == BEM_P1 ? m.nv : 3 * m.nt);
}

int kernel_op(int op)
{
    if (op == BEM_LAPLACE_ADLP) return BEM_LAPLACE_DLP;
    if (op == BEM_HELMHOLTZ_ADLP) return BEM_HELMHOLTZ_DLP;
    return op;
}

size_t out_elem_bytes(int op, int prec)
{
    const size_t real = prec == BEM_FP32 ? 4 : 8;
    return is_complex_op(op) ? 2 * real : real;
}

namespace {

// Per-thread scratch mapping triangles to lane slots.
struct StarScratch {
    std::vector<int32_t> slot_of;
    std::vector<uint32_t> stamp;
    uint32_t gen = 0;
    void prepare(int64_t nt)
    {
        if ((int64_t)stamp.size() < nt) {
            stamp.assign(nt, 0);
            slot_of.assign(nt, -1);
            gen = 0;
        }
        next_gen();
    }
    void next_gen()
    {
        if (++gen == 0) {
            std::fill(stamp.begin(), stamp.end(), 0);
            gen = 1;
        }
    }
};
thread_local StarScratch g_scratch;

size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

void expand_fixed(const bem_mesh &m, int space, const int32_t *dofs, int64_t n, Request &r)
{
    r.fix.clear();
    r.nstar = 0;
    if (space == BEM_P0) {
        r.fix.assign(dofs, dofs + n);
    } else if (space == BEM_P1) {
        // the fixed dofs' stars stay in the mesh's star table: ranges only
        r.fix.resize(2 * n);
        for (int64_t f = 0; f < n; ++f) {
            const int32_t v = dofs[f];
            r.fix[2 * f] = (int32_t)m.star_ptr[v];
            r.fix[2 * f + 1] = (int32_t)m.star_ptr[v + 1];
            r.nstar += m.star_ptr[v + 1] - m.star_ptr[v];
        }
    } else {
        // DP1: a dof is the one-triangle star (t, a), one entry of the star table
        r.fix.resize(2 * n);
        for (int64_t f = 0; f < n; ++f) {
            r.fix[2 * f] = m.dp1_star[dofs[f]];
            r.fix[2 * f + 1] = r.fix[2 * f] + 1;
        }
        r.nstar = n;
    }
    r.nfix = n;
}

void finalize_sizes(Request &r)
{
    const bem_mesh &m = *r.mesh;
    const int64_t q2 = (int64_t)m.q * m.q;
    r.elem_bytes = out_elem_bytes(r.op, r.prec);
    const int64_t fixed_tris = r.space == BEM_P0 ? r.nfix : r.nstar;
    r.evals = fixed_tris * r.ndistinct * q2;
    r.nblocks = r.nfix * r.nchunk;
    const size_t own = r.ext ? 0 : r.own.ints();
    r.in_bytes = align16(4 * own);
    r.out_bytes = align16((size_t)r.entries() * r.elem_bytes);
    r.batch_bytes = request_bytes(r);
}

}  // namespace

namespace {

// 30-bit Morton code of a point in the mesh's bounding box (10 bits per axis).
uint32_t morton3(double x, double y, double z, const double *lo, const double *inv)
{
    auto spread = [](uint32_t v) {
        v &= 1023u;
        v = (v | (v << 16)) & 0x030000FFu;
        v = (v | (v << 8)) & 0x0300F00Fu;
        v = (v | (v << 4)) & 0x030C30C3u;
        v = (v | (v << 2)) & 0x09249249u;
        return v;
    };
    auto q = [](double t) { return (uint32_t)std::min(1023.0, std::max(0.0, t * 1023.0)); };
    return spread(q((x - lo[0]) * inv[0])) | (spread(q((y - lo[1]) * inv[1])) << 1) |
           (spread(q((z - lo[2]) * inv[2])) << 2);
}

}  // namespace

void build_lane_set(const bem_mesh &m, int space, const int32_t *dofs, int64_t n, LaneSet &ls, bool reorder)
{
    ls.pos.clear();
    if (reorder && space != BEM_P0 && n > kBlockLanes) {
        std::vector<std::pair<uint32_t, int32_t>> key((size_t)n);
        for (int64_t i = 0; i < n; ++i) {
            // P1: the vertex; DP1: the first vertex of the dof's triangle
            const int32_t v = space == BEM_P1 ? dofs[i] : m.tri[3 * (size_t)(dofs[i] / 3)];
            const double *x = &m.xyz[3 * (size_t)v];
            key[i] = {morton3(x[0], x[1], x[2], m.box_lo, m.box_inv), (int32_t)i};
        }
        std::sort(key.begin(), key.end());
        std::vector<int32_t> sorted((size_t)n);
        ls.pos.resize((size_t)n);
        for (int64_t i = 0; i < n; ++i) {
            sorted[i] = dofs[key[i].second];
            ls.pos[i] = key[i].second;
        }
        std::vector<int32_t> keep;
        keep.swap(ls.pos);
        build_lane_set(m, space, sorted.data(), n, ls, false);
        ls.pos.swap(keep);
        return;
    }
    ls.ndof = n;
    ls.lane.clear();
    ls.chunk.clear();
    ls.seg_ptr.clear();
    ls.seg.clear();
    if (space == BEM_P0) {
        ls.lane.assign(dofs, dofs + n);
        ls.ndistinct = n;
        for (int64_t c0 = 0; c0 < n; c0 += kBlockLanes) {
            const int32_t len = (int32_t)std::min<int64_t>(kBlockLanes, n - c0);
            ls.chunk.insert(ls.chunk.end(), {(int32_t)c0, len, (int32_t)c0, len});
        }
        return;
    }
    // P1: walk the dofs in order; a dof joins the open chunk while the
    // union of the chunk's stars stays within kBlockLanes triangles
    StarScratch &sc = g_scratch;
    sc.prepare(m.nt);
    ls.seg_ptr.resize(n + 1);
    ls.seg_ptr[0] = 0;
    int32_t lane0 = 0, count = 0;
    int64_t dof0 = 0;
    auto close = [&](int64_t end) {
        ls.chunk.insert(ls.chunk.end(), {lane0, count, (int32_t)dof0, (int32_t)(end - dof0)});
        lane0 += count;
        count = 0;
        dof0 = end;
        sc.next_gen();
    };
    // the star-table range of a dof: its vertex's star (P1) or the one entry
    // of its triangle and local vertex (DP1)
    auto range = [&](int32_t d, int64_t &b, int64_t &e) {
        if (space == BEM_P1) {
            b = m.star_ptr[d];
            e = m.star_ptr[d + 1];
        } else {
            b = m.dp1_star[d];
            e = b + 1;
        }
    };
    for (int64_t c = 0; c < n; ++c) {
        int64_t sb, se;
        range(dofs[c], sb, se);
        int32_t fresh = 0;
        for (int64_t s = sb; s < se; ++s) fresh += sc.stamp[m.star[s] >> 2] != sc.gen;
        if (count + fresh > kBlockLanes && c > dof0) close(c);
        for (int64_t s = sb; s < se; ++s) {
            const int32_t t = m.star[s] >> 2;
            if (sc.stamp[t] != sc.gen) {
                sc.stamp[t] = sc.gen;
                sc.slot_of[t] = count++;
                ls.lane.push_back(t);
            }
            ls.seg.push_back((sc.slot_of[t] << 2) | (m.star[s] & 3));
        }
        ls.seg_ptr[c + 1] = (int32_t)ls.seg.size();
    }
    if (n > dof0) close(n);
    // distinct triangles over all chunks
    ls.ndistinct = 0;
    for (int32_t t : ls.lane)
        if (sc.stamp[t] != sc.gen) {
            sc.stamp[t] = sc.gen;
            ++ls.ndistinct;
        }
    sc.next_gen();
}

namespace {

// Largest |c| over a singular item's integration domain, where the device
// writes x - y = rho c with the radius rho in [0, 1] and the Helmholtz
// radial integrals take omega = k |c| (near.hip).  |c| is convex in each
// coordinate of the (bi)linear parameterisations, so its maximum sits at the
// corners of the parameter domain:
//   identical:     c runs along the three edge vectors, the longest edge;
//   common edge:   c = dh E + s1 a - s2 b on four faces, dh in {0, +-1},
//                  s1, s2 in {0, 1} at the corners;
//   common vertex: c = a(u) - z b(v) or z a(u) - b(v), u, v, z in {0, 1}.
double near_span(const NearItem &q)
{
    auto dist = [](const double *a, const double *b) {
        const double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
        return std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    };
    const double *v = q.v;
    if (q.kind == 0) return std::max(std::max(dist(v + 3, v), dist(v + 6, v + 3)), dist(v + 6, v));
    if (q.kind == 1) {
        double E[3], a[3], b[3];
        for (int d = 0; d < 3; ++d) {
            E[d] = v[3 + d] - v[d];
            a[d] = v[6 + d] - v[d];
            b[d] = v[9 + d] - v[d];
        }
        double best = 0.0;
        for (int face = 0; face < 4; ++face)
            for (int p = 0; p <= 1; ++p)
                for (int qq = 0; qq <= 1; ++qq) {
                    double dh, s1, s2;
                    if (face == 0) dh = p, s1 = (1 - p) * qq, s2 = 1;
                    else if (face == 1) dh = p, s1 = 1 - p, s2 = qq;
                    else if (face == 2) dh = -p, s1 = 1, s2 = (1 - p) * qq;
                    else dh = -p, s1 = qq, s2 = 1 - p;
                    double c2 = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        const double c = dh * E[d] + s1 * a[d] - s2 * b[d];
                        c2 += c * c;
                    }
                    best = std::max(best, std::sqrt(c2));
                }
        return best;
    }
    const double *P = v, *T[2] = {v + 3, v + 6}, *S[2] = {v + 9, v + 12};
    double best = 0.0;
    for (int i = 0; i < 2; ++i) {
        best = std::max(best, std::max(dist(T[i], P), dist(S[i], P)));
        for (int j = 0; j < 2; ++j) best = std::max(best, dist(T[i], S[j]));
    }
    return best;
}

// The 48-term radial series of the Helmholtz singular pairs holds ~1e-14
// relative accuracy at omega = 6 and ~5e-10 at 12, then fails quickly (its
// largest terms grow like omega^n / n!): requests whose items reach beyond
// kOmegaMax are refused.
constexpr double kOmegaMax = 12.0;

int check_near_omega(const Request &r)
{
    if (!is_complex_op(r.op)) return BEM_OK;
    double span = 0.0;
    for (const NearItem &q : r.near_items) span = std::max(span, near_span(q));
    if (r.k * span > kOmegaMax)
        return fail(BEM_E_ARG, "BEM_NEAR_SINGULAR Helmholtz pair with k |x - y| up to " + std::to_string(r.k * span) +
                                   " > 12: the singular scheme's radial series is accurate only below that (the mesh "
                                   "needs more than about one element per wavelength)");
    return BEM_OK;
}

// The vertex-sharing pairs of a P0 request in the layouts of NearItem.  The
// kernels' test triangle is the row's (the column's for the adjoint double
// layer, evaluated as the transposed double layer).
void build_near_items(Request &r)
{
    const bem_mesh &m = *r.mesh;
    const bool adj = is_adjoint_op(r.op);
    std::vector<std::pair<int32_t, int64_t>> colpos((size_t)r.ncols);
    for (int64_t c = 0; c < r.ncols; ++c) colpos[c] = {r.cols[c], c};
    std::sort(colpos.begin(), colpos.end());
    auto vtx = [&](int32_t t, int k) { return &m.xyz[3 * (size_t)m.tri[3 * (size_t)t + k]]; };
    auto put3 = [](double *dst, const double *src) {
        dst[0] = src[0];
        dst[1] = src[1];
        dst[2] = src[2];
    };
    auto cross_len = [&](int32_t t, double *n) {
        const double *a = vtx(t, 0), *b = vtx(t, 1), *c = vtx(t, 2);
        const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        const double N[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        const double J = std::sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
        if (n)
            for (int d = 0; d < 3; ++d) n[d] = N[d] / J;
        return J;
    };
    std::vector<int32_t> nb;
    for (int64_t ri = 0; ri < r.nrows; ++ri) {
        const int32_t a = r.rows[ri];
        nb.clear();
        for (int k = 0; k < 3; ++k) {
            const int32_t v = m.tri[3 * (size_t)a + k];
            for (int64_t s = m.star_ptr[v]; s < m.star_ptr[v + 1]; ++s) nb.push_back(m.star[s] >> 2);
        }
        std::sort(nb.begin(), nb.end());
        nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
        for (int32_t b : nb) {
            auto it = std::lower_bound(colpos.begin(), colpos.end(), std::make_pair(b, (int64_t)-1));
            for (; it != colpos.end() && it->first == b; ++it) {
                const int32_t T = adj ? b : a, S = adj ? a : b;   // kernel test and trial triangles
                NearItem q{};
                const int32_t *tv = &m.tri[3 * (size_t)T], *sv = &m.tri[3 * (size_t)S];
                int shared = 0, ts[3], ss[3];
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        if (tv[i] == sv[j]) {
                            ts[shared] = i;
                            ss[shared] = j;
                            ++shared;
                        }
                q.k = is_complex_op(r.op) ? r.k : 0.0;
                q.jt = cross_len(T, nullptr);
                q.js = cross_len(S, q.ny);
                if (shared == 3) {
                    // the double layer of a flat triangle on itself vanishes ((x - y).n_y = 0)
                    if (kernel_op(r.op) == BEM_LAPLACE_DLP || kernel_op(r.op) == BEM_HELMHOLTZ_DLP) continue;
                    q.kind = 0;
                    for (int k = 0; k < 3; ++k) put3(q.v + 3 * k, vtx(T, k));
                } else if (shared == 2) {
                    q.kind = 1;
                    put3(q.v, vtx(T, ts[0]));
                    put3(q.v + 3, vtx(T, ts[1]));
                    put3(q.v + 6, vtx(T, 3 - ts[0] - ts[1]));
                    put3(q.v + 9, vtx(S, 3 - ss[0] - ss[1]));
                } else {
                    q.kind = 2;
                    put3(q.v, vtx(T, ts[0]));
                    put3(q.v + 3, vtx(T, (ts[0] + 1) % 3));
                    put3(q.v + 6, vtx(T, (ts[0] + 2) % 3));
                    put3(q.v + 9, vtx(S, (ss[0] + 1) % 3));
                    put3(q.v + 12, vtx(S, (ss[0] + 2) % 3));
                }
                r.near_items.push_back(q);
                r.near_index.push_back(ri * r.ncols + it->second);
            }
        }
    }
}

// The vertex-sharing pairs of a P1 (or DP1) request and, per output entry,
// the local matrix values that sum into it.  A pair (a on the row side, b
// adjacent to it) counts if a lies in the star of a requested row vertex
// (DP1: is the triangle of a requested row dof) and b touches a requested
// column vertex (DP1: is the triangle of a requested column dof); its local
// matrix M[i][j] (kernel test vertex i, trial vertex j) goes to the entries
// of the row and column positions of those vertices (DP1: of the dofs (a, i)
// and (b, j), one entry each), exchanged for the adjoint double layer.
void build_near_items_p1(Request &r)
{
    const bem_mesh &m = *r.mesh;
    const bool adj = is_adjoint_op(r.op);
    const bool dlp = kernel_op(r.op) == BEM_LAPLACE_DLP || kernel_op(r.op) == BEM_HELMHOLTZ_DLP;
    const bool hyps = r.op == BEM_LAPLACE_HYPS, hhyps = r.op == BEM_HELMHOLTZ_HYPS;
    std::vector<std::pair<int32_t, int64_t>> rowpos((size_t)r.nrows), colpos((size_t)r.ncols);
    for (int64_t i = 0; i < r.nrows; ++i) rowpos[i] = {r.rows[i], i};
    for (int64_t i = 0; i < r.ncols; ++i) colpos[i] = {r.cols[i], i};
    std::sort(rowpos.begin(), rowpos.end());
    std::sort(colpos.begin(), colpos.end());
    auto first_of = [](const std::vector<std::pair<int32_t, int64_t>> &v, int32_t x) {
        return std::lower_bound(v.begin(), v.end(), std::make_pair(x, (int64_t)-1));
    };
    auto vtx = [&](int32_t t, int k) { return &m.xyz[3 * (size_t)m.tri[3 * (size_t)t + k]]; };
    auto put3 = [](double *dst, const double *src) {
        dst[0] = src[0];
        dst[1] = src[1];
        dst[2] = src[2];
    };
    auto cross_len = [&](int32_t t, double *n) {
        const double *a = vtx(t, 0), *b = vtx(t, 1), *c = vtx(t, 2);
        const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        const double N[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        const double J = std::sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
        if (n)
            for (int d = 0; d < 3; ++d) n[d] = N[d] / J;
        return J;
    };
    auto star_of = [&](const int32_t *verts, int nv, std::vector<int32_t> &out) {
        out.clear();
        for (int k = 0; k < nv; ++k)
            for (int64_t s = m.star_ptr[verts[k]]; s < m.star_ptr[verts[k] + 1]; ++s) out.push_back(m.star[s] >> 2);
        std::sort(out.begin(), out.end());
        out.erase(std::unique(out.begin(), out.end()), out.end());
    };
    // P1 dofs are vertices; a DP1 dof is (triangle t, local vertex) = 3 t + local
    const bool dp1 = r.space == BEM_DP1;
    auto dof_of = [&](int32_t t, int32_t v) -> int32_t {
        if (!dp1) return v;
        int i = 0;
        while (m.tri[3 * (size_t)t + i] != v) ++i;
        return 3 * t + i;
    };
    std::vector<int32_t> rt, nb;
    {
        std::vector<int32_t> rv(r.rows.begin(), r.rows.end());
        std::sort(rv.begin(), rv.end());
        rv.erase(std::unique(rv.begin(), rv.end()), rv.end());
        rt.clear();
        for (int32_t v : rv) {
            if (dp1) {
                rt.push_back(v / 3);
                continue;
            }
            for (int64_t s = m.star_ptr[v]; s < m.star_ptr[v + 1]; ++s) rt.push_back(m.star[s] >> 2);
        }
        std::sort(rt.begin(), rt.end());
        rt.erase(std::unique(rt.begin(), rt.end()), rt.end());
    }
    // surface curl of the hat function of global vertex v on triangle t: with
    // the mesh's vertex order (v0, v1, v2) and J = |(v1 - v0) x (v2 - v0)|,
    // curl lambda_i = (v_{i+1} - v_{i+2}) / J
    auto curl = [&](int32_t t, int32_t v, double *c) {
        int i = 0;
        while (m.tri[3 * (size_t)t + i] != v) ++i;
        const double *p1 = vtx(t, (i + 1) % 3), *p2 = vtx(t, (i + 2) % 3);
        const double J = cross_len(t, nullptr);
        for (int d = 0; d < 3; ++d) c[d] = (p1[d] - p2[d]) / J;
    };
    struct Contrib {
        int64_t entry;
        int32_t src;
        double wt;
        bool operator<(const Contrib &o) const { return entry != o.entry ? entry < o.entry : src < o.src; }
    };
    std::vector<Contrib> contrib;
    for (int32_t a : rt) {
        star_of(&m.tri[3 * (size_t)a], 3, nb);
        for (int32_t b : nb) {
            bool touches = false;
            for (int k = 0; k < 3 && !touches; ++k) {
                const int32_t v = dp1 ? 3 * b + k : m.tri[3 * (size_t)b + k];
                auto it = first_of(colpos, v);
                touches = it != colpos.end() && it->first == v;
            }
            if (!touches) continue;
            const int32_t T = adj ? b : a, S = adj ? a : b;   // kernel test and trial triangles
            const int32_t *tv = &m.tri[3 * (size_t)T], *sv = &m.tri[3 * (size_t)S];
            int shared = 0, ts[3], ss[3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    if (tv[i] == sv[j]) {
                        ts[shared] = i;
                        ss[shared] = j;
                        ++shared;
                    }
            if (shared == 3 && dlp) continue;   // (x - y).n_y = 0 on a flat triangle
            NearItem q{};
            q.k = is_complex_op(r.op) ? r.k : 0.0;
            int32_t tl[3], sl[3];   // global vertices in the kernel's local orders
            double nt[3];
            q.jt = cross_len(T, nt);
            q.js = cross_len(S, q.ny);
            if (shared == 3) {
                q.kind = 0;
                for (int k = 0; k < 3; ++k) {
                    put3(q.v + 3 * k, vtx(T, k));
                    tl[k] = sl[k] = tv[k];
                }
            } else if (shared == 2) {
                q.kind = 1;
                const int t3 = 3 - ts[0] - ts[1], s3 = 3 - ss[0] - ss[1];
                put3(q.v, vtx(T, ts[0]));
                put3(q.v + 3, vtx(T, ts[1]));
                put3(q.v + 6, vtx(T, t3));
                put3(q.v + 9, vtx(S, s3));
                tl[0] = tv[ts[0]], tl[1] = tv[ts[1]], tl[2] = tv[t3];
                sl[0] = sv[ss[0]], sl[1] = sv[ss[1]], sl[2] = sv[s3];
            } else {
                q.kind = 2;
                for (int k = 0; k < 3; ++k) {
                    put3(q.v + 3 * k, vtx(T, (ts[0] + k) % 3));
                    tl[k] = tv[(ts[0] + k) % 3];
                }
                put3(q.v + 9, vtx(S, (ss[0] + 1) % 3));
                put3(q.v + 12, vtx(S, (ss[0] + 2) % 3));
                for (int k = 0; k < 3; ++k) sl[k] = sv[(ss[0] + k) % 3];
            }
            const int32_t pi = (int32_t)r.near_items.size();
            r.near_items.push_back(q);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    const int32_t rv = adj ? dof_of(S, sl[j]) : dof_of(T, tl[i]);
                    const int32_t cv = adj ? dof_of(T, tl[i]) : dof_of(S, sl[j]);
                    double w = 1.0;
                    if (hyps || hhyps) {
                        double ct[3], cs[3];
                        curl(T, tl[i], ct);
                        curl(S, sl[j], cs);
                        w = ct[0] * cs[0] + ct[1] * cs[1] + ct[2] * cs[2];
                    }
                    // Helmholtz hypersingular: curl products times the P0 value (source 9 of the pair)
                    // minus k^2 n_x . n_y times the single layer's local matrix
                    const double wn = -r.k * r.k * (nt[0] * q.ny[0] + nt[1] * q.ny[1] + nt[2] * q.ny[2]);
                    for (auto ri = first_of(rowpos, rv); ri != rowpos.end() && ri->first == rv; ++ri)
                        for (auto ci = first_of(colpos, cv); ci != colpos.end() && ci->first == cv; ++ci) {
                            const int64_t e = ri->second * r.ncols + ci->second;
                            if (hhyps) {
                                contrib.push_back({e, pi * 10 + 9, w});
                                contrib.push_back({e, pi * 10 + 3 * i + j, wn});
                            } else {
                                contrib.push_back({e, hyps ? pi : pi * 9 + 3 * i + j, w});
                            }
                        }
                }
        }
    }
    std::sort(contrib.begin(), contrib.end());
    r.near_src.resize(contrib.size());
    if (hyps || hhyps) r.near_wt.resize(contrib.size());
    for (size_t k = 0; k < contrib.size(); ++k) {
        r.near_src[k] = contrib[k].src;
        if (hyps || hhyps) r.near_wt[k] = contrib[k].wt;
        if (k == 0 || contrib[k].entry != contrib[k - 1].entry)
            r.near_recs.push_back({contrib[k].entry, (int32_t)k, 0});
        ++r.near_recs.back().count;
    }
}

}  // namespace

static size_t align256_sz(size_t x) { return (x + 255) & ~(size_t)255; }

NearP1Layout near_p1_layout(int mode, int64_t items, int64_t recs, int64_t src)
{
    NearP1Layout L;
    L.per = mode == 1 ? 1 : (mode == 2 ? 18 : (mode == 3 ? 20 : 9));
    L.src_per = mode == 1 ? 1 : (mode == 3 ? 10 : 9);
    L.weighted = mode == 1 || mode == 3;
    L.cplx = mode >= 2;
    L.items = 0;
    L.recs = align256_sz(sizeof(NearItem) * (size_t)items);
    L.src = L.recs + align256_sz(sizeof(NearGather) * (size_t)recs);
    L.wt = L.src + align256_sz(sizeof(int32_t) * (size_t)src);
    L.local = L.wt + (L.weighted ? align256_sz(sizeof(double) * (size_t)src) : 0);
    L.bytes = L.local + align256_sz(L.per * sizeof(double) * (size_t)items);
    return L;
}

int near_p1_mode(const Request &r)
{
    return r.op == BEM_LAPLACE_HYPS ? 1 : (r.op == BEM_HELMHOLTZ_HYPS ? 3 : (is_complex_op(r.op) ? 2 : 0));
}

NearP1Layout near_p1_layout(const Request &r)
{
    return near_p1_layout(near_p1_mode(r), (int64_t)r.near_items.size(), (int64_t)r.near_recs.size(),
                          (int64_t)r.near_src.size());
}

int near_p1_group(const Request &r)
{
    const int kop = kernel_op(r.op);
    const int g = r.op == BEM_LAPLACE_HYPS   ? 2
                : r.op == BEM_HELMHOLTZ_HYPS ? 5
                : kop == BEM_HELMHOLTZ_SLP   ? 3
                : kop == BEM_HELMHOLTZ_DLP   ? 4
                                             : kop;
    return 2 * g + (r.prec == BEM_FP32 ? 1 : 0);
}

void stage_near_p1(const Request &r, const NearP1Layout &L, char *host, char *dev, char *out_dev, int64_t pb,
                   int64_t rb, int64_t sb)
{
    NearItem *q = reinterpret_cast<NearItem *>(host + L.items) + pb;
    for (size_t j = 0; j < r.near_items.size(); ++j) {
        q[j] = r.near_items[j];
        q[j].out = dev + L.local + L.per * sizeof(double) * ((size_t)pb + j);
    }
    NearGather *g = reinterpret_cast<NearGather *>(host + L.recs) + rb;
    for (size_t j = 0; j < r.near_recs.size(); ++j)
        g[j] = {out_dev + (size_t)r.near_recs[j].entry * r.elem_bytes, (int32_t)(sb + r.near_recs[j].first),
                r.near_recs[j].count};
    int32_t *src = reinterpret_cast<int32_t *>(host + L.src) + sb;
    for (size_t j = 0; j < r.near_src.size(); ++j) src[j] = (int32_t)(L.src_per * pb) + r.near_src[j];
    if (L.weighted && !r.near_wt.empty())
        std::memcpy(reinterpret_cast<double *>(host + L.wt) + sb, r.near_wt.data(), sizeof(double) * r.near_wt.size());
}

hipError_t launch_near_p1_region(int op, bool fp32, const NearP1Layout &L, char *dev, int64_t items, int64_t recs,
                                 hipStream_t s)
{
    hipError_t e = launch_near_p1(op, reinterpret_cast<const NearItem *>(dev + L.items), items, s);
    if (e != hipSuccess) return e;
    return launch_near_gather(fp32, L.cplx, reinterpret_cast<const NearGather *>(dev + L.recs), recs,
                              reinterpret_cast<const int32_t *>(dev + L.src),
                              L.weighted ? reinterpret_cast<const double *>(dev + L.wt) : nullptr,
                              reinterpret_cast<const double *>(dev + L.local), s);
}

int expand_request(Request &r)
{
    const bem_mesh &m = *r.mesh;
    if (r.op < 0 || r.op > 7) return fail(BEM_E_ARG, "unknown operator");
    if (r.space != BEM_P0 && r.space != BEM_P1 && r.space != BEM_DP1) return fail(BEM_E_ARG, "unknown space");
    if ((r.op == BEM_LAPLACE_HYPS || r.op == BEM_HELMHOLTZ_HYPS) && r.space != BEM_P1)
        return fail(BEM_E_ARG, "the hypersingular operator needs continuous (P1) functions");
    if (r.prec != BEM_FP32 && r.prec != BEM_FP64) return fail(BEM_E_ARG, "unknown precision");
    if (r.near != BEM_NEAR_ERROR && r.near != BEM_NEAR_SKIP && r.near != BEM_NEAR_SINGULAR)
        return fail(BEM_E_ARG, "unknown near-field policy");
    if (is_complex_op(r.op)) {
        if (!(std::isfinite(r.k) && r.k > 0.0)) return fail(BEM_E_ARG, "Helmholtz needs a finite wavenumber k > 0");
    } else if (r.k != 0.0) {
        return fail(BEM_E_ARG, "Laplace needs k = 0");
    }
    const int64_t ndof = space_ndof(m, r.space);
    for (int32_t v : r.rows)
        if (v < 0 || v >= ndof) return fail(BEM_E_ARG, "row index out of range");
    for (int32_t v : r.cols)
        if (v < 0 || v >= ndof) return fail(BEM_E_ARG, "column index out of range");
    if (r.nrows > INT32_MAX || r.ncols > INT32_MAX) return fail(BEM_E_ARG, "request dimension too large");

    r.ext = nullptr;
    // the smaller side is fixed; an adjoint double layer is evaluated as the
    // double layer with test and trial exchanged (Eqs. dlp, adlp:
    // [K'_h]_ij = [K_h]_ji for the same space on both sides)
    r.fixrows = r.ncols >= r.nrows ? 1 : 0;
    r.rowfix = is_adjoint_op(r.op) ? 1 - r.fixrows : r.fixrows;
    const std::vector<int32_t> &fix_dofs = r.fixrows ? r.rows : r.cols;
    const std::vector<int32_t> &lane_dofs = r.fixrows ? r.cols : r.rows;
    expand_fixed(m, r.space, fix_dofs.data(), (int64_t)fix_dofs.size(), r);
    build_lane_set(m, r.space, lane_dofs.data(), (int64_t)lane_dofs.size(), r.own, true);
    r.nlane = (int64_t)r.own.lane.size();
    r.nchunk = r.own.nchunk();
    r.ndistinct = r.own.ndistinct;
    r.near_items.clear();
    r.near_index.clear();
    r.near_recs.clear();
    r.near_src.clear();
    r.near_wt.clear();
    if (r.near == BEM_NEAR_SINGULAR) {
        if (r.space == BEM_P0)
            build_near_items(r);
        else
            build_near_items_p1(r);
        const int rc = check_near_omega(r);
        if (rc != BEM_OK) return rc;
    }
    finalize_sizes(r);
    return BEM_OK;
}

void expand_single_fixed(Request &r, int32_t dof, int rowfix, const LaneRef *ext)
{
    r.near_items.clear();
    r.near_index.clear();
    r.near_recs.clear();
    r.near_src.clear();
    r.near_wt.clear();
    r.ext = ext;
    r.fixrows = rowfix;
    r.rowfix = is_adjoint_op(r.op) ? 1 - rowfix : rowfix;
    r.own.lane.clear();
    r.own.chunk.clear();
    r.own.seg_ptr.clear();
    r.own.seg.clear();
    r.own.pos.clear();
    expand_fixed(*r.mesh, r.space, &dof, 1, r);
    r.nlane = ext->nlane;
    r.nchunk = ext->nchunk;
    r.ndistinct = ext->ndistinct;
    if (r.fixrows) {
        r.nrows = 1;
        r.ncols = ext->ndof;
    } else {
        r.nrows = ext->ndof;
        r.ncols = 1;
    }
    finalize_sizes(r);
}

size_t request_bytes(const Request &r)
{
    // descriptor, inputs, status, outputs, block table, launch-timing records
    return sizeof(ReqDev) + r.in_bytes + 8 + r.out_bytes + (size_t)r.nblocks * (sizeof(EntryBlock) + 16) +
           (r.space != BEM_P0 ? near_p1_layout(r).bytes : r.near_items.size() * sizeof(NearItem)) + 512;
}

void describe_request(const Request &r, ReqDev &d)
{
    const bem_mesh &m = *r.mesh;
    d.g32 = m.d_g32;
    d.g64 = m.d_g64;
    d.vtx = m.d_vtx;
    if (r.ext) {
        d.chunk = r.ext->chunk;
        d.lane = r.ext->lane;
        d.seg_ptr = r.ext->seg_ptr;
        d.seg = r.ext->seg;
    } else {
        d.chunk = nullptr;
        d.lane = d.seg_ptr = d.seg = nullptr;
    }
    d.lpos = nullptr;
    d.fstar = m.d_star;
    if (r.fixrows) {   // output position of (fixed f, lane-side dof d): out[f * sf + d * sl]
        d.sf = r.ncols;
        d.sl = 1;
    } else {
        d.sf = 1;
        d.sl = r.ncols;
    }
    d.nrows = (int32_t)r.nrows;
    d.ncols = (int32_t)r.ncols;
    d.nlane = (int32_t)r.nlane;
    d.nfix = (int32_t)r.nfix;
    d.rowfix = r.rowfix;
    d.near_error = r.near == BEM_NEAR_ERROR ? 1 : 0;
    d.k = r.k;
    d.kk = r.k / (2.0 * 3.14159265358979323846);
    d.out = nullptr;
    d.status = nullptr;
}

size_t stage_own_inputs(const Request &r, char *host_base, char *dev_base, size_t off, ReqDev &d)
{
    if (r.ext) return r.in_bytes;
    char *h = host_base + off;
    char *dv = dev_base + off;
    auto put = [&](const std::vector<int32_t> &v) -> const int32_t * {
        if (v.empty()) return nullptr;
        std::memcpy(h, v.data(), 4 * v.size());
        const int32_t *dp = reinterpret_cast<const int32_t *>(dv);
        h += 4 * v.size();
        dv += 4 * v.size();
        return dp;
    };
    // the chunk table (int4 records) goes first: the section starts 16-byte aligned
    d.chunk = reinterpret_cast<const int4 *>(put(r.own.chunk));
    d.lane = put(r.own.lane);
    d.seg_ptr = put(r.own.seg_ptr);
    d.seg = put(r.own.seg);
    d.lpos = put(r.own.pos);
    return r.in_bytes;
}

size_t stage_request_inputs(Request &r, char *host_base, char *dev_base, size_t off, ReqDev &d)
{
    describe_request(r, d);
    return stage_own_inputs(r, host_base, dev_base, off, d);
}

void finish_descriptor(const Request &r, char *dev_base, size_t off_out, size_t off_status, ReqDev &d)
{
    (void)r;
    d.out = dev_base + off_out;
    d.status = reinterpret_cast<int32_t *>(dev_base + off_status);
}

int64_t write_blocks(const Request &r, int32_t ri, EntryBlock *out)
{
    const bem_mesh &m = *r.mesh;
    const int32_t *ch = r.ext ? r.ext->chunk_host : r.own.chunk.data();
    const float *lgeo = r.ext ? r.ext->geo : nullptr;
    const int4 *lmeta = r.ext ? r.ext->meta : nullptr;
    int64_t n = 0;
    for (int32_t f = 0; f < (int32_t)r.nfix; ++f) {
        int32_t s0, s1;
        if (r.space == BEM_P0) {
            s0 = r.fix[f];
            s1 = s0 + 1;
        } else {
            s0 = r.fix[2 * f];
            s1 = r.fix[2 * f + 1];
        }
        for (int32_t c = 0; c < (int32_t)r.nchunk; ++c) {
            EntryBlock &b = out[n++];
            b.req = (ri << 1) | (r.rowfix ? 1 : 0);
            b.fixed = f;
            b.s0 = s0;
            b.s1 = s1;
            b.chunk = make_int4(ch[4 * c], ch[4 * c + 1], ch[4 * c + 2], ch[4 * c + 3]);
            b.lgeo = lgeo;
            b.lmeta = r.separated ? nullptr : lmeta;
            // the fixed side's records: P1 star records per star entry, P0
            // the mesh's triangle records
            b.sgeo = r.space != BEM_P0 ? m.d_sgeo : m.d_g32;
            b.smeta = r.space != BEM_P0 ? m.d_smeta : m.d_vtx;
        }
    }
    return n;
}

int request_key(const Request &r)
{
    return ((kernel_op(r.op) * 2 + kernel_space(r.space)) * 2 + r.prec) * 2 + (r.mesh->q == 6 ? 1 : 0);
}

void prebuild_staging(Request &r)
{
    r.key = request_key(r);
    r.pre_blocks.resize((size_t)r.nblocks);
    write_blocks(r, 0, r.pre_blocks.data());
    describe_request(r, r.pre_dev);
}

}  // namespace bem

// ---------------------------------------------------------------------------
// Mesh creation / destruction.
using namespace bem;

namespace bem {
int mesh_create_impl(const double *xyz, int64_t nv, const int32_t *tri, int64_t nt, int q, bem_mesh **out)
{
    if (!xyz || !tri || !out) return fail(BEM_E_ARG, "null pointer");
    if (nv < 3 || nt < 1) return fail(BEM_E_ARG, "mesh needs at least 3 vertices and 1 triangle");
    if (q != 4 && q != 6) return fail(BEM_E_ARG, "quad_points must be 4 or 6");
    if (nt > (INT32_MAX >> 2) || nv > INT32_MAX) return fail(BEM_E_ARG, "mesh too large for 32-bit indices");
    for (int64_t i = 0; i < 3 * nv; ++i)
        if (!std::isfinite(xyz[i])) return fail(BEM_E_ARG, "non-finite vertex coordinate");
    for (int64_t i = 0; i < 3 * nt; ++i)
        if (tri[i] < 0 || tri[i] >= nv) return fail(BEM_E_ARG, "triangle vertex index out of range");
    for (int64_t t = 0; t < nt; ++t)
        if (tri[3 * t] == tri[3 * t + 1] || tri[3 * t] == tri[3 * t + 2] || tri[3 * t + 1] == tri[3 * t + 2])
            return fail(BEM_E_ARG, "triangle with a repeated vertex");

    bem_mesh *m = new (std::nothrow) bem_mesh();
    if (!m) return fail(BEM_E_OOM, "host allocation failed");
    m->nv = nv;
    m->nt = nt;
    m->q = q;
    m->xyz.assign(xyz, xyz + 3 * nv);
    m->tri.assign(tri, tri + 3 * nt);
    m->star_ptr.assign(nv + 1, 0);
    for (int64_t i = 0; i < 3 * nt; ++i) m->star_ptr[tri[i] + 1]++;
    for (int64_t v = 0; v < nv; ++v) m->star_ptr[v + 1] += m->star_ptr[v];
    m->star.resize(3 * nt);
    {
        std::vector<int64_t> fill(m->star_ptr.begin(), m->star_ptr.end() - 1);
        for (int64_t t = 0; t < nt; ++t)
            for (int k = 0; k < 3; ++k) m->star[fill[tri[3 * t + k]]++] = (int32_t)((t << 2) | k);
    }
    m->dp1_star.resize(3 * nt);
    for (int64_t s = 0; s < 3 * nt; ++s) m->dp1_star[3 * (size_t)(m->star[s] >> 2) + (m->star[s] & 3)] = (int32_t)s;
    for (int64_t v = 0; v < nv; ++v) m->max_star = std::max<int>(m->max_star, (int)(m->star_ptr[v + 1] - m->star_ptr[v]));
    if (m->max_star > kBlockLanes) {
        delete m;
        return fail(BEM_E_ARG, "a vertex belongs to more than 256 triangles");
    }
    double sj = 0.0, se = 0.0;
    for (int64_t t = 0; t < nt; ++t) {
        const double *a = &xyz[3 * tri[3 * t]], *b = &xyz[3 * tri[3 * t + 1]], *c = &xyz[3 * tri[3 * t + 2]];
        double e1[3], e2[3];
        for (int d = 0; d < 3; ++d) {
            e1[d] = b[d] - a[d];
            e2[d] = c[d] - a[d];
        }
        const double N[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        sj += std::sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
        double e3[3] = {c[0] - b[0], c[1] - b[1], c[2] - b[2]};
        se += std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]) + std::sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]) +
              std::sqrt(e3[0] * e3[0] + e3[1] * e3[1] + e3[2] * e3[2]);
    }
    m->mean_J = sj / nt;
    m->mean_edge = se / (3.0 * nt);
    for (int d = 0; d < 3; ++d) {
        double lo = INFINITY, hi = -INFINITY;
        for (int64_t v = 0; v < nv; ++v) {
            lo = std::min(lo, xyz[3 * v + d]);
            hi = std::max(hi, xyz[3 * v + d]);
        }
        m->box_lo[d] = lo;
        m->box_inv[d] = hi > lo ? 1.0 / (hi - lo) : 0.0;
    }

    hipError_t e = hipGetDevice(&m->device);
    double *d_xyz = nullptr;
    int32_t *d_tri = nullptr, *d_bad = nullptr;
    const size_t b32 = sizeof(float) * kGeo32Stride * nt, b64 = sizeof(double) * kGeo64Stride * nt,
                 bv = sizeof(int4) * nt;
    int rc = BEM_OK;
    int32_t bad = 0;
    if (e == hipSuccess) e = hipMalloc(&m->d_g32, b32);
    if (e == hipSuccess) e = hipMalloc(&m->d_g64, b64);
    if (e == hipSuccess) e = hipMalloc(&m->d_vtx, bv);
    if (e == hipSuccess) e = hipMalloc(&d_xyz, sizeof(double) * 3 * nv);
    if (e == hipSuccess) e = hipMalloc(&d_tri, sizeof(int32_t) * 3 * nt);
    if (e == hipSuccess) e = hipMalloc(&d_bad, sizeof(int32_t));
    if (e == hipSuccess) e = hipMemcpy(d_xyz, xyz, sizeof(double) * 3 * nv, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_tri, tri, sizeof(int32_t) * 3 * nt, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_bad, &bad, sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_geometry(d_xyz, d_tri, nt, q, m->d_g32, m->d_g64, m->d_vtx, d_bad, 0);
    if (e == hipSuccess) e = hipMemcpy(&bad, d_bad, sizeof(int32_t), hipMemcpyDeviceToHost);
    // star tables: the packed star entries and, per entry, its triangle's
    // FP32 record and vertex ids with the local vertex in w
    const int64_t ns = 3 * nt;
    if (e == hipSuccess) e = hipMalloc(&m->d_star, sizeof(int32_t) * ns);
    if (e == hipSuccess) e = hipMalloc(&m->d_sgeo, sizeof(float) * kGeo32Stride * ns);
    if (e == hipSuccess) e = hipMalloc(&m->d_smeta, sizeof(int4) * ns);
    if (e == hipSuccess) e = hipMemcpy(m->d_star, m->star.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_gather(m->d_g32, m->d_vtx, m->d_star, 2, ns, m->d_sgeo, m->d_smeta, 0);
    if (e == hipSuccess) e = hipStreamSynchronize(0);
    if (d_xyz) (void)hipFree(d_xyz);
    if (d_tri) (void)hipFree(d_tri);
    if (d_bad) (void)hipFree(d_bad);
    if (e != hipSuccess)
        rc = fail(e == hipErrorOutOfMemory ? BEM_E_OOM : BEM_E_DEVICE, std::string("mesh upload: ") + hipGetErrorString(e));
    else if (bad)
        rc = fail(BEM_E_ARG, "degenerate triangle (zero area)");
    if (rc != BEM_OK) {
        for (void *p : {(void *)m->d_g32, (void *)m->d_g64, (void *)m->d_vtx, (void *)m->d_star, (void *)m->d_sgeo,
                        (void *)m->d_smeta})
            if (p) (void)hipFree(p);
        delete m;
        return rc;
    }
    m->dev_bytes = b32 + b64 + bv + 3 * (size_t)nt * (4 + 4 * kGeo32Stride + sizeof(int4));
    *out = m;
    return BEM_OK;
}

int mesh_destroy_impl(bem_mesh *m)
{
    if (!m) return fail(BEM_E_ARG, "null mesh");
    if (m->inflight.load() != 0) return fail(BEM_E_BUSY, "requests on this mesh are still in flight");
    for (void *p : {(void *)m->d_g32, (void *)m->d_g64, (void *)m->d_vtx, (void *)m->d_star, (void *)m->d_sgeo,
                    (void *)m->d_smeta})
        (void)hipFree(p);
    delete m;
    return BEM_OK;
}
}  // namespace bem
