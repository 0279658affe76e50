// Cluster tree and block tree (host, FP64), Section 2.1's geometric
// partition of the matrix into admissible (low-rank) and dense leaves.
//
//  * dof points: triangle centroids (P0, and the three dofs of a triangle
//    for DP1) or vertices (P1); every dof carries
//    a support box, the bounding box of the vertices of the triangles its
//    basis function lives on;
//  * a cluster with more than leaf_size dofs is split at the midpoint of the
//    longest side of its points' bounding box (lowest axis on ties); points
//    below the midpoint go to the first child, keeping their order; if one
//    side would be empty, the dofs are sorted by (coordinate, index) and the
//    first half goes to the first child;
//  * blocks start at (root, root); a block is admissible when the distance
//    of the two support boxes is positive, the smaller support-box
//    diameter is at most eta times that distance and (with max_block > 0)
//    neither cluster holds more than max_block dofs; otherwise it is dense
//    if either cluster is a leaf, else it splits into its four child pairs.
// Support boxes keep every vertex-sharing triangle pair out of admissible
// blocks, so ACA only ever requests regular entries.
#include "tree.hpp"

#include <algorithm>
#include <cmath>

namespace bem {

void dof_geometry(const bem_mesh &m, int space, std::vector<double> &pts, std::vector<double> &slo,
                  std::vector<double> &shi)
{
    const int64_t nt = m.nt, nv = m.nv;
    std::vector<double> tlo(3 * nt), thi(3 * nt);
    for (int64_t t = 0; t < nt; ++t)
        for (int d = 0; d < 3; ++d) {
            const double a = m.xyz[3 * m.tri[3 * t] + d], b = m.xyz[3 * m.tri[3 * t + 1] + d],
                         c = m.xyz[3 * m.tri[3 * t + 2] + d];
            tlo[3 * t + d] = std::min(std::min(a, b), c);
            thi[3 * t + d] = std::max(std::max(a, b), c);
        }
    if (space == BEM_P0 || space == BEM_DP1) {
        // a triangle's dofs (one for P0, three for DP1) sit at its centroid
        // and are supported on it
        const int per = space == BEM_P0 ? 1 : 3;
        pts.resize(3 * per * nt);
        slo.resize(3 * per * nt);
        shi.resize(3 * per * nt);
        for (int64_t t = 0; t < nt; ++t)
            for (int d = 0; d < 3; ++d) {
                const double c = ((m.xyz[3 * m.tri[3 * t] + d] + m.xyz[3 * m.tri[3 * t + 1] + d]) +
                                  m.xyz[3 * m.tri[3 * t + 2] + d]) / 3.0;
                for (int a = 0; a < per; ++a) {
                    pts[3 * (per * t + a) + d] = c;
                    slo[3 * (per * t + a) + d] = tlo[3 * t + d];
                    shi[3 * (per * t + a) + d] = thi[3 * t + d];
                }
            }
        return;
    }
    pts.assign(m.xyz.begin(), m.xyz.end());
    slo.assign(3 * nv, INFINITY);
    shi.assign(3 * nv, -INFINITY);
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k) {
            const int64_t v = m.tri[3 * t + k];
            for (int d = 0; d < 3; ++d) {
                slo[3 * v + d] = std::min(slo[3 * v + d], tlo[3 * t + d]);
                shi[3 * v + d] = std::max(shi[3 * v + d], thi[3 * t + d]);
            }
        }
}

namespace {

struct Builder {
    const std::vector<double> &pts, &slo, &shi;
    int leaf;
    std::vector<int32_t> &perm;
    std::vector<Cluster> &nodes;

    int make(int64_t b, int64_t e)
    {
        const int id = (int)nodes.size();
        nodes.push_back(Cluster());
        Cluster c;
        c.begin = b;
        c.end = e;
        for (int d = 0; d < 3; ++d) {
            c.lo[d] = INFINITY;
            c.hi[d] = -INFINITY;
            c.slo[d] = INFINITY;
            c.shi[d] = -INFINITY;
        }
        for (int64_t i = b; i < e; ++i) {
            const int64_t v = perm[i];
            for (int d = 0; d < 3; ++d) {
                c.lo[d] = std::min(c.lo[d], pts[3 * v + d]);
                c.hi[d] = std::max(c.hi[d], pts[3 * v + d]);
                c.slo[d] = std::min(c.slo[d], slo[3 * v + d]);
                c.shi[d] = std::max(c.shi[d], shi[3 * v + d]);
            }
        }
        nodes[id] = c;
        if (e - b <= leaf) return id;
        int axis = 0;
        double ext = c.hi[0] - c.lo[0];
        for (int d = 1; d < 3; ++d)
            if (c.hi[d] - c.lo[d] > ext) {
                ext = c.hi[d] - c.lo[d];
                axis = d;
            }
        const double mid = (c.lo[axis] + c.hi[axis]) / 2.0;
        auto first = perm.begin() + b, last = perm.begin() + e;
        auto cut = std::stable_partition(first, last, [&](int32_t v) { return pts[3 * v + axis] < mid; });
        int64_t split = b + (cut - first);
        if (split == b || split == e) {
            std::sort(first, last, [&](int32_t x, int32_t y) {
                const double cx = pts[3 * x + axis], cy = pts[3 * y + axis];
                return cx < cy || (cx == cy && x < y);
            });
            split = b + (e - b) / 2;
        }
        const int l = make(b, split);
        const int r = make(split, e);
        nodes[id].child[0] = l;
        nodes[id].child[1] = r;
        return id;
    }
};

double box_diam(const double *lo, const double *hi)
{
    const double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    return std::sqrt(dx * dx + dy * dy + dz * dz);
}

double box_dist(const Cluster &a, const Cluster &b)
{
    double g[3];
    for (int k = 0; k < 3; ++k) g[k] = std::max(0.0, std::max(a.slo[k] - b.shi[k], b.slo[k] - a.shi[k]));
    return std::sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
}

}  // namespace

bool admissible(const Cluster &a, const Cluster &b, double eta, int max_block)
{
    if (max_block > 0 && std::max(a.end - a.begin, b.end - b.begin) > max_block) return false;
    const double d = box_dist(a, b);
    if (!(d > 0.0)) return false;
    return std::min(box_diam(a.slo, a.shi), box_diam(b.slo, b.shi)) <= eta * d;
}

double support_distance(const Cluster &a, const Cluster &b) { return box_dist(a, b); }

void build_partition(const std::vector<double> &pts, const std::vector<double> &slo, const std::vector<double> &shi,
                     int leaf_size, double eta, int max_block, Partition &P)
{
    const int64_t n = (int64_t)pts.size() / 3;
    P.perm.resize(n);
    for (int64_t i = 0; i < n; ++i) P.perm[i] = (int32_t)i;
    P.nodes.clear();
    P.blocks.clear();
    if (n == 0) return;
    Builder B{pts, slo, shi, std::max(1, leaf_size), P.perm, P.nodes};
    B.make(0, n);
    std::vector<std::pair<int, int>> stack{{0, 0}};
    while (!stack.empty()) {
        const auto ts = stack.back();
        stack.pop_back();
        const Cluster &t = P.nodes[ts.first], &s = P.nodes[ts.second];
        if (admissible(t, s, eta, max_block)) {
            P.blocks.push_back({ts.first, ts.second, 1});
        } else if (t.child[0] < 0 || s.child[0] < 0) {
            P.blocks.push_back({ts.first, ts.second, 0});
        } else {
            stack.push_back({t.child[1], s.child[1]});
            stack.push_back({t.child[1], s.child[0]});
            stack.push_back({t.child[0], s.child[1]});
            stack.push_back({t.child[0], s.child[0]});
        }
    }
}

}  // namespace bem
