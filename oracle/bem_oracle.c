/*
 * FP64 CPU oracle for Galerkin boundary-element weak-form entries.
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
 * CPU-baseline leg may call it; the product library never does.  It shares no
 * source, header, table or constant with the HIP path.
 *
 * What it computes (Vater, Betcke, Dilba, "Simple and efficient GPU
 * parallelization of existing H-Matrix accelerated BEM code", Section 2):
 *
 *   single layer (Eq. slp)  [S]_ij = int_Ti int_Tj psi_i(x) g(x,y) phi_j(y)
 *   double layer (Eq. dlp)  [K]_ij = same with dg/dn_y (normal of the trial
 *                                    triangle, which carries y)
 *   adjoint double layer (Eq. adlp)
 *                           [K']_ij = same with dg/dn_x (normal of the test
 *                                    triangle, which carries x)
 *   hypersingular (Eq. hypsHelmholtz), P1 only
 *                           [D]_ij = int int g [curl psi_i . curl phi_j
 *                                    - k^2 psi_i phi_j n_x . n_y]
 *                           with curl u = n x grad_Gamma u, constant on each
 *                           triangle for the hat functions
 *   Green's function (Section 2, after Eq. hypsHelmholtz)
 *                           g = exp(i k r) / (4 pi r),  r = |x - y|,
 *                           Laplace is k = 0.
 *
 * Rows are test functions psi_i (variable x), columns trial functions phi_j
 * (variable y), as the equations write them.  Both integrals are evaluated
 * with the same symmetric Gauss rule on each triangle (Section 3.2.1: a
 * 6-point degree-4 rule; a 4-point degree-3 rule is the second option), only
 * for pairs of triangles that share no vertex (Section 3.2.3: regular pairs;
 * singular pairs are a different scheme).  Summation order per entry: test
 * point p outer, trial point q inner, for P1 test triangle m outer and trial
 * triangle n inner in ascending triangle index.
 *
 * Parity status: every function here is pinned by tests under
 * tests/test_oracle_*.py (closed forms, invariants, brute force).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "orc_internal.h"

static const double ORC_PI = 3.14159265358979323846264338327950288;

/* ------------------------------------------------------------------------ */
/* Quadrature on the reference triangle {(0,0),(1,0),(0,1)}; the weights sum
 * to 1/2 (its area).  Points are given by barycentric triples (l0, l1, l2)
 * with xi = l1, eta = l2.
 *
 * 6 points, degree 4 (Section 3.2.1 names the symmetric rule of order 4 with
 * six weights): two orbits (a, a, 1-2a) whose parameters and weights are the
 * roots of the degree-4 moment equations, in closed form
 *   a = (8 - sqrt10 +- sqrt(38 - 44 sqrt(2/5))) / 18,
 *   w = (620 +- sqrt(213125 - 53320 sqrt10)) / 3720   (weights summing to 1).
 * 4 points, degree 3: centroid with weight -27/48 and the orbit
 *   (3/5, 1/5, 1/5) with weight 25/48 each.                                  */
int orc_rule(int npts, double *xi, double *eta, double *w)
{
    if (npts == 6) {
        long double s10 = sqrtl(10.0L);
        long double r = sqrtl(38.0L - 44.0L * sqrtl(0.4L));
        long double a[2] = {(8.0L - s10 + r) / 18.0L, (8.0L - s10 - r) / 18.0L};
        long double q = sqrtl(213125.0L - 53320.0L * s10);
        long double ww[2] = {(620.0L + q) / 3720.0L, (620.0L - q) / 3720.0L};
        for (int o = 0; o < 2; ++o) {
            long double b[3][3] = {{1.0L - 2.0L * a[o], a[o], a[o]},
                                   {a[o], 1.0L - 2.0L * a[o], a[o]},
                                   {a[o], a[o], 1.0L - 2.0L * a[o]}};
            for (int k = 0; k < 3; ++k) {
                xi[3 * o + k] = (double)b[k][1];
                eta[3 * o + k] = (double)b[k][2];
                w[3 * o + k] = (double)(ww[o] / 2.0L);
            }
        }
        return 6;
    }
    if (npts == 4) {
        xi[0] = 1.0 / 3.0; eta[0] = 1.0 / 3.0; w[0] = -27.0 / 96.0;
        double b[3][3] = {{0.6, 0.2, 0.2}, {0.2, 0.6, 0.2}, {0.2, 0.2, 0.6}};
        for (int k = 0; k < 3; ++k) {
            xi[1 + k] = b[k][1];
            eta[1 + k] = b[k][2];
            w[1 + k] = 25.0 / 96.0;
        }
        return 4;
    }
    return ORC_E_ARG;
}

/* ------------------------------------------------------------------------ */
/* Kernel g, dg/dn_y or dg/dn_x at one point pair; out = (re, im).  `nrm` is
 * n_y (trial normal) for the double layer and n_x (test normal) for the
 * adjoint double layer.                                                      */
void orc_kernel(int op, double k, const double *x, const double *y, const double *nrm, double *out)
{
    const double *ny = nrm, *nx = nrm;
    double d0 = x[0] - y[0], d1 = x[1] - y[1], d2 = x[2] - y[2];
    double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    double g = 1.0 / (4.0 * ORC_PI * r);
    switch (op) {
    case ORC_LAPLACE_SLP:
        out[0] = g;
        out[1] = 0.0;
        return;
    case ORC_LAPLACE_DLP: {
        /* d/dn_y of 1/(4 pi |x-y|) = (x-y).n_y / (4 pi r^3) */
        double dn = d0 * ny[0] + d1 * ny[1] + d2 * ny[2];
        out[0] = g * dn / (r * r);
        out[1] = 0.0;
        return;
    }
    case ORC_HELMHOLTZ_SLP:
        out[0] = g * cos(k * r);
        out[1] = g * sin(k * r);
        return;
    case ORC_HELMHOLTZ_DLP: {
        /* d/dn_y exp(ikr)/(4 pi r) = exp(ikr) (1 - ikr) (x-y).n_y / (4 pi r^3) */
        double dn = d0 * ny[0] + d1 * ny[1] + d2 * ny[2];
        double c = cos(k * r), s = sin(k * r);
        double f = g * dn / (r * r);
        /* (c + i s)(1 - i k r) = (c + s k r) + i (s - c k r) */
        out[0] = f * (c + s * k * r);
        out[1] = f * (s - c * k * r);
        return;
    }
    case ORC_LAPLACE_ADLP: {
        /* d/dn_x of 1/(4 pi |x-y|) = (y-x).n_x / (4 pi r^3) */
        double dn = -(d0 * nx[0] + d1 * nx[1] + d2 * nx[2]);
        out[0] = g * dn / (r * r);
        out[1] = 0.0;
        return;
    }
    case ORC_HELMHOLTZ_ADLP: {
        /* d/dn_x exp(ikr)/(4 pi r) = exp(ikr) (1 - ikr) (y-x).n_x / (4 pi r^3) */
        double dn = -(d0 * nx[0] + d1 * nx[1] + d2 * nx[2]);
        double c = cos(k * r), s = sin(k * r);
        double f = g * dn / (r * r);
        out[0] = f * (c + s * k * r);
        out[1] = f * (s - c * k * r);
        return;
    }
    default:
        out[0] = out[1] = NAN;
    }
}

/* ------------------------------------------------------------------------ */


void orc_mesh_free(orc_mesh *m)
{
    if (!m) return;
    free(m->xyz); free(m->tri); free(m->J); free(m->n); free(m->qp);
    free(m->star_ptr); free(m->star);
    free(m);
}

orc_mesh *orc_mesh_new(const double *xyz, int64_t nv, const int32_t *tri, int64_t nt, int q)
{
    if (nv <= 0 || nt <= 0 || (q != 4 && q != 6)) return NULL;
    for (int64_t t = 0; t < 3 * nt; ++t)
        if (tri[t] < 0 || tri[t] >= nv) return NULL;
    orc_mesh *m = (orc_mesh *)calloc(1, sizeof(orc_mesh));
    m->nv = nv; m->nt = nt; m->q = q;
    orc_rule(q, m->qxi, m->qeta, m->qw);
    m->xyz = (double *)malloc(sizeof(double) * 3 * nv);
    memcpy(m->xyz, xyz, sizeof(double) * 3 * nv);
    m->tri = (int32_t *)malloc(sizeof(int32_t) * 3 * nt);
    memcpy(m->tri, tri, sizeof(int32_t) * 3 * nt);
    m->J = (double *)malloc(sizeof(double) * nt);
    m->n = (double *)malloc(sizeof(double) * 3 * nt);
    m->qp = (double *)malloc(sizeof(double) * 3 * q * nt);
    for (int64_t t = 0; t < nt; ++t) {
        const double *a = xyz + 3 * tri[3 * t], *b = xyz + 3 * tri[3 * t + 1], *c = xyz + 3 * tri[3 * t + 2];
        double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double N[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        double J = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
        m->J[t] = J;
        for (int d = 0; d < 3; ++d) m->n[3 * t + d] = N[d] / J;
        for (int p = 0; p < q; ++p)
            for (int d = 0; d < 3; ++d)
                m->qp[(t * q + p) * 3 + d] = a[d] + m->qxi[p] * e1[d] + m->qeta[p] * e2[d];
    }
    /* stars: counting sort, ascending triangle order within each vertex */
    m->star_ptr = (int64_t *)calloc(nv + 1, sizeof(int64_t));
    m->star = (int32_t *)malloc(sizeof(int32_t) * 3 * nt);
    for (int64_t t = 0; t < 3 * nt; ++t) m->star_ptr[tri[t] + 1]++;
    for (int64_t v = 0; v < nv; ++v) m->star_ptr[v + 1] += m->star_ptr[v];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * nv);
    memcpy(fill, m->star_ptr, sizeof(int64_t) * nv);
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k) m->star[fill[tri[3 * t + k]]++] = (int32_t)t;
    free(fill);
    return m;
}

int64_t orc_mesh_nt(const orc_mesh *m) { return m->nt; }
int64_t orc_mesh_nv(const orc_mesh *m) { return m->nv; }

/* geometry accessors for tests */
void orc_mesh_geometry(const orc_mesh *m, double *J, double *n, double *qp)
{
    if (J) memcpy(J, m->J, sizeof(double) * m->nt);
    if (n) memcpy(n, m->n, sizeof(double) * 3 * m->nt);
    if (qp) memcpy(qp, m->qp, sizeof(double) * 3 * m->q * m->nt);
}

/* Two triangles are adjacent if they share at least one vertex index; a
 * triangle is adjacent to itself (Section 3.2.3: identical, edge- or
 * vertex-sharing pairs need singular quadrature).                            */
int orc_adjacent(const orc_mesh *m, int64_t a, int64_t b)
{
    const int32_t *ta = m->tri + 3 * a, *tb = m->tri + 3 * b;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            if (ta[i] == tb[j]) return 1;
    return 0;
}

/* Barycentric basis value of local vertex `loc` at quadrature point p:
 * l0 = 1 - xi - eta, l1 = xi, l2 = eta.                                      */
static double orc_basis(const orc_mesh *m, int loc, int p)
{
    if (loc == 0) return 1.0 - m->qxi[p] - m->qeta[p];
    if (loc == 1) return m->qxi[p];
    return m->qeta[p];
}

/* Integral over one regular triangle pair (test tm, trial tn) with test basis
 * lam_a (a = -1: constant 1) and trial basis lam_b (b = -1: constant 1):
 *   J_m J_n sum_p sum_q w_p w_q psi(p) phi(q) K(x_p, y_q).                    */
void orc_pair(const orc_mesh *m, int op, double k, int64_t tm, int64_t tn,
              int a, int b, double *re, double *im)
{
    const int q = m->q;
    const int adj = op == ORC_LAPLACE_ADLP || op == ORC_HELMHOLTZ_ADLP;
    double sr = 0.0, si = 0.0;
    for (int p = 0; p < q; ++p) {
        const double *x = m->qp + (tm * q + p) * 3;
        double wp = m->qw[p] * (a < 0 ? 1.0 : orc_basis(m, a, p));
        for (int qq = 0; qq < q; ++qq) {
            const double *y = m->qp + (tn * q + qq) * 3;
            double wq = m->qw[qq] * (b < 0 ? 1.0 : orc_basis(m, b, qq));
            double kv[2];
            orc_kernel(op, k, x, y, m->n + 3 * (adj ? tm : tn), kv);
            sr += wp * wq * kv[0];
            si += wp * wq * kv[1];
        }
    }
    double JJ = m->J[tm] * m->J[tn];
    *re = JJ * sr;
    *im = JJ * si;
}

static int orc_local_index(const orc_mesh *m, int64_t t, int64_t v)
{
    for (int k = 0; k < 3; ++k)
        if (m->tri[3 * t + k] == v) return k;
    return -1;
}

/* Surface curl of the hat function of local vertex `loc` on triangle t:
 * curl u = n x grad_Gamma u.  The surface gradient is taken through the
 * triangle's metric: with tangents t1 = v1 - v0, t2 = v2 - v0 and the
 * reference derivatives (dl/dxi, dl/deta) = (-1,-1), (1,0), (0,1) for local
 * vertices 0, 1, 2, grad_Gamma l = sum_ij Ginv_ij (dl/dxi_i) t_j with
 * G_ij = t_i . t_j.                                                          */
void orc_curl(const orc_mesh *m, int64_t t, int loc, double *out)
{
    const double *v0 = m->xyz + 3 * m->tri[3 * t], *v1 = m->xyz + 3 * m->tri[3 * t + 1],
                 *v2 = m->xyz + 3 * m->tri[3 * t + 2];
    double t1[3], t2[3];
    for (int d = 0; d < 3; ++d) {
        t1[d] = v1[d] - v0[d];
        t2[d] = v2[d] - v0[d];
    }
    double g11 = t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2];
    double g12 = t1[0] * t2[0] + t1[1] * t2[1] + t1[2] * t2[2];
    double g22 = t2[0] * t2[0] + t2[1] * t2[1] + t2[2] * t2[2];
    double det = g11 * g22 - g12 * g12;
    double d1 = loc == 0 ? -1.0 : (loc == 1 ? 1.0 : 0.0);
    double d2 = loc == 0 ? -1.0 : (loc == 2 ? 1.0 : 0.0);
    /* coefficients of t1, t2: Ginv (d1, d2) */
    double c1 = (g22 * d1 - g12 * d2) / det;
    double c2 = (-g12 * d1 + g11 * d2) / det;
    double grad[3];
    for (int d = 0; d < 3; ++d) grad[d] = c1 * t1[d] + c2 * t2[d];
    const double *n = m->n + 3 * t;
    out[0] = n[1] * grad[2] - n[2] * grad[1];
    out[1] = n[2] * grad[0] - n[0] * grad[2];
    out[2] = n[0] * grad[1] - n[1] * grad[0];
}

/* One regular pair's hypersingular contribution, test triangle tm with hat
 * function of local vertex a, trial triangle tn with local vertex b:
 *   (curl_a . curl_b) int int g  -  k^2 (n_m . n_n) int int g lam_a lam_b.    */
static void orc_pair_hyps(const orc_mesh *m, double k, int64_t tm, int64_t tn, int a, int b, double *re,
                          double *im)
{
    const int slp = k == 0.0 ? ORC_LAPLACE_SLP : ORC_HELMHOLTZ_SLP;
    double s0r, s0i, s1r = 0.0, s1i = 0.0;
    orc_pair(m, slp, k, tm, tn, -1, -1, &s0r, &s0i);
    double ca[3], cb[3];
    orc_curl(m, tm, a, ca);
    orc_curl(m, tn, b, cb);
    double cc = ca[0] * cb[0] + ca[1] * cb[1] + ca[2] * cb[2];
    *re = cc * s0r;
    *im = cc * s0i;
    if (k != 0.0) {
        orc_pair(m, slp, k, tm, tn, a, b, &s1r, &s1i);
        const double *na = m->n + 3 * tm, *nb = m->n + 3 * tn;
        double nn = na[0] * nb[0] + na[1] * nb[1] + na[2] * nb[2];
        *re -= k * k * nn * s1r;
        *im -= k * k * nn * s1i;
    }
}

static int orc_is_hyps(int op) { return op == ORC_LAPLACE_HYPS || op == ORC_HELMHOLTZ_HYPS; }

/* One entry A[row, col]; returns ORC_OK or ORC_E_NEARFIELD. */
static int orc_entry(const orc_mesh *m, int op, int space, double k, int64_t row, int64_t col,
                     int near, double *re, double *im)
{
    *re = 0.0;
    *im = 0.0;
    if (space == ORC_P0) {
        if (orc_adjacent(m, row, col)) return near == ORC_NEAR_SKIP ? ORC_OK : ORC_E_NEARFIELD;
        orc_pair(m, op, k, row, col, -1, -1, re, im);
        return ORC_OK;
    }
    if (space == ORC_DP1) {
        /* discontinuous P1: dof 3 t + a is the barycentric function of local
         * vertex a on triangle t alone, so an entry is one triangle pair with
         * one basis function on each side */
        if (orc_adjacent(m, row / 3, col / 3)) return near == ORC_NEAR_SKIP ? ORC_OK : ORC_E_NEARFIELD;
        orc_pair(m, op, k, row / 3, col / 3, (int)(row % 3), (int)(col % 3), re, im);
        return ORC_OK;
    }
    /* P1: sum over test triangles m around vertex `row`, trial triangles n
     * around vertex `col`, both ascending. */
    double sr = 0.0, si = 0.0;
    for (int64_t a = m->star_ptr[row]; a < m->star_ptr[row + 1]; ++a) {
        int64_t tm = m->star[a];
        int la = orc_local_index(m, tm, row);
        for (int64_t b = m->star_ptr[col]; b < m->star_ptr[col + 1]; ++b) {
            int64_t tn = m->star[b];
            if (orc_adjacent(m, tm, tn)) {
                if (near == ORC_NEAR_SKIP) continue;
                return ORC_E_NEARFIELD;
            }
            int lb = orc_local_index(m, tn, col);
            double r, i;
            if (orc_is_hyps(op))
                orc_pair_hyps(m, k, tm, tn, la, lb, &r, &i);
            else
                orc_pair(m, op, k, tm, tn, la, lb, &r, &i);
            sr += r;
            si += i;
        }
    }
    *re = sr;
    *im = si;
    return ORC_OK;
}

static int orc_is_complex(int op)
{
    return op == ORC_HELMHOLTZ_SLP || op == ORC_HELMHOLTZ_DLP || op == ORC_HELMHOLTZ_ADLP || op == ORC_HELMHOLTZ_HYPS;
}

/* Sub-block A[rows, cols], row-major; complex operators write interleaved
 * (re, im).  nthreads <= 0 uses the OpenMP default.  Entries are independent;
 * threads only split the entry list.                                         */
int orc_entries(const orc_mesh *m, int op, int space, double k,
                const int32_t *rows, int64_t nr, const int32_t *cols, int64_t nc,
                int near, double *out, int nthreads)
{
    if (op < 0 || op > 7 || (space != ORC_P0 && space != ORC_P1 && space != ORC_DP1)) return ORC_E_ARG;
    if (orc_is_hyps(op) && space != ORC_P1) return ORC_E_ARG;   /* needs continuous trial/test functions */
    int64_t ndof = space == ORC_P0 ? m->nt : (space == ORC_P1 ? m->nv : 3 * m->nt);
    for (int64_t r = 0; r < nr; ++r)
        if (rows[r] < 0 || rows[r] >= ndof) return ORC_E_ARG;
    for (int64_t c = 0; c < nc; ++c)
        if (cols[c] < 0 || cols[c] >= ndof) return ORC_E_ARG;
    const int cplx = orc_is_complex(op);
    int status = ORC_OK;
    int64_t total = nr * nc;
#ifdef _OPENMP
    int nth = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) num_threads(nth)
#endif
    for (int64_t e = 0; e < total; ++e) {
        int64_t r = e / nc, c = e % nc;
        double re, im;
        int st = orc_entry(m, op, space, k, rows[r], cols[c], near, &re, &im);
        if (st != ORC_OK) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            status = st;
        }
        if (cplx) {
            out[2 * e] = re;
            out[2 * e + 1] = im;
        } else {
            out[e] = re;
        }
    }
    (void)nthreads;
    return status;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
