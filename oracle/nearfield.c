/*
 * Near-field fixture of the oracle (TEST INFRASTRUCTURE ONLY).
 *
 * The weak-form path evaluates regular (vertex-disjoint) triangle pairs only;
 * the paper hands identical and adjacent pairs to a separate singular scheme
 * (Section 3.2.3).  The closed-form checks on the unit sphere (the sum of the
 * single-layer matrix, its spectrum, the double-layer identity) and the
 * parity of the device's singular pairs need every pair, so this file
 * supplies a semi-analytic P0 value for near pairs:
 *
 *   inner integral over the flat trial triangle in closed form,
 *     single layer:  int_T 1/|x-y| dy          (potential of a uniform flat
 *                    triangle, Wilton et al. 1984 / Graglia 1993),
 *     double layer:  int_T (x-y).n_y/|x-y|^3 dy = -Omega(x), Omega the signed
 *                    solid angle of Van Oosterom & Strackee (1983),
 *   outer integral over the test triangle with the 6-point rule applied on
 *   4^L congruent sub-triangles.
 *
 * Helmholtz (Eq. slp/dlp with g = e^{ikr}/(4 pi r)): the kernel is expanded
 * around r = 0 and the singular and non-smooth terms are integrated in closed
 * form over the trial triangle,
 *     e^{ikr}/r             = 1/r + ik - (k^2/2) r + T(r),
 *     e^{ikr}(1 - ikr)/r^3  = 1/r^3 + (k^2/2)/r + i k^3/3 - (k^4/8) r + U(r)
 * ((x-y).n_y is the height of x over the trial plane, constant in y), with
 * int_T |x-y| dy in closed form as well; the remainders T = O(r^2) and
 * U = O(r^2) go to the subdivided 6-point rule on the trial triangle.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "orc_internal.h"

static const double NF_PI = 3.14159265358979323846264338327950288;

double orc_tri_solid_angle(const double *v0, const double *v1, const double *v2, const double *x);
int orc_subdivided_rule(int level, double *xi, double *eta, double *w);
static double nf_entry(const orc_mesh *m, int op, int64_t i, int64_t j, int npts, const double *xi,
                       const double *eta, const double *w);
static void nf_remainder(int dlp, double z, double *re, double *im);
static void nfc_entry(const orc_mesh *m, int op, double k, int64_t i, int64_t j, int npts, const double *xi,
                      const double *eta, const double *w, int nin, const double *ixi, const double *ieta,
                      const double *iw, double *re, double *im);

static void sub3(const double *a, const double *b, double *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* int_T 1/|x - y| dy for the flat triangle (v0, v1, v2). */
double orc_tri_potential(const double *v0, const double *v1, const double *v2, const double *x)
{
    const double *v[3] = {v0, v1, v2};
    double e1[3], e2[3], N[3], n[3], xv0[3], rho[3];
    sub3(v1, v0, e1);
    sub3(v2, v0, e2);
    cross3(e1, e2, N);
    double nn = sqrt(dot3(N, N));
    for (int d = 0; d < 3; ++d) n[d] = N[d] / nn;
    sub3(x, v0, xv0);
    double h = dot3(xv0, n);
    double ah = fabs(h);
    for (int d = 0; d < 3; ++d) rho[d] = x[d] - h * n[d];
    double sum = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double *pm = v[i], *pp = v[(i + 1) % 3];
        double s[3], m[3], a[3], b[3];
        sub3(pp, pm, s);
        double L = sqrt(dot3(s, s));
        for (int d = 0; d < 3; ++d) s[d] /= L;
        cross3(s, n, m); /* in-plane outward normal of the edge */
        sub3(pp, rho, a);
        sub3(pm, rho, b);
        double lp = dot3(a, s), lm = dot3(b, s);
        double t0 = dot3(b, m);
        double R0sq = t0 * t0 + h * h;
        double Rp = sqrt(R0sq + lp * lp), Rm = sqrt(R0sq + lm * lm);
        if (fabs(t0) > 0.0) {
            double lg;
            if (lp + lm >= 0.0)
                lg = log((Rp + lp) / (Rm + lm));
            else
                lg = log((Rm - lm) / (Rp - lp));
            sum += t0 * lg;
        }
        if (ah > 0.0)
            sum -= ah * (atan(t0 * lp / (R0sq + ah * Rp)) - atan(t0 * lm / (R0sq + ah * Rm)));
    }
    return sum;
}

/* ln(R + l) for R = sqrt(R0sq + l^2), in the form without cancellation
 * (R + l = R0sq / (R - l) for l < 0). */
static double nf_log_rl(double l, double R, double R0sq)
{
    return l >= 0.0 ? log(R + l) : log(R0sq / (R - l));
}

/* int_T |x - y| dy for the flat triangle (v0, v1, v2).  With y' = y - rho
 * (rho the projection of x on the plane, h the height of x over it) and
 * R = |x - y|, the surface divergence div(y' R) = 3R - h^2/R, so
 *   int_T R = (1/3) [ sum_e t_e int_e R dl + h^2 int_T 1/R ],
 * t_e the distance of rho from edge e's line along the edge's outward
 * in-plane normal, int_e R dl = (1/2) [l R + R0^2 ln(l + R)] between the
 * edge's ends (l along the edge from the foot of the perpendicular,
 * R0^2 = t_e^2 + h^2). */
double orc_tri_moment_r(const double *v0, const double *v1, const double *v2, const double *x)
{
    const double *v[3] = {v0, v1, v2};
    double e1[3], e2[3], N[3], n[3], xv0[3], rho[3];
    sub3(v1, v0, e1);
    sub3(v2, v0, e2);
    cross3(e1, e2, N);
    double nn = sqrt(dot3(N, N));
    for (int d = 0; d < 3; ++d) n[d] = N[d] / nn;
    sub3(x, v0, xv0);
    double h = dot3(xv0, n);
    for (int d = 0; d < 3; ++d) rho[d] = x[d] - h * n[d];
    double sum = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double *pm = v[i], *pp = v[(i + 1) % 3];
        double s[3], m[3], a[3], b[3];
        sub3(pp, pm, s);
        double L = sqrt(dot3(s, s));
        for (int d = 0; d < 3; ++d) s[d] /= L;
        cross3(s, n, m);
        sub3(pp, rho, a);
        sub3(pm, rho, b);
        double lp = dot3(a, s), lm = dot3(b, s);
        double t0 = dot3(b, m);
        double R0sq = t0 * t0 + h * h;
        double Rp = sqrt(R0sq + lp * lp), Rm = sqrt(R0sq + lm * lm);
        double edge = 0.5 * (lp * Rp - lm * Rm);
        if (R0sq > 0.0) edge += 0.5 * R0sq * (nf_log_rl(lp, Rp, R0sq) - nf_log_rl(lm, Rm, R0sq));
        sum += t0 * edge;
    }
    return (sum + h * h * orc_tri_potential(v0, v1, v2, x)) / 3.0;
}

/* Vector moments of the flat triangle (v0, v1, v2) seen from x, with rho the
 * projection of x on its plane: V1 = int_T (y - rho)/|x - y| dy and
 * V3 = int_T (y - rho)/|x - y|^3 dy.  The in-plane gradient of R = |x - y|
 * is (y - rho)/R and that of 1/R is -(y - rho)/R^3, so by the gradient
 * theorem V1 = sum_e m_e int_e R dl and V3 = -sum_e m_e int_e dl/R, m_e the
 * edge's outward in-plane normal; int_e dl/R = ln(l + R) between the ends.
 * V3 needs x off the edges' lines (R0 > 0); it returns zeros where R0 = 0. */
void orc_tri_vector_moments(const double *v0, const double *v1, const double *v2, const double *x, double *V1,
                            double *V3)
{
    const double *v[3] = {v0, v1, v2};
    double e1[3], e2[3], N[3], n[3], xv0[3], rho[3];
    sub3(v1, v0, e1);
    sub3(v2, v0, e2);
    cross3(e1, e2, N);
    double nn = sqrt(dot3(N, N));
    for (int d = 0; d < 3; ++d) n[d] = N[d] / nn;
    sub3(x, v0, xv0);
    double h = dot3(xv0, n);
    for (int d = 0; d < 3; ++d) rho[d] = x[d] - h * n[d];
    for (int d = 0; d < 3; ++d) V1[d] = V3[d] = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double *pm = v[i], *pp = v[(i + 1) % 3];
        double s[3], m[3], a[3], b[3];
        sub3(pp, pm, s);
        double L = sqrt(dot3(s, s));
        for (int d = 0; d < 3; ++d) s[d] /= L;
        cross3(s, n, m);
        sub3(pp, rho, a);
        sub3(pm, rho, b);
        double lp = dot3(a, s), lm = dot3(b, s);
        double t0 = dot3(b, m);
        double R0sq = t0 * t0 + h * h;
        double Rp = sqrt(R0sq + lp * lp), Rm = sqrt(R0sq + lm * lm);
        double lg = R0sq > 0.0 ? nf_log_rl(lp, Rp, R0sq) - nf_log_rl(lm, Rm, R0sq) : 0.0;
        double edge_r = 0.5 * (lp * Rp - lm * Rm + R0sq * lg);
        for (int d = 0; d < 3; ++d) {
            V1[d] += m[d] * edge_r;
            V3[d] -= m[d] * lg;
        }
    }
}

/* W1 = int_T (y - rho) |x - y| dy: the in-plane gradient of R^3/3 is
 * R (y - rho), so W1 = sum_e m_e int_e R^3/3 dl with
 * int_e R^3 dl = [l R^3/4 + 3 R0^2 l R/8 + 3 R0^4 ln(l + R)/8] between the
 * edge's ends. */
void orc_tri_vector_moment_r(const double *v0, const double *v1, const double *v2, const double *x, double *W1)
{
    const double *v[3] = {v0, v1, v2};
    double e1[3], e2[3], N[3], n[3], xv0[3], rho[3];
    sub3(v1, v0, e1);
    sub3(v2, v0, e2);
    cross3(e1, e2, N);
    double nn = sqrt(dot3(N, N));
    for (int d = 0; d < 3; ++d) n[d] = N[d] / nn;
    sub3(x, v0, xv0);
    double h = dot3(xv0, n);
    for (int d = 0; d < 3; ++d) rho[d] = x[d] - h * n[d];
    for (int d = 0; d < 3; ++d) W1[d] = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double *pm = v[i], *pp = v[(i + 1) % 3];
        double s[3], m[3], a[3], b[3];
        sub3(pp, pm, s);
        double L = sqrt(dot3(s, s));
        for (int d = 0; d < 3; ++d) s[d] /= L;
        cross3(s, n, m);
        sub3(pp, rho, a);
        sub3(pm, rho, b);
        double lp = dot3(a, s), lm = dot3(b, s);
        double t0 = dot3(b, m);
        double R0sq = t0 * t0 + h * h;
        double Rp = sqrt(R0sq + lp * lp), Rm = sqrt(R0sq + lm * lm);
        double lg = R0sq > 0.0 ? nf_log_rl(lp, Rp, R0sq) - nf_log_rl(lm, Rm, R0sq) : 0.0;
        double edge = (lp * Rp * Rp * Rp - lm * Rm * Rm * Rm) / 4.0 + 3.0 * R0sq * (lp * Rp - lm * Rm) / 8.0 +
                      3.0 * R0sq * R0sq * lg / 8.0;
        for (int d = 0; d < 3; ++d) W1[d] += m[d] * edge / 3.0;
    }
}

/* 3 x 3 local matrix of a triangle pair for the P1 hat functions restricted
 * to the pair, Laplace single (op 0) or double (op 1) layer:
 * M[a][b] = int_{T_i} phi_a(x) int_{T_j} psi_b(y) K(x, y) dy dx, a and b in
 * the mesh's vertex order of each triangle.  psi_b is affine, so with rho
 * the projection of x on the trial plane, psi_b(y) = psi_b(rho) +
 * grad psi_b . (y - rho) and the inner integrals are
 *   single layer: psi_b(rho) int 1/R + grad psi_b . V1,
 *   double layer: -psi_b(rho) Omega + h grad psi_b . V3  (h the height of x);
 * the outer integral takes the rule (xi, eta, w) on the test triangle. */
static void nf_p1_local(const orc_mesh *m, int op, int64_t i, int64_t j, int npts, const double *xi,
                        const double *eta, const double *w, double *M)
{
    const double *a = m->xyz + 3 * m->tri[3 * i], *b = m->xyz + 3 * m->tri[3 * i + 1],
                 *c = m->xyz + 3 * m->tri[3 * i + 2];
    const double *u[3] = {m->xyz + 3 * m->tri[3 * j], m->xyz + 3 * m->tri[3 * j + 1], m->xyz + 3 * m->tri[3 * j + 2]};
    const double *nj = m->n + 3 * j;
    const double Jj = m->J[j];
    double grad[3][3];   /* in-plane gradients of the trial barycentrics */
    for (int q = 0; q < 3; ++q) {
        double ed[3];
        sub3(u[(q + 2) % 3], u[(q + 1) % 3], ed);
        cross3(nj, ed, grad[q]);
        for (int d = 0; d < 3; ++d) grad[q][d] /= Jj;
    }
    for (int k = 0; k < 9; ++k) M[k] = 0.0;
    for (int p = 0; p < npts; ++p) {
        double x[3], xu[3], rho[3], V1[3], V3[3];
        for (int d = 0; d < 3; ++d) x[d] = a[d] + xi[p] * (b[d] - a[d]) + eta[p] * (c[d] - a[d]);
        const double phi[3] = {1.0 - xi[p] - eta[p], xi[p], eta[p]};
        sub3(x, u[0], xu);
        const double hgt = dot3(xu, nj);
        for (int d = 0; d < 3; ++d) rho[d] = x[d] - hgt * nj[d];
        double base;
        if (op == ORC_LAPLACE_SLP) {
            base = orc_tri_potential(u[0], u[1], u[2], x);
        } else {
            if (fabs(hgt) <= 1e-12 * sqrt(Jj)) continue;   /* (x - y).n_y = 0 */
            base = -orc_tri_solid_angle(u[0], u[1], u[2], x);
        }
        orc_tri_vector_moments(u[0], u[1], u[2], x, V1, V3);
        for (int q = 0; q < 3; ++q) {
            double r1[3], r2[3], cr[3];
            sub3(u[(q + 1) % 3], rho, r1);
            sub3(u[(q + 2) % 3], rho, r2);
            cross3(r1, r2, cr);
            const double lam = dot3(cr, nj) / Jj;   /* psi_q(rho) */
            const double inner = op == ORC_LAPLACE_SLP ? lam * base + dot3(grad[q], V1)
                                                       : lam * base + hgt * dot3(grad[q], V3);
            for (int t = 0; t < 3; ++t) M[3 * t + q] += w[p] * phi[t] * inner;
        }
    }
    for (int k = 0; k < 9; ++k) M[k] *= m->J[i] / (4.0 * NF_PI);
}

/* Complex 3 x 3 local matrix of the P1 hat functions for the Helmholtz single
 * (op 2) or double layer (op 3): the kernel expanded as for P0,
 *   single layer: psi_b . (1/R + ik - (k^2/2) R + T(R)),
 *   double layer: psi_b . h (1/R^3 + (k^2/2)/R + i k^3/3 - (k^4/8) R + U(R)),
 * each singular term over the trial triangle in closed form for the affine
 * psi_b = psi_b(rho) + grad psi_b . (y - rho) (potentials I0, I1 = int R,
 * solid angle, vector moments V1, V3, W1; int psi_b = |T|/3), the
 * remainder on the inner rule (ixi, ieta, iw); M is 9 complex values. */
static void nf_p1_local_c(const orc_mesh *m, int op, double k, int64_t i, int64_t j, int npts, const double *xi,
                          const double *eta, const double *w, int nin, const double *ixi, const double *ieta,
                          const double *iw, double *M)
{
    const double *a = m->xyz + 3 * m->tri[3 * i], *b = m->xyz + 3 * m->tri[3 * i + 1],
                 *c = m->xyz + 3 * m->tri[3 * i + 2];
    const double *u[3] = {m->xyz + 3 * m->tri[3 * j], m->xyz + 3 * m->tri[3 * j + 1], m->xyz + 3 * m->tri[3 * j + 2]};
    const double *nj = m->n + 3 * j;
    const double Jj = m->J[j], area3 = Jj / 6.0;
    const int dlp = op == ORC_HELMHOLTZ_DLP;
    double grad[3][3];
    for (int q = 0; q < 3; ++q) {
        double ed[3];
        sub3(u[(q + 2) % 3], u[(q + 1) % 3], ed);
        cross3(nj, ed, grad[q]);
        for (int d = 0; d < 3; ++d) grad[q][d] /= Jj;
    }
    for (int kk = 0; kk < 18; ++kk) M[kk] = 0.0;
    for (int p = 0; p < npts; ++p) {
        double x[3], xu[3], rho[3], V1[3], V3[3], W1[3];
        for (int d = 0; d < 3; ++d) x[d] = a[d] + xi[p] * (b[d] - a[d]) + eta[p] * (c[d] - a[d]);
        const double phi[3] = {1.0 - xi[p] - eta[p], xi[p], eta[p]};
        sub3(x, u[0], xu);
        const double hgt = dot3(xu, nj);
        if (dlp && fabs(hgt) <= 1e-12 * sqrt(Jj)) continue;   /* (x - y).n_y = 0 */
        for (int d = 0; d < 3; ++d) rho[d] = x[d] - hgt * nj[d];
        const double I0 = orc_tri_potential(u[0], u[1], u[2], x), I1 = orc_tri_moment_r(u[0], u[1], u[2], x);
        orc_tri_vector_moments(u[0], u[1], u[2], x, V1, V3);
        orc_tri_vector_moment_r(u[0], u[1], u[2], x, W1);
        const double Om = dlp ? orc_tri_solid_angle(u[0], u[1], u[2], x) : 0.0;
        /* remainder with the trial hat functions at the inner points */
        double rr[3] = {0, 0, 0}, ri[3] = {0, 0, 0};
        for (int q = 0; q < nin; ++q) {
            double y[3], d3[3];
            for (int d = 0; d < 3; ++d) y[d] = u[0][d] + ixi[q] * (u[1][d] - u[0][d]) + ieta[q] * (u[2][d] - u[0][d]);
            sub3(x, y, d3);
            double r = sqrt(dot3(d3, d3));
            if (r == 0.0) continue;
            double tr, ti;
            nf_remainder(dlp, k * r, &tr, &ti);
            const double sc = dlp ? iw[q] / (r * r * r) : iw[q] / r;
            const double psi[3] = {1.0 - ixi[q] - ieta[q], ixi[q], ieta[q]};
            for (int bb = 0; bb < 3; ++bb) {
                rr[bb] += sc * tr * psi[bb];
                ri[bb] += sc * ti * psi[bb];
            }
        }
        for (int q = 0; q < 3; ++q) {
            double r1[3], r2[3], cr[3];
            sub3(u[(q + 1) % 3], rho, r1);
            sub3(u[(q + 2) % 3], rho, r2);
            cross3(r1, r2, cr);
            const double lam = dot3(cr, nj) / Jj;
            double inr, ini;
            if (!dlp) {
                inr = lam * (I0 - 0.5 * k * k * I1) + dot3(grad[q], V1) - 0.5 * k * k * dot3(grad[q], W1) + Jj * rr[q];
                ini = k * area3 + Jj * ri[q];
            } else {
                inr = -lam * Om + hgt * dot3(grad[q], V3) +
                      hgt * (0.5 * k * k * (lam * I0 + dot3(grad[q], V1)) -
                             0.125 * k * k * k * k * (lam * I1 + dot3(grad[q], W1)) + Jj * rr[q]);
                ini = hgt * (k * k * k * area3 / 3.0 + Jj * ri[q]);
            }
            for (int t = 0; t < 3; ++t) {
                M[2 * (3 * t + q)] += w[p] * phi[t] * inr;
                M[2 * (3 * t + q) + 1] += w[p] * phi[t] * ini;
            }
        }
    }
    for (int kk = 0; kk < 18; ++kk) M[kk] *= m->J[i] / (4.0 * NF_PI);
}

/* Complex P1 local matrices of n pairs, Helmholtz single (op 2) or double
 * (op 3) layer, or the Helmholtz hypersingular operator (op 7, Eq.
 * hypsHelmholtz: curl_a . curl_b times the pair's P0 single-layer value minus
 * k^2 (n_x . n_y) times its P1 single-layer local matrix): outer rule on
 * 4^level, remainder on 4^inner_level sub-triangles; out holds n row-major
 * 3 x 3 complex (18 doubles). */
int orc_nearfield_p1_local_c(const orc_mesh *m, int op, double k, int64_t n, const int64_t *rows,
                             const int64_t *cols, int level, int inner_level, double *out)
{
    if ((op != ORC_HELMHOLTZ_SLP && op != ORC_HELMHOLTZ_DLP && op != ORC_HELMHOLTZ_HYPS) || level < 0 ||
        inner_level < 0)
        return ORC_E_ARG;
    int np = 6, ni = 6;
    for (int l = 0; l < level; ++l) np *= 4;
    for (int l = 0; l < inner_level; ++l) ni *= 4;
    double *xi = (double *)malloc(sizeof(double) * 3 * (np + ni));
    double *eta = xi + np, *w = xi + 2 * np, *ixi = xi + 3 * np, *ieta = ixi + ni, *iw = ixi + 2 * ni;
    orc_subdivided_rule(level, xi, eta, w);
    orc_subdivided_rule(inner_level, ixi, ieta, iw);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t t = 0; t < n; ++t) {
        if (op != ORC_HELMHOLTZ_HYPS) {
            nf_p1_local_c(m, op, k, rows[t], cols[t], np, xi, eta, w, ni, ixi, ieta, iw, out + 18 * t);
            continue;
        }
        double *M = out + 18 * t, v[2];
        nf_p1_local_c(m, ORC_HELMHOLTZ_SLP, k, rows[t], cols[t], np, xi, eta, w, ni, ixi, ieta, iw, M);
        nfc_entry(m, ORC_HELMHOLTZ_SLP, k, rows[t], cols[t], np, xi, eta, w, ni, ixi, ieta, iw, v, v + 1);
        const double *na = m->n + 3 * rows[t], *nb = m->n + 3 * cols[t];
        const double nn = na[0] * nb[0] + na[1] * nb[1] + na[2] * nb[2];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double ca[3], cb[3];
                orc_curl(m, rows[t], a, ca);
                orc_curl(m, cols[t], b, cb);
                const double cc = ca[0] * cb[0] + ca[1] * cb[1] + ca[2] * cb[2];
                double *e = M + 2 * (3 * a + b);
                e[0] = cc * v[0] - k * k * nn * e[0];
                e[1] = cc * v[1] - k * k * nn * e[1];
            }
    }
    free(xi);
    return ORC_OK;
}

/* P1 local matrices of n pairs (rows[t], cols[t]), Laplace single or double
 * layer, or the Laplace hypersingular operator (Eq. hypsHelmholtz at k = 0:
 * curl_a . curl_b times the pair's P0 single-layer integral, the hat
 * functions' surface curls being constant per triangle), outer rule on
 * 4^level sub-triangles; out holds n row-major 3 x 3. */
int orc_nearfield_p1_local(const orc_mesh *m, int op, int64_t n, const int64_t *rows, const int64_t *cols,
                           int level, double *out)
{
    if ((op != ORC_LAPLACE_SLP && op != ORC_LAPLACE_DLP && op != ORC_LAPLACE_HYPS) || level < 0) return ORC_E_ARG;
    int np = 6;
    for (int l = 0; l < level; ++l) np *= 4;
    double *xi = (double *)malloc(sizeof(double) * 3 * np);
    double *eta = xi + np, *w = xi + 2 * np;
    orc_subdivided_rule(level, xi, eta, w);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t t = 0; t < n; ++t) {
        if (op != ORC_LAPLACE_HYPS) {
            nf_p1_local(m, op, rows[t], cols[t], np, xi, eta, w, out + 9 * t);
            continue;
        }
        const double v = nf_entry(m, ORC_LAPLACE_SLP, rows[t], cols[t], np, xi, eta, w);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double ca[3], cb[3];
                orc_curl(m, rows[t], a, ca);
                orc_curl(m, cols[t], b, cb);
                out[9 * t + 3 * a + b] = (ca[0] * cb[0] + ca[1] * cb[1] + ca[2] * cb[2]) * v;
            }
    }
    free(xi);
    return ORC_OK;
}

/* Remainders of the Helmholtz kernels after the terms integrated in closed
 * form, at z = k r: T(r) r = sum_{n>=3} (iz)^n / n!, U(r) r^3 = sum_{n>=5}
 * (1 - n) (iz)^n / n!.  Power series below z = 2, the closed expressions
 * above (cos z - 1 + z^2/2 + i (sin z - z), and cos z + z sin z - 1 - z^2/2
 * + z^4/8 + i (sin z - z cos z - z^3/3)). */
static void nf_remainder(int dlp, double z, double *re, double *im)
{
    if (z < 2.0) {
        double t = 1.0, sr = 0.0, si = 0.0;   /* t = z^n / n! */
        for (int n = 1; n <= 40; ++n) {
            t *= z / n;
            if (n < (dlp ? 5 : 3)) continue;
            double c = dlp ? (double)(1 - n) : 1.0;
            switch (n & 3) {   /* i^n */
            case 0: sr += c * t; break;
            case 1: si += c * t; break;
            case 2: sr -= c * t; break;
            default: si -= c * t; break;
            }
        }
        *re = sr;
        *im = si;
        return;
    }
    double c = cos(z), s = sin(z);
    if (!dlp) {
        *re = c - 1.0 + 0.5 * z * z;
        *im = s - z;
    } else {
        *re = c + z * s - 1.0 - 0.5 * z * z + 0.125 * z * z * z * z;
        *im = s - z * c - z * z * z / 3.0;
    }
}

/* Signed solid angle of the triangle seen from x; positive when x lies on the
 * side opposite to (v1-v0) x (v2-v0). */
double orc_tri_solid_angle(const double *v0, const double *v1, const double *v2, const double *x)
{
    double a[3], b[3], c[3], bc[3];
    sub3(v0, x, a);
    sub3(v1, x, b);
    sub3(v2, x, c);
    double la = sqrt(dot3(a, a)), lb = sqrt(dot3(b, b)), lc = sqrt(dot3(c, c));
    cross3(b, c, bc);
    double num = dot3(a, bc);
    double den = la * lb * lc + dot3(a, b) * lc + dot3(a, c) * lb + dot3(b, c) * la;
    return 2.0 * atan2(num, den);
}

/* 6-point rule on 4^level congruent sub-triangles of the reference triangle.
 * Returns the number of points (6 * 4^level); weights sum to 1/2. */
int orc_subdivided_rule(int level, double *xi, double *eta, double *w)
{
    double qx[6], qe[6], qw[6];
    orc_rule(6, qx, qe, qw);
    int ntri = 1;
    for (int l = 0; l < level; ++l) ntri *= 4;
    double *T = (double *)malloc(sizeof(double) * 6 * ntri);
    double *U = (double *)malloc(sizeof(double) * 6 * ntri);
    T[0] = 0; T[1] = 0; T[2] = 1; T[3] = 0; T[4] = 0; T[5] = 1;
    int cur = 1;
    for (int l = 0; l < level; ++l) {
        for (int t = 0; t < cur; ++t) {
            double *P = T + 6 * t;
            double m01[2] = {0.5 * (P[0] + P[2]), 0.5 * (P[1] + P[3])};
            double m12[2] = {0.5 * (P[2] + P[4]), 0.5 * (P[3] + P[5])};
            double m20[2] = {0.5 * (P[4] + P[0]), 0.5 * (P[5] + P[1])};
            double sub[4][6] = {
                {P[0], P[1], m01[0], m01[1], m20[0], m20[1]},
                {m01[0], m01[1], P[2], P[3], m12[0], m12[1]},
                {m20[0], m20[1], m12[0], m12[1], P[4], P[5]},
                {m12[0], m12[1], m20[0], m20[1], m01[0], m01[1]},
            };
            memcpy(U + 24 * t, sub, sizeof(sub));
        }
        cur *= 4;
        double *tmp = T; T = U; U = tmp;
    }
    double scale = 1.0 / (double)ntri;
    int k = 0;
    for (int t = 0; t < ntri; ++t) {
        double *P = T + 6 * t;
        for (int p = 0; p < 6; ++p, ++k) {
            xi[k] = P[0] + qx[p] * (P[2] - P[0]) + qe[p] * (P[4] - P[0]);
            eta[k] = P[1] + qx[p] * (P[3] - P[1]) + qe[p] * (P[5] - P[1]);
            w[k] = qw[p] * scale;
        }
    }
    free(T);
    free(U);
    return 6 * ntri;
}

/* Semi-analytic P0 entry for one pair (test i, trial j), Laplace single or
 * double layer.  xi/eta/w: an outer rule on the reference triangle. */
static double nf_entry(const orc_mesh *m, int op, int64_t i, int64_t j, int npts,
                       const double *xi, const double *eta, const double *w)
{
    const double *a = m->xyz + 3 * m->tri[3 * i], *b = m->xyz + 3 * m->tri[3 * i + 1],
                 *c = m->xyz + 3 * m->tri[3 * i + 2];
    const double *u0 = m->xyz + 3 * m->tri[3 * j], *u1 = m->xyz + 3 * m->tri[3 * j + 1],
                 *u2 = m->xyz + 3 * m->tri[3 * j + 2];
    double s = 0.0;
    for (int p = 0; p < npts; ++p) {
        double x[3];
        for (int d = 0; d < 3; ++d) x[d] = a[d] + xi[p] * (b[d] - a[d]) + eta[p] * (c[d] - a[d]);
        double inner;
        if (op == ORC_LAPLACE_SLP) {
            inner = orc_tri_potential(u0, u1, u2, x) / (4.0 * NF_PI);
        } else {
            /* (x - y).n_y vanishes identically when x lies in the plane of the
             * trial triangle (the identical pair, coplanar neighbours); the
             * solid-angle formula would return the one-sided limit +-2 pi. */
            double xu[3];
            sub3(x, u0, xu);
            double hgt = dot3(xu, m->n + 3 * j);
            double scale = sqrt(m->J[j]);
            inner = fabs(hgt) <= 1e-12 * scale ? 0.0 : -orc_tri_solid_angle(u0, u1, u2, x) / (4.0 * NF_PI);
        }
        s += w[p] * inner;
    }
    return m->J[i] * s;
}

/* Semi-analytic P0 entry of the Helmholtz single (op 2) or double (op 3)
 * layer for one pair: the outer rule (xi, eta, w) on the test triangle, the
 * inner rule (ixi, ieta, iw) on the trial triangle for the smooth remainder. */
static void nfc_entry(const orc_mesh *m, int op, double k, int64_t i, int64_t j, int npts, const double *xi,
                      const double *eta, const double *w, int nin, const double *ixi, const double *ieta,
                      const double *iw, double *re, double *im)
{
    const double *a = m->xyz + 3 * m->tri[3 * i], *b = m->xyz + 3 * m->tri[3 * i + 1],
                 *c = m->xyz + 3 * m->tri[3 * i + 2];
    const double *u0 = m->xyz + 3 * m->tri[3 * j], *u1 = m->xyz + 3 * m->tri[3 * j + 1],
                 *u2 = m->xyz + 3 * m->tri[3 * j + 2];
    const double area = 0.5 * m->J[j];
    const int dlp = op == ORC_HELMHOLTZ_DLP;
    double sr = 0.0, si = 0.0;
    for (int p = 0; p < npts; ++p) {
        double x[3];
        for (int d = 0; d < 3; ++d) x[d] = a[d] + xi[p] * (b[d] - a[d]) + eta[p] * (c[d] - a[d]);
        /* smooth remainder: T(r) (single layer) or U(r) (double layer, times
         * the height below) over the trial triangle */
        double rr = 0.0, ri = 0.0;
        for (int q = 0; q < nin; ++q) {
            double y[3], d3[3];
            for (int d = 0; d < 3; ++d) y[d] = u0[d] + ixi[q] * (u1[d] - u0[d]) + ieta[q] * (u2[d] - u0[d]);
            sub3(x, y, d3);
            double r = sqrt(dot3(d3, d3));
            if (r == 0.0) continue;   /* both remainders vanish as r -> 0 (T/r, U/r^3 = O(r)) */
            double tr, ti;
            nf_remainder(dlp, k * r, &tr, &ti);
            double scale = dlp ? iw[q] / (r * r * r) : iw[q] / r;
            rr += scale * tr;
            ri += scale * ti;
        }
        rr *= m->J[j];
        ri *= m->J[j];
        double I0 = orc_tri_potential(u0, u1, u2, x), I1 = orc_tri_moment_r(u0, u1, u2, x);
        double inr, ini;
        if (!dlp) {
            inr = I0 - 0.5 * k * k * I1 + rr;
            ini = k * area + ri;
        } else {
            double xu[3];
            sub3(x, u0, xu);
            double hgt = dot3(xu, m->n + 3 * j);
            if (fabs(hgt) <= 1e-12 * sqrt(m->J[j])) {
                inr = ini = 0.0;   /* x in the trial plane: (x - y).n_y = 0 */
            } else {
                inr = -orc_tri_solid_angle(u0, u1, u2, x) + hgt * (0.5 * k * k * I0 - 0.125 * k * k * k * k * I1 + rr);
                ini = hgt * (k * k * k * area / 3.0 + ri);
            }
        }
        sr += w[p] * inr;
        si += w[p] * ini;
    }
    *re = m->J[i] * sr / (4.0 * NF_PI);
    *im = m->J[i] * si / (4.0 * NF_PI);
}

/* Near-field P0 entries of any of the four operators for n pairs (rows[t],
 * cols[t]) (outer rule on 4^level sub-triangles; the Helmholtz remainder on
 * 4^inner_level); out holds n complex values (imaginary parts 0 for Laplace). */
int orc_nearfield_entries_c(const orc_mesh *m, int op, double k, int64_t n, const int64_t *rows,
                            const int64_t *cols, int level, int inner_level, double *out)
{
    if (op < ORC_LAPLACE_SLP || op > ORC_HELMHOLTZ_DLP || level < 0 || inner_level < 0) return ORC_E_ARG;
    int np = 6, ni = 6;
    for (int l = 0; l < level; ++l) np *= 4;
    for (int l = 0; l < inner_level; ++l) ni *= 4;
    double *xi = (double *)malloc(sizeof(double) * 3 * (np + ni));
    double *eta = xi + np, *w = xi + 2 * np, *ixi = xi + 3 * np, *ieta = ixi + ni, *iw = ixi + 2 * ni;
    orc_subdivided_rule(level, xi, eta, w);
    orc_subdivided_rule(inner_level, ixi, ieta, iw);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t t = 0; t < n; ++t) {
        if (op <= ORC_LAPLACE_DLP) {
            out[2 * t] = nf_entry(m, op, rows[t], cols[t], np, xi, eta, w);
            out[2 * t + 1] = 0.0;
        } else {
            nfc_entry(m, op, k, rows[t], cols[t], np, xi, eta, w, ni, ixi, ieta, iw, out + 2 * t, out + 2 * t + 1);
        }
    }
    free(xi);
    return ORC_OK;
}

double orc_nearfield_entry(const orc_mesh *m, int op, int64_t i, int64_t j, int level)
{
    int np = 6;
    for (int l = 0; l < level; ++l) np *= 4;
    double *xi = (double *)malloc(sizeof(double) * np * 3);
    double *eta = xi + np, *w = xi + 2 * np;
    orc_subdivided_rule(level, xi, eta, w);
    double v = nf_entry(m, op, i, j, np, xi, eta, w);
    free(xi);
    return v;
}

/* Full nt x nt P0 matrix of the Laplace single (op 0) or double (op 1) layer:
 * pairs whose centroids are closer than near_dist, or that share a vertex,
 * take the semi-analytic value; all other pairs the regular oracle value.
 * Row-major output. */
int orc_p0_matrix_with_nearfield(const orc_mesh *m, int op, double near_dist, int level, double *out)
{
    if (op != ORC_LAPLACE_SLP && op != ORC_LAPLACE_DLP) return ORC_E_ARG;
    int np = 6;
    for (int l = 0; l < level; ++l) np *= 4;
    double *xi = (double *)malloc(sizeof(double) * np * 3);
    double *eta = xi + np, *w = xi + 2 * np;
    orc_subdivided_rule(level, xi, eta, w);
    const int64_t nt = m->nt;
    double *cen = (double *)malloc(sizeof(double) * 3 * nt);
    for (int64_t t = 0; t < nt; ++t)
        for (int d = 0; d < 3; ++d)
            cen[3 * t + d] = (m->xyz[3 * m->tri[3 * t] + d] + m->xyz[3 * m->tri[3 * t + 1] + d] +
                              m->xyz[3 * m->tri[3 * t + 2] + d]) / 3.0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t i = 0; i < nt; ++i) {
        for (int64_t j = 0; j < nt; ++j) {
            double dd[3];
            sub3(cen + 3 * i, cen + 3 * j, dd);
            double dist = sqrt(dot3(dd, dd));
            if (dist < near_dist || orc_adjacent(m, i, j)) {
                out[i * nt + j] = nf_entry(m, op, i, j, np, xi, eta, w);
            } else {
                double re, im;
                orc_pair(m, op, 0.0, i, j, -1, -1, &re, &im);
                out[i * nt + j] = re;
            }
        }
    }
    free(cen);
    free(xi);
    return ORC_OK;
}
