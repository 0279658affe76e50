/*
 * Internal declarations shared by the oracle's own C files (test
 * infrastructure; nothing in the product includes this).
 */
#ifndef ORC_INTERNAL_H
#define ORC_INTERNAL_H
#include <stdint.h>

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_NEARFIELD (-4)

enum {
    ORC_LAPLACE_SLP = 0,
    ORC_LAPLACE_DLP = 1,
    ORC_HELMHOLTZ_SLP = 2,
    ORC_HELMHOLTZ_DLP = 3,
    ORC_LAPLACE_ADLP = 4,
    ORC_HELMHOLTZ_ADLP = 5,
    ORC_LAPLACE_HYPS = 6,
    ORC_HELMHOLTZ_HYPS = 7
};
enum { ORC_P0 = 0, ORC_P1 = 1, ORC_DP1 = 2 };
enum { ORC_NEAR_ERROR = 0, ORC_NEAR_SKIP = 1 };

/* ------------------------------------------------------------------------ */
/* Mesh context: geometry per triangle and vertex stars.                      */
typedef struct {
    int64_t nv, nt;
    int q;
    double qxi[6], qeta[6], qw[6];
    double *xyz;      /* nv x 3 */
    int32_t *tri;     /* nt x 3 */
    double *J;        /* nt: |(b-a) x (c-a)| = twice the area */
    double *n;        /* nt x 3 unit normal along (b-a) x (c-a) */
    double *qp;       /* nt x q x 3 quadrature points */
    int64_t *star_ptr; /* nv + 1 */
    int32_t *star;    /* 3 nt: triangles around each vertex, ascending */
} orc_mesh;

int orc_rule(int npts, double *xi, double *eta, double *w);
void orc_kernel(int op, double k, const double *x, const double *y, const double *nrm, double *out);
int orc_adjacent(const orc_mesh *m, int64_t a, int64_t b);
/* surface curl n x grad of the hat function of local vertex loc on triangle t */
void orc_curl(const orc_mesh *m, int64_t t, int loc, double *out);
void orc_pair(const orc_mesh *m, int op, double k, int64_t tm, int64_t tn,
              int a, int b, double *re, double *im);

#endif
