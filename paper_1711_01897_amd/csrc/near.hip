// Singular (vertex-sharing) triangle pairs on the device: the Laplace and
// Helmholtz single and double layer, P0 and P1 (P1: 3 x 3 local matrices,
// summed into the entries by a fixed-order gather), and the P1 Laplace and
// Helmholtz hypersingular operator.
//
// The regular kernels integrate vertex-disjoint pairs only; Section 3.2.3
// gives identical, edge-adjacent and vertex-adjacent pairs to a separate
// singular scheme.  Here each such pair is written in coordinates around its
// singular set in which x - y is (radius) x (a vector of the remaining
// coordinates).  Both kernels are homogeneous in x - y (degree -1 for 1/r,
// -2 for (x-y).n_y / r^3, where only the test side's out-of-plane part
// survives in the numerator), so the radial integral is a polynomial one and
// is done in closed form; what remains is smooth and goes to a composite
// Gauss-Legendre rule:
//   identical:     the six-region decomposition of T x T over the reference
//                  triangle {0 <= x2 <= x1 <= 1} (Jacobian xi^3 eta1^2 eta2);
//                  x - y = xi eta1 eta2 c(eta3) with c one of three lines in
//                  the plane of the edges, so the single layer is
//                  (1/3) sum_c int_0^1 d(eta3) / |c(eta3)| and the double
//                  layer vanishes (x - y lies in the plane);
//   common edge:   affine coordinates x = P + u1 E + s1 a, y = P + u2 E + s2 b
//                  (E the shared edge, a, b to the third vertices); the three
//                  small coordinates (u1 - u2, s1, s2) in cone coordinates of
//                  radius rho = max(s2, s1 + u1 - u2) (or its mirror), the
//                  along-edge coordinate leaving a segment of length 1 - rho:
//                  radial factor int rho (1 - rho) = 1/6 (single layer) or
//                  int (1 - rho) = 1/2 (double layer), four faces of the
//                  unit cone, each a square or a collapsed square;
//   common vertex: Duffy coordinates from the shared vertex ordered by the
//                  larger radius s (Jacobian s^3 z), x - y = s (a(u) - z b(v))
//                  or s (z a(u) - b(v)): radial factor 1/3 or 1/2, a 3D
//                  integral over (z, u, v).
// Rules: 16 points per direction (two panels of the 8-point rule; 32 for the
// identical case's 1D integrals): about 1e-12 relative on these pairs, where
// the full 4D tensor rule with 8 points per direction left ~1e-8.
// Helmholtz: g = e^{ikr}/(4 pi r) and its normal derivative
// e^{ikr} (1 - ikr) (x-y).n_y / (4 pi r^3) are the Laplace kernels times a
// factor smooth in the radius, so the same coordinates apply with the radial
// integral int pi(rho) e^{i omega rho} (1 - i omega rho)^[double layer] d rho
// (omega = k |c|, pi the Laplace case's radial polynomial, identical pairs
// after folding xi eta1 eta2 into one radius with weight (1 - p)^2) taken
// as its power series sum_n (i omega)^n mu_n c_n / n! (mu_n the moments of
// pi, c_n = 1, or 1 - n with the double layer's factor), 48 terms in Horner
// form: ~1e-14 relative at omega = 6 (two elements per wavelength reach
// omega ~ 2 pi), 5e-10 at omega = 12 where the alternating terms cancel.
// The adjoint double layer is the double layer with test and trial exchanged
// (the host builds its items that way).
#include <hip/hip_runtime.h>

#include "bem_internal.hpp"

namespace bem {
namespace {

constexpr int kGL = 8;          // Gauss-Legendre points per panel
constexpr int kPts = 2 * kGL;   // composite rule: two panels per direction
constexpr int kIdPanels = 4;    // identical pairs: 1D integrals on four panels
constexpr int kIdPts = kIdPanels * kGL;
constexpr int kNearThreads = 256;
static_assert(kPts * kPts == kNearThreads, "common-vertex pairs take one (u, v) node per thread");
static_assert(4 * kPts * 4 == kNearThreads, "common-edge pairs take (face, p, q group) per thread");
static_assert(3 * kIdPts <= kNearThreads, "identical pairs take one (line, node) per thread");

// 8-point Gauss-Legendre rule on [0, 1] (nodes (1 + x)/2, weights w/2 of the
// published rule on [-1, 1]).
__constant__ double c_x[kGL] = {0.5 * (1.0 - 0.9602898564975363), 0.5 * (1.0 - 0.7966664774136267),
                                0.5 * (1.0 - 0.5255324099163290), 0.5 * (1.0 - 0.1834346424956498),
                                0.5 * (1.0 + 0.1834346424956498), 0.5 * (1.0 + 0.5255324099163290),
                                0.5 * (1.0 + 0.7966664774136267), 0.5 * (1.0 + 0.9602898564975363)};
__constant__ double c_w[kGL] = {0.5 * 0.1012285362903763, 0.5 * 0.2223810344533745, 0.5 * 0.3137066458778873,
                                0.5 * 0.3626837833783620, 0.5 * 0.3626837833783620, 0.5 * 0.3137066458778873,
                                0.5 * 0.2223810344533745, 0.5 * 0.1012285362903763};

constexpr double kInv4PiD = 0.0795774715459476678844418816862571;

struct V3 {
    double x, y, z;
};
__device__ __forceinline__ V3 ld(const double *p) { return {p[0], p[1], p[2]}; }
__device__ __forceinline__ V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 mul(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ V3 fma3(double s, V3 a, V3 b) { return {fma(s, a.x, b.x), fma(s, a.y, b.y), fma(s, a.z, b.z)}; }
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

struct Cx {
    double re, im;
};

// Power series of the radial integral: coefficients of omega^(2m) (real
// part) and omega^(2m+1) (imaginary part), signs of i^n included.
constexpr int kSeries = 48;
template <int POLY, bool DL>
struct RadialSeries {
    double re[kSeries / 2], im[kSeries / 2];
    constexpr RadialSeries() : re(), im()
    {
        double fact = 1.0;
        for (int n = 0; n < kSeries; ++n) {
            if (n > 0) fact *= n;
            const double nn = n;
            const double mu = POLY == 0 ? 2.0 / ((nn + 1) * (nn + 2) * (nn + 3))
                            : POLY == 1 ? 1.0 / ((nn + 2) * (nn + 3))
                            : POLY == 2 ? 1.0 / ((nn + 1) * (nn + 2))
                            : POLY == 3 ? 1.0 / (nn + 3)
                                        : 1.0 / (nn + 2);
            const double a = mu * (DL ? 1.0 - nn : 1.0) / fact;
            const int m = n / 2;
            const double sgn = (m % 2) ? -1.0 : 1.0;
            if (n % 2 == 0)
                re[m] = sgn * a;
            else
                im[m] = sgn * a;
        }
    }
};

// int_0^1 pi(rho) e^{i om rho} (1 - i om rho)^[DL] d rho.
template <int POLY, bool DL>
__device__ __forceinline__ Cx radial(double om)
{
    constexpr RadialSeries<POLY, DL> c{};
    const double w2 = om * om;
    double r = c.re[kSeries / 2 - 1], i = c.im[kSeries / 2 - 1];
#pragma unroll
    for (int m = kSeries / 2 - 2; m >= 0; --m) {
        r = fma(r, w2, c.re[m]);
        i = fma(i, w2, c.im[m]);
    }
    return {r, om * i};
}

// int_0^1 rho^A (1 - rho)^B e^{i om rho} (1 - i om rho)^[DL] d rho (B <= 2)
// by the same 48-term series (moments of rho^A (1 - rho)^B).
template <int A, int B, bool DL>
struct MomentSeries {
    double re[kSeries / 2], im[kSeries / 2];
    constexpr MomentSeries() : re(), im()
    {
        double fact = 1.0;
        for (int n = 0; n < kSeries; ++n) {
            if (n > 0) fact *= n;
            const double e = n + A;
            const double mu = B == 0 ? 1.0 / (e + 1) : B == 1 ? 1.0 / ((e + 1) * (e + 2)) : 2.0 / ((e + 1) * (e + 2) * (e + 3));
            const double a = mu * (DL ? 1.0 - n : 1.0) / fact;
            const int m = n / 2;
            const double sgn = (m % 2) ? -1.0 : 1.0;
            if (n % 2 == 0)
                re[m] = sgn * a;
            else
                im[m] = sgn * a;
        }
    }
};

template <int A, int B, bool DL>
__device__ __forceinline__ Cx moment(double om)
{
    constexpr MomentSeries<A, B, DL> c{};
    const double w2 = om * om;
    double r = c.re[kSeries / 2 - 1], i = c.im[kSeries / 2 - 1];
#pragma unroll
    for (int m = kSeries / 2 - 2; m >= 0; --m) {
        r = fma(r, w2, c.re[m]);
        i = fma(i, w2, c.im[m]);
    }
    return {r, om * i};
}

// Helmholtz share of this thread (op 2 single layer, op 3 double layer),
// without jt js / 4 pi (and (a.n_y) for common-edge double layers).
template <int OP>
__device__ Cx pair_part_helmholtz(const NearItem &it, const double *sx, const double *sw)
{
    constexpr bool DL = OP == 3;
    const int t = threadIdx.x;
    const double k = it.k;
    if (it.kind == 0) {
        if (DL || t >= 3 * kIdPts) return {0.0, 0.0};
        const V3 V0 = ld(it.v), V1 = ld(it.v + 3), V2 = ld(it.v + 6);
        const V3 E1 = sub(V1, V0), E2 = sub(V2, V1);
        const int line = t / kIdPts, kk = t - line * kIdPts;
        const double e = (c_x[kk % kGL] + (double)(kk / kGL)) * (1.0 / kIdPanels);
        const double w = c_w[kk % kGL] * (1.0 / kIdPanels);
        const V3 c = line == 0 ? fma3(e, E1, E2) : (line == 1 ? fma3(e, E2, E1) : fma3(-e, E1, mul(1.0 - e, E2)));
        const double ri = rsqrt(dot(c, c));
        const Cx rad = radial<0, false>(k / ri);
        return {w * ri * rad.re, w * ri * rad.im};
    }
    double ar = 0.0, ai = 0.0;
    if (it.kind == 1) {
        const V3 P = ld(it.v), Q = ld(it.v + 3), A = ld(it.v + 6), B = ld(it.v + 9);
        const V3 E = sub(Q, P), a = sub(A, P), b = sub(B, P);
        const int face = t >> 6, ip = (t >> 2) & (kPts - 1), g = t & 3;
        const double p = sx[ip], q1 = 1.0 - p;
        V3 c0, c1;
        double s1c, s1q, fw;
        if (face == 0) {
            c0 = sub(mul(p, E), b), c1 = mul(q1, a), s1c = 0.0, s1q = q1, fw = q1;
        } else if (face == 1) {
            c0 = fma3(p, E, mul(q1, a)), c1 = mul(-1.0, b), s1c = q1, s1q = 0.0, fw = 1.0;
        } else if (face == 2) {
            c0 = fma3(-p, E, a), c1 = mul(-q1, b), s1c = 1.0, s1q = 0.0, fw = q1;
        } else {
            c0 = fma3(-p, E, mul(-q1, b)), c1 = a, s1c = 0.0, s1q = 1.0, fw = 1.0;
        }
        for (int j = 0; j < kPts / 4; ++j) {
            const double q = sx[g + 4 * j];
            const V3 c = fma3(q, c1, c0);
            const double ri = rsqrt(dot(c, c));
            const Cx rad = radial<DL ? 2 : 1, DL>(k / ri);
            const double f = sw[g + 4 * j] * (DL ? fma(q, s1q, s1c) * ri * ri * ri : ri);
            ar += f * rad.re;
            ai += f * rad.im;
        }
        const double wf = sw[ip] * fw;
        return {wf * ar, wf * ai};
    }
    const V3 P = ld(it.v), A = ld(it.v + 3), B = ld(it.v + 6), C = ld(it.v + 9), D = ld(it.v + 12);
    const int iu = t / kPts, iv = t % kPts;
    const V3 a = fma3(sx[iu], sub(B, A), sub(A, P));
    const V3 b = fma3(sx[iv], sub(D, C), sub(C, P));
    const double an = DL ? dot(a, ld(it.ny)) : 1.0;
    for (int kz = 0; kz < kPts; ++kz) {
        const double z = sx[kz], wz = sw[kz] * z;
        const V3 d1 = fma3(-z, b, a), d2 = fma3(z, a, mul(-1.0, b));
        const double r1 = rsqrt(dot(d1, d1)), r2 = rsqrt(dot(d2, d2));
        const Cx g1 = radial<DL ? 4 : 3, DL>(k / r1), g2 = radial<DL ? 4 : 3, DL>(k / r2);
        const double f1 = wz * an * (DL ? r1 * r1 * r1 : r1);
        const double f2 = wz * an * (DL ? z * r2 * r2 * r2 : r2);
        ar += f1 * g1.re + f2 * g2.re;
        ai += f1 * g1.im + f2 * g2.im;
    }
    const double wuv = sw[iu] * sw[iv];
    return {wuv * ar, wuv * ai};
}

// Kernel of the remaining integral at the scaled difference c: 1/|c| for
// the single layer, num/|c|^3 for the double layer.
template <int OP>
__device__ __forceinline__ double kern(V3 c, double num)
{
    const double ri = rsqrt(dot(c, c));
    if constexpr (OP == 0) return ri;
    return num * ri * ri * ri;
}

// This thread's share of the pair integral (without jt js / 4 pi and the
// radial factor, which pair_scale gives); sx, sw hold the 16-point rule.
template <int OP>
__device__ double pair_part(const NearItem &it, const double *sx, const double *sw)
{
    const int t = threadIdx.x;
    if (it.kind == 0) {
        if constexpr (OP == 1) return 0.0;
        if (t >= 3 * kIdPts) return 0.0;
        const V3 V0 = ld(it.v), V1 = ld(it.v + 3), V2 = ld(it.v + 6);
        const V3 E1 = sub(V1, V0), E2 = sub(V2, V1);
        const int line = t / kIdPts, k = t - line * kIdPts;
        const double e = (c_x[k % kGL] + (double)(k / kGL)) * (1.0 / kIdPanels);
        const double w = c_w[k % kGL] * (1.0 / kIdPanels);
        const V3 c = line == 0 ? fma3(e, E1, E2) : (line == 1 ? fma3(e, E2, E1) : fma3(-e, E1, mul(1.0 - e, E2)));
        return w * kern<0>(c, 0.0);
    }
    if (it.kind == 1) {
        const V3 P = ld(it.v), Q = ld(it.v + 3), A = ld(it.v + 6), B = ld(it.v + 9);
        const V3 E = sub(Q, P), a = sub(A, P), b = sub(B, P);
        const int face = t >> 6, ip = (t >> 2) & (kPts - 1), g = t & 3;
        const double p = sx[ip], q1 = 1.0 - p;
        // c = c0 + q c1 on the face; s1 = s1c + q s1q is the test side's
        // distance from the edge (the double layer's numerator / (a.n_y))
        V3 c0, c1;
        double s1c, s1q, fw;
        if (face == 0) {          // s2 = 1, s1 = (1 - d) q
            c0 = sub(mul(p, E), b), c1 = mul(q1, a), s1c = 0.0, s1q = q1, fw = q1;
        } else if (face == 1) {   // s1 + d = 1, s2 = q
            c0 = fma3(p, E, mul(q1, a)), c1 = mul(-1.0, b), s1c = q1, s1q = 0.0, fw = 1.0;
        } else if (face == 2) {   // s1 = 1, s2 = (1 - e) q, d = -e
            c0 = fma3(-p, E, a), c1 = mul(-q1, b), s1c = 1.0, s1q = 0.0, fw = q1;
        } else {                  // s2 + e = 1, s1 = q, d = -e
            c0 = fma3(-p, E, mul(-q1, b)), c1 = a, s1c = 0.0, s1q = 1.0, fw = 1.0;
        }
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < kPts / 4; ++j) {
            const double q = sx[g + 4 * j];
            s += sw[g + 4 * j] * kern<OP>(fma3(q, c1, c0), fma(q, s1q, s1c));
        }
        return sw[ip] * fw * s;
    }
    const V3 P = ld(it.v), A = ld(it.v + 3), B = ld(it.v + 6), C = ld(it.v + 9), D = ld(it.v + 12);
    const int iu = t / kPts, iv = t % kPts;
    const V3 a = fma3(sx[iu], sub(B, A), sub(A, P));
    const V3 b = fma3(sx[iv], sub(D, C), sub(C, P));
    const double an = OP == 1 ? dot(a, ld(it.ny)) : 0.0;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kPts; ++k) {
        const double z = sx[k], wz = sw[k] * z;
        s += wz * (kern<OP>(fma3(-z, b, a), an) + (OP == 1 ? z : 1.0) * kern<OP>(fma3(z, a, mul(-1.0, b)), an));
    }
    return sw[iu] * sw[iv] * s;
}

// jt js / 4 pi times the closed-form radial integral of the pair's kind.
template <int OP>
__device__ double pair_scale(const NearItem &it)
{
    if constexpr (OP >= 2) {
        const double an = (OP == 3 && it.kind == 1) ? dot(sub(ld(it.v + 6), ld(it.v)), ld(it.ny)) : 1.0;
        return an * it.jt * it.js * kInv4PiD;
    }
    double radial;
    if (it.kind == 0)
        radial = OP == 0 ? 1.0 / 3.0 : 0.0;
    else if (it.kind == 1)
        radial = OP == 0 ? 1.0 / 6.0 : 0.5 * dot(sub(ld(it.v + 6), ld(it.v)), ld(it.ny));
    else
        radial = OP == 0 ? 1.0 / 3.0 : 0.5;
    return radial * it.jt * it.js * kInv4PiD;
}

template <int OP>
__device__ Cx pair_value(const NearItem &it)
{
    __shared__ double sx[kPts], sw[kPts];
    __shared__ double red[2][kNearThreads];
    const int t = threadIdx.x;
    if (t < kPts) {
        sx[t] = 0.5 * (c_x[t % kGL] + (double)(t / kGL));
        sw[t] = 0.5 * c_w[t % kGL];
    }
    __syncthreads();
    if constexpr (OP >= 2) {
        const Cx v = pair_part_helmholtz<OP>(it, sx, sw);
        red[0][t] = v.re;
        red[1][t] = v.im;
    } else {
        red[0][t] = pair_part<OP>(it, sx, sw);
        red[1][t] = 0.0;
    }
    __syncthreads();
    // fixed-order tree reduction over the workgroup
    for (int h = kNearThreads / 2; h > 0; h >>= 1) {
        if (t < h) {
            red[0][t] += red[0][t + h];
            red[1][t] += red[1][t + h];
        }
        __syncthreads();
    }
    const double sc = pair_scale<OP>(it);
    return {red[0][0] * sc, red[1][0] * sc};
}

template <int OP, bool FP32>
__global__ __launch_bounds__(kNearThreads) void k_near_p0(const NearItem *__restrict__ items, int64_t n)
{
    if ((int64_t)blockIdx.x >= n) return;
    const NearItem &it = items[blockIdx.x];
    const Cx v = pair_value<OP>(it);
    if (threadIdx.x == 0) {
        constexpr int kParts = OP >= 2 ? 2 : 1;   // complex entries: (re, im)
        if constexpr (FP32) {
            float *o = static_cast<float *>(it.out);
            o[0] = (float)((double)o[0] + v.re);
            if constexpr (kParts == 2) o[1] = (float)((double)o[1] + v.im);
        } else {
            double *o = static_cast<double *>(it.out);
            o[0] = o[0] + v.re;
            if constexpr (kParts == 2) o[1] = o[1] + v.im;
        }
    }
}

// ---------------------------------------------------------------------------
// P1 pairs: the 3 x 3 local matrix M[a][b] = int_T lambda_a int_S mu_b K of
// the pair's barycentrics in the item's vertex order (test (V0, V1, V2),
// (P, Q, A), (P, A, B); trial (V0, V1, V2), (P, Q, B), (P, C, D) for the
// identical, common-edge and common-vertex kinds).  Same coordinates and face
// rules as P0; the barycentrics are affine in the radius (bilinear in radius
// and along-edge coordinate; for identical pairs polynomial in xi, eta1,
// eta2), so those directions take Gauss rules exact for the degrees that
// occur: 3 points for the radius (degree 4), 2 for the rest (degree <= 3).

// 2- and 3-point Gauss-Legendre rules on [0, 1].
constexpr double kG2x[2] = {0.5 - 0.28867513459481288225, 0.5 + 0.28867513459481288225};
constexpr double kG3x[3] = {0.5 - 0.38729833462074168852, 0.5, 0.5 + 0.38729833462074168852};
constexpr double kG3w[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};

struct L3 {
    double v[3];
};

// acc[3a + b] += w * l[a] * m[b]
__device__ __forceinline__ void outer_acc(double *acc, double w, const L3 &l, const L3 &m)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double wa = w * l.v[a];
#pragma unroll
        for (int b = 0; b < 3; ++b) acc[3 * a + b] = fma(wa, m.v[b], acc[3 * a + b]);
    }
}

// This thread's share of the 9 local integrals (without jt js / 4 pi and,
// for the common-edge double layer, without (a.n_y)).
template <int OP>
__device__ void pair_part_p1(const NearItem &it, const double *sx, const double *sw, double *acc)
{
    const int t = threadIdx.x;
    if (it.kind == 0) {
        if (OP == 1 || t >= 3 * kIdPts) return;
        const V3 V0 = ld(it.v), V1 = ld(it.v + 3), V2 = ld(it.v + 6);
        const V3 E1 = sub(V1, V0), E2 = sub(V2, V1);
        const int line = t / kIdPts, kk = t - line * kIdPts;
        const double e3 = (c_x[kk % kGL] + (double)(kk / kGL)) * (1.0 / kIdPanels);
        const double w3 = c_w[kk % kGL] * (1.0 / kIdPanels);
        const V3 c = line == 0 ? fma3(e3, E1, E2) : (line == 1 ? fma3(e3, E2, E1) : fma3(-e3, E1, mul(1.0 - e3, E2)));
        const double ic = rsqrt(dot(c, c));
        // barycentrics of V0 + a E1 + b E2: (1 - a, a - b, b)
        auto lam = [](double a, double b) { return L3{{1.0 - a, a - b, b}}; };
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int l = 0; l < 2; ++l) {
                    const double xi = kG3x[i], e1 = kG2x[j], e2 = kG2x[l];
                    double xa, xb, ya, yb;
                    if (line == 0) {
                        xa = xi, xb = xi * (1.0 - e1 + e1 * e2), ya = xi * (1.0 - e1 * e2 * e3), yb = xi * (1.0 - e1);
                    } else if (line == 1) {
                        xa = xi, xb = xi * e1 * (1.0 - e2 + e2 * e3), ya = xi * (1.0 - e1 * e2), yb = xi * e1 * (1.0 - e2);
                    } else {
                        xa = xi * (1.0 - e1 * e2 * e3), xb = xi * e1 * (1.0 - e2 * e3), ya = xi, yb = xi * e1 * (1.0 - e2);
                    }
                    const L3 lx = lam(xa, xb), ly = lam(ya, yb);
                    const double w = w3 * kG3w[i] * 0.25 * xi * xi * e1 * ic;
                    // the region and its mirror (x and y exchanged)
                    outer_acc(acc, w, lx, ly);
                    outer_acc(acc, w, ly, lx);
                }
        return;
    }
    if (it.kind == 1) {
        const V3 P = ld(it.v), Q = ld(it.v + 3), A = ld(it.v + 6), B = ld(it.v + 9);
        const V3 E = sub(Q, P), a = sub(A, P), b = sub(B, P);
        const int face = t >> 6, ip = (t >> 2) & (kPts - 1), g = t & 3;
        const double p = sx[ip], q1 = 1.0 - p;
        for (int j = 0; j < kPts / 4; ++j) {
            const double q = sx[g + 4 * j];
            double dh, s1h, s2h, fw;
            if (face == 0)
                dh = p, s1h = q1 * q, s2h = 1.0, fw = q1;
            else if (face == 1)
                dh = p, s1h = q1, s2h = q, fw = 1.0;
            else if (face == 2)
                dh = -p, s1h = 1.0, s2h = q1 * q, fw = q1;
            else
                dh = -p, s1h = q, s2h = q1, fw = 1.0;
            const V3 c = fma3(dh, E, fma3(s1h, a, mul(-s2h, b)));
            const double ic = rsqrt(dot(c, c));
            const double K = sw[ip] * sw[g + 4 * j] * fw * (OP == 0 ? ic : s1h * ic * ic * ic);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int l = 0; l < 2; ++l) {
                    const double rho = kG3x[i], tau = kG2x[l];
                    double u1, u2;
                    if (face < 2) {
                        u2 = (1.0 - rho) * tau;
                        u1 = u2 + rho * dh;
                    } else {
                        u1 = (1.0 - rho) * tau;
                        u2 = u1 - rho * dh;
                    }
                    const double s1 = rho * s1h, s2 = rho * s2h;
                    const double rad = OP == 0 ? rho * (1.0 - rho) : 1.0 - rho;
                    outer_acc(acc, K * kG3w[i] * 0.5 * rad, L3{{1.0 - u1 - s1, u1, s1}}, L3{{1.0 - u2 - s2, u2, s2}});
                }
        }
        return;
    }
    const V3 P = ld(it.v), A = ld(it.v + 3), B = ld(it.v + 6), C = ld(it.v + 9), D = ld(it.v + 12);
    const int iu = t / kPts, iv = t % kPts;
    const double u = sx[iu], v = sx[iv];
    const V3 av = fma3(u, sub(B, A), sub(A, P));
    const V3 bv = fma3(v, sub(D, C), sub(C, P));
    const double an = OP == 1 ? dot(av, ld(it.ny)) : 1.0;
    const double wuv = sw[iu] * sw[iv];
    for (int kz = 0; kz < kPts; ++kz) {
        const double z = sx[kz];
        const V3 c1 = fma3(-z, bv, av), c2 = fma3(z, av, mul(-1.0, bv));
        const double i1 = rsqrt(dot(c1, c1)), i2 = rsqrt(dot(c2, c2));
        const double f = wuv * sw[kz] * z * an;
        const double k1 = f * (OP == 0 ? i1 : i1 * i1 * i1), k2 = f * (OP == 0 ? i2 : z * i2 * i2 * i2);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double s = kG3x[i], sz = s * z;
            const double rad = kG3w[i] * (OP == 0 ? s * s : s);
            outer_acc(acc, rad * k1, L3{{1.0 - s, s * (1.0 - u), s * u}}, L3{{1.0 - sz, sz * (1.0 - v), sz * v}});
            outer_acc(acc, rad * k2, L3{{1.0 - sz, sz * (1.0 - u), sz * u}}, L3{{1.0 - s, s * (1.0 - v), s * v}});
        }
    }
}

// The three series J_m = int rho^(A0 + m) (1 - rho)^B e^{i om rho} (...)
// (m = 0, 1, 2) evaluated together from a coefficient table staged in LDS
// (interleaved re/im of the three per power of om^2): literal FP64
// coefficients would otherwise be held in registers across the face loops.
template <int A0, int B, bool DL>
struct MomentTable3 {
    double v[6 * (kSeries / 2)];
    constexpr MomentTable3() : v()
    {
        const MomentSeries<A0, B, DL> s0{};
        const MomentSeries<A0 + 1, B, DL> s1{};
        const MomentSeries<A0 + 2, B, DL> s2{};
        for (int m = 0; m < kSeries / 2; ++m) {
            v[6 * m] = s0.re[m], v[6 * m + 1] = s0.im[m];
            v[6 * m + 2] = s1.re[m], v[6 * m + 3] = s1.im[m];
            v[6 * m + 4] = s2.re[m], v[6 * m + 5] = s2.im[m];
        }
    }
};
constexpr int kTab3 = 6 * (kSeries / 2);
__constant__ MomentTable3<2, 0, false> c_tab_s20{};   // identical and common-vertex single layer
__constant__ MomentTable3<1, 1, false> c_tab_s11{};   // common-edge single layer
__constant__ MomentTable3<1, 0, true> c_tab_d10{};    // common-vertex double layer
__constant__ MomentTable3<0, 1, true> c_tab_d01{};    // common-edge double layer

__device__ __forceinline__ void moment3(double om, const double *tab, Cx &J0, Cx &J1, Cx &J2)
{
    const double w2 = om * om;
    const double *t = tab + 6 * (kSeries / 2 - 1);
    double r0 = t[0], i0 = t[1], r1 = t[2], i1 = t[3], r2 = t[4], i2 = t[5];
#pragma unroll 4
    for (int m = kSeries / 2 - 2; m >= 0; --m) {
        t = tab + 6 * m;
        r0 = fma(r0, w2, t[0]);
        i0 = fma(i0, w2, t[1]);
        r1 = fma(r1, w2, t[2]);
        i1 = fma(i1, w2, t[3]);
        r2 = fma(r2, w2, t[4]);
        i2 = fma(i2, w2, t[5]);
    }
    J0 = {r0, om * i0};
    J1 = {r1, om * i1};
    J2 = {r2, om * i2};
}

// acc[3a + b] += K (alpha_a gamma_b J0 + (alpha_a delta_b + beta_a gamma_b) J1
// + beta_a delta_b J2): the radial integral of (alpha + beta rho)(gamma +
// delta rho) against the moments J_m (complex), times K.
__device__ __forceinline__ void moment_acc(double *ar, double *ai, double K, const L3 &al, const L3 &be, const L3 &ga,
                                           const L3 &de, const Cx &J0, const Cx &J1, const Cx &J2)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const double c0 = K * al.v[a] * ga.v[b], c1 = K * (al.v[a] * de.v[b] + be.v[a] * ga.v[b]),
                         c2 = K * be.v[a] * de.v[b];
            ar[3 * a + b] += c0 * J0.re + c1 * J1.re + c2 * J2.re;
            ai[3 * a + b] += c0 * J0.im + c1 * J1.im + c2 * J2.im;
        }
}

// P1 Helmholtz (op 2 single, op 3 double layer): the Laplace P1 scheme with
// the radial factor e^{ikr}: at each face point the barycentrics are
// alpha + beta rho (test) and gamma + delta rho (trial), and the radial
// integrals are three moment series (identical pairs: the radius xi, the
// moments at omega eta1 eta2, eta1 and eta2 on the 8-point rule).
// tr: the radial table of identical and common-vertex pairs, te: of
// common-edge pairs (both in LDS).
template <int OP>
__device__ void pair_part_p1_helmholtz(const NearItem &it, const double *sx, const double *sw, const double *tr,
                                       const double *te, double *ar, double *ai)
{
    constexpr bool DL = OP == 3;
    const int t = threadIdx.x;
    const double k = it.k;
    if (it.kind == 0) {
        if (DL || t >= 3 * kIdPts) return;
        const V3 V0 = ld(it.v), V1 = ld(it.v + 3), V2 = ld(it.v + 6);
        const V3 E1 = sub(V1, V0), E2 = sub(V2, V1);
        const int line = t / kIdPts, kk = t - line * kIdPts;
        const double e3 = (c_x[kk % kGL] + (double)(kk / kGL)) * (1.0 / kIdPanels);
        const double w3 = c_w[kk % kGL] * (1.0 / kIdPanels);
        const V3 c = line == 0 ? fma3(e3, E1, E2) : (line == 1 ? fma3(e3, E2, E1) : fma3(-e3, E1, mul(1.0 - e3, E2)));
        const double ic = rsqrt(dot(c, c));
        const double om = k / ic;
        // loops kept rolled: the unrolled series would hold every node's
        // coefficients in registers
#pragma unroll 1
        for (int j = 0; j < kGL; ++j)
#pragma unroll 1
            for (int l = 0; l < kGL; ++l) {
                const double e1 = c_x[j], e2 = c_x[l];
                // x = xi (A1, B1), y = xi (A2, B2) in the (a, b) coordinates
                double A1, B1, A2, B2;
                if (line == 0) {
                    A1 = 1.0, B1 = 1.0 - e1 + e1 * e2, A2 = 1.0 - e1 * e2 * e3, B2 = 1.0 - e1;
                } else if (line == 1) {
                    A1 = 1.0, B1 = e1 * (1.0 - e2 + e2 * e3), A2 = 1.0 - e1 * e2, B2 = e1 * (1.0 - e2);
                } else {
                    A1 = 1.0 - e1 * e2 * e3, B1 = e1 * (1.0 - e2 * e3), A2 = 1.0, B2 = e1 * (1.0 - e2);
                }
                const double w = w3 * c_w[j] * c_w[l] * e1 * ic;
                const double oe = om * e1 * e2;
                Cx J0, J1, J2;
                moment3(oe, tr, J0, J1, J2);
                const L3 al{{1.0, 0.0, 0.0}}, bx{{-A1, A1 - B1, B1}}, by{{-A2, A2 - B2, B2}};
                moment_acc(ar, ai, w, al, bx, al, by, J0, J1, J2);   // the region
                moment_acc(ar, ai, w, al, by, al, bx, J0, J1, J2);   // and its mirror
            }
        return;
    }
    if (it.kind == 1) {
        const V3 P = ld(it.v), Q = ld(it.v + 3), A = ld(it.v + 6), B = ld(it.v + 9);
        const V3 E = sub(Q, P), a = sub(A, P), b = sub(B, P);
        const int face = t >> 6, ip = (t >> 2) & (kPts - 1), g = t & 3;
        const double p = sx[ip], q1 = 1.0 - p;
#pragma unroll 1
        for (int j = 0; j < kPts / 4; ++j) {
            const double q = sx[g + 4 * j];
            double dh, s1h, s2h, fw;
            if (face == 0)
                dh = p, s1h = q1 * q, s2h = 1.0, fw = q1;
            else if (face == 1)
                dh = p, s1h = q1, s2h = q, fw = 1.0;
            else if (face == 2)
                dh = -p, s1h = 1.0, s2h = q1 * q, fw = q1;
            else
                dh = -p, s1h = q, s2h = q1, fw = 1.0;
            const V3 c = fma3(dh, E, fma3(s1h, a, mul(-s2h, b)));
            const double ic = rsqrt(dot(c, c));
            const double om = k / ic;
            const double K = sw[ip] * sw[g + 4 * j] * fw * (DL ? s1h * ic * ic * ic : ic);
            Cx J0, J1, J2;
            moment3(om, te, J0, J1, J2);
#pragma unroll
            for (int l = 0; l < 2; ++l) {
                const double tau = kG2x[l];
                L3 al, be, ga, de;
                al = L3{{1.0 - tau, tau, 0.0}};
                ga = L3{{1.0 - tau, tau, 0.0}};
                if (face < 2) {   // u2 = (1 - rho) tau, u1 = u2 + rho dh
                    be = L3{{tau - dh - s1h, dh - tau, s1h}};
                    de = L3{{tau - s2h, -tau, s2h}};
                } else {          // u1 = (1 - rho) tau, u2 = u1 - rho dh
                    be = L3{{tau - s1h, -tau, s1h}};
                    de = L3{{tau + dh - s2h, -dh - tau, s2h}};
                }
                moment_acc(ar, ai, 0.5 * K, al, be, ga, de, J0, J1, J2);
            }
        }
        return;
    }
    const V3 P = ld(it.v), A = ld(it.v + 3), B = ld(it.v + 6), C = ld(it.v + 9), D = ld(it.v + 12);
    const int iu = t / kPts, iv = t % kPts;
    const double u = sx[iu], v = sx[iv];
    const V3 av = fma3(u, sub(B, A), sub(A, P));
    const V3 bv = fma3(v, sub(D, C), sub(C, P));
    const double an = DL ? dot(av, ld(it.ny)) : 1.0;
    const double wuv = sw[iu] * sw[iv];
    const L3 al{{1.0, 0.0, 0.0}}, bu{{-1.0, 1.0 - u, u}}, bvv{{-1.0, 1.0 - v, v}};
#pragma unroll 1
    for (int kz = 0; kz < kPts; ++kz) {
        const double z = sx[kz];
        const V3 c1 = fma3(-z, bv, av), c2 = fma3(z, av, mul(-1.0, bv));
        const double i1 = rsqrt(dot(c1, c1)), i2 = rsqrt(dot(c2, c2));
        const double f = wuv * sw[kz] * z * an;
        const double k1 = f * (DL ? i1 * i1 * i1 : i1), k2 = f * (DL ? z * i2 * i2 * i2 : i2);
        Cx J0, J1, J2, H0, H1, H2;
        moment3(k / i1, tr, J0, J1, J2);
        moment3(k / i2, tr, H0, H1, H2);
        const L3 zbv{{-z, z * (1.0 - v), z * v}}, zbu{{-z, z * (1.0 - u), z * u}};
        moment_acc(ar, ai, k1, al, bu, al, zbv, J0, J1, J2);    // x = P + s a(u), y = P + s z b(v)
        moment_acc(ar, ai, k2, al, zbu, al, bvv, H0, H1, H2);   // x = P + s z a(u), y = P + s b(v)
    }
}

// WITH_P0 (the Helmholtz hypersingular operator): the pair's P0 single-layer
// value follows the 9 complex local-matrix values (20 doubles per pair).
template <int OP, bool WITH_P0>
__global__ __launch_bounds__(kNearThreads) void k_near_p1_helmholtz(const NearItem *__restrict__ items, int64_t n)
{
    if ((int64_t)blockIdx.x >= n) return;
    const NearItem &it = items[blockIdx.x];
    __shared__ double sx[kPts], sw[kPts];
    __shared__ double tr[kTab3], te[kTab3];
    __shared__ double red[18][kNearThreads];
    const int t = threadIdx.x;
    if (t < kPts) {
        sx[t] = 0.5 * (c_x[t % kGL] + (double)(t / kGL));
        sw[t] = 0.5 * c_w[t % kGL];
    }
    for (int i = t; i < kTab3; i += kNearThreads) {
        tr[i] = OP == 3 ? c_tab_d10.v[i] : c_tab_s20.v[i];
        te[i] = OP == 3 ? c_tab_d01.v[i] : c_tab_s11.v[i];
    }
    __syncthreads();
    double ar[9], ai[9];
#pragma unroll
    for (int kk = 0; kk < 9; ++kk) ar[kk] = ai[kk] = 0.0;
    pair_part_p1_helmholtz<OP>(it, sx, sw, tr, te, ar, ai);
#pragma unroll
    for (int kk = 0; kk < 9; ++kk) {
        red[2 * kk][t] = ar[kk];
        red[2 * kk + 1][t] = ai[kk];
    }
    __syncthreads();
    for (int h = kNearThreads / 2; h > 0; h >>= 1) {
        if (t < h)
#pragma unroll
            for (int kk = 0; kk < 18; ++kk) red[kk][t] += red[kk][t + h];
        __syncthreads();
    }
    if (t < 18) {
        const double an = (OP == 3 && it.kind == 1) ? dot(sub(ld(it.v + 6), ld(it.v)), ld(it.ny)) : 1.0;
        static_cast<double *>(it.out)[t] = red[t][0] * an * it.jt * it.js * kInv4PiD;
    }
    if constexpr (WITH_P0) {
        const Cx v = pair_value<2>(it);
        if (t == 0) {
            static_cast<double *>(it.out)[18] = v.re;
            static_cast<double *>(it.out)[19] = v.im;
        }
    }
}

template <int OP>
__global__ __launch_bounds__(kNearThreads) void k_near_p1(const NearItem *__restrict__ items, int64_t n)
{
    if ((int64_t)blockIdx.x >= n) return;
    const NearItem &it = items[blockIdx.x];
    __shared__ double sx[kPts], sw[kPts];
    __shared__ double red[9][kNearThreads];
    const int t = threadIdx.x;
    if (t < kPts) {
        sx[t] = 0.5 * (c_x[t % kGL] + (double)(t / kGL));
        sw[t] = 0.5 * c_w[t % kGL];
    }
    __syncthreads();
    double acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = 0.0;
    pair_part_p1<OP>(it, sx, sw, acc);
#pragma unroll
    for (int k = 0; k < 9; ++k) red[k][t] = acc[k];
    __syncthreads();
    for (int h = kNearThreads / 2; h > 0; h >>= 1) {
        if (t < h)
#pragma unroll
            for (int k = 0; k < 9; ++k) red[k][t] += red[k][t + h];
        __syncthreads();
    }
    if (t < 9) {
        const double an = (OP == 1 && it.kind == 1) ? dot(sub(ld(it.v + 6), ld(it.v)), ld(it.ny)) : 1.0;
        static_cast<double *>(it.out)[t] = red[t][0] * an * it.jt * it.js * kInv4PiD;
    }
}

// Laplace hypersingular operator (Eq. hypsHelmholtz at k = 0): the hat
// functions' surface curls are constant per triangle, so a pair's local
// matrix is curl_a . curl_b times its P0 single-layer integral; the pair
// kernel stores that integral, the gather applies the curl products.
__global__ __launch_bounds__(kNearThreads) void k_near_slp_value(const NearItem *__restrict__ items, int64_t n)
{
    if ((int64_t)blockIdx.x >= n) return;
    const NearItem &it = items[blockIdx.x];
    const Cx v = pair_value<0>(it);
    if (threadIdx.x == 0) *static_cast<double *>(it.out) = v.re;
}

// Each record sums its sources (indices into the local values, times the
// source's weight when wt is given) in order and adds the sum to its entry.
template <bool FP32, bool CPLX>
__global__ void k_near_gather(const NearGather *__restrict__ recs, int64_t n, const int32_t *__restrict__ src,
                              const double *__restrict__ wt, const double *__restrict__ local)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const NearGather g = recs[i];
    if constexpr (CPLX) {   // complex local values (re, im) and entries
        double sr = 0.0, si = 0.0;
        for (int32_t k = 0; k < g.count; ++k) {
            const int64_t q = 2 * (int64_t)src[g.first + k];
            const double w = wt ? wt[g.first + k] : 1.0;
            sr += w * local[q];
            si += w * local[q + 1];
        }
        if constexpr (FP32) {
            float *o = static_cast<float *>(g.out);
            o[0] = (float)((double)o[0] + sr);
            o[1] = (float)((double)o[1] + si);
        } else {
            double *o = static_cast<double *>(g.out);
            o[0] = o[0] + sr;
            o[1] = o[1] + si;
        }
        return;
    }
    double s = 0.0;
    if (wt)
        for (int32_t k = 0; k < g.count; ++k) s += wt[g.first + k] * local[src[g.first + k]];
    else
        for (int32_t k = 0; k < g.count; ++k) s += local[src[g.first + k]];
    if constexpr (FP32) {
        float *o = static_cast<float *>(g.out);
        *o = (float)((double)*o + s);
    } else {
        double *o = static_cast<double *>(g.out);
        *o = *o + s;
    }
}

}  // namespace

hipError_t launch_near_p1(int op, const NearItem *items, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (n > INT32_MAX || op < 0 || (op > 3 && op != BEM_LAPLACE_HYPS && op != BEM_HELMHOLTZ_HYPS))
        return hipErrorInvalidValue;
    if (op == 2)
        hipLaunchKernelGGL((k_near_p1_helmholtz<2, false>), dim3((unsigned)n), dim3(kNearThreads), 0, s, items, n);
    else if (op == 3)
        hipLaunchKernelGGL((k_near_p1_helmholtz<3, false>), dim3((unsigned)n), dim3(kNearThreads), 0, s, items, n);
    else if (op == BEM_HELMHOLTZ_HYPS)
        hipLaunchKernelGGL((k_near_p1_helmholtz<2, true>), dim3((unsigned)n), dim3(kNearThreads), 0, s, items, n);
    else if (op == BEM_LAPLACE_HYPS)
        hipLaunchKernelGGL(k_near_slp_value, dim3((unsigned)n), dim3(kNearThreads), 0, s, items, n);
    else if (op == 0)
        hipLaunchKernelGGL((k_near_p1<0>), dim3((unsigned)n), dim3(kNearThreads), 0, s, items, n);
    else
        hipLaunchKernelGGL((k_near_p1<1>), dim3((unsigned)n), dim3(kNearThreads), 0, s, items, n);
    return hipGetLastError();
}

hipError_t launch_near_gather(bool fp32, bool cplx, const NearGather *recs, int64_t n, const int32_t *src,
                              const double *wt, const double *local, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks), block(256);
    if (cplx) {
        if (fp32)
            hipLaunchKernelGGL((k_near_gather<true, true>), grid, block, 0, s, recs, n, src, wt, local);
        else
            hipLaunchKernelGGL((k_near_gather<false, true>), grid, block, 0, s, recs, n, src, wt, local);
    } else if (fp32) {
        hipLaunchKernelGGL((k_near_gather<true, false>), grid, block, 0, s, recs, n, src, wt, local);
    } else {
        hipLaunchKernelGGL((k_near_gather<false, false>), grid, block, 0, s, recs, n, src, wt, local);
    }
    return hipGetLastError();
}

hipError_t launch_near(int op, bool fp32, const NearItem *items, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (n > INT32_MAX || op < 0 || op > 3) return hipErrorInvalidValue;
    const dim3 grid((unsigned)n), block(kNearThreads);
#define BEM_NEAR_LAUNCH(O)                                                              \
    do {                                                                                \
        if (fp32)                                                                       \
            hipLaunchKernelGGL((k_near_p0<O, true>), grid, block, 0, s, items, n);      \
        else                                                                            \
            hipLaunchKernelGGL((k_near_p0<O, false>), grid, block, 0, s, items, n);     \
    } while (0)
    switch (op) {
    case 0: BEM_NEAR_LAUNCH(0); break;
    case 1: BEM_NEAR_LAUNCH(1); break;
    case 2: BEM_NEAR_LAUNCH(2); break;
    default: BEM_NEAR_LAUNCH(3); break;
    }
#undef BEM_NEAR_LAUNCH
    return hipGetLastError();
}

}  // namespace bem
