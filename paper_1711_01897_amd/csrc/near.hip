// Singular (vertex-sharing) P0 triangle pairs of the Laplace single and
// double layer on the device.
//
// The regular kernels integrate vertex-disjoint pairs only; Section 3.2.3
// gives identical, edge-adjacent and vertex-adjacent pairs to a separate
// singular scheme.  Here each such pair is mapped to the unit 4-cube by a
// transformation whose Jacobian vanishes where x = y to the order of the
// kernel's singularity, so the transformed integrand is smooth and a tensor
// Gauss-Legendre rule (8 points per dimension) converges fast:
//   identical:   the six-region decomposition of T x T over the reference
//                triangle {0 <= x2 <= x1 <= 1}, Jacobian xi^3 eta1^2 eta2;
//   common edge: Duffy coordinates from each triangle's third vertex
//                (distance s1, s2 from the edge, position t, t' along it),
//                then t - t' of either sign and the three pyramids of the
//                (|t - t'|, s1, s2) cube, Jacobian rho^2 (1 - |t - t'|);
//   common vertex: Duffy coordinates from the shared vertex, ordered by the
//                larger radius, Jacobian s^3 z.
// All three map polynomial integrands exactly (checked against product
// rules on the two triangles) and meet the closed-form inner integrals of
// the oracle's near-field fixture.
#include <hip/hip_runtime.h>

#include "bem_internal.hpp"

namespace bem {
namespace {

constexpr int kGL = 8;   // Gauss-Legendre points per dimension (6 points leave ~2e-7 on these pairs)
constexpr int kNearThreads = 256;

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

// Kernel without 1/4pi: single layer 1/r, double layer (x-y).n_y / r^3.
template <int OP>
__device__ __forceinline__ double green(V3 x, V3 y, V3 ny)
{
    const V3 d = sub(x, y);
    const double r2 = d.x * d.x + d.y * d.y + d.z * d.z;
    const double ri = rsqrt(r2);
    if constexpr (OP == 0) return ri;
    return (d.x * ny.x + d.y * ny.y + d.z * ny.z) * ri * ri * ri;
}

template <int OP>
__device__ double pair_value(const NearItem &it)
{
    const int t = threadIdx.x;
    const V3 ny = ld(it.ny);
    double acc = 0.0;
    constexpr int n4 = kGL * kGL * kGL * kGL;
    if (it.kind == 0) {
        const V3 V0 = ld(it.v), V1 = ld(it.v + 3), V2 = ld(it.v + 6);
        const V3 E1 = sub(V1, V0), E2 = sub(V2, V1);
        auto F = [&](double a, double b) { return add(V0, add(mul(a, E1), mul(b, E2))); };
        for (int k = t; k < n4; k += kNearThreads) {
            const int i0 = k % kGL, i1 = (k / kGL) % kGL, i2 = (k / (kGL * kGL)) % kGL, i3 = k / (kGL * kGL * kGL);
            const double xi = c_x[i0], e1 = c_x[i1], e2 = c_x[i2], e3 = c_x[i3];
            const double w = c_w[i0] * c_w[i1] * c_w[i2] * c_w[i3] * xi * xi * xi * e1 * e1 * e2;
            double s = green<OP>(F(xi, xi * (1.0 - e1 + e1 * e2)), F(xi * (1.0 - e1 * e2 * e3), xi * (1.0 - e1)), ny);
            s += green<OP>(F(xi * (1.0 - e1 * e2 * e3), xi * (1.0 - e1)), F(xi, xi * (1.0 - e1 + e1 * e2)), ny);
            s += green<OP>(F(xi, xi * e1 * (1.0 - e2 + e2 * e3)), F(xi * (1.0 - e1 * e2), xi * e1 * (1.0 - e2)), ny);
            s += green<OP>(F(xi * (1.0 - e1 * e2), xi * e1 * (1.0 - e2)), F(xi, xi * e1 * (1.0 - e2 + e2 * e3)), ny);
            s += green<OP>(F(xi * (1.0 - e1 * e2 * e3), xi * e1 * (1.0 - e2 * e3)), F(xi, xi * e1 * (1.0 - e2)), ny);
            s += green<OP>(F(xi, xi * e1 * (1.0 - e2)), F(xi * (1.0 - e1 * e2 * e3), xi * e1 * (1.0 - e2 * e3)), ny);
            acc += w * s;
        }
    } else if (it.kind == 1) {
        const V3 P = ld(it.v), Q = ld(it.v + 3), A = ld(it.v + 6), B = ld(it.v + 9);
        const V3 E = sub(Q, P);
        for (int k = t; k < 6 * n4; k += kNearThreads) {
            const int reg = k / n4, kk = k - reg * n4;
            const int i0 = kk % kGL, i1 = (kk / kGL) % kGL, i2 = (kk / (kGL * kGL)) % kGL, i3 = kk / (kGL * kGL * kGL);
            const double rho = c_x[i0], w1 = c_x[i1], w2 = c_x[i2], tau = c_x[i3];
            const int pyr = reg % 3;
            const double d = pyr == 0 ? rho : rho * w1;
            const double s1 = pyr == 1 ? rho : (pyr == 0 ? rho * w1 : rho * w2);
            const double s2 = pyr == 2 ? rho : rho * w2;
            double tx, ty;
            if (reg < 3) {
                ty = (1.0 - d) * tau;
                tx = ty + d;
            } else {
                tx = (1.0 - d) * tau;
                ty = tx + d;
            }
            const V3 ex = add(P, mul(tx, E)), ey = add(P, mul(ty, E));
            const V3 x = sub(ex, mul(s1, sub(ex, A)));
            const V3 y = sub(ey, mul(s2, sub(ey, B)));
            const double w = c_w[i0] * c_w[i1] * c_w[i2] * c_w[i3] * rho * rho * (1.0 - d) * (1.0 - s1) * (1.0 - s2);
            acc += w * green<OP>(x, y, ny);
        }
    } else {
        const V3 P = ld(it.v), A = ld(it.v + 3), B = ld(it.v + 6), C = ld(it.v + 9), D = ld(it.v + 12);
        for (int k = t; k < n4; k += kNearThreads) {
            const int i0 = k % kGL, i1 = (k / kGL) % kGL, i2 = (k / (kGL * kGL)) % kGL, i3 = k / (kGL * kGL * kGL);
            const double s = c_x[i0], z = c_x[i1], u = c_x[i2], v = c_x[i3];
            const V3 a = add(mul(1.0 - u, sub(A, P)), mul(u, sub(B, P)));
            const V3 b = add(mul(1.0 - v, sub(C, P)), mul(v, sub(D, P)));
            const double w = c_w[i0] * c_w[i1] * c_w[i2] * c_w[i3] * s * s * s * z;
            acc += w * (green<OP>(add(P, mul(s, a)), add(P, mul(s * z, b)), ny) +
                        green<OP>(add(P, mul(s * z, a)), add(P, mul(s, b)), ny));
        }
    }
    // fixed-order tree reduction over the workgroup
    __shared__ double red[kNearThreads];
    red[t] = acc;
    __syncthreads();
    for (int h = kNearThreads / 2; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    return red[0] * it.jt * it.js * kInv4PiD;
}

template <int OP, bool FP32>
__global__ __launch_bounds__(kNearThreads) void k_near_p0(const NearItem *__restrict__ items, int64_t n)
{
    if ((int64_t)blockIdx.x >= n) return;
    const NearItem &it = items[blockIdx.x];
    const double v = pair_value<OP>(it);
    if (threadIdx.x == 0) {
        if constexpr (FP32) {
            float *o = static_cast<float *>(it.out);
            *o = (float)((double)*o + v);
        } else {
            double *o = static_cast<double *>(it.out);
            *o = *o + v;
        }
    }
}

}  // namespace

hipError_t launch_near(int op, bool fp32, const NearItem *items, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (n > INT32_MAX || (op != 0 && op != 1)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)n), block(kNearThreads);
    if (op == 0) {
        if (fp32)
            hipLaunchKernelGGL((k_near_p0<0, true>), grid, block, 0, s, items, n);
        else
            hipLaunchKernelGGL((k_near_p0<0, false>), grid, block, 0, s, items, n);
    } else {
        if (fp32)
            hipLaunchKernelGGL((k_near_p0<1, true>), grid, block, 0, s, items, n);
        else
            hipLaunchKernelGGL((k_near_p0<1, false>), grid, block, 0, s, items, n);
    }
    return hipGetLastError();
}

}  // namespace bem
