// Per-triangle geometry, computed once on the device when a mesh is created
// and kept resident (Section 3.2.1: normals, Jacobians and global quadrature
// points are precomputed on the device and laid out for coalesced access).
// The FP32 record keeps the two edge vectors instead of the quadrature
// points (64 bytes instead of 128); the kernels form the points from them.
#include <algorithm>
#include <cstdint>

#include "bem_internal.hpp"
#include "quad_rules.hpp"

namespace bem {

template <int Q>
__global__ __launch_bounds__(256) void k_geometry(const double *__restrict__ xyz, const int32_t *__restrict__ tri,
                                                  int64_t nt, float *__restrict__ g32, double *__restrict__ g64,
                                                  int4 *__restrict__ vtx, int32_t *__restrict__ bad)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const int i0 = tri[3 * t], i1 = tri[3 * t + 1], i2 = tri[3 * t + 2];
    const double a[3] = {xyz[3 * i0], xyz[3 * i0 + 1], xyz[3 * i0 + 2]};
    const double b[3] = {xyz[3 * i1], xyz[3 * i1 + 1], xyz[3 * i1 + 2]};
    const double c[3] = {xyz[3 * i2], xyz[3 * i2 + 1], xyz[3 * i2 + 2]};
    double e1[3], e2[3];
    for (int d = 0; d < 3; ++d) {
        e1[d] = b[d] - a[d];
        e2[d] = c[d] - a[d];
    }
    const double N[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double J = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
    if (!(J > 0.0)) atomicOr(bad, 1);
    const double inv = 1.0 / J;
    double cen[3];
    for (int d = 0; d < 3; ++d) cen[d] = ((a[d] + b[d]) + c[d]) / 3.0;

    double *r64 = g64 + t * kGeo64Stride;
    float r32[kGeo32Stride];
    for (int d = 0; d < 3; ++d) {
        r64[d] = N[d] * inv;
        const float hi = (float)cen[d];
        r32[d] = hi;
        r32[4 + d] = (float)(cen[d] - (double)hi);
        r32[8 + d] = (float)e1[d];
        r32[12 + d] = (float)e2[d];
    }
    r64[3] = J;
    r32[3] = (float)J;
    r32[7] = (float)(N[0] * inv);
    r32[11] = (float)(N[1] * inv);
    r32[15] = (float)(N[2] * inv);
    float4 *o32 = reinterpret_cast<float4 *>(g32 + t * kGeo32Stride);
    for (int i = 0; i < kGeo32Stride / 4; ++i) o32[i] = make_float4(r32[4 * i], r32[4 * i + 1], r32[4 * i + 2], r32[4 * i + 3]);
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        for (int d = 0; d < 3; ++d) r64[4 + 3 * p + d] = a[d] + rule::Rule<Q>::l1[p] * e1[d] + rule::Rule<Q>::l2[p] * e2[d];
    }
    for (int i = 4 + 3 * Q; i < kGeo64Stride; ++i) r64[i] = 0.0;
    vtx[t] = make_int4(i0, i1, i2, 0);
}

// Gathered copies of triangle records: record i of the copy is the FP32
// record (kGeo32Stride words) of triangle index[i] >> shift, and meta[i] its
// vertex ids with w = index[i] & 3 when shift == 2 (the local vertex of a
// packed star entry), else 0.  One thread per word.
__global__ __launch_bounds__(256) void k_gather(const float *__restrict__ g32, const int4 *__restrict__ vtx,
                                                const int32_t *__restrict__ index, int shift, int64_t n,
                                                float *__restrict__ geo, int4 *__restrict__ meta)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n * kGeo32Stride) return;
    const int64_t i = j / kGeo32Stride;
    const int w = (int)(j - i * kGeo32Stride);
    const int32_t pk = index[i];
    const int32_t t = pk >> shift;
    geo[j] = g32[(int64_t)t * kGeo32Stride + w];
    if (w == 0) {
        int4 v = vtx[t];
        v.w = shift == 2 ? (pk & 3) : 0;
        meta[i] = v;
    }
}

hipError_t launch_gather(const float *g32, const int4 *vtx, const int32_t *index, int shift, int64_t n, float *geo,
                         int4 *meta, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t words = n * kGeo32Stride;
    const int64_t grid = (words + 255) / 256;
    if (grid > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)grid), dim3(256), 0, s, g32, vtx, index, shift, n, geo, meta);
    return hipGetLastError();
}

// Batch staging copy: n 16-byte words from host staging (its device
// address) to the device arena, on the compute queue of the stream, so the
// entry kernels that follow need no wait on a copy engine.
__global__ __launch_bounds__(256) void k_stage_copy(const int4 *__restrict__ src, int4 *__restrict__ dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) dst[j] = src[j];
}

hipError_t launch_stage_copy(const void *src, void *dst, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    if ((bytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15)) return hipErrorInvalidValue;
    const int64_t n = (int64_t)(bytes / 16);
    const int64_t grid = std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_stage_copy, dim3((unsigned)grid), dim3(256), 0, s, static_cast<const int4 *>(src),
                       static_cast<int4 *>(dst), n);
    return hipGetLastError();
}

hipError_t launch_geometry(const double *xyz, const int32_t *tri, int64_t nt, int q, float *g32, double *g64,
                           int4 *vtx, int32_t *bad, hipStream_t s)
{
    const int block = 256;
    const unsigned grid = (unsigned)((nt + block - 1) / block);
    if (q == 6)
        hipLaunchKernelGGL(k_geometry<6>, dim3(grid), dim3(block), 0, s, xyz, tri, nt, g32, g64, vtx, bad);
    else
        hipLaunchKernelGGL(k_geometry<4>, dim3(grid), dim3(block), 0, s, xyz, tri, nt, g32, g64, vtx, bad);
    return hipGetLastError();
}

}  // namespace bem
