// Weak-form entry kernels for gfx950.
//
// One 256-thread workgroup (four wavefronts) per block of work.  A block
// pairs one "fixed" item (a test or trial triangle for P0, the star of a
// test or trial vertex for P1) with up to 256 "lane" triangles, one per
// thread.  The lane triangles are gathered from the resident per-triangle
// records (one 128-byte FP32 or 192-byte FP64 record each); for P1 the
// fixed star's records are staged once per workgroup in LDS, so the waves
// read them at LDS latency instead of walking the star through dependent
// global loads.  Every lane evaluates the Green's function at all Q x Q
// pairs of quadrature points (Section 3.3: kernel values at all pairs of
// Gauss points, then weights times basis values for every pair of local
// dofs).  Test-fixed (row) and trial-fixed (column) requests share one
// kernel and launch; the side is a workgroup-uniform branch.
//
// FP32 path: positions are centroid-relative (bem_internal.hpp), 1/r is the
// hardware reciprocal square root; the Helmholtz phase k r is split into
// k |D| (centroid distance, FP64 per triangle pair, reduced to a turn) and
// k (r - |D|) from small quantities in FP32 (see Phase), and the turn in
// [-1/2, 1/2] is fed to the hardware sine and cosine, which take their
// argument in turns.  The inner sum over one
// triangle's quadrature points is a plain FP32 sum; every coarser sum (over
// the other triangle's points for P0, over triangle pairs for P1, and the
// final per-entry reduction) is compensated with TwoSum (Knuth).
// FP64 path: absolute FP64 positions, FP64 reciprocal square root and
// sincos, plain sums.
//
// P1 entries are sums over the triangles of two vertex stars (hat basis
// functions, Section 2); each lane keeps the three partial sums of its lane
// triangle (one per local vertex) over the fixed star in LDS, and after a
// workgroup barrier each entry of the chunk adds the partials that belong to
// it in a fixed order.  No atomics touch the results, so results do not
// depend on which other requests share a launch.
#include <hip/hip_ext.h>

#include "bem_internal.hpp"
#include "quad_rules.hpp"

namespace bem {

namespace {

constexpr int LSLP = BEM_LAPLACE_SLP, LDLP = BEM_LAPLACE_DLP, HSLP = BEM_HELMHOLTZ_SLP, HDLP = BEM_HELMHOLTZ_DLP;
constexpr int LHYP = BEM_LAPLACE_HYPS, HHYP = BEM_HELMHOLTZ_HYPS;
constexpr float kInv4PiF = 0.0795774715459476679f;
constexpr double kInv4Pi = 0.0795774715459476678844418816862571;

// Memory access helpers.  Relaxed atomics at device scope go to the point of
// coherence of the device, at system scope to host memory; they carry no
// cache invalidation or writeback.
template <typename T>
__device__ __forceinline__ T ld_dev(const T *p)
{
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_dev(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_sys(const T *p)
{
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
template <typename T>
__device__ __forceinline__ void st_sys(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
template <typename P>
__device__ __forceinline__ P ld_ptr_sys(P const *p)
{
    return reinterpret_cast<P>(ld_sys(reinterpret_cast<const uint64_t *>(p)));
}
template <typename P>
__device__ __forceinline__ P ld_ptr_dev(P const *p)
{
    return reinterpret_cast<P>(ld_dev(reinterpret_cast<const uint64_t *>(p)));
}
// Loads and stores through global rather than generic pointers.  The
// records, tables and outputs these kernels touch are device or
// host-coherent memory reached through generic pointers, which compile to
// flat accesses; a flat access also counts against the LDS wait counter, so
// every wait for an LDS access (or for a scalar load) would wait for it too.
// The vector types keep the accesses in the global address space (a struct
// copy would go back through a generic reference).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ldg(const float4 *p)
{
    const f32x4 v = *(const __attribute__((address_space(1))) f32x4 *)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ int4 ldg(const int4 *p)
{
    const i32x4 v = *(const __attribute__((address_space(1))) i32x4 *)p;
    return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ int32_t ldg(const int32_t *p) { return *(const __attribute__((address_space(1))) int32_t *)p; }
__device__ __forceinline__ void stg(float *p, float v) { *(__attribute__((address_space(1))) float *)p = v; }
__device__ __forceinline__ void stg(float2 *p, float2 v)
{
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    f32x2 w;
    w.x = v.x;
    w.y = v.y;
    *(__attribute__((address_space(1))) f32x2 *)p = w;
}

// Waits until this wavefront's vector memory operations, stores included
// (gfx9 counts both in vmcnt), have completed; also a compiler barrier.
__device__ __forceinline__ void wait_memory() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }


// Results, near-field flags and clock records go to host-coherent staging.
// A launched kernel stores them plainly: the end of the kernel makes them
// visible to the host.  A persistent launch (SYS = true) reports each batch
// while it keeps running, so it stores them at system scope, written through
// to host memory instead of staying in the device cache.
template <bool SYS>
__device__ __forceinline__ void put(float *p, float v)
{
    if constexpr (SYS) st_sys(reinterpret_cast<uint32_t *>(p), __float_as_uint(v));
    else stg(p, v);
}
template <bool SYS>
__device__ __forceinline__ void put(double *p, double v)
{
    if constexpr (SYS) st_sys(reinterpret_cast<uint64_t *>(p), (uint64_t)__double_as_longlong(v));
    else *p = v;
}
template <bool SYS>
__device__ __forceinline__ void put(float2 *p, float2 v)
{
    if constexpr (SYS) st_sys(reinterpret_cast<uint64_t *>(p), ((uint64_t)__float_as_uint(v.y) << 32) | __float_as_uint(v.x));
    else stg(p, v);
}
template <bool SYS>
__device__ __forceinline__ void put(double2 *p, double2 v)
{
    if constexpr (SYS) {
        st_sys(reinterpret_cast<uint64_t *>(p), (uint64_t)__double_as_longlong(v.x));
        st_sys(reinterpret_cast<uint64_t *>(p) + 1, (uint64_t)__double_as_longlong(v.y));
    } else {
        *p = v;
    }
}
template <bool SYS>
__device__ __forceinline__ void put(int32_t *p, int32_t v)
{
    if constexpr (SYS) st_sys(p, v);
    else *p = v;
}
template <bool SYS>
__device__ __forceinline__ void put(unsigned long long *p, unsigned long long v)
{
    if constexpr (SYS) st_sys(p, v);
    else *p = v;
}


template <int OP>
constexpr bool is_cplx() { return OP == HSLP || OP == HDLP || OP == HHYP; }
template <int OP>
constexpr bool is_hyp() { return OP == LHYP || OP == HHYP; }
template <int OP>
constexpr bool is_dlp() { return OP == LDLP || OP == HDLP; }

template <int Q>
constexpr int n32() { return (12 + 3 * Q + 3) / 4 * 4; }
template <int Q>
constexpr int n64() { return (4 + 3 * Q + 1) / 2 * 2; }
// A staged P1 star record on the trial side: the FP32 record with its
// quadrature offsets scaled by -2, then |o_q|^2 per point (see pair_p1_*).
template <int Q>
constexpr int nstar32() { return (n32<Q>() + Q + 3) / 4 * 4; }

// Edges from quadrature points.  The last orbit of each rule has barycentric
// coordinates (1 - 2 alpha, alpha, alpha) rotated to each vertex: point
// vpt(a) sits on the median through vertex a with x - c = (1 - 3 alpha)
// (v_a - c), so the edge opposite a, v_{a+1} - v_{a+2}, is
// (x_{vpt(a+1)} - x_{vpt(a+2)}) * vscale.
template <int Q>
constexpr int vpt(int a) { return Q - 3 + a; }
template <int Q>
constexpr double vscale() { return 1.0 / (1.0 - 3.0 * rule::Rule<Q>::l1[Q - 3]); }

// Working layout (n32<Q>() words) of a packed FP32 triangle record (see
// bem_internal.hpp): centroid parts, J and normal copied, the quadrature
// points relative to the centroid formed from the two edges as
// x_p - c = (xi_p - 1/3) e1 + (eta_p - 1/3) e2.  Every kernel expands a
// record with this one function, so a triangle's points are the same bits
// wherever it is used.
template <int Q>
__device__ __forceinline__ void expand32(const float4 &r0, const float4 &r1, const float4 &r2, const float4 &r3,
                                         float *v)
{
    v[0] = r0.x;
    v[1] = r0.y;
    v[2] = r0.z;
    v[3] = r0.w;
    v[4] = r1.x;
    v[5] = r1.y;
    v[6] = r1.z;
    v[7] = 0.0f;
    v[8] = r1.w;
    v[9] = r2.w;
    v[10] = r3.w;
    v[11] = 0.0f;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const float a = (float)(rule::Rule<Q>::l1[p] - 1.0 / 3.0), b = (float)(rule::Rule<Q>::l2[p] - 1.0 / 3.0);
        v[12 + 3 * p] = fmaf(b, r3.x, a * r2.x);
        v[13 + 3 * p] = fmaf(b, r3.y, a * r2.y);
        v[14 + 3 * p] = fmaf(b, r3.z, a * r2.z);
    }
#pragma unroll
    for (int i = 12 + 3 * Q; i < n32<Q>(); ++i) v[i] = 0.0f;
}

template <int Q>
__device__ __forceinline__ void load32(const float *__restrict__ g, int t, float *v)
{
    const float4 *p = reinterpret_cast<const float4 *>(g + (size_t)t * kGeo32Stride);
    expand32<Q>(ldg(p), ldg(p + 1), ldg(p + 2), ldg(p + 3), v);
}

template <int Q>
__device__ __forceinline__ void load64(const double *__restrict__ g, int t, double *v)
{
    const double2 *p = reinterpret_cast<const double2 *>(g + (size_t)t * kGeo64Stride);
#pragma unroll
    for (int i = 0; i < n64<Q>() / 2; ++i) {
        const double2 x = p[i];
        v[2 * i] = x.x;
        v[2 * i + 1] = x.y;
    }
}

__device__ __forceinline__ bool share_vertex(int4 a, int4 b)
{
    return a.x == b.x || a.x == b.y || a.x == b.z || a.y == b.x || a.y == b.y || a.y == b.z || a.z == b.x ||
           a.z == b.y || a.z == b.z;
}

// hi + lo += x, error-free (TwoSum).
__device__ __forceinline__ void two_sum_acc(float &hi, float &lo, float x)
{
    const float s = hi + x;
    const float bp = s - hi;
    const float ap = s - bp;
    lo += (hi - ap) + (x - bp);
    hi = s;
}

// Launch timing: with tc set, workgroup b stores the constant-rate device
// clock at its start in tc[2b] and, once all its wavefronts are done, at its
// end in tc[2b + 1] (plain stores, one slot per workgroup).
__device__ __forceinline__ void clock_start(unsigned long long *tc)
{
    if (tc && threadIdx.x == 0) put<false>(tc + 2 * blockIdx.x, (unsigned long long)wall_clock64());
}

__device__ __forceinline__ void clock_end(unsigned long long *tc)
{
    if (tc) {   // workgroup-uniform
        __syncthreads();
        if (threadIdx.x == 0) put<false>(tc + 2 * blockIdx.x + 1, (unsigned long long)wall_clock64());
    }
}

// Helmholtz phase on the FP32 path.  With D the centroid difference of the
// pair and d = o_p - o_q the offset difference of two quadrature points,
// r = |D + d| and k r = k |D| + k (r - |D|).  The first term is formed once
// per triangle pair in FP64 from the exact centroid parts and reduced to a
// turn (t0); the second from N = r^2 - |D|^2 = 2 D.d + |d|^2, a sum of small
// terms, as k (r - |D|) = k N / (r + |D|) in FP32.  The phase error is then
// about k h 1e-7 (h the element size) instead of k r 1e-7.
struct Phase {
    float t0;     // frac(k |D| / 2 pi), in [-1/2, 1/2]
    float dn;     // |D|
    float dsq;    // |D_f|^2 of the FP32 centroid difference
    float kkf;    // k / 2 pi
};

__device__ __forceinline__ Phase phase_base(const float *T, const float *S, double kk, float dcx, float dcy,
                                            float dcz)
{
    const double dx = ((double)T[0] - (double)S[0]) + ((double)T[4] - (double)S[4]);
    const double dy = ((double)T[1] - (double)S[1]) + ((double)T[5] - (double)S[5]);
    const double dz = ((double)T[2] - (double)S[2]) + ((double)T[6] - (double)S[6]);
    const double d = __builtin_sqrt(dx * dx + dy * dy + dz * dz);
    const double t = kk * d;
    Phase ph;
    ph.t0 = (float)(t - __builtin_rint(t));
    ph.dn = (float)d;
    ph.dsq = fmaf(dcx, dcx, fmaf(dcy, dcy, dcz * dcz));
    ph.kkf = (float)kk;
    return ph;
}

// Green's function factors at one point pair, FP32.  r2 = |x - y|^2; for
// Helmholtz also n = r^2 - |D|^2 (see Phase).
// SLP: accumulates w/r;   DLP: w/r^3 (the (x-y).n_y factor is applied per
// test point by the caller: the trial offsets lie in the trial plane, so
// (x_p - y_q).n_y = (x_p - c_y).n_y for every q).
template <int OP>
__device__ __forceinline__ void kern_f32(float r2, float n, float w, float kf, const Phase &ph, float &sr, float &si)
{
    const float ri = __builtin_amdgcn_rsqf(r2);
    if constexpr (OP == LSLP) {
        sr = fmaf(w, ri, sr);
    } else if constexpr (OP == LDLP) {
        sr = fmaf(w, ri * ri * ri, sr);
    } else {
        const float r = r2 * ri;
        const float delta = n * __builtin_amdgcn_rcpf(r + ph.dn);   // r - |D|
        float f = fmaf(ph.kkf, delta, ph.t0);                         // phase in turns
        f = f - __builtin_rintf(f);                                   // reduced to [-1/2, 1/2]
        const float sn = __builtin_amdgcn_sinf(f);                    // sin(2 pi f)
        const float cs = __builtin_amdgcn_cosf(f);
        if constexpr (OP == HSLP) {
            const float g = w * ri;
            sr = fmaf(g, cs, sr);
            si = fmaf(g, sn, si);
        } else {
            // exp(ikr)(1 - ikr) = (cos + kr sin) + i (sin - kr cos)
            const float g = w * ri * ri * ri;
            const float kr = kf * r;
            sr = fmaf(g, fmaf(sn, kr, cs), sr);
            si = fmaf(g, fmaf(-cs, kr, sn), si);
        }
    }
}

template <int OP>
__device__ __forceinline__ void kern_f64(double dx, double dy, double dz, const double *n, double w, double k,
                                         double &sr, double &si)
{
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double ri = rsqrt(r2);
    if constexpr (OP == LSLP) {
        sr += w * ri;
    } else if constexpr (OP == LDLP) {
        const double dn = dx * n[0] + dy * n[1] + dz * n[2];
        sr += w * dn * ri * ri * ri;
    } else {
        const double r = r2 * ri;
        double sn, cs;
        sincos(k * r, &sn, &cs);
        if constexpr (OP == HSLP) {
            const double g = w * ri;
            sr += g * cs;
            si += g * sn;
        } else {
            const double dn = dx * n[0] + dy * n[1] + dz * n[2];
            const double g = w * dn * ri * ri * ri;
            const double kr = k * r;
            sr += g * (cs + sn * kr);
            si += g * (sn - cs * kr);
        }
    }
}

// ---------------------------------------------------------------------------
// P0 pair value sum_p sum_q w_p w_q K(x_p, y_q) (without J_x J_y / 4 pi).
template <int OP, int Q>
__device__ __forceinline__ void pair_p0_f32(const float *T, const float *S, float kf, double kk, float &vr, float &vi)
{
    const float dcx = (T[0] - S[0]) + (T[4] - S[4]);
    const float dcy = (T[1] - S[1]) + (T[5] - S[5]);
    const float dcz = (T[2] - S[2]) + (T[6] - S[6]);
    float hr = 0.f, lr = 0.f, hi = 0.f, li = 0.f;
    if constexpr (is_cplx<OP>()) {
        // n = r^2 - |D|^2 = (A'_p + B_q) + (-2 a_p).o_q with a_p = D + o_p,
        // A'_p = 2 D.o_p + |o_p|^2, B_q = |o_q|^2; r^2 = n + |D|^2
        const Phase ph = phase_base(T, S, kk, dcx, dcy, dcz);
        float B[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q)
            B[q] = fmaf(S[12 + 3 * q], S[12 + 3 * q], fmaf(S[13 + 3 * q], S[13 + 3 * q], S[14 + 3 * q] * S[14 + 3 * q]));
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            const float ox = T[12 + 3 * p], oy = T[13 + 3 * p], oz = T[14 + 3 * p];
            const float ax = dcx + ox, ay = dcy + oy, az = dcz + oz;
            const float mx = -2.0f * ax, my = -2.0f * ay, mz = -2.0f * az;
            const float Ap = fmaf(2.0f * dcx + ox, ox, fmaf(2.0f * dcy + oy, oy, (2.0f * dcz + oz) * oz));
            float sr = 0.f, si = 0.f;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const float n = fmaf(mx, S[12 + 3 * q], fmaf(my, S[13 + 3 * q], fmaf(mz, S[14 + 3 * q], Ap + B[q])));
                kern_f32<OP>(n + ph.dsq, n, (float)rule::Rule<Q>::w[q], kf, ph, sr, si);
            }
            float wp = (float)rule::Rule<Q>::w[p];
            if constexpr (is_dlp<OP>()) wp *= fmaf(ax, S[8], fmaf(ay, S[9], az * S[10]));
            two_sum_acc(hr, lr, wp * sr);
            two_sum_acc(hi, li, wp * si);
        }
    } else {
        const Phase ph{};
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            const float ax = dcx + T[12 + 3 * p], ay = dcy + T[13 + 3 * p], az = dcz + T[14 + 3 * p];
            float sr = 0.f, si = 0.f;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const float dx = ax - S[12 + 3 * q], dy = ay - S[13 + 3 * q], dz = az - S[14 + 3 * q];
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                kern_f32<OP>(r2, 0.f, (float)rule::Rule<Q>::w[q], kf, ph, sr, si);
            }
            float wp = (float)rule::Rule<Q>::w[p];
            if constexpr (is_dlp<OP>()) wp *= fmaf(ax, S[8], fmaf(ay, S[9], az * S[10]));
            two_sum_acc(hr, lr, wp * sr);
        }
    }
    vr = hr + lr;
    vi = hi + li;
}

template <int OP>
constexpr int f64_unroll() { return is_cplx<OP>() ? 1 : 8; }

template <int OP, int Q>
__device__ __forceinline__ void pair_p0_f64(const double *T, const double *S, double k, double &vr, double &vi)
{
    double ar = 0.0, ai = 0.0;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        double sr = 0.0, si = 0.0;
#pragma unroll f64_unroll<OP>()
        for (int q = 0; q < Q; ++q)
            kern_f64<OP>(T[4 + 3 * p] - S[4 + 3 * q], T[5 + 3 * p] - S[5 + 3 * q], T[6 + 3 * p] - S[6 + 3 * q], S,
                         rule::Rule<Q>::w[q], k, sr, si);
        ar += rule::Rule<Q>::w[p] * sr;
        ai += rule::Rule<Q>::w[p] * si;
    }
    vr = ar;
    vi = ai;
}

// ---------------------------------------------------------------------------
// P1 pair values for the three local vertices of the lane triangle.
//
// Test side fixed with local vertex a (basis lam_a at the test points), trial
// side on the lane with all three local vertices e:
//   v_e = sum_q w_q lam_e(q) [ sum_p w_p lam_a(p) K(x_p, y_q) ].
//
// The trial offsets arrive scaled by -2 (m_q = -2 o_q, exact) with
// Bq[q] = |o_q|^2, both formed once per trial triangle.
template <int OP, int Q>
__device__ __forceinline__ void pair_p1_testfix_f32(const float *T, int a, const float *S, const float *Bq, float kf,
                                                    double kk, float *vr, float *vi)
{
    // x_p - y_q = a_p - o_q with a_p the test point relative to the trial
    // centroid; r^2 = (|a_p|^2 + |o_q|^2) + a_p . (-2 o_q) costs one add and
    // three fma per point pair.  Helmholtz: the same chain started from
    // A'_p = |a_p|^2 - |D|^2 = 2 D.o_p + |o_p|^2 gives n = r^2 - |D|^2.
    const float dcx = (T[0] - S[0]) + (T[4] - S[4]);
    const float dcy = (T[1] - S[1]) + (T[5] - S[5]);
    const float dcz = (T[2] - S[2]) + (T[6] - S[6]);
    Phase ph{};
    if constexpr (is_cplx<OP>()) ph = phase_base(T, S, kk, dcx, dcy, dcz);
    float mx[Q], my[Q], mz[Q], A[Q], wa[Q];
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const float ox = T[12 + 3 * p], oy = T[13 + 3 * p], oz = T[14 + 3 * p];
        const float ax = dcx + ox, ay = dcy + oy, az = dcz + oz;
        mx[p] = ax;
        my[p] = ay;
        mz[p] = az;
        if constexpr (is_cplx<OP>())
            A[p] = fmaf(2.0f * dcx + ox, ox, fmaf(2.0f * dcy + oy, oy, (2.0f * dcz + oz) * oz));
        else
            A[p] = fmaf(ax, ax, fmaf(ay, ay, az * az));
        const float l = (float)(a == 0 ? rule::Rule<Q>::l0[p] : (a == 1 ? rule::Rule<Q>::l1[p] : rule::Rule<Q>::l2[p]));
        wa[p] = (float)rule::Rule<Q>::w[p] * l;
        if constexpr (is_dlp<OP>()) wa[p] *= fmaf(ax, S[8], fmaf(ay, S[9], az * S[10]));
    }
#pragma unroll
    for (int e = 0; e < 3; ++e) vr[e] = vi[e] = 0.f;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const float ox = S[12 + 3 * q], oy = S[13 + 3 * q], oz = S[14 + 3 * q];
        const float B = Bq[q];
        float tr = 0.f, ti = 0.f;
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            const float v = fmaf(mx[p], ox, fmaf(my[p], oy, fmaf(mz[p], oz, A[p] + B)));
            if constexpr (is_cplx<OP>())
                kern_f32<OP>(v + ph.dsq, v, wa[p], kf, ph, tr, ti);
            else
                kern_f32<OP>(v, 0.f, wa[p], kf, ph, tr, ti);
        }
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const float wl = (float)(rule::Rule<Q>::w[q] * rule::lam<Q>(e, q));
            vr[e] = fmaf(wl, tr, vr[e]);
            if constexpr (is_cplx<OP>()) vi[e] = fmaf(wl, ti, vi[e]);
        }
    }
}

// Trial side fixed with local vertex b, test side on the lane with all three
// local vertices d:  v_d = sum_p w_p lam_d(p) [ sum_q w_q lam_b(q) K(x_p, y_q) ].
// S is a staged trial record (nstar32 layout: offsets scaled by -2, then
// |o_q|^2).
template <int OP, int Q>
__device__ __forceinline__ void pair_p1_trialfix_f32(const float *T, const float *S, int b, float kf, double kk,
                                                     float *vr, float *vi)
{
    const float dcx = (T[0] - S[0]) + (T[4] - S[4]);
    const float dcy = (T[1] - S[1]) + (T[5] - S[5]);
    const float dcz = (T[2] - S[2]) + (T[6] - S[6]);
    Phase ph{};
    if constexpr (is_cplx<OP>()) ph = phase_base(T, S, kk, dcx, dcy, dcz);
    float wb[Q], B[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const float l = (float)(b == 0 ? rule::Rule<Q>::l0[q] : (b == 1 ? rule::Rule<Q>::l1[q] : rule::Rule<Q>::l2[q]));
        wb[q] = (float)rule::Rule<Q>::w[q] * l;
        B[q] = S[n32<Q>() + q];
    }
#pragma unroll
    for (int e = 0; e < 3; ++e) vr[e] = vi[e] = 0.f;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const float ox = T[12 + 3 * p], oy = T[13 + 3 * p], oz = T[14 + 3 * p];
        const float ax = dcx + ox, ay = dcy + oy, az = dcz + oz;
        const float mx = ax, my = ay, mz = az;
        float A;
        if constexpr (is_cplx<OP>())
            A = fmaf(2.0f * dcx + ox, ox, fmaf(2.0f * dcy + oy, oy, (2.0f * dcz + oz) * oz));
        else
            A = fmaf(ax, ax, fmaf(ay, ay, az * az));
        float tr = 0.f, ti = 0.f;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const float v = fmaf(mx, S[12 + 3 * q], fmaf(my, S[13 + 3 * q], fmaf(mz, S[14 + 3 * q], A + B[q])));
            if constexpr (is_cplx<OP>())
                kern_f32<OP>(v + ph.dsq, v, wb[q], kf, ph, tr, ti);
            else
                kern_f32<OP>(v, 0.f, wb[q], kf, ph, tr, ti);
        }
        if constexpr (is_dlp<OP>()) {
            const float an = fmaf(ax, S[8], fmaf(ay, S[9], az * S[10]));
            tr *= an;
            ti *= an;
        }
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const float wl = (float)(rule::Rule<Q>::w[p] * rule::lam<Q>(e, p));
            vr[e] = fmaf(wl, tr, vr[e]);
            if constexpr (is_cplx<OP>()) vi[e] = fmaf(wl, ti, vi[e]);
        }
    }
}

// Hypersingular operator (Eq. hypsHelmholtz), P1, FP32.  On a flat triangle
// the surface curl of the hat function of local vertex e is E_e / J with
// E_e = v_{e+1} - v_{e+2} the edge opposite e, so one regular pair adds
//   (E_a . E_b) / (J_x J_y) int int g  -  k^2 (n_x . n_y) int int g lam_a lam_b
// to entry (a, b).  T is the test triangle, S the trial triangle (offsets
// scaled by -2 with |o_q|^2 in Bq: the lane's for row requests, the staged
// record's own for column requests).  TESTFIX: test vertex `fix` given, the
// three trial vertices returned; else trial vertex `fix` given, the three
// test vertices returned.  Returned values are divided by J_x J_y (the
// caller multiplies by J_x J_y / 4 pi).
template <int OP, int Q, bool TESTFIX>
__device__ __forceinline__ void pair_p1_hyp_f32(const float *T, const float *S, int fix, const float *Bq, float kf,
                                                double kk, float *vr, float *vi)
{
    const float dcx = (T[0] - S[0]) + (T[4] - S[4]);
    const float dcy = (T[1] - S[1]) + (T[5] - S[5]);
    const float dcz = (T[2] - S[2]) + (T[6] - S[6]);
    Phase ph{};
    if constexpr (is_cplx<OP>()) ph = phase_base(T, S, kk, dcx, dcy, dcz);
    // g without 1/4pi at r^2 = v (+ |D|^2 for Helmholtz, see Phase)
    auto green = [&](float v, float &gr, float &gi) {
        if constexpr (is_cplx<OP>()) {
            const float r2 = v + ph.dsq;
            const float ri = __builtin_amdgcn_rsqf(r2);
            const float r = r2 * ri;
            const float delta = v * __builtin_amdgcn_rcpf(r + ph.dn);
            float f = fmaf(ph.kkf, delta, ph.t0);
            f = f - __builtin_rintf(f);
            gr = ri * __builtin_amdgcn_cosf(f);
            gi = ri * __builtin_amdgcn_sinf(f);
        } else {
            gr = __builtin_amdgcn_rsqf(v);
            gi = 0.f;
        }
    };
    float t0r = 0.f, t0i = 0.f;                              // sum w_p w_q g
    float t1r[3] = {0.f, 0.f, 0.f}, t1i[3] = {0.f, 0.f, 0.f};   // Helmholtz: with both bases
    if constexpr (TESTFIX) {
        float ax[Q], ay[Q], az[Q], A[Q];
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            const float ox = T[12 + 3 * p], oy = T[13 + 3 * p], oz = T[14 + 3 * p];
            ax[p] = dcx + ox;
            ay[p] = dcy + oy;
            az[p] = dcz + oz;
            if constexpr (is_cplx<OP>())
                A[p] = fmaf(2.0f * dcx + ox, ox, fmaf(2.0f * dcy + oy, oy, (2.0f * dcz + oz) * oz));
            else
                A[p] = fmaf(ax[p], ax[p], fmaf(ay[p], ay[p], az[p] * az[p]));
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const float mx = S[12 + 3 * q], my = S[13 + 3 * q], mz = S[14 + 3 * q];
            const float B = Bq[q];
            float ur = 0.f, ui = 0.f, br = 0.f, bi = 0.f;
#pragma unroll
            for (int p = 0; p < Q; ++p) {
                const float v = fmaf(ax[p], mx, fmaf(ay[p], my, fmaf(az[p], mz, A[p] + B)));
                float gr, gi;
                green(v, gr, gi);
                const float w = (float)rule::Rule<Q>::w[p];
                ur = fmaf(w, gr, ur);
                if constexpr (is_cplx<OP>()) {
                    ui = fmaf(w, gi, ui);
                    const float l = (float)(fix == 0 ? rule::Rule<Q>::l0[p] : (fix == 1 ? rule::Rule<Q>::l1[p] : rule::Rule<Q>::l2[p]));
                    br = fmaf(w * l, gr, br);
                    bi = fmaf(w * l, gi, bi);
                }
            }
            const float wq = (float)rule::Rule<Q>::w[q];
            t0r = fmaf(wq, ur, t0r);
            if constexpr (is_cplx<OP>()) {
                t0i = fmaf(wq, ui, t0i);
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    const float wl = (float)(rule::Rule<Q>::w[q] * rule::lam<Q>(e, q));
                    t1r[e] = fmaf(wl, br, t1r[e]);
                    t1i[e] = fmaf(wl, bi, t1i[e]);
                }
            }
        }
    } else {
        float B[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) B[q] = S[n32<Q>() + q];
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            const float ox = T[12 + 3 * p], oy = T[13 + 3 * p], oz = T[14 + 3 * p];
            const float ax = dcx + ox, ay = dcy + oy, az = dcz + oz;
            float A;
            if constexpr (is_cplx<OP>())
                A = fmaf(2.0f * dcx + ox, ox, fmaf(2.0f * dcy + oy, oy, (2.0f * dcz + oz) * oz));
            else
                A = fmaf(ax, ax, fmaf(ay, ay, az * az));
            float ur = 0.f, ui = 0.f, br = 0.f, bi = 0.f;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const float v = fmaf(ax, S[12 + 3 * q], fmaf(ay, S[13 + 3 * q], fmaf(az, S[14 + 3 * q], A + B[q])));
                float gr, gi;
                green(v, gr, gi);
                const float w = (float)rule::Rule<Q>::w[q];
                ur = fmaf(w, gr, ur);
                if constexpr (is_cplx<OP>()) {
                    ui = fmaf(w, gi, ui);
                    const float l = (float)(fix == 0 ? rule::Rule<Q>::l0[q] : (fix == 1 ? rule::Rule<Q>::l1[q] : rule::Rule<Q>::l2[q]));
                    br = fmaf(w * l, gr, br);
                    bi = fmaf(w * l, gi, bi);
                }
            }
            const float wp = (float)rule::Rule<Q>::w[p];
            t0r = fmaf(wp, ur, t0r);
            if constexpr (is_cplx<OP>()) {
                t0i = fmaf(wp, ui, t0i);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const float wl = (float)(rule::Rule<Q>::w[p] * rule::lam<Q>(d, p));
                    t1r[d] = fmaf(wl, br, t1r[d]);
                    t1i[d] = fmaf(wl, bi, t1i[d]);
                }
            }
        }
    }
    // curl products: test edges from unscaled offsets, trial edges from the
    // -2-scaled ones
    const float vs = (float)vscale<Q>();
    float ET[3][3], ES[3][3];
#pragma unroll
    for (int e = 0; e < 3; ++e)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int i1 = 12 + 3 * vpt<Q>((e + 1) % 3) + c, i2 = 12 + 3 * vpt<Q>((e + 2) % 3) + c;
            ET[e][c] = (T[i1] - T[i2]) * vs;
            ES[e][c] = (S[i1] - S[i2]) * (-0.5f * vs);
        }
    const float inv = 1.0f / (T[3] * S[3]);
    float nn = 0.f;
    if constexpr (is_cplx<OP>()) nn = fmaf(T[8], S[8], fmaf(T[9], S[9], T[10] * S[10])) * kf * kf;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const float *et = TESTFIX ? (fix == 0 ? ET[0] : (fix == 1 ? ET[1] : ET[2])) : ET[e];
        const float *es = TESTFIX ? ES[e] : (fix == 0 ? ES[0] : (fix == 1 ? ES[1] : ES[2]));
        const float cc = fmaf(et[0], es[0], fmaf(et[1], es[1], et[2] * es[2])) * inv;
        vr[e] = cc * t0r;
        vi[e] = cc * t0i;
        if constexpr (is_cplx<OP>()) {
            vr[e] = fmaf(-nn, t1r[e], vr[e]);
            vi[e] = fmaf(-nn, t1i[e], vi[e]);
        }
    }
}

// Hypersingular operator, P1, FP64: the same terms from absolute points.
template <int OP, int Q, bool TESTFIX>
__device__ __forceinline__ void pair_p1_hyp_f64(const double *T, const double *S, int fix, double k, double *vr,
                                                double *vi)
{
    constexpr int G = is_cplx<OP>() ? HSLP : LSLP;
    double t0r = 0.0, t0i = 0.0, t1r[3] = {0.0, 0.0, 0.0}, t1i[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        double ur = 0.0, ui = 0.0, br[3] = {0.0, 0.0, 0.0}, bi[3] = {0.0, 0.0, 0.0};
#pragma unroll f64_unroll<OP>()
        for (int q = 0; q < Q; ++q) {
            double gr = 0.0, gi = 0.0;
            kern_f64<G>(T[4 + 3 * p] - S[4 + 3 * q], T[5 + 3 * p] - S[5 + 3 * q], T[6 + 3 * p] - S[6 + 3 * q], S, 1.0,
                        k, gr, gi);
            const double w = rule::Rule<Q>::w[q];
            ur += w * gr;
            ui += w * gi;
            if constexpr (is_cplx<OP>()) {
                if constexpr (TESTFIX) {
#pragma unroll
                    for (int e = 0; e < 3; ++e) {
                        br[e] += w * rule::lam<Q>(e, q) * gr;
                        bi[e] += w * rule::lam<Q>(e, q) * gi;
                    }
                } else {
                    const double l = fix == 0 ? rule::Rule<Q>::l0[q] : (fix == 1 ? rule::Rule<Q>::l1[q] : rule::Rule<Q>::l2[q]);
                    br[0] += w * l * gr;
                    bi[0] += w * l * gi;
                }
            }
        }
        const double wp = rule::Rule<Q>::w[p];
        t0r += wp * ur;
        t0i += wp * ui;
        if constexpr (is_cplx<OP>()) {
            if constexpr (TESTFIX) {
                const double l = fix == 0 ? rule::Rule<Q>::l0[p] : (fix == 1 ? rule::Rule<Q>::l1[p] : rule::Rule<Q>::l2[p]);
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    t1r[e] += wp * l * br[e];
                    t1i[e] += wp * l * bi[e];
                }
            } else {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    t1r[d] += wp * rule::lam<Q>(d, p) * br[0];
                    t1i[d] += wp * rule::lam<Q>(d, p) * bi[0];
                }
            }
        }
    }
    const double vs = vscale<Q>();
    double ET[3][3], ES[3][3];
#pragma unroll
    for (int e = 0; e < 3; ++e)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int i1 = 4 + 3 * vpt<Q>((e + 1) % 3) + c, i2 = 4 + 3 * vpt<Q>((e + 2) % 3) + c;
            ET[e][c] = (T[i1] - T[i2]) * vs;
            ES[e][c] = (S[i1] - S[i2]) * vs;
        }
    const double inv = 1.0 / (T[3] * S[3]);
    const double nn = is_cplx<OP>() ? (T[0] * S[0] + T[1] * S[1] + T[2] * S[2]) * k * k : 0.0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const double *et = TESTFIX ? (fix == 0 ? ET[0] : (fix == 1 ? ET[1] : ET[2])) : ET[e];
        const double *es = TESTFIX ? ES[e] : (fix == 0 ? ES[0] : (fix == 1 ? ES[1] : ES[2]));
        const double cc = (et[0] * es[0] + et[1] * es[1] + et[2] * es[2]) * inv;
        vr[e] = cc * t0r - nn * t1r[e];
        vi[e] = cc * t0i - nn * t1i[e];
    }
}

// FP64: general form with explicit test basis (a) and trial basis (b); the
// free side (a or b == -1) is returned for all three local vertices.
template <int OP, int Q, bool TESTFIX>
__device__ __forceinline__ void pair_p1_f64(const double *T, const double *S, int fixloc, double k, double *vr,
                                            double *vi)
{
#pragma unroll
    for (int e = 0; e < 3; ++e) vr[e] = vi[e] = 0.0;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        double sr[3] = {0.0, 0.0, 0.0}, si[3] = {0.0, 0.0, 0.0};
#pragma unroll f64_unroll<OP>()
        for (int q = 0; q < Q; ++q) {
            double kr = 0.0, ki = 0.0;
            kern_f64<OP>(T[4 + 3 * p] - S[4 + 3 * q], T[5 + 3 * p] - S[5 + 3 * q], T[6 + 3 * p] - S[6 + 3 * q], S,
                         rule::Rule<Q>::w[q], k, kr, ki);
            if constexpr (TESTFIX) {
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    sr[e] += rule::lam<Q>(e, q) * kr;
                    si[e] += rule::lam<Q>(e, q) * ki;
                }
            } else {
                const double l = fixloc == 0 ? rule::Rule<Q>::l0[q] : (fixloc == 1 ? rule::Rule<Q>::l1[q] : rule::Rule<Q>::l2[q]);
                sr[0] += l * kr;
                si[0] += l * ki;
            }
        }
        if constexpr (TESTFIX) {
            const double l = fixloc == 0 ? rule::Rule<Q>::l0[p] : (fixloc == 1 ? rule::Rule<Q>::l1[p] : rule::Rule<Q>::l2[p]);
            const double w = rule::Rule<Q>::w[p] * l;
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                vr[e] += w * sr[e];
                vi[e] += w * si[e];
            }
        } else {
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                const double w = rule::Rule<Q>::w[p] * rule::lam<Q>(e, p);
                vr[e] += w * sr[0];
                vi[e] += w * si[0];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Kernels.
//
// Workgroup B covers the lane chunk B.chunk against fixed position B.fixed
// (star entries [B.s0, B.s1), or triangle B.s0 for P0); thread t takes lane
// t of the chunk.  Threads past the end of the
// chunk repeat its first lane (valid loads) and store nothing; a wavefront
// with no valid lane skips the arithmetic.

template <int OP, int Q, bool ROWFIX, bool SYS = false>
__device__ __forceinline__ void p0_body_f32(const ReqDev &R, const EntryBlock &B)
{
    const int4 ch = B.chunk;   // first lane, lanes, first dof, dofs
    const int t = threadIdx.x;
    if ((t & ~63) >= ch.y) return;
    const bool act = t < ch.y;
    const int li = ch.x + (act ? t : 0);
    // the lane's record: gathered per lane position for resident lane sets,
    // else through its triangle index; the fixed triangle's from the mesh
    // records the block names (no request field on the way)
    const int tf = B.s0;
    const bool sep = B.lgeo && !B.lmeta;   // separated sides: no vertex-sharing pair (workgroup-uniform)
    const float *lg;
    int4 vl = make_int4(-1, -1, -1, -1);
    if (B.lgeo) {
        if (!sep) vl = ldg(B.lmeta + li);
        lg = B.lgeo + (size_t)li * kGeo32Stride;
    } else {
        const int tn = ldg(R.lane + li);
        vl = ldg(R.vtx + tn);
        lg = R.g32 + (size_t)tn * kGeo32Stride;
    }
    const int4 vf = sep ? make_int4(-2, -2, -2, -2) : ldg(B.smeta + tf);
    const float4 *fp = reinterpret_cast<const float4 *>(B.sgeo + (size_t)tf * kGeo32Stride);
    const float4 *lp = reinterpret_cast<const float4 *>(lg);
    // both records are loaded before the adjacency test (a vertex-sharing
    // pair is rare and its records are valid), and the request's fields
    // after them: the host-link round trip for those overlaps the loads
    const float4 f0 = ldg(fp), f1 = ldg(fp + 1), f2 = ldg(fp + 2), f3 = ldg(fp + 3);
    const float4 l0 = ldg(lp), l1 = ldg(lp + 1), l2 = ldg(lp + 2), l3 = ldg(lp + 3);
    asm volatile("" ::: "memory");
    const float kf = (float)R.k;
    const double kk = R.kk;
    void *const out = R.out;
    const int64_t o = (int64_t)B.fixed * R.sf + (int64_t)(ch.z + t) * R.sl;
    const bool adj = !sep && share_vertex(vf, vl);
    float vr = 0.f, vi = 0.f;
    if (!adj) {
        float F[n32<Q>()], L[n32<Q>()];
        expand32<Q>(f0, f1, f2, f3, F);
        expand32<Q>(l0, l1, l2, l3, L);
        if constexpr (ROWFIX)
            pair_p0_f32<OP, Q>(F, L, kf, kk, vr, vi);
        else
            pair_p0_f32<OP, Q>(L, F, kf, kk, vr, vi);
        const float sc = F[3] * L[3] * kInv4PiF;
        vr *= sc;
        vi *= sc;
    } else if (act && R.near_error) {
        put<SYS>(R.status, 1);
    }
    if (act) {
        if constexpr (is_cplx<OP>())
            put<SYS>(reinterpret_cast<float2 *>(out) + o, make_float2(vr, vi));
        else
            put<SYS>(reinterpret_cast<float *>(out) + o, vr);
    }
}

template <int OP, int Q>
__global__ __launch_bounds__(kBlockLanes) void k_p0_f32(const ReqDev *__restrict__ reqs,
                                                        const EntryBlock *__restrict__ blocks, int64_t nblocks,
                                                        unsigned long long *tclock)
{
    if ((int64_t)blockIdx.x >= nblocks) return;
    clock_start(tclock);
    const EntryBlock B = blocks[blockIdx.x];
    const ReqDev &R = reqs[B.req >> 1];
    if (B.req & 1)
        p0_body_f32<OP, Q, true>(R, B);
    else
        p0_body_f32<OP, Q, false>(R, B);
    clock_end(tclock);
}

template <int OP, int Q, bool ROWFIX, bool SYS = false>
__device__ __forceinline__ void p0_body_f64(const ReqDev &R, const EntryBlock &B)
{
    const int4 ch = B.chunk;
    const int t = threadIdx.x;
    if ((t & ~63) >= ch.y) return;
    const bool act = t < ch.y;
    const int li = ch.x + (act ? t : 0);
    const int tf = B.s0;
    const int tn = R.lane[li];
    const int test = ROWFIX ? tf : tn, trial = ROWFIX ? tn : tf;
    const bool sep = B.lgeo && !B.lmeta;   // separated sides: no vertex-sharing pair (workgroup-uniform)
    const bool adj = !sep && share_vertex(R.vtx[test], R.vtx[trial]);
    double vr = 0.0, vi = 0.0;
    if (!adj) {
        double T[n64<Q>()], S[n64<Q>()];
        load64<Q>(R.g64, test, T);
        load64<Q>(R.g64, trial, S);
        pair_p0_f64<OP, Q>(T, S, R.k, vr, vi);
        const double sc = T[3] * S[3] * kInv4Pi;
        vr *= sc;
        vi *= sc;
    } else if (act && R.near_error) {
        put<SYS>(R.status, 1);
    }
    if (act) {
        const int64_t o = (int64_t)B.fixed * R.sf + (int64_t)(ch.z + t) * R.sl;
        if constexpr (is_cplx<OP>())
            put<SYS>(reinterpret_cast<double2 *>(R.out) + o, make_double2(vr, vi));
        else
            put<SYS>(reinterpret_cast<double *>(R.out) + o, vr);
    }
}

template <int OP, int Q>
__global__ __launch_bounds__(kBlockLanes) void k_p0_f64(const ReqDev *__restrict__ reqs,
                                                        const EntryBlock *__restrict__ blocks, int64_t nblocks,
                                                        unsigned long long *tclock)
{
    if ((int64_t)blockIdx.x >= nblocks) return;
    clock_start(tclock);
    const EntryBlock B = blocks[blockIdx.x];
    const ReqDev &R = reqs[B.req >> 1];
    if (B.req & 1)
        p0_body_f64<OP, Q, true>(R, B);
    else
        p0_body_f64<OP, Q, false>(R, B);
    clock_end(tclock);
}

// Stages up to kStage triangles of the fixed star, starting at star entry
// sb, into LDS: W words of geometry per triangle (one word per thread), the
// vertex ids and the local vertex of the star's dof.  Every thread of the
// workgroup calls it (it synchronises).
template <typename R_T, int W>
__device__ __forceinline__ int stage_star(const ReqDev &R, const R_T *__restrict__ g, int stride, int sb, int s1,
                                          R_T (*sG)[W], int4 *sV, int *sL)
{
    const int t = threadIdx.x;
    const int ns = min(kStage, s1 - sb);
    __syncthreads();   // the previous stage has been read
    if (t < ns * W) {
        const int k = t / W, w = t - k * W;
        sG[k][w] = g[(size_t)(R.fstar[sb + k] >> 2) * stride + w];
    }
    if (t < ns) {
        const int pk = R.fstar[sb + t];
        sV[t] = R.vtx[pk >> 2];
        sL[t] = pk & 3;
    }
    __syncthreads();
    return ns;
}

// The request fields that phase 2 of a P1 block uses: segment lists, output
// positions, output address and strides.  A block reads them all at its
// start, together with its first loads: the descriptor of a direct batch
// sits in host memory, and a read at each point of use would add a host-link
// round trip to the path of every workgroup.
struct Phase2Req {
    const int32_t *seg_ptr, *seg, *lpos;
    void *out;
    int64_t sf, sl;
    __device__ __forceinline__ explicit Phase2Req(const ReqDev &R)
        : seg_ptr(R.seg_ptr), seg(R.seg), lpos(R.lpos), out(R.out), sf(R.sf), sl(R.sl)
    {
    }
};

// The first kN segments of thread t's first entry (dof ch.z + t of the
// chunk), loaded ahead of use.
struct SegPrefetch {
    static constexpr int kN = 8;
    int g0 = 0, g1 = 0;
    int seg[kN];
    __device__ __forceinline__ void fetch(const Phase2Req &P, const int4 &ch, int t)
    {
        if (t >= ch.w) return;
        const int d = ch.z + t;
        g0 = ldg(P.seg_ptr + d);
        g1 = ldg(P.seg_ptr + d + 1);
#pragma unroll
        for (int i = 0; i < kN; ++i) seg[i] = g0 + i < g1 ? ldg(P.seg + g0 + i) : 0;
    }
};

// Star records of the fixed side, staged kStage entries at a time: thread
// t < ns loads entry sb + t of block B's star table into registers
// (load_star), then, once the previous stage has been read, expands it into
// LDS (put_star).  A trial-side star (TRIAL) is staged in the nstar32 layout:
// offsets scaled by -2 (exact) and |o_q|^2 appended; a test-side star as the
// plain record.  Loading apart from storing lets the first stage's loads be
// issued together with the lane records.
struct StarRec {
    float4 r0, r1, r2, r3;
    int4 m;
};

__device__ __forceinline__ StarRec load_star(const EntryBlock &B, int e)
{
    const float4 *p = reinterpret_cast<const float4 *>(B.sgeo + (size_t)e * kGeo32Stride);
    return StarRec{ldg(p), ldg(p + 1), ldg(p + 2), ldg(p + 3), ldg(B.smeta + e)};
}

template <int Q, bool TRIAL>
__device__ __forceinline__ void put_star(const StarRec &x, int ns, float (*sG)[nstar32<Q>()], int4 *sV, int *sL)
{
    constexpr int W = n32<Q>();
    const int t = threadIdx.x;
    __syncthreads();   // the previous stage has been read
    if (t < ns) {
        float v[W];
        expand32<Q>(x.r0, x.r1, x.r2, x.r3, v);
        if constexpr (TRIAL) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                float *o = v + 12 + 3 * q;
                sG[t][W + q] = fmaf(o[0], o[0], fmaf(o[1], o[1], o[2] * o[2]));
                o[0] *= -2.0f;
                o[1] *= -2.0f;
                o[2] *= -2.0f;
            }
        }
#pragma unroll
        for (int w = 0; w < W; ++w) sG[t][w] = v[w];
        sV[t] = x.m;
        sL[t] = x.m.w;
    }
    __syncthreads();
}

// P1, FP32.  Phase 1: lane triangle against the fixed vertex star; the three
// compensated partial sums (one per local vertex of the lane triangle) go to
// LDS.  Phase 2: thread j adds, for dof j of the chunk, the partials its
// segment list names, in order, compensated, and stores the entry.
// Lane groups of a P1 chunk.  A chunk of at most 64 (128) lane triangles
// runs on all four wavefronts: the workgroup is cut into 4 (2) groups of one
// (two) wavefronts, every group holds all lanes and takes every 4th (2nd)
// triangle of the fixed star, and the groups' partial sums are combined in
// group order before the per-entry reduction.  Small requests (the rows and
// columns of small admissible blocks) then keep every wavefront busy
// instead of leaving three of four idle.  Workgroup-uniform.
struct LaneGroups {
    int size;    // threads (lanes) per group
    int count;   // groups: 4, 2 or 1
    __device__ __forceinline__ explicit LaneGroups(int lanes)
    {
        size = lanes <= 64 ? 64 : (lanes <= 128 ? 128 : kBlockLanes);
        count = kBlockLanes / size;
    }
};

// Combines the groups' compensated partials of lane t < G.size into sP[t]
// (group order).  Every thread of the workgroup calls it (it synchronises).
template <bool CPLX>
__device__ __forceinline__ void combine_groups_f32(const LaneGroups &G, int lanes, float4 (*sP)[3])
{
    if (G.count == 1) return;
    const int t = threadIdx.x;
    float4 c[3];
    const bool mine = t < G.size && t < lanes;
    if (mine) {
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            c[e] = sP[t][e];
            for (int g = 1; g < G.count; ++g) {
                const float4 v = sP[t + g * G.size][e];
                two_sum_acc(c[e].x, c[e].y, v.x);
                c[e].y += v.y;
                if constexpr (CPLX) {
                    two_sum_acc(c[e].z, c[e].w, v.z);
                    c[e].w += v.w;
                }
            }
        }
    }
    __syncthreads();   // every group's partials have been read
    if (mine) {
#pragma unroll
        for (int e = 0; e < 3; ++e) sP[t][e] = c[e];
    }
    __syncthreads();
}

template <int OP, int Q, bool ROWFIX, bool SYS = false>
__device__ __forceinline__ void p1_body_f32(const ReqDev &R, const EntryBlock &B, float (*sG)[nstar32<Q>()], int4 *sV,
                                            int *sL, float4 (*sP)[3])
{
    const int4 ch = B.chunk;   // first lane, lanes, first dof, dofs
    const int t = threadIdx.x;
    const LaneGroups G(ch.y);
    const int lt = t % G.size;             // lane of this thread
    const int grp = t / G.size;            // its group: star entries s0 + grp, s0 + grp + G.count, ...
    const bool wact = (lt & ~63) < ch.y;   // wave-uniform
    const bool act = lt < ch.y;
    const int li = ch.x + (act ? lt : 0);
    const bool sep = B.lgeo && !B.lmeta;   // separated sides: no vertex-sharing pair (workgroup-uniform)
    const float4 *lrec;
    int4 vn = make_int4(-1, -1, -1, -1);
    if (B.lgeo && ch.y > 0) {
        // lane records gathered per lane position
        if (!sep) vn = ldg(B.lmeta + li);
        lrec = reinterpret_cast<const float4 *>(B.lgeo + (size_t)li * kGeo32Stride);
    } else {
        const int tn = ch.y > 0 ? ldg(R.lane + li) : 0;   // a chunk of dofs without triangles has no lanes
        vn = ldg(R.vtx + tn);
        lrec = reinterpret_cast<const float4 *>(R.g32 + (size_t)tn * kGeo32Stride);
    }
    const float4 r0 = ldg(lrec), r1 = ldg(lrec + 1), r2 = ldg(lrec + 2), r3 = ldg(lrec + 3);
    const int s0 = B.s0, s1 = B.s1;
    StarRec first{};
    if (t < min(kStage, s1 - s0)) first = load_star(B, s0 + t);   // the first stage
    // the request's phase-2 fields are read once the lane and star loads are
    // issued: waiting for them (a host-link round trip in direct batches)
    // then overlaps those loads instead of holding them back
    asm volatile("" ::: "memory");
    const Phase2Req P(R);
    float L[n32<Q>()];
    expand32<Q>(r0, r1, r2, r3, L);
    // row requests: the lane is the trial side; its offsets scaled by -2 and
    // |o_q|^2 serve every star triangle
    float Bq[ROWFIX ? Q : 1];
    if constexpr (ROWFIX) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            float *o = L + 12 + 3 * q;
            Bq[q] = fmaf(o[0], o[0], fmaf(o[1], o[1], o[2] * o[2]));
            o[0] *= -2.0f;
            o[1] *= -2.0f;
            o[2] *= -2.0f;
        }
    }
    float hr[3] = {0.f, 0.f, 0.f}, lr[3] = {0.f, 0.f, 0.f}, hi[3] = {0.f, 0.f, 0.f}, lo[3] = {0.f, 0.f, 0.f};
    // phase 2 of this thread's first entry: its segment list, fetched while
    // phase 1 computes (after the first stage, so the stage barrier does not
    // wait for it)
    SegPrefetch pf;
    static_assert(kStage % 4 == 0, "every stage starts a new round of the lane groups");
    // this thread's pairs with the ns staged star triangles
    auto pairs = [&](int ns) {
        if (!wact) return;
        for (int s = grp; s < ns; s += G.count) {
            if (!sep && share_vertex(sV[s], vn)) {
                if (act && R.near_error) put<SYS>(R.status, 1);
                continue;
            }
            constexpr int FW = ROWFIX ? n32<Q>() : nstar32<Q>();
            float F[FW];
#pragma unroll
            for (int i = 0; i < FW; ++i) F[i] = sG[s][i];
            const int loc = sL[s];
            float vr[3], vi[3];
            if constexpr (is_hyp<OP>()) {
                if constexpr (ROWFIX)
                    pair_p1_hyp_f32<OP, Q, true>(F, L, loc, Bq, (float)R.k, R.kk, vr, vi);
                else
                    pair_p1_hyp_f32<OP, Q, false>(L, F, loc, nullptr, (float)R.k, R.kk, vr, vi);
            } else if constexpr (ROWFIX) {
                pair_p1_testfix_f32<OP, Q>(F, loc, L, Bq, (float)R.k, R.kk, vr, vi);
            } else {
                pair_p1_trialfix_f32<OP, Q>(L, F, loc, (float)R.k, R.kk, vr, vi);
            }
            const float sc = F[3] * L[3] * kInv4PiF;
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                two_sum_acc(hr[e], lr[e], sc * vr[e]);
                if constexpr (is_cplx<OP>()) two_sum_acc(hi[e], lo[e], sc * vi[e]);
            }
        }
    };
    if (s0 < s1) {
        // the first stage, loaded above (its registers are free after this)
        const int ns = min(kStage, s1 - s0);
        put_star<Q, !ROWFIX>(first, ns, sG, sV, sL);
        pf.fetch(P, ch, t);
        pairs(ns);
    }
    for (int sb = s0 + kStage; sb < s1; sb += kStage) {
        const int ns = min(kStage, s1 - sb);
        StarRec x{};
        if (t < ns) x = load_star(B, sb + t);
        put_star<Q, !ROWFIX>(x, ns, sG, sV, sL);
        pairs(ns);
    }
    if (act) {
#pragma unroll
        for (int e = 0; e < 3; ++e) sP[t][e] = make_float4(hr[e], lr[e], hi[e], lo[e]);
    }
    if (s0 == s1) pf.fetch(P, ch, t);
    __syncthreads();
    combine_groups_f32<is_cplx<OP>()>(G, ch.y, sP);
    for (int j = t; j < ch.w; j += kBlockLanes) {
        const int d = ch.z + j;
        int g0, g1;
        if (j == t) {
            g0 = pf.g0;
            g1 = pf.g1;
        } else {
            g0 = ldg(P.seg_ptr + d);
            g1 = ldg(P.seg_ptr + d + 1);
        }
        float ar = 0.f, br = 0.f, ai = 0.f, bi = 0.f;
        auto add = [&](int pk) {
            const float4 v = sP[pk >> 2][pk & 3];
            two_sum_acc(ar, br, v.x);
            br += v.y;
            if constexpr (is_cplx<OP>()) {
                two_sum_acc(ai, bi, v.z);
                bi += v.w;
            }
        };
        int g = g0;
        if (j == t) {
#pragma unroll
            for (int i = 0; i < SegPrefetch::kN; ++i)
                if (g0 + i < g1) add(pf.seg[i]);
            g = g0 + SegPrefetch::kN;
        }
        for (; g < g1; ++g) add(ldg(P.seg + g));
        const int32_t dp = P.lpos ? ldg(P.lpos + d) : d;   // lane-side output position
        const int64_t o = (int64_t)B.fixed * P.sf + (int64_t)dp * P.sl;
        if constexpr (is_cplx<OP>())
            put<SYS>(reinterpret_cast<float2 *>(P.out) + o, make_float2(ar + br, ai + bi));
        else
            put<SYS>(reinterpret_cast<float *>(P.out) + o, ar + br);
    }
}

template <int OP, int Q>
__global__ __launch_bounds__(kBlockLanes) void k_p1_f32(const ReqDev *__restrict__ reqs,
                                                        const EntryBlock *__restrict__ blocks, int64_t nblocks,
                                                        unsigned long long *tclock)
{
    __shared__ float sG[kStage][nstar32<Q>()];
    __shared__ int4 sV[kStage];
    __shared__ int sL[kStage];
    __shared__ float4 sP[kBlockLanes][3];
    if ((int64_t)blockIdx.x >= nblocks) return;
    clock_start(tclock);
    const EntryBlock B = blocks[blockIdx.x];
    const ReqDev &R = reqs[B.req >> 1];
    if (B.req & 1)
        p1_body_f32<OP, Q, true>(R, B, sG, sV, sL, sP);
    else
        p1_body_f32<OP, Q, false>(R, B, sG, sV, sL, sP);
    clock_end(tclock);
}

// P1, FP64: the same two phases with plain FP64 sums.
template <int OP, int Q, bool ROWFIX, bool SYS = false>
__device__ __forceinline__ void p1_body_f64(const ReqDev &R, const EntryBlock &B, double (*sG)[n64<Q>()], int4 *sV,
                                            int *sL, double2 (*sP)[3])
{
    const int4 ch = B.chunk;
    const int t = threadIdx.x;
    const LaneGroups G(ch.y);
    const int lt = t % G.size;
    const int grp = t / G.size;
    const bool wact = (lt & ~63) < ch.y;
    const bool act = lt < ch.y;
    const int li = ch.x + (act ? lt : 0);
    const Phase2Req P(R);
    const bool sep = B.lgeo && !B.lmeta;   // separated sides: no vertex-sharing pair (workgroup-uniform)
    const int tn = ch.y > 0 ? R.lane[li] : 0;
    const int4 vn = sep ? make_int4(-1, -1, -1, -1) : R.vtx[tn];
    double L[n64<Q>()];
    load64<Q>(R.g64, tn, L);
    double ar[3] = {0.0, 0.0, 0.0}, ai[3] = {0.0, 0.0, 0.0};
    const int s0 = B.s0, s1 = B.s1;
    SegPrefetch pf;
    for (int sb = s0; sb < s1; sb += kStage) {
        const int ns = stage_star<double, n64<Q>()>(R, R.g64, kGeo64Stride, sb, s1, sG, sV, sL);
        if (sb == s0) pf.fetch(P, ch, t);
        if (!wact) continue;
        for (int s = grp; s < ns; s += G.count) {
            if (!sep && share_vertex(sV[s], vn)) {
                if (act && R.near_error) put<SYS>(R.status, 1);
                continue;
            }
            double F[n64<Q>()];
#pragma unroll
            for (int i = 0; i < n64<Q>(); ++i) F[i] = sG[s][i];
            const int loc = sL[s];
            double vr[3], vi[3];
            if constexpr (is_hyp<OP>()) {
                if constexpr (ROWFIX)
                    pair_p1_hyp_f64<OP, Q, true>(F, L, loc, R.k, vr, vi);
                else
                    pair_p1_hyp_f64<OP, Q, false>(L, F, loc, R.k, vr, vi);
            } else if constexpr (ROWFIX) {
                pair_p1_f64<OP, Q, true>(F, L, loc, R.k, vr, vi);
            } else {
                pair_p1_f64<OP, Q, false>(L, F, loc, R.k, vr, vi);
            }
            const double sc = F[3] * L[3] * kInv4Pi;
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                ar[e] += sc * vr[e];
                ai[e] += sc * vi[e];
            }
        }
    }
    if (act) {
#pragma unroll
        for (int e = 0; e < 3; ++e) sP[t][e] = make_double2(ar[e], ai[e]);
    }
    if (s0 == s1) pf.fetch(P, ch, t);
    __syncthreads();
    if (G.count > 1) {
        // the groups' partials of lane t, added in group order
        double2 c[3];
        const bool mine = t < G.size && t < ch.y;
        if (mine) {
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                c[e] = sP[t][e];
                for (int g = 1; g < G.count; ++g) {
                    c[e].x += sP[t + g * G.size][e].x;
                    c[e].y += sP[t + g * G.size][e].y;
                }
            }
        }
        __syncthreads();
        if (mine) {
#pragma unroll
            for (int e = 0; e < 3; ++e) sP[t][e] = c[e];
        }
        __syncthreads();
    }
    for (int j = t; j < ch.w; j += kBlockLanes) {
        const int d = ch.z + j;
        int g0, g1;
        if (j == t) {
            g0 = pf.g0;
            g1 = pf.g1;
        } else {
            g0 = ldg(P.seg_ptr + d);
            g1 = ldg(P.seg_ptr + d + 1);
        }
        double xr = 0.0, xi = 0.0;
        auto add = [&](int pk) {
            const double2 v = sP[pk >> 2][pk & 3];
            xr += v.x;
            xi += v.y;
        };
        int g = g0;
        if (j == t) {
#pragma unroll
            for (int i = 0; i < SegPrefetch::kN; ++i)
                if (g0 + i < g1) add(pf.seg[i]);
            g = g0 + SegPrefetch::kN;
        }
        for (; g < g1; ++g) add(ldg(P.seg + g));
        const int32_t dp = P.lpos ? ldg(P.lpos + d) : d;   // lane-side output position
        const int64_t o = (int64_t)B.fixed * P.sf + (int64_t)dp * P.sl;
        if constexpr (is_cplx<OP>())
            put<SYS>(reinterpret_cast<double2 *>(P.out) + o, make_double2(xr, xi));
        else
            put<SYS>(reinterpret_cast<double *>(P.out) + o, xr);
    }
}

template <int OP, int Q>
__global__ __launch_bounds__(kBlockLanes) void k_p1_f64(const ReqDev *__restrict__ reqs,
                                                        const EntryBlock *__restrict__ blocks, int64_t nblocks,
                                                        unsigned long long *tclock)
{
    __shared__ double sG[kStage][n64<Q>()];
    __shared__ int4 sV[kStage];
    __shared__ int sL[kStage];
    __shared__ double2 sP[kBlockLanes][3];
    if ((int64_t)blockIdx.x >= nblocks) return;
    clock_start(tclock);
    const EntryBlock B = blocks[blockIdx.x];
    const ReqDev &R = reqs[B.req >> 1];
    if (B.req & 1)
        p1_body_f64<OP, Q, true>(R, B, sG, sV, sL, sP);
    else
        p1_body_f64<OP, Q, false>(R, B, sG, sV, sL, sP);
    clock_end(tclock);
}

// ---------------------------------------------------------------------------
// Persistent launches (layout and protocol in bem_internal.hpp).
//
// Words shared between workgroups are read and written with relaxed atomics
// at device scope, host words at system scope: those accesses go to the
// point of coherence instead of a cache that may hold an older copy, and
// they carry no cache invalidation or writeback, which would cost the
// geometry its L2 residency.  Order comes from two rules: a load that
// depends on another is issued only after that one has returned (its value
// decides whether it is issued), and a word that publishes data is stored
// only after the stores of that data have completed (wait_memory).  Results
// reach host memory through put<true>(), so a batch's completion word can follow
// its entries while the launch runs on.

__device__ __forceinline__ uint64_t claim_word(uint64_t seq, int64_t nblk)
{
    return ((seq & 0xffffull) << 48) | ((uint64_t)nblk << 32);
}

// The watching thread: copies each published ring entry to device memory,
// then makes its blocks claimable; ends on the host's stop word or after
// idle_ticks without a new entry.
__device__ void persist_watch(const PersistArgs &a)
{
    uint64_t seq = a.seq0;
    uint64_t last = wall_clock64();
    for (;;) {
        const PersistEntry *e = &a.host->ring[seq % kPersistRing];
        if (ld_sys(&e->seq1) == seq + 1) {
            PersistItem *d = &a.ctl->item[seq % kPersistRing];
            const int64_t nb = ld_sys(&e->nblk);
            st_dev(reinterpret_cast<uint64_t *>(&d->reqs), reinterpret_cast<uint64_t>(ld_ptr_sys(&e->reqs)));
            st_dev(reinterpret_cast<uint64_t *>(&d->blocks), reinterpret_cast<uint64_t>(ld_ptr_sys(&e->blocks)));
            st_dev(reinterpret_cast<uint64_t *>(&d->clock), reinterpret_cast<uint64_t>(ld_ptr_sys(&e->clock)));
            st_dev(&d->nblk, nb);
            wait_memory();   // the entry is in place before its blocks can be claimed
            st_dev(&a.ctl->claim[seq % kPersistRing][0], (unsigned long long)claim_word(seq, nb));
            ++seq;
            last = wall_clock64();
            continue;
        }
        if (ld_sys(&a.host->stop) >= a.id || (long long)(wall_clock64() - last) > a.idle_ticks) break;
        __builtin_amdgcn_s_sleep(2);
    }
    st_dev(&a.ctl->stop, 1u);
    wait_memory();
    st_sys(a.exit_word, (a.id << 40) | (seq + 1));
}

// What a workgroup works on (LDS, written by thread 0).  The records are
// kept as 64-bit words, the form they are read in, and decoded with memcpy.
struct PersistBlock {
    uint64_t R[sizeof(ReqDev) / 8];
    uint64_t B[sizeof(EntryBlock) / 8];
    unsigned long long *clock;
    int64_t idx, nblk;
    uint64_t seq;
    int go;
};
static_assert(sizeof(ReqDev) % 8 == 0 && sizeof(EntryBlock) % 8 == 0, "records are read in 8-byte words");
static_assert(offsetof(EntryBlock, req) == 0, "the request index is the block record's first word");

// Workgroup-uniform copy of a record held in LDS words (32-bit halves
// through readfirstlane, so the per-block code keeps its scalar addressing).
template <typename T>
__device__ __forceinline__ T uniform_copy(const uint64_t *src)
{
    constexpr int n = (int)(sizeof(T) / 4);
    int u[n];
#pragma unroll
    for (int i = 0; i < n; ++i) {
        const uint64_t wv = src[i / 2];
        u[i] = __builtin_amdgcn_readfirstlane((int)(uint32_t)((i & 1) ? (wv >> 32) : wv));
    }
    T out;
    __builtin_memcpy(&out, u, sizeof(T));
    return out;
}

// Claims the next block for the workgroup, oldest batch first from the
// workgroup's cursor *c (LDS, thread 0's), and reads its block record and
// request descriptor from the host-coherent staging into w.  False (for the
// whole workgroup) once the launch is ending.
__device__ bool persist_claim(const PersistArgs &a, uint64_t *cp, PersistBlock &w)
{
    if (threadIdx.x == 0) {
        int go = 1;
        uint64_t c = *cp, s = 0;
        int64_t idx = 0, nb = 0;
        for (;;) {
            unsigned long long *cw = &a.ctl->claim[c % kPersistRing][0];
            const uint64_t v = __hip_atomic_fetch_add(cw, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // the batch this claim belongs to: c + ds (ds < 0: an earlier batch
            // still holds the entry, batch c is not published yet)
            const int64_t ds = (int16_t)(uint16_t)((v >> 48) - (c & 0xffff));
            idx = (int64_t)(v & 0xffffffffull);
            nb = (int64_t)((v >> 32) & 0xffff);
            if (ds >= 0) {
                s = c + (uint64_t)ds;
                if (idx < nb) break;   // block idx of batch s
                // batch s has no unclaimed block: step on (an entry that holds a
                // later batch than c means batch c ended long ago)
                if (s == c) {
                    unsigned long long cur = c;
                    __hip_atomic_compare_exchange_strong(&a.ctl->cur, &cur, (unsigned long long)(c + 1),
                                                         __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                }
                ++c;
                const uint64_t cur = ld_dev(&a.ctl->cur);
                if (cur > c) c = cur;
                continue;
            }
            // batch c is not published yet: wait for it, for the cursor to pass
            // it or for the end of the launch (the claim word every round, the
            // other two every eighth)
            for (int round = 1;; ++round) {
                if ((uint16_t)(ld_dev(cw) >> 48) == (uint16_t)(c & 0xffff)) break;
                if ((round & 7) == 0) {
                    const uint64_t cur = ld_dev(&a.ctl->cur);
                    if (cur > c) {
                        c = cur;
                        break;
                    }
                    if (ld_dev(&a.ctl->stop) != 0u) {
                        go = 0;
                        break;
                    }
                }
                __builtin_amdgcn_s_sleep(24);
            }
            if (!go) break;
        }
        *cp = c;
        w.go = go;
        if (go) {
            const PersistItem *it = &a.ctl->item[s % kPersistRing];
            const EntryBlock *blocks = ld_ptr_dev(&it->blocks);
            const ReqDev *reqs = ld_ptr_dev(&it->reqs);
            w.clock = ld_ptr_dev(&it->clock);
            w.idx = idx;
            w.nblk = nb;
            w.seq = s;
            // the block record, then its request's descriptor: all words of a
            // record in flight together, stored to LDS once they have arrived
            constexpr int nb8 = (int)(sizeof(EntryBlock) / 8), nr8 = (int)(sizeof(ReqDev) / 8);
            const uint64_t *bs = reinterpret_cast<const uint64_t *>(blocks + idx);
            uint64_t bw[nb8], rw[nr8];
#pragma unroll
            for (int i = 0; i < nb8; ++i) bw[i] = ld_sys(bs + i);
            const int32_t req = (int32_t)(uint32_t)bw[0];   // EntryBlock::req, the record's first word
            const uint64_t *rs = reinterpret_cast<const uint64_t *>(reqs + (req >> 1));
#pragma unroll
            for (int i = 0; i < nr8; ++i) rw[i] = ld_sys(rs + i);
#pragma unroll
            for (int i = 0; i < nb8; ++i) w.B[i] = bw[i];
#pragma unroll
            for (int i = 0; i < nr8; ++i) w.R[i] = rw[i];
            if (w.clock) put<true>(w.clock + 2 * idx, (unsigned long long)wall_clock64());
        }
    }
    __syncthreads();
    return w.go != 0;
}

// After a block: once every thread's entries and status words are written,
// the block counts as finished; the last block of a batch stores the
// batch's completion word.
__device__ void persist_finish(const PersistArgs &a, PersistBlock &w)
{
    wait_memory();
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint64_t s = w.seq;
        if (w.clock) put<true>(w.clock + 2 * w.idx + 1, (unsigned long long)wall_clock64());
        wait_memory();
        unsigned int *cnt = &a.ctl->done[s % kPersistRing][0];
        const unsigned int n = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((int64_t)n + 1 == w.nblk) {
            st_dev(cnt, 0u);
            wait_memory();
            st_sys(&a.done[8 * (s % kPersistRing)], s + 1);
        }
    }
}

template <int OP, int Q>
__global__ __launch_bounds__(kBlockLanes) void kp_p0_f32(PersistArgs a)
{
    __shared__ PersistBlock w;
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) persist_watch(a);
        return;
    }
    __shared__ uint64_t cursor;   // thread 0's, kept out of registers across the block's code
    if (threadIdx.x == 0) cursor = a.seq0;
    while (persist_claim(a, &cursor, w)) {
        const EntryBlock B = uniform_copy<EntryBlock>(w.B);
        const ReqDev R = uniform_copy<ReqDev>(w.R);
        if (B.req & 1)
            p0_body_f32<OP, Q, true, true>(R, B);
        else
            p0_body_f32<OP, Q, false, true>(R, B);
        persist_finish(a, w);
    }
}

template <int OP, int Q>
__global__ __launch_bounds__(kBlockLanes) void kp_p0_f64(PersistArgs a)
{
    __shared__ PersistBlock w;
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) persist_watch(a);
        return;
    }
    __shared__ uint64_t cursor;   // thread 0's, kept out of registers across the block's code
    if (threadIdx.x == 0) cursor = a.seq0;
    while (persist_claim(a, &cursor, w)) {
        const EntryBlock B = uniform_copy<EntryBlock>(w.B);
        const ReqDev R = uniform_copy<ReqDev>(w.R);
        if (B.req & 1)
            p0_body_f64<OP, Q, true, true>(R, B);
        else
            p0_body_f64<OP, Q, false, true>(R, B);
        persist_finish(a, w);
    }
}

template <int OP, int Q>
__global__ __launch_bounds__(kBlockLanes) void kp_p1_f32(PersistArgs a)
{
    __shared__ float sG[kStage][nstar32<Q>()];
    __shared__ int4 sV[kStage];
    __shared__ int sL[kStage];
    __shared__ float4 sP[kBlockLanes][3];
    __shared__ PersistBlock w;
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) persist_watch(a);
        return;
    }
    __shared__ uint64_t cursor;   // thread 0's, kept out of registers across the block's code
    if (threadIdx.x == 0) cursor = a.seq0;
    while (persist_claim(a, &cursor, w)) {
        const EntryBlock B = uniform_copy<EntryBlock>(w.B);
        const ReqDev R = uniform_copy<ReqDev>(w.R);
        if (B.req & 1)
            p1_body_f32<OP, Q, true, true>(R, B, sG, sV, sL, sP);
        else
            p1_body_f32<OP, Q, false, true>(R, B, sG, sV, sL, sP);
        persist_finish(a, w);
    }
}

template <int OP, int Q>
__global__ __launch_bounds__(kBlockLanes) void kp_p1_f64(PersistArgs a)
{
    __shared__ double sG[kStage][n64<Q>()];
    __shared__ int4 sV[kStage];
    __shared__ int sL[kStage];
    __shared__ double2 sP[kBlockLanes][3];
    __shared__ PersistBlock w;
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) persist_watch(a);
        return;
    }
    __shared__ uint64_t cursor;   // thread 0's, kept out of registers across the block's code
    if (threadIdx.x == 0) cursor = a.seq0;
    while (persist_claim(a, &cursor, w)) {
        const EntryBlock B = uniform_copy<EntryBlock>(w.B);
        const ReqDev R = uniform_copy<ReqDev>(w.R);
        if (B.req & 1)
            p1_body_f64<OP, Q, true, true>(R, B, sG, sV, sL, sP);
        else
            p1_body_f64<OP, Q, false, true>(R, B, sG, sV, sL, sP);
        persist_finish(a, w);
    }
}

// Resets the control block of a launch that starts at sequence number seq0:
// no batch claimable (every entry tagged with an earlier batch), nothing
// finished.  One workgroup of kPersistRing threads.
__global__ void k_persist_reset(PersistCtl *ctl, uint64_t seq0)
{
    const int i = threadIdx.x;
    if (i == 0) {
        ctl->cur = seq0;
        ctl->stop = 0u;
    }
    if (i < kPersistRing) {
        ctl->claim[i][0] = claim_word(seq0 - 1, 0);
        ctl->done[i][0] = 0u;
    }
}

typedef void (*PersistKernel)(PersistArgs);

template <int OP, int Q>
PersistKernel pick_persist(int space, int prec)
{
    if constexpr (is_hyp<OP>()) {
        if (space == BEM_P0) return nullptr;
    } else {
        if (space == BEM_P0) return prec == BEM_FP32 ? kp_p0_f32<OP, Q> : kp_p0_f64<OP, Q>;
    }
    return prec == BEM_FP32 ? kp_p1_f32<OP, Q> : kp_p1_f64<OP, Q>;
}

template <int OP>
PersistKernel pick_persist_q(int space, int prec, int q)
{
    return q == 6 ? pick_persist<OP, 6>(space, prec) : pick_persist<OP, 4>(space, prec);
}

PersistKernel select_persist(const Variant &v)
{
    switch (v.op) {
    case LSLP: return pick_persist_q<LSLP>(v.space, v.prec, v.q);
    case LDLP: return pick_persist_q<LDLP>(v.space, v.prec, v.q);
    case HSLP: return pick_persist_q<HSLP>(v.space, v.prec, v.q);
    case HDLP: return pick_persist_q<HDLP>(v.space, v.prec, v.q);
    case LHYP: return pick_persist_q<LHYP>(v.space, v.prec, v.q);
    case HHYP: return pick_persist_q<HHYP>(v.space, v.prec, v.q);
    default: return nullptr;
    }
}

// ---------------------------------------------------------------------------
// Dispatch.
typedef void (*EntryKernel)(const ReqDev *, const EntryBlock *, int64_t, unsigned long long *);

template <int OP, int Q>
EntryKernel pick(int space, int prec)
{
    if constexpr (is_hyp<OP>()) {
        if (space == BEM_P0) return nullptr;   // the hypersingular operator needs P1 (host-checked)
    } else {
        if (space == BEM_P0) return prec == BEM_FP32 ? k_p0_f32<OP, Q> : k_p0_f64<OP, Q>;
    }
    return prec == BEM_FP32 ? k_p1_f32<OP, Q> : k_p1_f64<OP, Q>;
}

template <int OP>
EntryKernel pick_q(int space, int prec, int q)
{
    return q == 6 ? pick<OP, 6>(space, prec) : pick<OP, 4>(space, prec);
}

EntryKernel select_kernel(const Variant &v)
{
    switch (v.op) {
    case LSLP: return pick_q<LSLP>(v.space, v.prec, v.q);
    case LDLP: return pick_q<LDLP>(v.space, v.prec, v.q);
    case HSLP: return pick_q<HSLP>(v.space, v.prec, v.q);
    case HDLP: return pick_q<HDLP>(v.space, v.prec, v.q);
    case LHYP: return pick_q<LHYP>(v.space, v.prec, v.q);
    case HHYP: return pick_q<HHYP>(v.space, v.prec, v.q);
    default: return nullptr;
    }
}

// ---------------------------------------------------------------------------
// Pair-based P1 blocks (dense assembly).
//
// Section 3's dense assembly evaluates the kernel at all pairs of Gauss
// points of a triangle pair once, weights the values with the basis
// functions of every pair of local dofs and adds the results to the global
// entries.  The star kernels above integrate a pair once per test vertex
// (three times for a full block); here a block's pairs are integrated once
// into their 3 x 3 local matrices (k_local_*, one lane per trial triangle
// against a tile of test triangles staged in LDS), stored plane by plane
// (L[(m 9 + 3 a + b) ntrial + n] for test triangle m, trial triangle n), and
// every entry then adds its pairs' local values in a fixed order, test
// triangles of its row's star outer, trial triangles of its column's star
// inner (k_gather_dense_*; compensated in FP32).  Vertex-sharing pairs
// contribute zero (regular part).
constexpr int kLocalTile = 8;   // test triangles staged per workgroup

// 3 x 3 local matrix of a regular pair, FP32, without J_x J_y / 4 pi:
// M[a][b] = sum_q w_q lam_b(q) sum_p w_p lam_a(p) K(x_p, y_q).  T is the test
// record, S the trial record with its offsets scaled by -2 and Bq[q] =
// |o_q|^2 (see pair_p1_testfix_f32).
template <int OP, int Q>
__device__ __forceinline__ void pair_local_f32(const float *T, const float *S, const float *Bq, float kf, double kk,
                                               float (*Mr)[3], float (*Mi)[3])
{
    const float dcx = (T[0] - S[0]) + (T[4] - S[4]);
    const float dcy = (T[1] - S[1]) + (T[5] - S[5]);
    const float dcz = (T[2] - S[2]) + (T[6] - S[6]);
    Phase ph{};
    if constexpr (is_cplx<OP>()) ph = phase_base(T, S, kk, dcx, dcy, dcz);
    float mx[Q], my[Q], mz[Q], A[Q], wa[3][Q];
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const float ox = T[12 + 3 * p], oy = T[13 + 3 * p], oz = T[14 + 3 * p];
        const float ax = dcx + ox, ay = dcy + oy, az = dcz + oz;
        mx[p] = ax;
        my[p] = ay;
        mz[p] = az;
        if constexpr (is_cplx<OP>())
            A[p] = fmaf(2.0f * dcx + ox, ox, fmaf(2.0f * dcy + oy, oy, (2.0f * dcz + oz) * oz));
        else
            A[p] = fmaf(ax, ax, fmaf(ay, ay, az * az));
        float wn = (float)rule::Rule<Q>::w[p];
        if constexpr (is_dlp<OP>()) wn *= fmaf(ax, S[8], fmaf(ay, S[9], az * S[10]));
#pragma unroll
        for (int a = 0; a < 3; ++a) wa[a][p] = wn * (float)rule::lam<Q>(a, p);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) Mr[a][b] = Mi[a][b] = 0.f;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const float ox = S[12 + 3 * q], oy = S[13 + 3 * q], oz = S[14 + 3 * q];
        const float B = Bq[q];
        float ur[3] = {0.f, 0.f, 0.f}, ui[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            const float v = fmaf(mx[p], ox, fmaf(my[p], oy, fmaf(mz[p], oz, A[p] + B)));
            float kr = 0.f, ki = 0.f;
            if constexpr (is_cplx<OP>())
                kern_f32<OP>(v + ph.dsq, v, 1.0f, kf, ph, kr, ki);
            else
                kern_f32<OP>(v, 0.f, 1.0f, kf, ph, kr, ki);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                ur[a] = fmaf(wa[a][p], kr, ur[a]);
                if constexpr (is_cplx<OP>()) ui[a] = fmaf(wa[a][p], ki, ui[a]);
            }
        }
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const float wl = (float)(rule::Rule<Q>::w[q] * rule::lam<Q>(b, q));
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                Mr[a][b] = fmaf(wl, ur[a], Mr[a][b]);
                if constexpr (is_cplx<OP>()) Mi[a][b] = fmaf(wl, ui[a], Mi[a][b]);
            }
        }
    }
}

// The same in FP64 from absolute points.
template <int OP, int Q>
__device__ __forceinline__ void pair_local_f64(const double *T, const double *S, double k, double (*Mr)[3],
                                               double (*Mi)[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) Mr[a][b] = Mi[a][b] = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        double ur[3] = {0.0, 0.0, 0.0}, ui[3] = {0.0, 0.0, 0.0};
#pragma unroll f64_unroll<OP>()
        for (int p = 0; p < Q; ++p) {
            double kr = 0.0, ki = 0.0;
            kern_f64<OP>(T[4 + 3 * p] - S[4 + 3 * q], T[5 + 3 * p] - S[5 + 3 * q], T[6 + 3 * p] - S[6 + 3 * q], S,
                         rule::Rule<Q>::w[p], k, kr, ki);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                ur[a] += rule::lam<Q>(a, p) * kr;
                ui[a] += rule::lam<Q>(a, p) * ki;
            }
        }
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const double wl = rule::Rule<Q>::w[q] * rule::lam<Q>(b, q);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                Mr[a][b] += wl * ur[a];
                Mi[a][b] += wl * ui[a];
            }
        }
    }
}

// Local matrices of the pairs (test[m], trial[n]) for m in this workgroup's
// tile of kLocalTile test triangles, n = one lane per trial triangle.
template <int OP, int Q>
__global__ __launch_bounds__(kBlockLanes) void k_local_f32(const float *__restrict__ g32, const int4 *__restrict__ vtx,
                                                           const int32_t *__restrict__ test, int ntest,
                                                           const int32_t *__restrict__ trial, int ntrial,
                                                           float *__restrict__ Lr, float *__restrict__ Li, float kf,
                                                           double kk)
{
    constexpr int W = n32<Q>();
    __shared__ float sT[kLocalTile][W];
    __shared__ int4 sV[kLocalTile];
    const int t = threadIdx.x;
    const int m0 = blockIdx.y * kLocalTile;
    const int nm = min(kLocalTile, ntest - m0);
    if (t < nm) {
        float v[W];
        load32<Q>(g32, test[m0 + t], v);
#pragma unroll
        for (int w = 0; w < W; ++w) sT[t][w] = v[w];
        sV[t] = vtx[test[m0 + t]];
    }
    __syncthreads();
    const int n = blockIdx.x * kBlockLanes + t;
    if (n >= ntrial) return;   // no barrier below
    float S[W], Bq[Q];
    load32<Q>(g32, trial[n], S);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        float *o = S + 12 + 3 * q;
        Bq[q] = fmaf(o[0], o[0], fmaf(o[1], o[1], o[2] * o[2]));
        o[0] *= -2.0f;
        o[1] *= -2.0f;
        o[2] *= -2.0f;
    }
    const int4 vs = vtx[trial[n]];
    for (int i = 0; i < nm; ++i) {
        float Mr[3][3], Mi[3][3];
        if (share_vertex(sV[i], vs)) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) Mr[a][b] = Mi[a][b] = 0.f;
        } else {
            float T[W];
#pragma unroll
            for (int w = 0; w < W; ++w) T[w] = sT[i][w];
            pair_local_f32<OP, Q>(T, S, Bq, kf, kk, Mr, Mi);
            const float sc = T[3] * S[3] * kInv4PiF;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    Mr[a][b] *= sc;
                    Mi[a][b] *= sc;
                }
        }
        float *lr = Lr + (size_t)(m0 + i) * 9 * ntrial + n;
        float *li = is_cplx<OP>() ? Li + (size_t)(m0 + i) * 9 * ntrial + n : nullptr;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            lr[(size_t)k * ntrial] = Mr[k / 3][k % 3];
            if constexpr (is_cplx<OP>()) li[(size_t)k * ntrial] = Mi[k / 3][k % 3];
        }
    }
}

template <int OP, int Q>
__global__ __launch_bounds__(kBlockLanes) void k_local_f64(const double *__restrict__ g64, const int4 *__restrict__ vtx,
                                                           const int32_t *__restrict__ test, int ntest,
                                                           const int32_t *__restrict__ trial, int ntrial,
                                                           double *__restrict__ Lr, double *__restrict__ Li, double k)
{
    constexpr int W = n64<Q>();
    __shared__ double sT[kLocalTile][W];
    __shared__ int4 sV[kLocalTile];
    const int t = threadIdx.x;
    const int m0 = blockIdx.y * kLocalTile;
    const int nm = min(kLocalTile, ntest - m0);
    for (int i = t; i < nm * W; i += kBlockLanes) {
        const int kk = i / W, w = i - kk * W;
        sT[kk][w] = g64[(size_t)test[m0 + kk] * kGeo64Stride + w];
    }
    if (t < nm) sV[t] = vtx[test[m0 + t]];
    __syncthreads();
    const int n = blockIdx.x * kBlockLanes + t;
    if (n >= ntrial) return;
    double S[W];
    load64<Q>(g64, trial[n], S);
    const int4 vs = vtx[trial[n]];
    for (int i = 0; i < nm; ++i) {
        double Mr[3][3], Mi[3][3];
        if (share_vertex(sV[i], vs)) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) Mr[a][b] = Mi[a][b] = 0.0;
        } else {
            double T[W];
#pragma unroll
            for (int w = 0; w < W; ++w) T[w] = sT[i][w];
            pair_local_f64<OP, Q>(T, S, k, Mr, Mi);
            const double sc = T[3] * S[3] * kInv4Pi;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    Mr[a][b] *= sc;
                    Mi[a][b] *= sc;
                }
        }
        double *lr = Lr + (size_t)(m0 + i) * 9 * ntrial + n;
        double *li = is_cplx<OP>() ? Li + (size_t)(m0 + i) * 9 * ntrial + n : nullptr;
#pragma unroll
        for (int kk = 0; kk < 9; ++kk) {
            lr[(size_t)kk * ntrial] = Mr[kk / 3][kk % 3];
            if constexpr (is_cplx<OP>()) li[(size_t)kk * ntrial] = Mi[kk / 3][kk % 3];
        }
    }
}

// Entry (r, c) of a panel: sum over the row's star (rsrc[rptr[r] ..], packed
// test index << 2 | local vertex) and the column's star (csrc[cptr[c] ..],
// trial index << 2 | local vertex) of the local values, in that order.
template <bool CPLX>
__global__ __launch_bounds__(kBlockLanes) void k_gather_dense_f32(const float *__restrict__ Lr,
                                                                  const float *__restrict__ Li, int ntrial,
                                                                  const int32_t *__restrict__ rptr,
                                                                  const int32_t *__restrict__ rsrc,
                                                                  const int32_t *__restrict__ cptr,
                                                                  const int32_t *__restrict__ csrc, int ncols,
                                                                  void *__restrict__ out)
{
    const int c = blockIdx.x * kBlockLanes + threadIdx.x;
    const int r = blockIdx.y;
    if (c >= ncols) return;
    float hr = 0.f, lr = 0.f, hi = 0.f, li = 0.f;
    const int c0 = cptr[c], c1 = cptr[c + 1];
    for (int i = rptr[r]; i < rptr[r + 1]; ++i) {
        const int ms = rsrc[i];
        const size_t base = ((size_t)(ms >> 2) * 9 + 3 * (ms & 3)) * ntrial;
        for (int j = c0; j < c1; ++j) {
            const int ns = csrc[j];
            const size_t o = base + (size_t)(ns & 3) * ntrial + (ns >> 2);
            two_sum_acc(hr, lr, Lr[o]);
            if constexpr (CPLX) two_sum_acc(hi, li, Li[o]);
        }
    }
    const size_t e = (size_t)r * ncols + c;
    if constexpr (CPLX)
        reinterpret_cast<float2 *>(out)[e] = make_float2(hr + lr, hi + li);
    else
        reinterpret_cast<float *>(out)[e] = hr + lr;
}

template <bool CPLX>
__global__ __launch_bounds__(kBlockLanes) void k_gather_dense_f64(const double *__restrict__ Lr,
                                                                  const double *__restrict__ Li, int ntrial,
                                                                  const int32_t *__restrict__ rptr,
                                                                  const int32_t *__restrict__ rsrc,
                                                                  const int32_t *__restrict__ cptr,
                                                                  const int32_t *__restrict__ csrc, int ncols,
                                                                  void *__restrict__ out)
{
    const int c = blockIdx.x * kBlockLanes + threadIdx.x;
    const int r = blockIdx.y;
    if (c >= ncols) return;
    double sr = 0.0, si = 0.0;
    const int c0 = cptr[c], c1 = cptr[c + 1];
    for (int i = rptr[r]; i < rptr[r + 1]; ++i) {
        const int ms = rsrc[i];
        const size_t base = ((size_t)(ms >> 2) * 9 + 3 * (ms & 3)) * ntrial;
        for (int j = c0; j < c1; ++j) {
            const int ns = csrc[j];
            const size_t o = base + (size_t)(ns & 3) * ntrial + (ns >> 2);
            sr += Lr[o];
            if constexpr (CPLX) si += Li[o];
        }
    }
    const size_t e = (size_t)r * ncols + c;
    if constexpr (CPLX)
        reinterpret_cast<double2 *>(out)[e] = make_double2(sr, si);
    else
        reinterpret_cast<double *>(out)[e] = sr;
}

template <int OP>
hipError_t local_launch(bool fp32, int q, const bem_mesh &m, const int32_t *test, int ntest, const int32_t *trial,
                        int ntrial, void *Lr, void *Li, double k, hipStream_t s)
{
    const dim3 grid((unsigned)((ntrial + kBlockLanes - 1) / kBlockLanes),
                    (unsigned)((ntest + kLocalTile - 1) / kLocalTile));
    const float kf = (float)k;
    const double kk = k / (2.0 * 3.14159265358979323846);
    if (fp32) {
        if (q == 6)
            hipLaunchKernelGGL((k_local_f32<OP, 6>), grid, dim3(kBlockLanes), 0, s, m.d_g32, m.d_vtx, test, ntest,
                               trial, ntrial, (float *)Lr, (float *)Li, kf, kk);
        else
            hipLaunchKernelGGL((k_local_f32<OP, 4>), grid, dim3(kBlockLanes), 0, s, m.d_g32, m.d_vtx, test, ntest,
                               trial, ntrial, (float *)Lr, (float *)Li, kf, kk);
    } else {
        if (q == 6)
            hipLaunchKernelGGL((k_local_f64<OP, 6>), grid, dim3(kBlockLanes), 0, s, m.d_g64, m.d_vtx, test, ntest,
                               trial, ntrial, (double *)Lr, (double *)Li, k);
        else
            hipLaunchKernelGGL((k_local_f64<OP, 4>), grid, dim3(kBlockLanes), 0, s, m.d_g64, m.d_vtx, test, ntest,
                               trial, ntrial, (double *)Lr, (double *)Li, k);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_entries(const Variant &v, const ReqDev *reqs, const EntryBlock *blocks, int64_t nblocks, hipStream_t s,
                          unsigned long long *tclock, hipEvent_t start, hipEvent_t stop)
{
    if (nblocks <= 0) return hipSuccess;
    if (nblocks > INT32_MAX) return hipErrorInvalidValue;
    const EntryKernel k = select_kernel(v);
    if (!k) return hipErrorInvalidValue;
    if (start || stop)
        hipExtLaunchKernelGGL(k, dim3((unsigned)nblocks), dim3(kBlockLanes), 0, s, start, stop, 0, reqs, blocks,
                              nblocks, tclock);
    else
        hipLaunchKernelGGL(k, dim3((unsigned)nblocks), dim3(kBlockLanes), 0, s, reqs, blocks, nblocks, tclock);
    return hipGetLastError();
}

hipError_t launch_persistent(const Variant &v, const PersistArgs &a, int groups, hipStream_t s, hipEvent_t start,
                             hipEvent_t stop)
{
    const PersistKernel k = select_persist(v);
    if (!k || groups < 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_persist_reset, dim3(1), dim3(kPersistRing), 0, s, a.ctl, a.seq0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (start || stop)
        hipExtLaunchKernelGGL(k, dim3((unsigned)groups), dim3(kBlockLanes), 0, s, start, stop, 0, a);
    else
        hipLaunchKernelGGL(k, dim3((unsigned)groups), dim3(kBlockLanes), 0, s, a);
    return hipGetLastError();
}

int persistent_occupancy(const Variant &v)
{
    const PersistKernel k = select_persist(v);
    if (!k) return 0;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, kBlockLanes, 0) != hipSuccess) return 0;
    return n;
}

}  // namespace bem

namespace bem {

hipError_t launch_dense_local(int op, bool fp32, const bem_mesh &m, const int32_t *test, int ntest,
                              const int32_t *trial, int ntrial, void *Lr, void *Li, double k, hipStream_t s)
{
    if (ntest <= 0 || ntrial <= 0) return hipSuccess;
    if ((ntest + kLocalTile - 1) / kLocalTile > 65535) return hipErrorInvalidValue;
    switch (op) {
    case LSLP: return local_launch<LSLP>(fp32, m.q, m, test, ntest, trial, ntrial, Lr, Li, k, s);
    case LDLP: return local_launch<LDLP>(fp32, m.q, m, test, ntest, trial, ntrial, Lr, Li, k, s);
    case HSLP: return local_launch<HSLP>(fp32, m.q, m, test, ntest, trial, ntrial, Lr, Li, k, s);
    case HDLP: return local_launch<HDLP>(fp32, m.q, m, test, ntest, trial, ntrial, Lr, Li, k, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dense_gather(bool fp32, bool cplx, const void *Lr, const void *Li, int ntrial, const int32_t *rptr,
                               const int32_t *rsrc, int nrows, const int32_t *cptr, const int32_t *csrc, int ncols,
                               void *out, hipStream_t s)
{
    if (nrows <= 0 || ncols <= 0) return hipSuccess;
    if (nrows > 65535) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((ncols + kBlockLanes - 1) / kBlockLanes), (unsigned)nrows);
    if (fp32) {
        if (cplx)
            hipLaunchKernelGGL(k_gather_dense_f32<true>, grid, dim3(kBlockLanes), 0, s, (const float *)Lr,
                               (const float *)Li, ntrial, rptr, rsrc, cptr, csrc, ncols, out);
        else
            hipLaunchKernelGGL(k_gather_dense_f32<false>, grid, dim3(kBlockLanes), 0, s, (const float *)Lr,
                               (const float *)Li, ntrial, rptr, rsrc, cptr, csrc, ncols, out);
    } else {
        if (cplx)
            hipLaunchKernelGGL(k_gather_dense_f64<true>, grid, dim3(kBlockLanes), 0, s, (const double *)Lr,
                               (const double *)Li, ntrial, rptr, rsrc, cptr, csrc, ncols, out);
        else
            hipLaunchKernelGGL(k_gather_dense_f64<false>, grid, dim3(kBlockLanes), 0, s, (const double *)Lr,
                               (const double *)Li, ntrial, rptr, rsrc, cptr, csrc, ncols, out);
    }
    return hipGetLastError();
}

}  // namespace bem
