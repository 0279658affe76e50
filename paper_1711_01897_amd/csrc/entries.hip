// Weak-form entry kernels for gfx950.
//
// One wavefront per tile.  A tile pairs one "fixed" item, shared by all 64
// lanes (a test or trial triangle for P0, the star of a test or trial vertex
// for P1), with up to 64 "lane" triangles, one per lane.  The fixed item's
// geometry is wave-uniform; the lane triangles are gathered from the
// resident per-triangle records (one 128-byte FP32 or 192-byte FP64 record
// each).  Every lane evaluates the Green's function at all Q x Q pairs of
// quadrature points (Section 3.3: kernel values at all pairs of Gauss
// points, then weights times basis values for every pair of local dofs).
//
// FP32 path: positions are centroid-relative (bem_internal.hpp), 1/r is the
// hardware reciprocal square root, the Helmholtz phase k r is formed and
// reduced to a turn in [-1/2, 1/2] in FP64 and fed to the hardware sine and
// cosine, which take their argument in turns.  The inner sum over one
// triangle's quadrature points is a plain FP32 sum; every coarser sum (over
// the other triangle's points for P0, over triangle pairs for P1, and the
// final per-entry reduction) is compensated with TwoSum (Knuth).
// FP64 path: absolute FP64 positions, FP64 reciprocal square root and
// sincos, plain sums.
//
// P1 entries are sums over the triangles of two vertex stars (hat basis
// functions, Section 2); each lane keeps the three partial sums of its lane
// triangle (one per local vertex) over the fixed star, and a second kernel
// adds the partials that belong to each requested entry in a fixed order.
// No atomics touch the results, so results do not depend on which other
// requests share a launch.
#include "bem_internal.hpp"
#include "quad_rules.hpp"

namespace bem {

namespace {

constexpr int LSLP = BEM_LAPLACE_SLP, LDLP = BEM_LAPLACE_DLP, HSLP = BEM_HELMHOLTZ_SLP, HDLP = BEM_HELMHOLTZ_DLP;
constexpr float kInv4PiF = 0.0795774715459476679f;
constexpr double kInv4Pi = 0.0795774715459476678844418816862571;

template <int OP>
constexpr bool is_cplx() { return OP == HSLP || OP == HDLP; }
template <int OP>
constexpr bool is_dlp() { return OP == LDLP || OP == HDLP; }

template <int Q>
constexpr int n32() { return (12 + 3 * Q + 3) / 4 * 4; }
template <int Q>
constexpr int n64() { return (4 + 3 * Q + 1) / 2 * 2; }

template <int Q>
__device__ __forceinline__ void load32(const float *__restrict__ g, int t, float *v)
{
    const float4 *p = reinterpret_cast<const float4 *>(g + (size_t)t * kGeo32Stride);
#pragma unroll
    for (int i = 0; i < n32<Q>() / 4; ++i) {
        const float4 x = p[i];
        v[4 * i] = x.x;
        v[4 * i + 1] = x.y;
        v[4 * i + 2] = x.z;
        v[4 * i + 3] = x.w;
    }
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

// Green's function factors at one point pair, FP32.  d = x - y, r2 = |d|^2.
// SLP: accumulates w/r;   DLP: w/r^3 (the (x-y).n_y factor is applied per
// test point by the caller: the trial offsets lie in the trial plane, so
// (x_p - y_q).n_y = (x_p - c_y).n_y for every q).
template <int OP>
__device__ __forceinline__ void kern_f32(float r2, float w, float kf, double kk, float &sr, float &si)
{
    const float ri = __builtin_amdgcn_rsqf(r2);
    if constexpr (OP == LSLP) {
        sr = fmaf(w, ri, sr);
    } else if constexpr (OP == LDLP) {
        sr = fmaf(w, ri * ri * ri, sr);
    } else {
        const float r = r2 * ri;
        const double t = (double)r * kk;               // phase in turns, FP64
        const float f = (float)(t - __builtin_rint(t)); // reduced to [-1/2, 1/2]
        const float sn = __builtin_amdgcn_sinf(f);      // sin(2 pi f)
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
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const float ax = dcx + T[12 + 3 * p], ay = dcy + T[13 + 3 * p], az = dcz + T[14 + 3 * p];
        float sr = 0.f, si = 0.f;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const float dx = ax - S[12 + 3 * q], dy = ay - S[13 + 3 * q], dz = az - S[14 + 3 * q];
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            kern_f32<OP>(r2, (float)rule::Rule<Q>::w[q], kf, kk, sr, si);
        }
        float wp = (float)rule::Rule<Q>::w[p];
        if constexpr (is_dlp<OP>()) wp *= fmaf(ax, S[8], fmaf(ay, S[9], az * S[10]));
        two_sum_acc(hr, lr, wp * sr);
        if constexpr (is_cplx<OP>()) two_sum_acc(hi, li, wp * si);
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
template <int OP, int Q>
__device__ __forceinline__ void pair_p1_testfix_f32(const float *T, int a, const float *S, float kf, double kk,
                                                    float *vr, float *vi)
{
    // x_p - y_q = a_p - o_q with a_p the test point relative to the trial
    // centroid; r^2 = (|a_p|^2 + |o_q|^2) + (-2 a_p) . o_q costs one add and
    // three fma per point pair.
    const float dcx = (T[0] - S[0]) + (T[4] - S[4]);
    const float dcy = (T[1] - S[1]) + (T[5] - S[5]);
    const float dcz = (T[2] - S[2]) + (T[6] - S[6]);
    float mx[Q], my[Q], mz[Q], A[Q], wa[Q];
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const float ax = dcx + T[12 + 3 * p], ay = dcy + T[13 + 3 * p], az = dcz + T[14 + 3 * p];
        mx[p] = -2.0f * ax;
        my[p] = -2.0f * ay;
        mz[p] = -2.0f * az;
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
        const float B = fmaf(ox, ox, fmaf(oy, oy, oz * oz));
        float tr = 0.f, ti = 0.f;
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            const float r2 = fmaf(mx[p], ox, fmaf(my[p], oy, fmaf(mz[p], oz, A[p] + B)));
            kern_f32<OP>(r2, wa[p], kf, kk, tr, ti);
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
template <int OP, int Q>
__device__ __forceinline__ void pair_p1_trialfix_f32(const float *T, const float *S, int b, float kf, double kk,
                                                     float *vr, float *vi)
{
    const float dcx = (T[0] - S[0]) + (T[4] - S[4]);
    const float dcy = (T[1] - S[1]) + (T[5] - S[5]);
    const float dcz = (T[2] - S[2]) + (T[6] - S[6]);
    float wb[Q], B[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const float l = (float)(b == 0 ? rule::Rule<Q>::l0[q] : (b == 1 ? rule::Rule<Q>::l1[q] : rule::Rule<Q>::l2[q]));
        wb[q] = (float)rule::Rule<Q>::w[q] * l;
        B[q] = fmaf(S[12 + 3 * q], S[12 + 3 * q], fmaf(S[13 + 3 * q], S[13 + 3 * q], S[14 + 3 * q] * S[14 + 3 * q]));
    }
#pragma unroll
    for (int e = 0; e < 3; ++e) vr[e] = vi[e] = 0.f;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const float ax = dcx + T[12 + 3 * p], ay = dcy + T[13 + 3 * p], az = dcz + T[14 + 3 * p];
        const float mx = -2.0f * ax, my = -2.0f * ay, mz = -2.0f * az;
        const float A = fmaf(ax, ax, fmaf(ay, ay, az * az));
        float tr = 0.f, ti = 0.f;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const float r2 = fmaf(mx, S[12 + 3 * q], fmaf(my, S[13 + 3 * q], fmaf(mz, S[14 + 3 * q], A + B[q])));
            kern_f32<OP>(r2, wb[q], kf, kk, tr, ti);
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
template <int OP, int Q, bool ROWFIX>
__global__ __launch_bounds__(256) void k_p0_f32(const ReqDev *__restrict__ reqs, const Tile *__restrict__ tiles,
                                                int64_t ntiles)
{
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    const ReqDev &R = reqs[tl.req];
    const bool act = lane < tl.nlanes;
    const int li = tl.lane0 + (act ? lane : 0);
    const int tf = R.fix[tl.fixed];
    const int tn = R.lane[li];
    const int test = ROWFIX ? tf : tn, trial = ROWFIX ? tn : tf;
    const bool adj = share_vertex(R.vtx[test], R.vtx[trial]);
    float vr = 0.f, vi = 0.f;
    if (!adj) {
        float T[n32<Q>()], S[n32<Q>()];
        load32<Q>(R.g32, test, T);
        load32<Q>(R.g32, trial, S);
        pair_p0_f32<OP, Q>(T, S, (float)R.k, R.kk, vr, vi);
        const float sc = T[3] * S[3] * kInv4PiF;
        vr *= sc;
        vi *= sc;
    } else if (act && R.near_error) {
        atomicOr(R.status, 1);
    }
    if (act) {
        const int64_t o = (int64_t)tl.fixed * R.sf + (int64_t)li * R.sl;
        if constexpr (is_cplx<OP>())
            reinterpret_cast<float2 *>(R.out)[o] = make_float2(vr, vi);
        else
            reinterpret_cast<float *>(R.out)[o] = vr;
    }
}

template <int OP, int Q, bool ROWFIX>
__global__ __launch_bounds__(256) void k_p0_f64(const ReqDev *__restrict__ reqs, const Tile *__restrict__ tiles,
                                                int64_t ntiles)
{
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    const ReqDev &R = reqs[tl.req];
    const bool act = lane < tl.nlanes;
    const int li = tl.lane0 + (act ? lane : 0);
    const int tf = R.fix[tl.fixed];
    const int tn = R.lane[li];
    const int test = ROWFIX ? tf : tn, trial = ROWFIX ? tn : tf;
    const bool adj = share_vertex(R.vtx[test], R.vtx[trial]);
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
        atomicOr(R.status, 1);
    }
    if (act) {
        const int64_t o = (int64_t)tl.fixed * R.sf + (int64_t)li * R.sl;
        if constexpr (is_cplx<OP>())
            reinterpret_cast<double2 *>(R.out)[o] = make_double2(vr, vi);
        else
            reinterpret_cast<double *>(R.out)[o] = vr;
    }
}

// Per-entry reduction of P1 partials in the fixed order of the segment list
// (ascending lane triangle), compensated in FP32.
template <bool CPLX>
__device__ __forceinline__ void reduce_entry_f32(const ReqDev &R, int64_t idx)
{
    const int64_t r = idx / R.ncols, c = idx - r * R.ncols;
    const int64_t f = R.rowfix ? r : c;
    const int64_t op = R.rowfix ? c : r;
    const int s0 = R.seg_ptr[op], s1 = R.seg_ptr[op + 1];
    float hr = 0.f, lr = 0.f, hi = 0.f, li = 0.f;
    for (int s = s0; s < s1; ++s) {
        const int pk = R.seg[s];
        const int64_t at = (f * R.nlane + (pk >> 2)) * 3 + (pk & 3);
        if constexpr (CPLX) {
            const float4 v = reinterpret_cast<const float4 *>(R.part)[at];
            two_sum_acc(hr, lr, v.x);
            lr += v.y;
            two_sum_acc(hi, li, v.z);
            li += v.w;
        } else {
            const float2 v = reinterpret_cast<const float2 *>(R.part)[at];
            two_sum_acc(hr, lr, v.x);
            lr += v.y;
        }
    }
    if constexpr (CPLX)
        reinterpret_cast<float2 *>(R.out)[idx] = make_float2(hr + lr, hi + li);
    else
        reinterpret_cast<float *>(R.out)[idx] = hr + lr;
}

template <bool CPLX>
__global__ __launch_bounds__(kReduceBlock) void k_p1_reduce_f32(const ReqDev *__restrict__ reqs,
                                                               const RTile *__restrict__ tiles, int64_t ntiles)
{
    const RTile tl = tiles[blockIdx.x];
    if ((int)threadIdx.x >= tl.count) return;
    reduce_entry_f32<CPLX>(reqs[tl.req], tl.e0 + threadIdx.x);
}

template <bool CPLX>
__device__ __forceinline__ void reduce_entry_f64(const ReqDev &R, int64_t idx)
{
    const int64_t r = idx / R.ncols, c = idx - r * R.ncols;
    const int64_t f = R.rowfix ? r : c;
    const int64_t op = R.rowfix ? c : r;
    const int s0 = R.seg_ptr[op], s1 = R.seg_ptr[op + 1];
    double ar = 0.0, ai = 0.0;
    for (int s = s0; s < s1; ++s) {
        const int pk = R.seg[s];
        const int64_t at = (f * R.nlane + (pk >> 2)) * 3 + (pk & 3);
        if constexpr (CPLX) {
            const double2 v = reinterpret_cast<const double2 *>(R.part)[at];
            ar += v.x;
            ai += v.y;
        } else {
            ar += reinterpret_cast<const double *>(R.part)[at];
        }
    }
    if constexpr (CPLX)
        reinterpret_cast<double2 *>(R.out)[idx] = make_double2(ar, ai);
    else
        reinterpret_cast<double *>(R.out)[idx] = ar;
}

template <bool CPLX>
__global__ __launch_bounds__(kReduceBlock) void k_p1_reduce_f64(const ReqDev *__restrict__ reqs,
                                                               const RTile *__restrict__ tiles, int64_t ntiles)
{
    const RTile tl = tiles[blockIdx.x];
    if ((int)threadIdx.x >= tl.count) return;
    reduce_entry_f64<CPLX>(reqs[tl.req], tl.e0 + threadIdx.x);
}

// Fused reduction of small P1 requests: after its partials are stored, each
// tile counts itself in with a device-scope release fence and an atomic;
// the tile that arrives last (acquire fence) reduces every entry of the
// request, 64 entries at a time.
template <bool F32, bool CPLX>
__device__ __forceinline__ void fused_reduce_tail(const ReqDev &R, int lane)
{
    if (!R.counter) return;
    __threadfence();
    int last = 0;
    if (lane == 0) last = atomicAdd(R.counter, 1) == R.ntiles_req - 1 ? 1 : 0;
    last = __builtin_amdgcn_readfirstlane(last);
    if (!last) return;
    __threadfence();
    const int64_t n = (int64_t)R.nrows * R.ncols;
    for (int64_t idx = lane; idx < n; idx += 64) {
        if constexpr (F32)
            reduce_entry_f32<CPLX>(R, idx);
        else
            reduce_entry_f64<CPLX>(R, idx);
    }
}

// P1: lane triangle against the fixed vertex star; writes the three
// compensated partial sums (one per local vertex of the lane triangle).
template <int OP, int Q, bool ROWFIX>
__global__ __launch_bounds__(256) void k_p1_f32(const ReqDev *__restrict__ reqs, const Tile *__restrict__ tiles,
                                                int64_t ntiles)
{
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    const ReqDev &R = reqs[tl.req];
    const bool act = lane < tl.nlanes;
    const int li = tl.lane0 + (act ? lane : 0);
    const int tn = R.lane[li];
    const int4 vn = R.vtx[tn];
    float L[n32<Q>()];
    load32<Q>(R.g32, tn, L);
    float hr[3] = {0.f, 0.f, 0.f}, lr[3] = {0.f, 0.f, 0.f}, hi[3] = {0.f, 0.f, 0.f}, lo[3] = {0.f, 0.f, 0.f};
    const int s0 = R.fix[tl.fixed], s1 = R.fix[tl.fixed + 1];
    for (int s = s0; s < s1; ++s) {
        const int pk = R.fstar[s];
        const int tf = pk >> 2, loc = pk & 3;
        if (share_vertex(R.vtx[tf], vn)) {
            if (act && R.near_error) atomicOr(R.status, 1);
            continue;
        }
        float F[n32<Q>()];
        load32<Q>(R.g32, tf, F);
        float vr[3], vi[3];
        if constexpr (ROWFIX)
            pair_p1_testfix_f32<OP, Q>(F, loc, L, (float)R.k, R.kk, vr, vi);
        else
            pair_p1_trialfix_f32<OP, Q>(L, F, loc, (float)R.k, R.kk, vr, vi);
        const float sc = F[3] * L[3] * kInv4PiF;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            two_sum_acc(hr[e], lr[e], sc * vr[e]);
            if constexpr (is_cplx<OP>()) two_sum_acc(hi[e], lo[e], sc * vi[e]);
        }
    }
    if (act) {
        const int64_t base = ((int64_t)tl.fixed * R.nlane + li) * 3;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            if constexpr (is_cplx<OP>())
                reinterpret_cast<float4 *>(R.part)[base + e] = make_float4(hr[e], lr[e], hi[e], lo[e]);
            else
                reinterpret_cast<float2 *>(R.part)[base + e] = make_float2(hr[e], lr[e]);
        }
    }
    fused_reduce_tail<true, is_cplx<OP>()>(R, lane);
}

template <int OP, int Q, bool ROWFIX>
__global__ __launch_bounds__(256) void k_p1_f64(const ReqDev *__restrict__ reqs, const Tile *__restrict__ tiles,
                                                int64_t ntiles)
{
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    const ReqDev &R = reqs[tl.req];
    const bool act = lane < tl.nlanes;
    const int li = tl.lane0 + (act ? lane : 0);
    const int tn = R.lane[li];
    const int4 vn = R.vtx[tn];
    double L[n64<Q>()];
    load64<Q>(R.g64, tn, L);
    double ar[3] = {0.0, 0.0, 0.0}, ai[3] = {0.0, 0.0, 0.0};
    const int s0 = R.fix[tl.fixed], s1 = R.fix[tl.fixed + 1];
    for (int s = s0; s < s1; ++s) {
        const int pk = R.fstar[s];
        const int tf = pk >> 2, loc = pk & 3;
        if (share_vertex(R.vtx[tf], vn)) {
            if (act && R.near_error) atomicOr(R.status, 1);
            continue;
        }
        double F[n64<Q>()];
        load64<Q>(R.g64, tf, F);
        double vr[3], vi[3];
        if constexpr (ROWFIX)
            pair_p1_f64<OP, Q, true>(F, L, loc, R.k, vr, vi);
        else
            pair_p1_f64<OP, Q, false>(L, F, loc, R.k, vr, vi);
        const double sc = F[3] * L[3] * kInv4Pi;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            ar[e] += sc * vr[e];
            ai[e] += sc * vi[e];
        }
    }
    if (act) {
        const int64_t base = ((int64_t)tl.fixed * R.nlane + li) * 3;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            if constexpr (is_cplx<OP>())
                reinterpret_cast<double2 *>(R.part)[base + e] = make_double2(ar[e], ai[e]);
            else
                reinterpret_cast<double *>(R.part)[base + e] = ar[e];
        }
    }
    fused_reduce_tail<false, is_cplx<OP>()>(R, lane);
}

// ---------------------------------------------------------------------------
// Tile tables.  Thread t finds its request by binary search in the group's
// exclusive prefix of per-request tile counts and writes the tile record.
__global__ __launch_bounds__(256) void k_build_tiles(const ReqDev *__restrict__ reqs, const int32_t *__restrict__ greq,
                                                     const int64_t *__restrict__ gpre, int ng, int64_t ntiles,
                                                     Tile *__restrict__ tiles)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    int lo = 0, hi = ng;  // gpre[lo] <= t < gpre[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (gpre[mid] <= t)
            lo = mid;
        else
            hi = mid;
    }
    const int r = greq[lo];
    const ReqDev &R = reqs[r];
    const int64_t u = t - gpre[lo];
    const int ntl = (R.nlane + kTileLanes - 1) / kTileLanes;
    const int f = (int)(u / ntl);
    const int c = (int)(u - (int64_t)f * ntl);
    Tile tl;
    tl.req = r;
    tl.fixed = f;
    tl.lane0 = c * kTileLanes;
    tl.nlanes = min(kTileLanes, R.nlane - c * kTileLanes);
    tiles[t] = tl;
}

__global__ __launch_bounds__(256) void k_build_rtiles(const ReqDev *__restrict__ reqs,
                                                      const int32_t *__restrict__ greq,
                                                      const int64_t *__restrict__ gpre, int ng, int64_t ntiles,
                                                      RTile *__restrict__ tiles)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    int lo = 0, hi = ng;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (gpre[mid] <= t)
            lo = mid;
        else
            hi = mid;
    }
    const int r = greq[lo];
    const ReqDev &R = reqs[r];
    const int64_t u = t - gpre[lo];
    const int64_t n = (int64_t)R.nrows * R.ncols;
    RTile tl;
    tl.req = r;
    tl.e0 = u * kReduceBlock;
    tl.count = (int32_t)min((int64_t)kReduceBlock, n - tl.e0);
    tiles[t] = tl;
}

__global__ __launch_bounds__(256) void k_build_all(const ReqDev *__restrict__ reqs,
                                                   const GroupDesc *__restrict__ groups, int ngroups, int64_t total)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    int glo = 0, ghi = ngroups;  // groups[glo].tile0 <= t < groups[ghi].tile0
    while (ghi - glo > 1) {
        const int mid = (glo + ghi) >> 1;
        if (groups[mid].tile0 <= t)
            glo = mid;
        else
            ghi = mid;
    }
    const GroupDesc &G = groups[glo];
    const int64_t tt = t - G.tile0;
    int lo = 0, hi = G.ng;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (G.gpre[mid] <= tt)
            lo = mid;
        else
            hi = mid;
    }
    const int r = G.greq[lo];
    const ReqDev &R = reqs[r];
    const int64_t u = tt - G.gpre[lo];
    if (G.kind == 0) {
        const int ntl = (R.nlane + kTileLanes - 1) / kTileLanes;
        const int f = (int)(u / ntl);
        const int c = (int)(u - (int64_t)f * ntl);
        Tile tl;
        tl.req = r;
        tl.fixed = f;
        tl.lane0 = c * kTileLanes;
        tl.nlanes = min(kTileLanes, R.nlane - c * kTileLanes);
        reinterpret_cast<Tile *>(G.tiles)[tt] = tl;
    } else {
        const int64_t n = (int64_t)R.nrows * R.ncols;
        RTile tl;
        tl.req = r;
        tl.e0 = u * kReduceBlock;
        tl.count = (int32_t)min((int64_t)kReduceBlock, n - tl.e0);
        reinterpret_cast<RTile *>(G.tiles)[tt] = tl;
    }
}

// ---------------------------------------------------------------------------
// Dispatch.
typedef void (*EntryKernel)(const ReqDev *, const Tile *, int64_t);

template <int OP, int Q, bool RF>
EntryKernel pick(int space, int prec)
{
    if (space == BEM_P0) return prec == BEM_FP32 ? k_p0_f32<OP, Q, RF> : k_p0_f64<OP, Q, RF>;
    return prec == BEM_FP32 ? k_p1_f32<OP, Q, RF> : k_p1_f64<OP, Q, RF>;
}

template <int OP, int Q>
EntryKernel pick_rf(int space, int prec, int rowfix)
{
    return rowfix ? pick<OP, Q, true>(space, prec) : pick<OP, Q, false>(space, prec);
}

template <int OP>
EntryKernel pick_q(int space, int prec, int q, int rowfix)
{
    return q == 6 ? pick_rf<OP, 6>(space, prec, rowfix) : pick_rf<OP, 4>(space, prec, rowfix);
}

EntryKernel select_kernel(const Variant &v)
{
    switch (v.op) {
    case LSLP: return pick_q<LSLP>(v.space, v.prec, v.q, v.rowfix);
    case LDLP: return pick_q<LDLP>(v.space, v.prec, v.q, v.rowfix);
    case HSLP: return pick_q<HSLP>(v.space, v.prec, v.q, v.rowfix);
    default: return pick_q<HDLP>(v.space, v.prec, v.q, v.rowfix);
    }
}

}  // namespace

hipError_t launch_build_tiles(const ReqDev *reqs, const int32_t *greq, const int64_t *gpre, int ng, int64_t ntiles,
                              Tile *tiles, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((ntiles + 255) / 256);
    hipLaunchKernelGGL(k_build_tiles, dim3(grid), dim3(256), 0, s, reqs, greq, gpre, ng, ntiles, tiles);
    return hipGetLastError();
}

hipError_t launch_build_all(const ReqDev *reqs, const GroupDesc *groups, int ngroups, int64_t total, hipStream_t s)
{
    if (total <= 0 || ngroups <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(k_build_all, dim3(grid), dim3(256), 0, s, reqs, groups, ngroups, total);
    return hipGetLastError();
}

hipError_t launch_build_rtiles(const ReqDev *reqs, const int32_t *greq, const int64_t *gpre, int ng, int64_t ntiles,
                               RTile *tiles, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((ntiles + 255) / 256);
    hipLaunchKernelGGL(k_build_rtiles, dim3(grid), dim3(256), 0, s, reqs, greq, gpre, ng, ntiles, tiles);
    return hipGetLastError();
}

hipError_t launch_entries(const Variant &v, const ReqDev *reqs, const Tile *tiles, int64_t ntiles, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((ntiles + kWavesPerBlock - 1) / kWavesPerBlock);
    hipLaunchKernelGGL(select_kernel(v), dim3(grid), dim3(64 * kWavesPerBlock), 0, s, reqs, tiles, ntiles);
    return hipGetLastError();
}

hipError_t launch_p1_reduce(int prec, bool cplx, const ReqDev *reqs, const RTile *tiles, int64_t ntiles,
                            hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    if (prec == BEM_FP32) {
        if (cplx)
            hipLaunchKernelGGL(k_p1_reduce_f32<true>, dim3(ntiles), dim3(kReduceBlock), 0, s, reqs, tiles, ntiles);
        else
            hipLaunchKernelGGL(k_p1_reduce_f32<false>, dim3(ntiles), dim3(kReduceBlock), 0, s, reqs, tiles, ntiles);
    } else {
        if (cplx)
            hipLaunchKernelGGL(k_p1_reduce_f64<true>, dim3(ntiles), dim3(kReduceBlock), 0, s, reqs, tiles, ntiles);
        else
            hipLaunchKernelGGL(k_p1_reduce_f64<false>, dim3(ntiles), dim3(kReduceBlock), 0, s, reqs, tiles, ntiles);
    }
    return hipGetLastError();
}

}  // namespace bem
