// Internal declarations of libbem (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "bem.h"

namespace bem {

// ---------------------------------------------------------------------------
// Device layout of one triangle.
//
// FP32 record, 32 floats (128 B), for the compensated FP32 path:
//   [0..2]  centroid, high part (float of the FP64 centroid)   [3]  J = |(b-a)x(c-a)|
//   [4..6]  centroid, low part  (float of the FP64 remainder)  [7]  0
//   [8..10] unit normal                                        [11] 0
//   [12..]  quadrature points relative to the centroid, point-major (x,y,z)
// Differences of two triangles' positions are formed as (hi_a - hi_b) +
// (lo_a - lo_b) + (offset_p - offset_q): the large centroid parts cancel
// first, so the result keeps FP32 relative accuracy in |x - y| wherever the
// mesh sits in space.
//
// FP64 record, 24 doubles (192 B), for the plain FP64 path:
//   [0..2] unit normal  [3] J  [4..] absolute quadrature points, point-major.
constexpr int kGeo32Stride = 32;
constexpr int kGeo64Stride = 24;
constexpr int kTileLanes = 64;      // one wavefront per tile
constexpr int kWavesPerBlock = 4;   // 256-thread workgroups
constexpr int kReduceBlock = 256;

// One request as the entry kernels see it.
//
// "fixed" side: one triangle (P0) or one vertex star (P1) shared by the 64
// lanes of a tile; "lane" side: one triangle per lane.  rowfix = 1 means the
// fixed side is the test (row) side.
struct ReqDev {
    const float *g32;
    const double *g64;
    const int4 *vtx;           // vertex ids per triangle (x, y, z; w unused)
    const int32_t *fix;        // P0: triangle per fixed position; P1: star ranges (nfix + 1)
    const int32_t *fstar;      // P1: packed (triangle << 2 | local vertex) of fixed stars
    const int32_t *lane;       // triangle per lane position
    const int32_t *seg_ptr;    // P1: per output position on the lane side, range into seg
    const int32_t *seg;        // P1: packed (lane slot << 2 | local vertex)
    void *part;                // P1: per (fixed pos, lane slot, local vertex) partial sums
    void *out;                 // final output, row-major nrows x ncols
    int32_t *status;           // bit 0: a vertex-sharing pair was met under BEM_NEAR_ERROR
    int32_t *counter;          // P1 with fused reduction: tiles finished so far (zeroed); else null
    int64_t sf, sl;            // P0: out index = fixed_pos * sf + lane_pos * sl
    int32_t nrows, ncols;
    int32_t nlane;             // lane-side item count
    int32_t nfix;              // fixed-side positions
    int32_t rowfix;
    int32_t near_error;
    int32_t ntiles_req;        // entry tiles of this request (fused reduction: the last one reduces)
    int32_t pad0;
    double k;                  // wavenumber
    double kk;                 // k / (2 pi): phase in turns per unit length
};

struct Tile {        // one wavefront of entry work
    int32_t req;
    int32_t fixed;   // fixed position
    int32_t lane0;   // first lane position
    int32_t nlanes;  // active lanes (<= 64)
};

struct RTile {       // one workgroup of P1 reduction work
    int32_t req;
    int32_t count;   // entries (<= kReduceBlock)
    int64_t e0;      // first flat output index
};

// Kernel variant: one compiled instantiation of the entry kernel.
struct Variant {
    int op, space, prec, q, rowfix;
    bool operator<(const Variant &o) const {
        if (op != o.op) return op < o.op;
        if (space != o.space) return space < o.space;
        if (prec != o.prec) return prec < o.prec;
        if (q != o.q) return q < o.q;
        return rowfix < o.rowfix;
    }
};

// Launchers (entries.hip).  Return hipSuccess or the launch error.
// Tile tables are built on the device from per-group request lists and
// exclusive prefix sums of per-request tile counts (gpre has ng + 1 entries).
hipError_t launch_build_tiles(const ReqDev *reqs, const int32_t *greq, const int64_t *gpre, int ng, int64_t ntiles,
                              Tile *tiles, hipStream_t s);
hipError_t launch_build_rtiles(const ReqDev *reqs, const int32_t *greq, const int64_t *gpre, int ng, int64_t ntiles,
                               RTile *tiles, hipStream_t s);
// All groups of a batch in one launch: group g covers global tiles
// [tile0, tile0 + ntiles) and writes Tile (kind 0) or RTile (kind 1) records.
struct GroupDesc {
    int64_t tile0, ntiles;
    const int32_t *greq;
    const int64_t *gpre;
    void *tiles;
    int32_t ng, kind;
};
hipError_t launch_build_all(const ReqDev *reqs, const GroupDesc *groups, int ngroups, int64_t total, hipStream_t s);
hipError_t launch_entries(const Variant &v, const ReqDev *reqs, const Tile *tiles, int64_t ntiles, hipStream_t s);
hipError_t launch_p1_reduce(int prec, bool cplx, const ReqDev *reqs, const RTile *tiles, int64_t ntiles,
                            hipStream_t s);
hipError_t launch_geometry(const double *xyz, const int32_t *tri, int64_t nt, int q, float *g32, double *g64,
                           int4 *vtx, int32_t *bad, hipStream_t s);

// ---------------------------------------------------------------------------
// Errors
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
#define BEM_HIP_TRY(expr)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::bem::fail(BEM_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

double now_seconds();

}  // namespace bem

// ---------------------------------------------------------------------------
// Mesh handle (host copies for request expansion and trees, device geometry).
struct bem_mesh {
    int64_t nv = 0, nt = 0;
    int q = 6;
    std::vector<double> xyz;          // nv x 3
    std::vector<int32_t> tri;         // nt x 3
    std::vector<int64_t> star_ptr;    // nv + 1
    std::vector<int32_t> star;        // packed (triangle << 2 | local vertex), ascending triangles
    double mean_J = 0.0, mean_edge = 0.0;
    int max_star = 0;
    int device = 0;
    float *d_g32 = nullptr;
    double *d_g64 = nullptr;
    int4 *d_vtx = nullptr;
    size_t dev_bytes = 0;
    std::atomic<int64_t> inflight{0};

    bool adjacent(int64_t a, int64_t b) const {
        const int32_t *ta = &tri[3 * a], *tb = &tri[3 * b];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                if (ta[i] == tb[j]) return true;
        return false;
    }
};

namespace bem {

// ---------------------------------------------------------------------------
// Lane side of a request: the triangles the lanes run over and, for P1, the
// map from each requested lane-side dof to its (triangle, local vertex)
// partial sums.  Computed once per dof list; device-resident copies are
// shared by every request of an H-matrix block.
struct LaneSet {
    int64_t ndof = 0;                 // lane-side output positions
    std::vector<int32_t> lane;        // P0: the dofs themselves; P1: distinct triangles, ascending
    std::vector<int32_t> seg_ptr;     // P1: ndof + 1
    std::vector<int32_t> seg;         // P1: packed (slot << 2 | local vertex)
    size_t ints() const { return lane.size() + seg_ptr.size() + seg.size(); }
};

struct LaneRef {                      // device pointers of a resident LaneSet
    const int32_t *lane = nullptr, *seg_ptr = nullptr, *seg = nullptr;
    int64_t ndof = 0, nlane = 0, nseg = 0;
};

void build_lane_set(const bem_mesh &m, int space, const int32_t *dofs, int64_t n, LaneSet &ls);

// ---------------------------------------------------------------------------
// A request on its way through the server.
struct Request {
    bem_mesh *mesh = nullptr;
    int op = 0, space = 0, prec = 0, near = 0;
    double k = 0.0;
    int64_t nrows = 0, ncols = 0;
    std::vector<int32_t> rows, cols;
    void *out_host = nullptr;   // destination (host); null with borrow = true
    bool borrow = false;        // completion hands out a pointer into pinned staging instead
    const void *result = nullptr;
    void *batch = nullptr;      // batch holding a borrowed result

    // expansion
    int rowfix = 1;
    std::vector<int32_t> fix, fstar;   // fixed side
    LaneSet own;                       // lane side, when not external
    const LaneRef *ext = nullptr;      // device-resident lane side
    int64_t nfix = 0, nlane = 0;
    size_t elem_bytes = 0, part_elem_bytes = 0;
    size_t in_bytes = 0, out_bytes = 0, part_bytes = 0;
    int64_t evals = 0;          // Q^2 x (fixed, lane) triangle pairs, vertex-sharing pairs included
    int64_t ntiles = 0, nrtiles = 0;
    bool fuse_reduce = false;   // P1: the request's last entry tile performs the per-entry reduction
    size_t batch_bytes = 0;     // request_bytes(), cached at expansion

    // completion
    std::mutex mu;
    std::condition_variable cv;
    bool done = false;
    int status = 0;
    double t_submit = 0.0, t_done = 0.0;
    // Completion callback, called from the server's completion thread with all
    // finished requests of one batch that share (on_done, cb_ctx); requests
    // with a callback are not signalled through cv.
    void (*on_done)(Request **, size_t, void *) = nullptr;
    void *cb_ctx = nullptr;
    int64_t tag = 0;            // caller's bookkeeping

    // placement inside a batch
    size_t off_out = 0, off_status = 0;

    int64_t entries() const { return nrows * ncols; }
};

bool is_complex_op(int op);
size_t out_elem_bytes(int op, int prec);

// Validate and expand a request (host; runs on the submitting thread).
int expand_request(Request &r);
// Fast path for requests whose lane side is a resident LaneRef and whose
// fixed side is a single dof known to be valid (H-matrix blocks).
void expand_single_fixed(Request &r, int32_t dof, int rowfix, const LaneRef *ext);

// Device bytes a request needs inside a batch (inputs, outputs, partials, tiles).
size_t request_bytes(const Request &r);

// Writes the request's inputs at host_base + off (staging) and fills its
// descriptor with device addresses at dev_base + off; returns the bytes used.
size_t stage_request_inputs(Request &r, char *host_base, char *dev_base, size_t off, ReqDev &d);
// off_status addresses two int32 per request: status word, then the arrival
// counter of the fused P1 reduction.
void finish_descriptor(const Request &r, char *dev_base, size_t off_out, size_t off_part, size_t off_status,
                       ReqDev &d);
// P1 requests with at most this many entries reduce inside the entry kernel
// (last-arriving tile); 0 = always a separate reduction launch.  Set by the
// BEM_FUSE_REDUCE_MAX environment variable, read once.
int64_t fuse_reduce_max_entries();

// Server
int server_submit(Request *r);
int server_submit_many(Request *const *rs, size_t n);
int server_wait(Request *r, double timeout_s);
void server_release(Request *r);           // return a borrowed result
int server_ensure_started();
bool server_running();

}  // namespace bem
