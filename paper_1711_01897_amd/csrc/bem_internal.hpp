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

struct Request;

// ---------------------------------------------------------------------------
// Device layout of one triangle.
//
// FP32 record, 16 floats (64 B, one load of four float4), for the
// compensated FP32 path:
//   [0..2]   centroid, high part (float of the FP64 centroid)   [3]  J = |(b-a)x(c-a)|
//   [4..6]   centroid, low part  (float of the FP64 remainder)  [7]  n_x
//   [8..10]  e1 = b - a                                         [11] n_y
//   [12..14] e2 = c - a                                         [15] n_z
// (n the unit normal).  Kernels expand it in registers to the working
// layout of n32<Q>() words: [0..2] centroid high, [3] J, [4..6] centroid
// low, [8..10] n, and from [12] the quadrature points relative to the
// centroid, x_p - c = (xi_p - 1/3) e1 + (eta_p - 1/3) e2, point-major.
// Differences of two triangles' positions are formed as (hi_a - hi_b) +
// (lo_a - lo_b) + (offset_p - offset_q): the large centroid parts cancel
// first, so the result keeps FP32 relative accuracy in |x - y| wherever the
// mesh sits in space.
//
// FP64 record, 24 doubles (192 B), for the plain FP64 path:
//   [0..2] unit normal  [3] J  [4..] absolute quadrature points, point-major.
constexpr int kGeo32Stride = 16;
constexpr int kGeo64Stride = 24;
constexpr int kBlockLanes = 256;    // lane-side items per workgroup (4 wavefronts)
constexpr int kStage = 8;           // fixed-side triangles staged in LDS at a time

// One request as the entry kernels see it.
//
// "fixed" side: one triangle (P0) or one vertex star (P1) shared by the
// lanes of a workgroup; "lane" side: one triangle per lane, grouped in
// chunks of at most kBlockLanes lanes.  rowfix = 1 means the fixed side is
// the test (row) side.  Output position (fixed f, lane-side dof d) is
// out[f * sf + d * sl].
struct ReqDev {
    const float *g32;
    const double *g64;
    const int4 *vtx;           // vertex ids per triangle (x, y, z; w unused)
    const int32_t *fstar;      // P1: the mesh star table (packed triangle << 2 | local vertex); block
                               // records name the fixed dof's entries [s0, s1)
    const int32_t *lane;       // triangle per lane position
    const int4 *chunk;         // per chunk: first lane, lanes, first dof, dofs
    const int32_t *seg_ptr;    // P1: per lane-side dof, range into seg
    const int32_t *seg;        // P1: packed (lane slot within the chunk << 2 | local vertex)
    const int32_t *lpos;       // P1: output position of each lane-side dof (null: its own index)
    void *out;                 // final output, row-major nrows x ncols
    int32_t *status;           // set to 1: a vertex-sharing pair was met under BEM_NEAR_ERROR
    int64_t sf, sl;
    int32_t nrows, ncols;
    int32_t nlane;             // lane-side items over all chunks
    int32_t nfix;              // fixed-side positions
    int32_t rowfix;
    int32_t near_error;
    double k;                  // wavenumber
    double kk;                 // k / (2 pi): phase in turns per unit length
};

struct EntryBlock {  // one workgroup of entry work (64 bytes, read with one scalar load)
    int32_t req;           // (request index << 1) | 1 if the test side is fixed (row request): the kernel
                           // picks its code path before the request descriptor arrives
    int32_t fixed;         // fixed position
    int32_t s0, s1;        // P1: the fixed dof's star, entries [s0, s1) of the mesh star table; P0: s0 = the fixed triangle
    int4 chunk;            // lane side: first lane, lanes, first dof, dofs
    const float *lgeo;     // lane records gathered per lane position (or null: gather through R.lane)
    const int4 *lmeta;     // their vertex ids; null with lgeo set: the sides are separated (no vertex-sharing
                           // pair can occur, the kernels skip the test)
    const float *sgeo;     // P1: the mesh's star records (FP32), indexed by star entry; P0: its triangle records
    const int4 *smeta;     // their vertex ids (P1: w = local vertex of the star's dof)
};

// Kernel variant: one compiled instantiation of the entry kernel (it serves
// both fixed sides).
struct Variant {
    int op, space, prec, q;
    int persist = 0;   // statistics only: the resident (persistent) form of the kernel
    bool operator<(const Variant &o) const {
        if (op != o.op) return op < o.op;
        if (space != o.space) return space < o.space;
        if (prec != o.prec) return prec < o.prec;
        if (q != o.q) return q < o.q;
        return persist < o.persist;
    }
};

// Block table of a request, written by the host: request index `ri` inside
// its batch, blocks in (fixed, chunk) order; returns the count.
int64_t write_blocks(const Request &r, int32_t ri, EntryBlock *out);

// Launchers (entries.hip).  Return hipSuccess or the launch error.
// tclock (optional, device memory, 2 * nblocks entries): receives each
// workgroup's start and end on the device's constant-rate clock.
// start/stop (optional): HIP events recorded around the launch on its stream.
hipError_t launch_entries(const Variant &v, const ReqDev *reqs, const EntryBlock *blocks, int64_t nblocks, hipStream_t s,
                          unsigned long long *tclock = nullptr, hipEvent_t start = nullptr, hipEvent_t stop = nullptr);

// ---------------------------------------------------------------------------
// Persistent service of batches.
//
// One launch of the entry kernel stays resident and serves a stream of
// batches of one kernel variant.  The host publishes each batch (its
// descriptors and block records already in host-coherent staging) as an
// entry of a ring in host-coherent memory, in sequence order.  Workgroup 0
// watches the ring (one thread) and copies each published entry to device
// memory together with its claim word; the other workgroups claim blocks
// with atomic adds on the claim words, oldest batch first, and run the same
// per-block code as the launched kernels.  Any workgroup can claim any
// block, so a launch never depends on all of its workgroups being resident.
// The workgroup that ends a batch's last block stores seq + 1 into the
// batch's completion word in host memory.  The launch ends when the host asks
// it to or no entry has been published for a given number of device-clock
// ticks: the watching thread stores the first sequence number it did not
// take into the exit word, and every waiting workgroup returns.  The host
// publishes entry i again only after the batch it last held has completed.
constexpr int kPersistRing = 64;    // ring entries (more than batches in flight)

struct PersistEntry {               // host-coherent; seq1 written last
    const ReqDev *reqs;
    const EntryBlock *blocks;
    unsigned long long *clock;      // per block {start, end} device clock, or null
    int64_t nblk;
    uint64_t seq1;                  // sequence number + 1 once published
    uint64_t pad[3];
};
static_assert(sizeof(PersistEntry) == 64, "ring entries are 64 bytes");

struct PersistHost {                // host-coherent words shared by the persistent launches
    PersistEntry ring[kPersistRing];
    uint64_t done[kPersistRing][8];   // done[i][0] = seq + 1 of the last batch of ring entry i completed
    uint64_t stop;                    // the host asks launches with id <= stop to end
    uint64_t pad0[7];
    uint64_t exit_word;               // id << 40 | (first sequence number not taken + 1), stored by a
                                      // launch as it ends
    uint64_t pad1[7];
};

struct PersistItem {                // a published batch as the workers read it (device memory)
    const ReqDev *reqs;
    const EntryBlock *blocks;
    unsigned long long *clock;
    int64_t nblk;
    uint64_t pad[4];
};

// Claim word of ring entry i: (seq mod 2^16) << 48 | nblk << 32 | blocks
// claimed, seq the batch the entry holds.  An atomic add of one claims
// block "blocks claimed" when that is below nblk; the tag names the batch
// the claim belongs to whatever batch the claimer expected (a workgroup's
// cursor is never 2^15 batches away from the batches an entry can hold), so
// no claim is lost when an entry is reused.
struct PersistCtl {                 // device memory, reset before each launch
    unsigned long long cur;         // every batch before cur has no unclaimed block
    unsigned long long pad0[15];
    unsigned int stop;              // the watcher has left: waiting workgroups return
    unsigned int pad1[31];
    PersistItem item[kPersistRing];
    unsigned long long claim[kPersistRing][16];   // one 128-byte line each
    unsigned int done[kPersistRing][32];          // blocks finished, one line each
};
constexpr int kPersistMaxBlocks = 65535;   // per batch (the claim word's nblk field)

struct PersistArgs {
    const PersistHost *host;        // device address of the host words
    uint64_t *done;                 // device address of host->done
    uint64_t *exit_word;            // device address of host->exit_word
    PersistCtl *ctl;
    uint64_t seq0;                  // first sequence number this launch serves
    uint64_t id;                    // launch number: the launch ends once host->stop >= id
    long long idle_ticks;           // device-clock ticks without a new entry before the launch ends
};

// Enqueues the reset of a.ctl for a launch that starts at sequence number
// a.seq0, then the persistent launch of variant v with `groups` workgroups
// (workgroup 0 watches the ring); start/stop events (optional) around the
// persistent launch.
hipError_t launch_persistent(const Variant &v, const PersistArgs &a, int groups, hipStream_t s,
                             hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
// Resident workgroups per compute unit of the persistent kernel of variant v
// (0 if there is none).
int persistent_occupancy(const Variant &v);

hipError_t launch_geometry(const double *xyz, const int32_t *tri, int64_t nt, int q, float *g32, double *g64,
                           int4 *vtx, int32_t *bad, hipStream_t s);
// geo[i] = FP32 record of triangle index[i] >> shift, meta[i] = its vertex
// ids (w = index[i] & 3 when shift == 2, else 0); i < n.
hipError_t launch_gather(const float *g32, const int4 *vtx, const int32_t *index, int shift, int64_t n, float *geo,
                         int4 *meta, hipStream_t s);
// One vertex-sharing (singular) P0 triangle pair of a BEM_NEAR_SINGULAR
// request, integrated by near.hip.  Vertices in the layout of its kind:
//   kind 0, identical:   v = V0, V1, V2 (the triangle in its own order)
//   kind 1, common edge: v = P, Q, A, B (shared edge P-Q; A the test
//                        triangle's third vertex, B the trial triangle's)
//   kind 2, common vertex: v = P, A, B, C, D (shared P; A, B the test
//                        triangle's others, C, D the trial triangle's)
// ny: unit normal of the trial triangle; jt, js: |cross| of the test and
// trial triangles (twice their areas).  out: the entry's address; the
// kernel adds the pair's value to what the entry kernel stored there.
struct NearItem {
    double v[15];
    double ny[3];
    double jt, js;
    double k;   // wavenumber (Helmholtz)
    void *out;
    int32_t kind;
    int32_t pad;
};
static_assert(sizeof(NearItem) == 184, "near items are 184 bytes");

// Adds each item's singular pair integral (FP64; radial integral in closed
// form for Laplace, by an 8-point rule for Helmholtz; composite
// Gauss-Legendre for the rest) to its entry: the Laplace single (op 0) or
// double layer (op 1), the Helmholtz single (op 2) or double layer (op 3),
// into float / complex<float> (fp32 = true) or double / complex<double>
// entries.  One workgroup per item.
// P1 singular region of a request: items | gather records | sources |
// source weights (hypersingular operator) | local values (9 per pair, 1 for
// the hypersingular operator); offsets from the region's start, each
// 256-byte aligned.
struct NearP1Layout {
    size_t items, recs, src, wt, local, bytes;
    int per;       // doubles per pair in the local values
    int src_per;   // gather source units per pair (9 values, 9 complex values, or 1)
    bool weighted, cplx;
};
// mode: 0 real 3 x 3 local matrices, 1 Laplace hypersingular (one value per
// pair, weighted sources), 2 complex 3 x 3 local matrices, 3 Helmholtz
// hypersingular (complex 3 x 3 single-layer local matrix and P0 value,
// weighted sources)
NearP1Layout near_p1_layout(int mode, int64_t items, int64_t recs, int64_t src);
int near_p1_mode(const Request &r);
NearP1Layout near_p1_layout(const Request &r);
// Writes request r's part of a region's host image at host (dev: the region's
// device address, out_dev: r's output on the device), its pairs, records and
// sources after the first pb, rb and sb of the region (requests of one
// kernel and precision share a region).
void stage_near_p1(const Request &r, const NearP1Layout &L, char *host, char *dev, char *out_dev, int64_t pb,
                   int64_t rb, int64_t sb);
// Enqueues the P1 singular pairs of a staged region (local matrices, then the
// gather into the entries).
hipError_t launch_near_p1_region(int op, bool fp32, const NearP1Layout &L, char *dev, int64_t items, int64_t recs,
                                 hipStream_t s);
// Index of the P1 singular run of a request (kernel and precision), 0..11:
// 2 g + fp32 with g = 0 single, 1 double layer, 2 hypersingular (Laplace),
// 3 single, 4 double layer, 5 hypersingular (Helmholtz).
int near_p1_group(const Request &r);

hipError_t launch_near(int op, bool fp32, const NearItem *items, int64_t n, hipStream_t s);

// P1: one entry's singular contributions, src[first .. first + count) into
// the pairs' local matrices (9 doubles per pair, row-major test x trial).
struct NearGather {
    void *out;
    int32_t first, count;
};
static_assert(sizeof(NearGather) == 16, "gather records are 16 bytes");

// P1 Laplace single (op 0) or double layer (op 1): each item's 3 x 3 local
// matrix (FP64) into the 9 doubles at item.out; Helmholtz single (op 2) or
// double layer (op 3): 9 complex values (18 doubles); Laplace hypersingular
// operator (op 6): the pair's P0 single-layer integral into the double at
// item.out.  One workgroup per item.
hipError_t launch_near_p1(int op, const NearItem *items, int64_t n, hipStream_t s);
// Adds each record's fixed-order sum of local values (times the source
// weights when wt is not null) to its float (fp32) or double entry.  One
// thread per record.
hipError_t launch_near_gather(bool fp32, bool cplx, const NearGather *recs, int64_t n, const int32_t *src,
                              const double *wt, const double *local, hipStream_t s);

// Copies bytes (a multiple of 16, both addresses 16-byte aligned) from src
// (device-visible host staging) to dst (device) with a kernel on stream s.
hipError_t launch_stage_copy(const void *src, void *dst, size_t bytes, hipStream_t s);

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
    std::vector<int32_t> dp1_star;    // 3 nt: star-table position of (triangle t, local vertex a) at 3 t + a
    double mean_J = 0.0, mean_edge = 0.0;
    double box_lo[3] = {0.0, 0.0, 0.0}, box_inv[3] = {0.0, 0.0, 0.0};   // bounding box: low corner, 1/extent
    int max_star = 0;
    int device = 0;
    float *d_g32 = nullptr;
    double *d_g64 = nullptr;
    int4 *d_vtx = nullptr;
    int32_t *d_star = nullptr;   // star table on the device (packed triangle << 2 | local vertex)
    float *d_sgeo = nullptr;     // FP32 record per star entry
    int4 *d_smeta = nullptr;     // vertex ids per star entry, w = local vertex
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
// Lane side of a request: the triangles the lanes run over, in chunks of at
// most kBlockLanes, and, for P1, the map from each requested lane-side dof to
// its (triangle, local vertex) partial sums.  A P1 chunk holds a run of
// consecutive lane-side dofs together with every triangle of their stars, so
// one workgroup finishes those entries on its own (triangles on a chunk
// border appear in both chunks).  Computed once per dof list; device-resident
// copies are shared by every request of an H-matrix block.
struct LaneSet {
    int64_t ndof = 0;                 // lane-side output positions
    int64_t ndistinct = 0;            // distinct lane triangles (P0: ndof)
    std::vector<int32_t> lane;        // P0: the dofs themselves; P1: triangles, chunk by chunk
    std::vector<int32_t> chunk;       // 4 per chunk: first lane, lanes, first dof, dofs
    std::vector<int32_t> seg_ptr;     // P1: ndof + 1
    std::vector<int32_t> seg;         // P1: packed (slot within the chunk << 2 | local vertex)
    std::vector<int32_t> pos;         // P1: output position of each lane-side dof when the set was
                                      // reordered for locality (empty: identity)
    int64_t nchunk() const { return (int64_t)chunk.size() / 4; }
    size_t ints() const { return chunk.size() + lane.size() + seg_ptr.size() + seg.size() + pos.size(); }
};

struct LaneRef {                      // device pointers of a resident LaneSet
    const int32_t *lane = nullptr, *seg_ptr = nullptr, *seg = nullptr;
    const int4 *chunk = nullptr;
    const int32_t *chunk_host = nullptr;   // host copy of the chunk table (block records carry it)
    const float *geo = nullptr;            // FP32 records gathered per lane position
    const int4 *meta = nullptr;            // their vertex ids
    int64_t ndof = 0, nlane = 0, nseg = 0, nchunk = 0, ndistinct = 0;
};

// Lane set of a dof list.  With reorder, a P1 list longer than one chunk is
// first ordered along a Morton curve of the vertex positions (ls.pos keeps
// each entry's position in the caller's list): chunks then hold the stars of
// neighbouring vertices instead of whatever the caller's order groups, which
// keeps the duplicated border lanes few.
void build_lane_set(const bem_mesh &m, int space, const int32_t *dofs, int64_t n, LaneSet &ls,
                    bool reorder = false);

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
    int fixrows = 1;            // the fixed items are the request's rows (else its columns)
    int rowfix = 1;             // kernel side: the fixed items are test functions (differs from fixrows
                                // for the adjoint double layer, evaluated as the double layer transposed)
    std::vector<int32_t> fix;   // fixed side: P0 triangles; P1 star ranges [s0, s1) per fixed dof (2 each)
    LaneSet own;                       // lane side, when not external
    const LaneRef *ext = nullptr;      // device-resident lane side
    // the supports of the fixed and lane sides have a positive distance (the
    // blocks of an admissible partition): no pair can share a vertex, so the
    // kernels neither load vertex ids for the lanes nor test for sharing
    bool separated = false;
    int64_t nfix = 0, nlane = 0, nchunk = 0, ndistinct = 0;
    int64_t nstar = 0;          // P1: triangles over the fixed dofs' stars
    size_t elem_bytes = 0;
    size_t in_bytes = 0, out_bytes = 0;
    int64_t evals = 0;          // Q^2 x distinct (fixed, lane) triangle pairs, vertex-sharing pairs included
    int64_t nblocks = 0;
    size_t batch_bytes = 0;     // request_bytes(), cached at expansion

    // staging records built by the submitting thread (prebuild_staging); the
    // server's dispatcher copies them into a batch and fills in what depends
    // on the batch: the request index of each block, the staged inputs, the
    // output and status addresses
    std::vector<NearItem> near_items;     // BEM_NEAR_SINGULAR: the request's vertex-sharing pairs
    std::vector<int64_t> near_index;      // P0: their entries' positions in the output
    struct NearRec {
        int64_t entry;                    // position in the output
        int32_t first, count;             // into near_src
    };
    std::vector<NearRec> near_recs;       // P1: entries with singular contributions, ascending
    std::vector<int32_t> near_src;        // P1: pair * 9 + 3 a + b of each contribution, per entry ascending
                                          // (hypersingular operator: the pair)
    std::vector<double> near_wt;          // P1 hypersingular operator: curl_a . curl_b of each contribution
    int key = 0;                          // launch group (operator, space, precision, rule)
    std::vector<EntryBlock> pre_blocks;   // `req` holds the fixed-side bit only
    ReqDev pre_dev{};

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
    bool fast = false;          // written into its batch by the submitter (server fast path)

    int64_t entries() const { return nrows * ncols; }
};

bool is_complex_op(int op);
// Dofs of a space on a mesh: triangles (P0), vertices (P1), 3 x triangles (DP1).
int64_t space_ndof(const bem_mesh &m, int space);
// The entry kernels' space: P0 kernels for P0, the P1 kernels (fixed star
// against lane triangles, per-dof reduction) for P1 and DP1 (a DP1 dof is a
// one-triangle star).
inline int kernel_space(int space) { return space == BEM_P0 ? BEM_P0 : BEM_P1; }
bool is_adjoint_op(int op);
// The operator the entry kernels evaluate: the adjoint double layer runs as
// the double layer with test and trial exchanged.
int kernel_op(int op);
size_t out_elem_bytes(int op, int prec);

// Validate and expand a request (host; runs on the submitting thread).
int expand_request(Request &r);
// Fast path for requests whose lane side is a resident LaneRef and whose
// fixed side is a single dof known to be valid (H-matrix blocks).
void expand_single_fixed(Request &r, int32_t dof, int rowfix, const LaneRef *ext);

// Device bytes a request needs inside a batch (inputs, outputs, block table).
size_t request_bytes(const Request &r);

// Writes the request's inputs at host_base + off (staging) and fills its
// descriptor with device addresses at dev_base + off; returns the bytes used.
size_t stage_request_inputs(Request &r, char *host_base, char *dev_base, size_t off, ReqDev &d);
// The descriptor fields that do not depend on where the request is staged.
void describe_request(const Request &r, ReqDev &d);
// Copies a request's own lane-side arrays into staging at `off` and points d
// at their device copies (no-op for a device-resident lane side); returns
// the bytes used (r.in_bytes).
size_t stage_own_inputs(const Request &r, char *host_base, char *dev_base, size_t off, ReqDev &d);
// Launch group of a request: (kernel operator, kernel space, precision, rule).
int request_key(const Request &r);
// Fills r.key, r.pre_blocks and r.pre_dev (called by the submitting thread).
void prebuild_staging(Request &r);
// off_status addresses the request's int32 status word (zeroed by the caller).
void finish_descriptor(const Request &r, char *dev_base, size_t off_out, size_t off_status, ReqDev &d);

// Server
int server_submit(Request *r);
int server_submit_many(Request *const *rs, size_t n);
// With BEM_DEBUG_TIMING set: prints and resets per-phase host times of the
// dispatch and completion threads (stderr).
void server_print_phases();
int server_wait(Request *r, double timeout_s);
// Status of a finished request handed to a completion callback (requests
// submitted through the server's fast path carry it in the batch).
int server_request_status(const Request *r);
// Completion time of such a request (library clock).
double server_request_done_time(const Request *r);
void server_release(Request *r);           // return a borrowed result
void server_release_batch(void *batch, int n);   // return n borrowed results of one batch (Request::batch)
int server_ensure_started();
bool server_running();

}  // namespace bem
