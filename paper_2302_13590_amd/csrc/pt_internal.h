// Internal declarations shared by the kernels and the host side of libpt.
// Device layouts of the flow field and of the tracking-kernel parameters.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pt {

// Per-cell flag word of the packed layouts.  Bits 0-1 are the cell's own
// PT_CELL_* flags; for each face f (0 = -i, 1 = +i, 2 = -j, 3 = +j, 4 = -k,
// 5 = +k) bit NB_OUT+f says the neighbour across f is outside the domain,
// NB_INACTIVE+f that it is inactive, NB_SINK+f that it is a sink cell.  With
// these the transfer to the next cell is decided from the current record.
enum : int32_t {
    CF_ACTIVE = 1,
    CF_SINK = 2,
    NB_OUT = 2,
    NB_INACTIVE = 8,
    NB_SINK = 14,
};

// 64-byte FP64 record: the six face velocities u = Q/(n V) (low/high face of
// i, j, k) and the flag word.  64-byte aligned: one gather touches one half
// of a 128-byte cache line.
struct alignas(64) CellRec64 {
    double u[6];
    int32_t flags;
    int32_t pad0;
    double pad1;
};
static_assert(sizeof(CellRec64) == 64, "CellRec64 must be 64 bytes");

// 32-byte FP32 record for the mixed-precision path.
struct alignas(32) CellRec32 {
    float u[6];
    int32_t flags;
    int32_t pad0;
};
static_assert(sizeof(CellRec32) == 32, "CellRec32 must be 32 bytes");

// Quadtree grids: the same 64-byte record (u = total face flow / (n V), own flags in the flag
// word), with the cell's first subface and the subface count of each face (5 bits per face,
// face f at bit 5f) in the padding.  A subface's extent in the face's two tangential local
// coordinates is {lo_u, lo_v, hi_u, hi_v}.
struct alignas(64) QuadRec {
    double u[6];
    int32_t flags;
    int32_t sub_base;
    uint32_t counts;
    int32_t pad0;
};
static_assert(sizeof(QuadRec) == 64, "QuadRec must be 64 bytes");
constexpr int kMaxSubPerFace = 31;
struct QuadBox {
    double lo[3];   // x_lo, y_lo, z_lo
    double h[3];    // hx, hy, hz
};

// One flow field as the kernels see it.
struct GridDev {
    const CellRec64* rec64;
    const CellRec32* rec32;
    const double* qx;
    const double* qy;
    const double* qz;
    const double* por;      // nullptr -> por_scalar
    const int32_t* flags;   // own flags only (faces layout)
    double por_scalar;
    double dx, dy, dz, x0, y0, z0;
    double V;               // (dx*dy)*dz
    int32_t nx, ny, nz, plane;   // plane = nx ny (structured), 1 (quadtree)
    // quadtree grids (nx = number of cells, ny = nz = 1; rec64 points at QuadRec records)
    const QuadBox* qbox;
    const int32_t* sub_nb;
    const double4* sub_rect;
};

constexpr int kXcd = 8;   // accelerator complex dies; workgroup b runs on die b mod 8
constexpr int kDieChunk = 16;   // static kernel: consecutive blocks of work dealt to one die at a time

// Counters of a run (device), cleared by the reset kernel.
struct Counters {
    unsigned long long crossings;
    unsigned long long status[8];
    unsigned long long cr_ambiguous;  // correctly rounded evaluations left undecided
    unsigned long long queue[kXcd];   // next slot handed out in each die's segment
    unsigned long long path_dropped;  // pathline records outside their slot range
    unsigned long long recheck_tracks;  // particles handed to the careful pass (may exceed its capacity)
    unsigned long long pad[12];
};
static_assert(sizeof(Counters) == 32 * 8, "Counters is 32 words");

// One pathline record (the layout of pt_path_record).
struct PathRec {
    double t, x, y, z;
    int32_t cell, face;
};
static_assert(sizeof(PathRec) == 40, "PathRec is 40 bytes");

// Capacity of the careful pass's particle list in pt_track.
constexpr int64_t kRecheckTracksMax = (int64_t)1 << 20;

struct TrackParams {
    int64_t n;
    int32_t* cell;
    double* xi;
    double* eta;
    double* zeta;
    double* t;
    int32_t* status;
    int32_t* ncross;
    uint64_t* hash;
    // batched runs: device copies of the group table and of the grid views
    const int64_t* group_offsets;
    const int32_t* group_grid;
    const GridDev* grids;
    int32_t n_groups;
    int32_t n_grids;
    GridDev g0;             // grids[0], by value for single-grid runs
    double t_max;
    int64_t max_steps;
    double sign;            // +1 forward, -1 backward
    int32_t stop_at_sink;
    int32_t n_snap;
    const double* snap_times;
    double* snap_xyz;
    double* out_xyz;
    Counters* counters;
    int32_t refill;
    int32_t steps_per_refill;
    int32_t chunk;
    int32_t pad_chunk;
    // Processing order: slot s of the work holds particle order[s] (nullptr: s itself).  The
    // static kernel deals the slots to the dies in chunks of kDieChunk blocks; the persistent
    // queue has one segment per die.
    const int32_t* order;
    // Pathline output (O_PATH kernels).  Count pass (path_count): path_off[p+1] receives the
    // crossings of particle p and no state is written back.  Record pass: the records of p go to
    // slots [path_off[p], path_off[p+1]) that are also below path_cap.
    int64_t* path_off;
    int32_t path_count;
    int32_t path_stage;   // record pass: records staged per lane in LDS, written in 64-byte segments
    int64_t path_cap;
    PathRec* path_rec;
    // Transient flow (batched kernels): grids[s] is the field of time step s, valid until
    // tstep_end[s]; the lane's grid index is its current time step.
    int32_t n_tsteps;
    int32_t pad_ts;
    const double* tstep_end;
    // Careful pass (FP64).  A correctly rounded evaluation that the accurate phase cannot decide
    // (a value within 2^-96 of a rounding midpoint) is not settled in the tracking kernels, whose
    // registers are sized for the common path: the particle's pid goes to recheck_pid and it is
    // tracked again from its input state by the careful kernel.
    int32_t* recheck_pid;
    int32_t recheck_cap;          // entries of recheck_pid (0: no careful pass)
    int32_t pad_recheck;
};

// Output form of a tracking kernel (template argument).
enum : int { O_END = 0, O_SERIES = 1, O_PATH = 2 };

// Inclusive prefix sum of v[0..n) in place (the pathline offsets), three kernels: tile sums,
// a scan of the tile sums, then the tile offsets added.
constexpr int kScanBlock = 1024;
constexpr int kScanPer = 8;
constexpr int64_t kScanTile = (int64_t)kScanBlock * kScanPer;
struct ScanParams {
    int64_t* v;
    int64_t n;
    int64_t* part;     // [ceil(n / kScanTile)] tile sums, then their exclusive scan
    int64_t ntiles;
    int64_t* head;     // element written 0 before v (path_off[0]); may be null
};

// Spatial ordering of particles by starting cell (one bucket per cell, or per run of 2^shift
// cells on grids of more than kMaxBuckets cells), in two levels without global returning
// atomics: tiles of kSortTile particles count their particles per super-bucket (a run of `fine`
// consecutive buckets) in LDS, an exclusive scan of those counts (super-bucket-major) places
// every tile's share of every super-bucket, and one block per super-bucket then orders its range
// by bucket with an LDS histogram.
constexpr int kSortTile = 4096;      // particles per tile (256 threads x 16)
constexpr int kFineMax = 8192;       // buckets per super-bucket at most (a 32 KB LDS histogram)
constexpr int kMaxSuper = 2048;      // super-buckets at most (kMaxBuckets / kFineMax)
constexpr int kFineBlock = 1024;     // threads of the per-super-bucket pass (= kScanBlock)
static_assert(kFineBlock == kScanBlock, "the second level uses the block scan of kScanBlock threads");
struct SortParams {
    int64_t n;
    const int32_t* cell;
    const int32_t* status;
    const int64_t* group_offsets;   // batched runs: group table and the first global cell id
    const int32_t* group_grid;      //   of each grid
    const int64_t* grid_base;
    int32_t n_groups;
    int32_t shift;                  // bucket = global cell id >> shift
    int32_t nbuckets;
    int32_t fine;                   // buckets per super-bucket
    int32_t nsuper;                 // super-buckets
    int32_t ptiles;                 // tiles of kSortTile particles
    int64_t ncnt;                   // nsuper * ptiles
    int32_t ntiles;                 // tiles of kScanTile entries in the scan of cnt
    int32_t pad;
    unsigned* cnt;                  // [nsuper][ptiles] particles of each tile in each super-bucket,
                                    //   then their exclusive prefix sums (super-bucket-major)
    unsigned* part;                 // [ntiles] scan tile totals, then their exclusive prefix sums
    unsigned* bucket;               // [n] bucket of each particle
    unsigned* sbucket;              // [n] buckets in super-bucket order
    int32_t* sidx;                  // [n] particle indices in super-bucket order
    int32_t* order;                 // [n]
};
constexpr int64_t kMaxBuckets = (int64_t)1 << 24;   // one bucket per cell up to 2^24 cells
static_assert((int64_t)kMaxSuper * kFineMax >= kMaxBuckets, "super-buckets cover every bucket");

enum Precision { P64 = 0, PMIX = 1 };
enum Layout { L_FACES = 1, L_CELL = 2, L_QUAD = 3 };
enum Sched { S_STATIC = 1, S_PERSISTENT = 2 };

struct KernelKey {
    int precision, layout, out, batched, sched;   // out: O_END / O_SERIES / O_PATH
};

// Kernel lookup (defined in pt_kernels.hip).
const void* track_kernel(const KernelKey& k);
const void* careful_kernel(const KernelKey& k);        // FP64 keys only
const void* reset_kernel();
const void* sort_tiles_kernel();
const void* sort_scan_tiles_kernel();
const void* sort_scan_partials_kernel();
const void* sort_scan_add_kernel();
const void* sort_spread_kernel();
const void* sort_fine_kernel();
const void* scan_tiles_kernel();
const void* scan_partials_kernel();
const void* scan_add_kernel();
const void* build_kernel();
const void* build_quad_kernel();

// Grid build kernel arguments.
struct BuildParams {
    GridDev g;
    CellRec64* rec64;
    CellRec32* rec32;
    double balance_tol;
    int* err;               // [4]: non-finite flow, bad porosity, bad flags, unbalanced
};

// Quadtree grid build kernel arguments.
struct BuildQuadParams {
    int64_t ncell;
    const QuadBox* box;
    const int32_t* sub_off;     // [ncell*6 + 1]
    const double* sub_q;
    const double* por;          // nullptr -> por_scalar
    double por_scalar;
    const int32_t* flags;       // nullptr -> all active
    QuadRec* rec;
    double balance_tol;
    int* err;                   // [4]: non-finite flow, bad porosity, bad flags, unbalanced
};

// Allocation-free entry point (pt_track_noalloc).  Its per-call tables are written by small
// fill kernels whose argument carries the bytes (no staging buffer, nothing read from host
// memory after the call returns), and its counter block is copied into the caller's counts.
struct FillArgs {
    unsigned char* dst;
    uint32_t nbytes;
    uint32_t pad;
    unsigned char bytes[2048];
};
struct CountsParams {
    const Counters* c;
    int64_t* out;          // PT_COUNTS_WORDS int64, device
    int32_t path_pass;     // 0: none, 1: count pass, 2: record pass
    int32_t pad;
};
const void* fill_kernel();
const void* counts_kernel();

constexpr int kMaxSnapLds = 1024;

// Slot of one lane for deferred snapshots (static kernel, timeseries, packed layouts): the
// step-start state and the range [ks0, ks0 + cnt) of snapshot indices; cnt = 0 when free.  The
// kernel takes blockDim.x slots of dynamic LDS.  R: the precision of the local coordinates.
template <typename R>
struct SnapJob {
    double t;
    R x[3];
    int32_t c, i, j, k;
    int32_t g, pid, ks0, cnt;
    int32_t start;        // first pair index of the slot in a flush
    uint32_t amb;         // FP64: a snapshot of this lane's particle was left undecided (careful pass)
};
static_assert(sizeof(SnapJob<double>) == 72 && sizeof(SnapJob<float>) == 64, "SnapJob layout");

// Staging of one lane's pathline records (record pass): the bytes of the current 64-byte segment
// of the particle's record stream and the overflow of the last record (12 doubles), and the
// particle's first record slot.  The kernel takes blockDim.x slots of dynamic LDS.
struct PathStage {
    double buf[12];
    int64_t q0;
    int64_t pad;
};
static_assert(sizeof(PathStage) == 112, "PathStage layout");

}  // namespace pt
