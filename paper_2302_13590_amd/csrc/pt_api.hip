// Host side of libpt: argument validation, handles, device memory, launches.
// Implements the C ABI declared in include/pt.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "pt.h"
#include "pt_internal.h"

using namespace pt;

// Scratch of the allocation-free entry point (pt_track_noalloc), one copy per device.  Host code
// never uses this name as an address: it takes the array's device address once per device with
// hipGetSymbolAddress (scratch_of below).
static __device__ __align__(256) unsigned char scratch[PT_NOALLOC_SCRATCH_BYTES];

static_assert(sizeof(pt_path_record) == sizeof(PathRec) && offsetof(pt_path_record, cell) == offsetof(PathRec, cell) &&
                  offsetof(pt_path_record, face) == offsetof(PathRec, face) && offsetof(pt_path_record, z) == offsetof(PathRec, z),
              "pt_path_record and the kernels' record differ");

// ---------------------------------------------------------------------------------------------
// errors
namespace {

// Message of the last failing call of this thread (a fixed buffer: no call allocates for it).
struct ErrBuf {
    char s[512];
    void clear() { s[0] = 0; }
    const char* c_str() const { return s; }
};
thread_local ErrBuf g_err = {{0}};

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err.s, sizeof g_err.s, fmt, ap);
    va_end(ap);
    return code;
}

int hip_code(hipError_t e) {
    switch (e) {
        case hipErrorOutOfMemory: return PT_ERR_OOM;
        case hipErrorNoDevice:
        case hipErrorInvalidDevice:
        case hipErrorInsufficientDriver: return PT_ERR_NO_DEVICE;
        default: return PT_ERR_DEVICE;
    }
}

#define HIP_TRY(call)                                                                             \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            (void)hipGetLastError();                                                              \
            return fail(hip_code(e_), "%s failed: %s", #call, hipGetErrorString(e_));             \
        }                                                                                         \
    } while (0)

// ---------------------------------------------------------------------------------------------
// handles

constexpr uint32_t kGridMagic = 0x50544744u;  // "PTGD"
constexpr uint32_t kRunMagic = 0x5054524eu;   // "PTRN"

std::mutex g_mu;
std::unordered_set<void*> g_live;

bool take_handle(void* h, uint32_t* magic_out) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_live.find(h);
    if (it == g_live.end()) return false;
    *magic_out = *reinterpret_cast<uint32_t*>(h);
    g_live.erase(it);
    return true;
}

bool is_live(const void* h, uint32_t magic) {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_live.count(const_cast<void*>(h)) && *reinterpret_cast<const uint32_t*>(h) == magic;
}

void add_live(void* h) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_live.insert(h);
}

int current_device(int* dev, int* n_cu) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return fail(PT_ERR_NO_DEVICE, "no HIP device available (%s)",
                    e == hipSuccess ? "device count is 0" : hipGetErrorString(e));
    }
    HIP_TRY(hipGetDevice(dev));
    if (n_cu) HIP_TRY(hipDeviceGetAttribute(n_cu, hipDeviceAttributeMultiprocessorCount, *dev));
    return PT_OK;
}

bool is_fin(double v) { return std::isfinite(v); }

}  // namespace

struct pt_grid {
    uint32_t magic;
    int device;
    bool quad = false;   // a quadtree grid (QuadRec records, boxes, subfaces)
    GridDev gd;
    std::vector<void*> allocs;
};

struct pt_run {
    uint32_t magic;
    int device;
    hipStream_t stream;
    Counters* d_counters = nullptr;
    Counters* h_counters = nullptr;     // pinned
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_done = nullptr;
    hipEvent_t evk0 = nullptr, evk1 = nullptr;   // around the tracking kernel alone
    bool launched = false;
    int sched = 0, layout = 0, block = 0, grid = 0;
    // per-run device tables (batched runs, snapshot times) and their pinned staging
    void* d_tables = nullptr;
    size_t d_tables_bytes = 0;
    void* d_sort = nullptr;             // order [n], ranks [n], buckets [n], histogram, tile sums
    size_t d_sort_bytes = 0;
    void* d_scan = nullptr;             // pathline count pass: tile sums of the offset scan
    size_t d_scan_bytes = 0;
    void* d_recheck = nullptr;          // careful pass: particle and snapshot lists
    size_t d_recheck_bytes = 0;
    int path_pass = 0;                  // 0: no pathline, 1: count pass, 2: record pass
    void* h_tables = nullptr;
    size_t h_tables_bytes = 0;
    // cached graph: [reset counters, track] for one exact set of kernel arguments
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<unsigned char> graph_key;
};

namespace {

std::vector<pt_run*> g_pool;  // released runs kept for reuse (guarded by g_mu)
// Released runs kept: enough for a few dozen calls in flight on one stream (each keeps its
// cached graph, events, counters and ordering buffers); pt_shutdown frees them.
constexpr size_t kPoolMax = 32;

void destroy_run(pt_run* r) {
    if (r->exec) (void)hipGraphExecDestroy(r->exec);
    if (r->graph) (void)hipGraphDestroy(r->graph);
    if (r->ev0) (void)hipEventDestroy(r->ev0);
    if (r->ev1) (void)hipEventDestroy(r->ev1);
    if (r->ev_done) (void)hipEventDestroy(r->ev_done);
    if (r->evk0) (void)hipEventDestroy(r->evk0);
    if (r->evk1) (void)hipEventDestroy(r->evk1);
    if (r->d_counters) (void)hipFree(r->d_counters);
    if (r->h_counters) (void)hipHostFree(r->h_counters);
    if (r->d_tables) (void)hipFree(r->d_tables);
    if (r->h_tables) (void)hipHostFree(r->h_tables);
    if (r->d_sort) (void)hipFree(r->d_sort);
    if (r->d_scan) (void)hipFree(r->d_scan);
    if (r->d_recheck) (void)hipFree(r->d_recheck);
    delete r;
}

int new_run(int device, pt_run** out) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (size_t q = 0; q < g_pool.size(); ++q) {
            if (g_pool[q]->device == device) {
                *out = g_pool[q];
                g_pool.erase(g_pool.begin() + q);
                (*out)->launched = false;
                return PT_OK;
            }
        }
    }
    pt_run* r = new pt_run();
    r->magic = kRunMagic;
    r->device = device;
    hipError_t e = hipMalloc(&r->d_counters, sizeof(Counters));
    if (e == hipSuccess) e = hipHostMalloc(&r->h_counters, sizeof(Counters), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreate(&r->ev0);
    if (e == hipSuccess) e = hipEventCreate(&r->ev1);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&r->ev_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreate(&r->evk0);
    if (e == hipSuccess) e = hipEventCreate(&r->evk1);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        destroy_run(r);
        return fail(hip_code(e), "run allocation failed: %s", hipGetErrorString(e));
    }
    *out = r;
    return PT_OK;
}

int ensure_tables(pt_run* r, size_t bytes) {
    if (bytes <= r->d_tables_bytes) return PT_OK;
    if (r->d_tables) (void)hipFree(r->d_tables);
    if (r->h_tables) (void)hipHostFree(r->h_tables);
    r->d_tables = r->h_tables = nullptr;
    r->d_tables_bytes = r->h_tables_bytes = 0;
    if (r->exec) {
        (void)hipGraphExecDestroy(r->exec);
        (void)hipGraphDestroy(r->graph);
        r->exec = nullptr;
        r->graph = nullptr;
        r->graph_key.clear();
    }
    HIP_TRY(hipMalloc(&r->d_tables, bytes));
    HIP_TRY(hipHostMalloc(&r->h_tables, bytes, hipHostMallocDefault));
    r->d_tables_bytes = r->h_tables_bytes = bytes;
    return PT_OK;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int ensure_sort(pt_run* r, size_t bytes) {
    if (bytes <= r->d_sort_bytes) return PT_OK;
    if (r->d_sort) (void)hipFree(r->d_sort);
    r->d_sort = nullptr;
    r->d_sort_bytes = 0;
    HIP_TRY(hipMalloc(&r->d_sort, bytes));
    r->d_sort_bytes = bytes;
    return PT_OK;
}

int ensure_recheck(pt_run* r, size_t bytes) {
    if (bytes <= r->d_recheck_bytes) return PT_OK;
    if (r->d_recheck) (void)hipFree(r->d_recheck);
    r->d_recheck = nullptr;
    r->d_recheck_bytes = 0;
    HIP_TRY(hipMalloc(&r->d_recheck, bytes));
    r->d_recheck_bytes = bytes;
    return PT_OK;
}

int ensure_scan(pt_run* r, size_t bytes) {
    if (bytes <= r->d_scan_bytes) return PT_OK;
    if (r->d_scan) (void)hipFree(r->d_scan);
    r->d_scan = nullptr;
    r->d_scan_bytes = 0;
    HIP_TRY(hipMalloc(&r->d_scan, bytes));
    r->d_scan_bytes = bytes;
    return PT_OK;
}

// One kernel launch of a run: launched eagerly in order, or as a chain of graph nodes.
struct Launch {
    const void* fn;
    dim3 grid, block;
    void* arg;
    size_t bytes;       // size of *arg
    size_t lds = 0;     // dynamic LDS bytes per block
};

// ---------------------------------------------------------------------------------------------
// grid validation of host-resident inputs (device-resident inputs are checked by k_build)

int check_host_grid(const pt_grid_desc* d) {
    const int64_t nx = d->nx, ny = d->ny, nz = d->nz;
    const int64_t nfx = (nx + 1) * ny * nz, nfy = nx * (ny + 1) * nz, nfz = nx * ny * (nz + 1);
    const int64_t ncell = nx * ny * nz;
    for (int64_t q = 0; q < nfx; ++q)
        if (!is_fin(d->qx[q])) return fail(PT_ERR_INVALID_ARG, "qx[%lld] is not finite", (long long)q);
    for (int64_t q = 0; q < nfy; ++q)
        if (!is_fin(d->qy[q])) return fail(PT_ERR_INVALID_ARG, "qy[%lld] is not finite", (long long)q);
    for (int64_t q = 0; q < nfz; ++q)
        if (!is_fin(d->qz[q])) return fail(PT_ERR_INVALID_ARG, "qz[%lld] is not finite", (long long)q);
    if (d->porosity)
        for (int64_t c = 0; c < ncell; ++c)
            if (!(d->porosity[c] > 0.0) || !is_fin(d->porosity[c]))
                return fail(PT_ERR_INVALID_ARG, "porosity[%lld] must be finite and > 0", (long long)c);
    if (d->flags)
        for (int64_t c = 0; c < ncell; ++c)
            if (d->flags[c] & ~(PT_CELL_ACTIVE | PT_CELL_SINK))
                return fail(PT_ERR_INVALID_ARG, "flags[%lld] has unknown bits", (long long)c);
    if (d->balance_tol >= 0.0) {
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    const int64_t c = (k * ny + j) * nx + i;
                    const int32_t f = d->flags ? d->flags[c] : PT_CELL_ACTIVE;
                    if (!(f & PT_CELL_ACTIVE) || (f & PT_CELL_SINK)) continue;
                    const int64_t fx = (k * ny + j) * (nx + 1) + i;
                    const int64_t fy = (k * (ny + 1) + j) * nx + i;
                    const int64_t fz = (k * ny + j) * nx + i;
                    const double q[6] = {d->qx[fx], d->qx[fx + 1], d->qy[fy], d->qy[fy + nx],
                                         d->qz[fz], d->qz[fz + nx * ny]};
                    const double net = (q[0] - q[1]) + (q[2] - q[3]) + (q[4] - q[5]);
                    double gross = 0.0;
                    for (double v : q) gross += std::fabs(v);
                    if (std::fabs(net) > d->balance_tol * gross)
                        return fail(PT_ERR_UNBALANCED,
                                    "cell (%lld,%lld,%lld): net flow %.3e exceeds %.3e of %.3e",
                                    (long long)i, (long long)j, (long long)k, net, d->balance_tol, gross);
                }
    }
    return PT_OK;
}

void free_grid(pt_grid* g) {
    for (void* p : g->allocs) (void)hipFree(p);
    delete g;
}

// Launch one kernel through the HIP module-less API.
hipError_t launch(const void* fn, dim3 grid, dim3 block, void* arg, size_t lds, hipStream_t s) {
    void* args[] = {arg};
    return hipLaunchKernel(fn, grid, block, args, lds, s);
}


// ---------------------------------------------------------------------------------------------
// pt_track and pt_track_noalloc share the argument checks, the launch plan (kernel, shape,
// table and ordering-buffer layout), the binding of the kernel arguments to device buffers and
// the launch sequence; they differ in where those buffers come from.

// Checks every argument of a tracking call (no device work); *dev and *n_cu describe the
// current device.
int check_track_args(const pt_grid* const* grids, int32_t n_grids, const pt_particles* p, const pt_track_opts* o,
                     int* dev, int* n_cu) {
    if (!grids || n_grids < 1) return fail(PT_ERR_INVALID_ARG, "need at least one grid");
    if (n_grids > 4096) return fail(PT_ERR_UNSUPPORTED, "at most 4096 grids per call");
    for (int32_t q = 0; q < n_grids; ++q)
        if (!grids[q] || !is_live(grids[q], kGridMagic))
            return fail(PT_ERR_BAD_HANDLE, "grids[%d] is not a live grid handle", q);
    if (!p || !o) return fail(PT_ERR_INVALID_ARG, "particles and options must not be NULL");
    if (p->n < 0) return fail(PT_ERR_INVALID_ARG, "n must be >= 0");
    if (p->n >= (int64_t(1) << 31)) return fail(PT_ERR_UNSUPPORTED, "at most 2^31 - 1 particles per call");
    if (p->n > 0 && (!p->cell || !p->xi || !p->eta || !p->zeta || !p->t || !p->status || !p->ncross ||
                     !p->path_hash))
        return fail(PT_ERR_INVALID_ARG, "a particle state array is NULL");
    if (o->mode != PT_ENDPOINT && o->mode != PT_TIMESERIES && o->mode != PT_PATHLINE)
        return fail(PT_ERR_INVALID_ARG, "bad mode");
    if (o->precision != PT_FP64 && o->precision != PT_MIXED) return fail(PT_ERR_INVALID_ARG, "bad precision");
    if (o->schedule < PT_SCHED_AUTO || o->schedule > PT_SCHED_PERSISTENT)
        return fail(PT_ERR_INVALID_ARG, "bad schedule");
    if (o->layout < PT_LAYOUT_AUTO || o->layout > PT_LAYOUT_CELL) return fail(PT_ERR_INVALID_ARG, "bad layout");
    if (o->direction != 1 && o->direction != -1) return fail(PT_ERR_INVALID_ARG, "direction must be +1 or -1");
    if (o->stop_at_sink != 0 && o->stop_at_sink != 1) return fail(PT_ERR_INVALID_ARG, "stop_at_sink must be 0 or 1");
    if (std::isnan(o->t_max)) return fail(PT_ERR_INVALID_ARG, "t_max is NaN");
    if (o->max_steps < 1 || o->max_steps > INT32_MAX)
        return fail(PT_ERR_INVALID_ARG, "max_steps must be in [1, 2^31-1]");
    if (o->block != 0 && (o->block < 64 || o->block > 1024 || o->block % 64))
        return fail(PT_ERR_INVALID_ARG, "block must be 0 or a multiple of 64 in [64, 1024]");
    if (o->block > 256) return fail(PT_ERR_UNSUPPORTED, "block > 256 exceeds the kernels' launch bounds");
    if (o->refill < 0 || o->refill > 64) return fail(PT_ERR_INVALID_ARG, "refill must be in [0, 64]");
    if (o->sort < PT_SORT_AUTO || o->sort > PT_SORT_CELL) return fail(PT_ERR_INVALID_ARG, "bad sort");
    if (o->steps_per_refill < 0 || o->blocks_per_cu < 0 || o->chunk < 0)
        return fail(PT_ERR_INVALID_ARG, "steps_per_refill, blocks_per_cu and chunk must be >= 0");
    if (o->precision == PT_MIXED && o->layout == PT_LAYOUT_FACES)
        return fail(PT_ERR_UNSUPPORTED, "mixed precision needs the packed cell layout");
    const bool ts = o->mode == PT_TIMESERIES;
    if (ts) {
        if (o->n_snap < 1 || !o->snap_times || !o->snap_xyz)
            return fail(PT_ERR_INVALID_ARG, "timeseries needs snap_times, n_snap >= 1 and snap_xyz");
        for (int32_t q = 0; q < o->n_snap; ++q) {
            if (!is_fin(o->snap_times[q])) return fail(PT_ERR_INVALID_ARG, "snap_times[%d] is not finite", q);
            if (q && o->snap_times[q] < o->snap_times[q - 1])
                return fail(PT_ERR_INVALID_ARG, "snap_times must be non-decreasing");
        }
    }
    const bool path = o->mode == PT_PATHLINE;
    const bool path_count = path && o->path_count_only;
    if (path) {
        if (o->path_count_only != 0 && o->path_count_only != 1)
            return fail(PT_ERR_INVALID_ARG, "path_count_only must be 0 or 1");
        if (!o->path_offsets) return fail(PT_ERR_INVALID_ARG, "pathline needs path_offsets [n+1]");
        if (!path_count) {
            if (o->path_cap < 0) return fail(PT_ERR_INVALID_ARG, "path_cap must be >= 0");
            if (o->path_cap > 0 && !o->path_records)
                return fail(PT_ERR_INVALID_ARG, "the record pass needs path_records");
        }
    }
    const int32_t n_groups = p->n_groups;
    if (n_groups < 0) return fail(PT_ERR_INVALID_ARG, "n_groups must be >= 0");
    const bool transient = o->n_tsteps != 0;
    bool quad = false;
    for (int32_t q = 0; q < n_grids; ++q) quad = quad || grids[q]->quad;
    if (quad) {
        if (n_grids != 1 || n_groups != 0 || transient)
            return fail(PT_ERR_UNSUPPORTED, "a quadtree grid is tracked alone (one grid, no groups, steady flow)");
        if (o->precision != PT_FP64) return fail(PT_ERR_UNSUPPORTED, "quadtree grids are tracked in FP64");
        if (o->layout == PT_LAYOUT_FACES) return fail(PT_ERR_UNSUPPORTED, "quadtree grids use the packed layout");
    }
    if (transient) {
        if (o->n_tsteps < 0 || !o->tstep_end) return fail(PT_ERR_INVALID_ARG, "transient flow needs n_tsteps >= 1 and tstep_end");
        if (o->n_tsteps != n_grids) return fail(PT_ERR_INVALID_ARG, "transient flow needs one grid per time step");
        if (n_groups != 0) return fail(PT_ERR_UNSUPPORTED, "transient flow with particle groups");
        if (o->direction != 1) return fail(PT_ERR_UNSUPPORTED, "transient flow is tracked forward only");
        for (int32_t q = 0; q < o->n_tsteps; ++q) {
            if (std::isnan(o->tstep_end[q])) return fail(PT_ERR_INVALID_ARG, "tstep_end[%d] is NaN", q);
            if (q && !(o->tstep_end[q] > o->tstep_end[q - 1]))
                return fail(PT_ERR_INVALID_ARG, "tstep_end must be strictly increasing");
            const GridDev& a = grids[q]->gd;
            const GridDev& b = grids[0]->gd;
            if (a.nx != b.nx || a.ny != b.ny || a.nz != b.nz || a.dx != b.dx || a.dy != b.dy || a.dz != b.dz ||
                a.x0 != b.x0 || a.y0 != b.y0 || a.z0 != b.z0)
                return fail(PT_ERR_INVALID_ARG, "the grids of the time steps must have the same geometry");
        }
    } else if (n_grids > 1 && n_groups == 0) {
        return fail(PT_ERR_INVALID_ARG, "several grids need particle groups");
    }
    if (n_groups > 0) {
        if (!p->group_offsets || !p->group_grid)
            return fail(PT_ERR_INVALID_ARG, "group_offsets and group_grid must not be NULL");
        if (p->group_offsets[0] != 0 || p->group_offsets[n_groups] != p->n)
            return fail(PT_ERR_INVALID_ARG, "group_offsets must start at 0 and end at n");
        for (int32_t q = 0; q < n_groups; ++q) {
            if (p->group_offsets[q + 1] < p->group_offsets[q])
                return fail(PT_ERR_INVALID_ARG, "group_offsets must be non-decreasing");
            if (p->group_grid[q] < 0 || p->group_grid[q] >= n_grids)
                return fail(PT_ERR_INVALID_ARG, "group_grid[%d] out of range", q);
        }
    }
    int rc = current_device(dev, n_cu);
    if (rc != PT_OK) return rc;
    for (int32_t q = 0; q < n_grids; ++q)
        if (grids[q]->device != *dev)
            return fail(PT_ERR_INVALID_ARG, "grids[%d] lives on device %d, current is %d", q, grids[q]->device, *dev);
    return PT_OK;
}

// What one tracking call launches, and the layout of the device buffers it needs.
struct Plan {
    KernelKey key;
    const void* fn = nullptr;
    bool ts = false, path = false, path_count = false, transient = false, batched = false, multi = false;
    bool sort = false;
    int32_t n_groups = 0;
    int block = 0, grid = 0;
    size_t lds = 0;                 // dynamic LDS of the tracking kernel
    // per-call tables (256-byte aligned segments): grid views, group table, snapshot times, time
    // step ends, first global cell of each grid (batched ordering)
    size_t b_grids = 0, b_offs = 0, b_gg = 0, b_snap = 0, b_tstep = 0, b_base = 0, tables = 0;
    // ordering by starting cell: order, bucket, super-bucket-ordered buckets and indices [n] each,
    // the tiles' super-bucket counts, scan tile sums
    int32_t shift = 0, nbuckets = 0, fine = 0, nsuper = 0, ptiles = 0, ntiles = 0;
    int64_t ncnt = 0;
    size_t b_order = 0, b_cnt = 0, sort_bytes = 0;
    // pathline count pass: tile sums of the offset scan
    int64_t scan_ntiles = 0;
    size_t scan_bytes = 0;
    // careful pass (FP64): capacity of the particle list and its bytes
    int32_t recheck_cap = 0;
    size_t recheck_bytes = 0;
};

// The plan of a checked call.  `sort_budget`: the largest ordering buffer the caller can
// provide; PT_SORT_AUTO orders only when it fits, PT_SORT_CELL beyond it is refused.
int make_plan(const pt_grid* const* grids, int32_t n_grids, const pt_particles* p, const pt_track_opts* o,
              int n_cu, size_t sort_budget, int64_t recheck_max, Plan* pl) {
    Plan& P = *pl;
    P.ts = o->mode == PT_TIMESERIES;
    P.path = o->mode == PT_PATHLINE;
    P.path_count = P.path && o->path_count_only;
    P.transient = o->n_tsteps != 0;
    P.n_groups = p->n_groups;
    P.batched = P.n_groups > 0;
    P.multi = P.batched || P.transient;   // the kernels that read a per-lane grid
    bool quad = false;
    for (int32_t q = 0; q < n_grids; ++q) quad = quad || grids[q]->quad;
    P.key.precision = o->precision == PT_MIXED ? PMIX : P64;
    P.key.layout = quad ? L_QUAD : (o->layout == PT_LAYOUT_FACES ? L_FACES : L_CELL);
    P.key.out = P.ts ? O_SERIES : (P.path ? O_PATH : O_END);
    P.key.batched = P.multi ? 1 : 0;
    P.key.sched = o->schedule == PT_SCHED_STATIC ? S_STATIC : S_PERSISTENT;
    P.fn = track_kernel(P.key);
    P.block = o->block ? o->block : 256;
    if (P.key.sched == S_STATIC) {
        // a multiple of 8 chunks of blocks: chunks are dealt to the dies round robin
        const int64_t nb = std::max<int64_t>(1, (p->n + P.block - 1) / P.block);
        const int64_t m = (int64_t)kXcd * kDieChunk;
        P.grid = (int)((nb + m - 1) / m * m);
    } else {
        int per_cu = o->blocks_per_cu;
        if (!per_cu) {
            int occ = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, P.fn, P.block, 0) != hipSuccess || occ < 1) {
                (void)hipGetLastError();
                occ = 2;
            }
            per_cu = occ;
        }
        P.grid = std::max(1, n_cu * per_cu);
        const int64_t need = (p->n + P.block - 1) / P.block;
        if (need < P.grid) P.grid = (int)std::max<int64_t>(1, need);
    }
    P.b_grids = P.multi ? align_up(sizeof(GridDev) * n_grids, 256) : 0;
    P.b_offs = P.batched ? align_up(sizeof(int64_t) * (P.n_groups + 1), 256) : 0;
    P.b_gg = P.batched ? align_up(sizeof(int32_t) * P.n_groups, 256) : 0;
    P.b_snap = P.ts ? align_up(sizeof(double) * o->n_snap, 256) : 0;
    P.b_tstep = P.transient ? align_up(sizeof(double) * o->n_tsteps, 256) : 0;
    const bool want_sort = o->sort == PT_SORT_CELL || (o->sort == PT_SORT_AUTO && p->n >= (1 << 16));
    if (want_sort) {
        int64_t cells = 0;
        for (int32_t q = 0; q < (P.batched ? n_grids : 1); ++q)
            cells += (int64_t)grids[q]->gd.nx * grids[q]->gd.ny * grids[q]->gd.nz;
        int shift = 0;
        while ((cells >> shift) >= kMaxBuckets) ++shift;
        P.shift = shift;
        P.nbuckets = (int32_t)(cells >> shift) + 1;
        // about 512 super-buckets (one block each in the second level: two resident per CU) of at
        // most kFineMax buckets
        P.fine = (int32_t)std::min<int64_t>(kFineMax, std::max<int64_t>(1, (P.nbuckets + 511) / 512));
        P.nsuper = (P.nbuckets + P.fine - 1) / P.fine;
        P.ptiles = (int32_t)((p->n + kSortTile - 1) / kSortTile);
        P.ncnt = (int64_t)P.nsuper * P.ptiles;
        P.ntiles = (int32_t)((P.ncnt + kScanTile - 1) / kScanTile);
        P.b_order = align_up(sizeof(int32_t) * (size_t)p->n, 256);
        P.b_cnt = align_up(sizeof(unsigned) * (size_t)P.ncnt, 256);
        P.sort_bytes = 4 * P.b_order + P.b_cnt + sizeof(unsigned) * (size_t)P.ntiles;
        P.sort = P.sort_bytes <= sort_budget;
        if (!P.sort && o->sort == PT_SORT_CELL)
            return fail(PT_ERR_UNSUPPORTED, "ordering %lld particles needs %zu bytes of buffer, above the %zu available",
                        (long long)p->n, P.sort_bytes, sort_budget);
        if (!P.sort) P.sort_bytes = 0;
    }
    P.b_base = (P.sort && P.batched) ? align_up(sizeof(int64_t) * n_grids, 256) : 0;
    P.tables = P.b_grids + P.b_offs + P.b_gg + P.b_snap + P.b_tstep + P.b_base;
    if (P.path_count) {
        P.scan_ntiles = (p->n + kScanTile - 1) / kScanTile;
        P.scan_bytes = sizeof(int64_t) * (size_t)std::max<int64_t>(1, P.scan_ntiles);
    }
    if (P.key.precision == P64 && p->n > 0) {
        P.recheck_cap = (int32_t)std::min<int64_t>(p->n, recheck_max);
        P.recheck_bytes = align_up(sizeof(int32_t) * (size_t)P.recheck_cap, 256);
    }
    // the static timeseries kernels on packed layouts keep one deferred-snapshot slot per thread
    // in dynamic LDS; the pathline record pass stages each lane's records there
    const bool snap_slots = P.key.out == O_SERIES && P.key.sched == S_STATIC && P.key.layout != L_FACES;
    const size_t slot = P.key.precision == P64 ? sizeof(SnapJob<double>) : sizeof(SnapJob<float>);
    const bool stage = P.path && !P.path_count && (reinterpret_cast<uintptr_t>(o->path_records) % 64 == 0);
    P.lds = snap_slots ? slot * (size_t)P.block : (stage ? sizeof(PathStage) * (size_t)P.block : 0);
    return PT_OK;
}

// The bytes of the per-call tables, segment by segment: put(offset, source, bytes).  Offsets
// follow the plan's layout; the gaps between segments are never read.
template <class Put>
void write_tables(const Plan& P, const pt_grid* const* grids, int32_t n_grids, const pt_particles* p,
                  const pt_track_opts* o, Put&& put) {
    size_t off = 0;
    if (P.multi) {
        for (int32_t q = 0; q < n_grids; ++q) put(off + sizeof(GridDev) * q, &grids[q]->gd, sizeof(GridDev));
        off += P.b_grids;
    }
    if (P.batched) {
        put(off, p->group_offsets, sizeof(int64_t) * (P.n_groups + 1));
        off += P.b_offs;
        put(off, p->group_grid, sizeof(int32_t) * P.n_groups);
        off += P.b_gg;
    }
    if (P.ts) {
        put(off, o->snap_times, sizeof(double) * o->n_snap);
        off += P.b_snap;
    }
    if (P.transient) {
        put(off, o->tstep_end, sizeof(double) * o->n_tsteps);
        off += P.b_tstep;
    }
    if (P.b_base) {
        int64_t acc = 0;
        for (int32_t q = 0; q < n_grids; ++q) {
            put(off + sizeof(int64_t) * q, &acc, sizeof acc);
            acc += (int64_t)grids[q]->gd.nx * grids[q]->gd.ny * grids[q]->gd.nz;
        }
    }
}

// Kernel arguments of a call whose buffers are at d_tables (P.tables bytes), d_sort
// (P.sort_bytes), d_scan (P.scan_bytes) and d_counters.
void bind_params(const Plan& PL, const pt_grid* const* grids, int32_t n_grids, const pt_particles* p,
                 const pt_track_opts* o, unsigned char* d_tables, unsigned char* d_sort, int64_t* d_scan,
                 unsigned char* d_recheck, Counters* d_counters, TrackParams& P, SortParams& SP, ScanParams& SC) {
    std::memset(&P, 0, sizeof P);
    std::memset(&SP, 0, sizeof SP);
    std::memset(&SC, 0, sizeof SC);
    size_t off = 0;
    if (PL.multi) {
        P.grids = reinterpret_cast<const GridDev*>(d_tables + off);
        off += PL.b_grids;
    }
    if (PL.batched) {
        P.group_offsets = reinterpret_cast<const int64_t*>(d_tables + off);
        off += PL.b_offs;
        P.group_grid = reinterpret_cast<const int32_t*>(d_tables + off);
        off += PL.b_gg;
    }
    if (PL.ts) {
        P.snap_times = reinterpret_cast<const double*>(d_tables + off);
        off += PL.b_snap;
    }
    if (PL.transient) {
        P.tstep_end = reinterpret_cast<const double*>(d_tables + off);
        off += PL.b_tstep;
    }
    P.n = p->n;
    P.cell = p->cell;
    P.xi = p->xi;
    P.eta = p->eta;
    P.zeta = p->zeta;
    P.t = p->t;
    P.status = p->status;
    P.ncross = p->ncross;
    P.hash = p->path_hash;
    P.n_groups = PL.n_groups;
    P.n_grids = n_grids;
    P.n_tsteps = PL.transient ? o->n_tsteps : 0;
    P.g0 = grids[0]->gd;
    P.t_max = o->t_max;
    P.max_steps = o->max_steps;
    P.sign = o->direction < 0 ? -1.0 : 1.0;
    P.stop_at_sink = o->stop_at_sink;
    P.n_snap = PL.ts ? o->n_snap : 0;
    P.snap_xyz = PL.ts ? o->snap_xyz : nullptr;
    P.out_xyz = o->out_xyz;
    P.counters = d_counters;
    if (PL.recheck_cap > 0) {
        P.recheck_pid = reinterpret_cast<int32_t*>(d_recheck);
        P.recheck_cap = PL.recheck_cap;
    }
    P.refill = o->refill ? o->refill : 1;
    P.steps_per_refill = o->steps_per_refill ? o->steps_per_refill : 1;
    P.chunk = o->chunk ? o->chunk : 64;
    if (PL.path) {
        P.path_off = o->path_offsets;
        P.path_count = PL.path_count ? 1 : 0;
        if (!PL.path_count) {
            P.path_cap = o->path_cap;
            P.path_rec = reinterpret_cast<PathRec*>(o->path_records);
            // staged record writes need 64-byte aligned segments of the record array
            P.path_stage = (reinterpret_cast<uintptr_t>(o->path_records) % 64 == 0) ? 1 : 0;
        }
    }
    if (PL.path_count) {   // the per-particle counts become offsets (scan of path_offsets[1..n])
        SC.v = o->path_offsets + 1;
        SC.n = p->n;
        SC.ntiles = PL.scan_ntiles;
        SC.head = o->path_offsets;
        SC.part = d_scan;
    }
    if (PL.sort) {
        SP.nbuckets = PL.nbuckets;
        SP.shift = PL.shift;
        SP.fine = PL.fine;
        SP.nsuper = PL.nsuper;
        SP.ptiles = PL.ptiles;
        SP.ncnt = PL.ncnt;
        SP.ntiles = PL.ntiles;
        SP.n = p->n;
        SP.cell = p->cell;
        SP.status = p->status;
        SP.n_groups = PL.batched ? PL.n_groups : 0;
        SP.group_offsets = P.group_offsets;
        SP.group_grid = P.group_grid;
        SP.grid_base = PL.batched ? reinterpret_cast<const int64_t*>(d_tables + (PL.tables - PL.b_base)) : nullptr;
        SP.order = reinterpret_cast<int32_t*>(d_sort);
        SP.bucket = reinterpret_cast<unsigned*>(d_sort + PL.b_order);
        SP.sbucket = reinterpret_cast<unsigned*>(d_sort + 2 * PL.b_order);
        SP.sidx = reinterpret_cast<int32_t*>(d_sort + 3 * PL.b_order);
        SP.cnt = reinterpret_cast<unsigned*>(d_sort + 4 * PL.b_order);
        SP.part = reinterpret_cast<unsigned*>(d_sort + 4 * PL.b_order + PL.b_cnt);
        P.order = SP.order;
    }
}

// The kernels of one call, in order (fixed capacity: no host allocation).
struct LaunchSeq {
    Launch v[16];
    int n = 0;
    int track_at = -1;   // index of the tracking kernel
    void push(const void* fn, dim3 grid, dim3 block, void* arg, size_t bytes, size_t lds = 0) {
        v[n].fn = fn;
        v[n].grid = grid;
        v[n].block = block;
        v[n].arg = arg;
        v[n].bytes = bytes;
        v[n].lds = lds;
        ++n;
    }
};

// Counter reset, ordering sort, tracking kernel, pathline offset scan.  The argument blocks
// are referenced, not copied: they must outlive the launches (or graph construction).
void build_seq(const Plan& PL, int64_t n, Counters** cptr, TrackParams* P, SortParams* SP, ScanParams* SC,
               LaunchSeq& seq) {
    seq.push(reset_kernel(), dim3(1), dim3(64), cptr, sizeof *cptr);
    if (n > 0) {
        if (PL.sort) {
            const unsigned nt = (unsigned)SP->ptiles;
            seq.push(sort_tiles_kernel(), dim3(nt), dim3(256), SP, sizeof *SP);
            seq.push(sort_scan_tiles_kernel(), dim3((unsigned)SP->ntiles), dim3(kScanBlock), SP, sizeof *SP);
            seq.push(sort_scan_partials_kernel(), dim3(1), dim3(kScanBlock), SP, sizeof *SP);
            if (SP->ntiles > 1)
                seq.push(sort_scan_add_kernel(), dim3((unsigned)SP->ntiles), dim3(kScanBlock), SP, sizeof *SP);
            seq.push(sort_spread_kernel(), dim3(nt), dim3(256), SP, sizeof *SP);
            seq.push(sort_fine_kernel(), dim3((unsigned)SP->nsuper), dim3(kFineBlock), SP, sizeof *SP);
        }
        seq.track_at = seq.n;
        seq.push(PL.fn, dim3(PL.grid), dim3(PL.block), P, sizeof *P, PL.lds);
        if (PL.recheck_cap > 0) {
            // careful pass: a fixed grid that strides over the (usually empty) lists
            const unsigned cb = 64;
            const unsigned ct = (unsigned)std::min<int64_t>(256, (PL.recheck_cap + cb - 1) / cb);
            seq.push(careful_kernel(PL.key), dim3(ct), dim3(cb), P, sizeof *P,
                     P->path_stage ? sizeof(PathStage) * cb : 0);
        }
        if (PL.path_count)
            seq.push(scan_tiles_kernel(), dim3((unsigned)SC->ntiles), dim3(kScanBlock), SC, sizeof *SC);
    }
    if (PL.path_count) {
        seq.push(scan_partials_kernel(), dim3(1), dim3(kScanBlock), SC, sizeof *SC);
        if (SC->ntiles > 1) seq.push(scan_add_kernel(), dim3((unsigned)SC->ntiles), dim3(kScanBlock), SC, sizeof *SC);
    }
}

// ---------------------------------------------------------------------------------------------
// Scratch of the allocation-free entry point: one array per device, in the library's code
// object, holding the counter block, the per-call tables, the ordering buffers and the
// pathline scan's tile sums of one call at a time.  Its device address is taken once per
// device (hipGetSymbolAddress, with that device current) and used for every access from the
// host: the array's own name is only a host-side stand-in.
constexpr size_t kScratchBytes = (size_t)PT_NOALLOC_SCRATCH_BYTES;
constexpr size_t kScratchCounters = 0;                       // Counters (256 B)
constexpr size_t kScratchTables = 256;                       // per-call tables, up to kScratchTablesMax
constexpr size_t kScratchTablesMax = (size_t)64 << 10;
constexpr size_t kScratchScan = kScratchTables + kScratchTablesMax;   // pathline tile sums
constexpr size_t kScratchScanMax = (size_t)64 << 10;
constexpr size_t kScratchRecheck = kScratchScan + kScratchScanMax;    // careful pass particle list
constexpr int64_t kScratchRecheckTracks = (int64_t)1 << 18;           //   (1 MiB)
constexpr size_t kScratchRecheckMax = sizeof(int32_t) * kScratchRecheckTracks;
constexpr size_t kScratchSort = kScratchRecheck + kScratchRecheckMax; // ordering buffers: the rest
static_assert(sizeof(Counters) <= kScratchTables, "counter block fits its scratch slot");
static_assert(kScratchSort < kScratchBytes, "scratch layout");


constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (taken on the first call on the device).
int scratch_of(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(PT_ERR_UNSUPPORTED, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(hip_code(e), "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = static_cast<unsigned char*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return PT_OK;
}

// Writes the per-call tables into device memory through small fill kernels whose arguments
// carry the bytes: no staging buffer and no copy from host memory that could still be in use.
struct TableFill {
    unsigned char* dst;   // device table region
    FillArgs A;
    hipStream_t s;
    hipError_t err = hipSuccess;
    void flush() {
        if (A.nbytes && err == hipSuccess) err = launch(fill_kernel(), dim3(1), dim3(256), &A, 0, s);
        A.nbytes = 0;
    }
    void put(size_t off, const void* src, size_t bytes) {
        const unsigned char* b = static_cast<const unsigned char*>(src);
        while (bytes) {
            if (A.nbytes && (A.dst + A.nbytes != dst + off || A.nbytes == sizeof A.bytes)) flush();
            if (!A.nbytes) A.dst = dst + off;
            const size_t take = std::min(bytes, sizeof A.bytes - (size_t)A.nbytes);
            std::memcpy(A.bytes + A.nbytes, b, take);
            A.nbytes += (uint32_t)take;
            b += take;
            off += take;
            bytes -= take;
        }
    }
};

}  // namespace

// =============================================================================================
extern "C" {

int pt_version(void) { return 104; }

const char* pt_last_error(void) { return g_err.c_str(); }

void pt_default_opts(pt_track_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->mode = PT_ENDPOINT;
    o->precision = PT_FP64;
    o->schedule = PT_SCHED_AUTO;
    o->layout = PT_LAYOUT_AUTO;
    o->direction = 1;
    o->stop_at_sink = 1;
    o->t_max = HUGE_VAL;
    o->max_steps = 1 << 20;
}

int pt_load_grid(const pt_grid_desc* d, void* hip_stream, pt_grid** out) {
    g_err.clear();
    if (!d || !out) return fail(PT_ERR_INVALID_ARG, "desc and out must not be NULL");
    *out = nullptr;
    if (d->nx < 1 || d->ny < 1 || d->nz < 1)
        return fail(PT_ERR_INVALID_ARG, "nx, ny, nz must be >= 1 (got %d, %d, %d)", d->nx, d->ny, d->nz);
    const int64_t ncell = (int64_t)d->nx * d->ny * d->nz;
    if (ncell >= (int64_t(1) << 31) || (int64_t)(d->nx + 1) * d->ny * d->nz >= (int64_t(1) << 31))
        return fail(PT_ERR_UNSUPPORTED, "grid too large: %lld cells (limit 2^31)", (long long)ncell);
    if (!(d->dx > 0) || !(d->dy > 0) || !(d->dz > 0) || !is_fin(d->dx) || !is_fin(d->dy) || !is_fin(d->dz))
        return fail(PT_ERR_INVALID_ARG, "dx, dy, dz must be finite and > 0");
    if (!is_fin(d->x0) || !is_fin(d->y0) || !is_fin(d->z0))
        return fail(PT_ERR_INVALID_ARG, "x0, y0, z0 must be finite");
    if (!d->qx || !d->qy || !d->qz) return fail(PT_ERR_INVALID_ARG, "qx, qy, qz must not be NULL");
    if (!d->porosity && (!(d->porosity_scalar > 0) || !is_fin(d->porosity_scalar)))
        return fail(PT_ERR_INVALID_ARG, "porosity_scalar must be finite and > 0 when porosity is NULL");
    if (d->mem != PT_MEM_HOST && d->mem != PT_MEM_DEVICE)
        return fail(PT_ERR_INVALID_ARG, "mem must be PT_MEM_HOST or PT_MEM_DEVICE");
    if (std::isnan(d->balance_tol)) return fail(PT_ERR_INVALID_ARG, "balance_tol is NaN");
    if (d->mem == PT_MEM_HOST) {
        int rc = check_host_grid(d);
        if (rc != PT_OK) return rc;
    }
    int dev = 0;
    int rc = current_device(&dev, nullptr);
    if (rc != PT_OK) return rc;

    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const int64_t nx = d->nx, ny = d->ny, nz = d->nz;
    const size_t bx = sizeof(double) * (nx + 1) * ny * nz, by = sizeof(double) * nx * (ny + 1) * nz,
                 bz = sizeof(double) * nx * ny * (nz + 1), bc = sizeof(double) * ncell,
                 bf = sizeof(int32_t) * ncell;
    pt_grid* g = new pt_grid();
    g->magic = kGridMagic;
    g->device = dev;
    auto alloc = [&](size_t bytes, void** p) -> hipError_t {
        hipError_t e = hipMalloc(p, bytes);
        if (e == hipSuccess) g->allocs.push_back(*p);
        return e;
    };
    void *qx, *qy, *qz, *por = nullptr, *flags, *r64, *r32, *err;
    hipError_t e = alloc(bx, &qx);
    if (e == hipSuccess) e = alloc(by, &qy);
    if (e == hipSuccess) e = alloc(bz, &qz);
    if (e == hipSuccess && d->porosity) e = alloc(bc, &por);
    if (e == hipSuccess) e = alloc(bf, &flags);
    if (e == hipSuccess) e = alloc(sizeof(CellRec64) * ncell, &r64);
    if (e == hipSuccess) e = alloc(sizeof(CellRec32) * ncell, &r32);
    if (e == hipSuccess) e = alloc(4 * sizeof(int), &err);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_grid(g);
        return fail(hip_code(e), "grid allocation failed: %s", hipGetErrorString(e));
    }
    const hipMemcpyKind kind = d->mem == PT_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    e = hipMemcpyAsync(qx, d->qx, bx, kind, s);
    if (e == hipSuccess) e = hipMemcpyAsync(qy, d->qy, by, kind, s);
    if (e == hipSuccess) e = hipMemcpyAsync(qz, d->qz, bz, kind, s);
    if (e == hipSuccess && d->porosity) e = hipMemcpyAsync(por, d->porosity, bc, kind, s);
    if (e == hipSuccess && d->flags) e = hipMemcpyAsync(flags, d->flags, bf, kind, s);
    if (e == hipSuccess) e = hipMemsetAsync(err, 0, 4 * sizeof(int), s);
    if (e == hipSuccess && !d->flags) {
        std::vector<int32_t> ones(ncell, PT_CELL_ACTIVE);
        e = hipMemcpyAsync(flags, ones.data(), bf, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    GridDev& gd = g->gd;
    gd.rec64 = static_cast<CellRec64*>(r64);
    gd.rec32 = static_cast<CellRec32*>(r32);
    gd.qx = static_cast<double*>(qx);
    gd.qy = static_cast<double*>(qy);
    gd.qz = static_cast<double*>(qz);
    gd.por = static_cast<double*>(por);
    gd.flags = static_cast<int32_t*>(flags);
    gd.por_scalar = d->porosity ? 0.0 : d->porosity_scalar;
    gd.dx = d->dx; gd.dy = d->dy; gd.dz = d->dz;
    gd.x0 = d->x0; gd.y0 = d->y0; gd.z0 = d->z0;
    gd.V = (d->dx * d->dy) * d->dz;
    gd.nx = d->nx; gd.ny = d->ny; gd.nz = d->nz; gd.plane = d->nx * d->ny;
    BuildParams B;
    B.g = gd;
    B.rec64 = static_cast<CellRec64*>(r64);
    B.rec32 = static_cast<CellRec32*>(r32);
    B.balance_tol = d->balance_tol;
    B.err = static_cast<int*>(err);
    if (e == hipSuccess)
        e = launch(build_kernel(), dim3((unsigned)((ncell + 255) / 256)), dim3(256), &B, 0, s);
    int herr[4] = {0, 0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(herr, err, sizeof herr, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_grid(g);
        return fail(hip_code(e), "grid upload failed: %s", hipGetErrorString(e));
    }
    if (herr[0] || herr[1] || herr[2] || herr[3]) {
        free_grid(g);
        if (herr[0]) return fail(PT_ERR_INVALID_ARG, "a face flow is not finite");
        if (herr[1]) return fail(PT_ERR_INVALID_ARG, "a porosity is not finite and > 0");
        if (herr[2]) return fail(PT_ERR_INVALID_ARG, "a cell flag has unknown bits");
        return fail(PT_ERR_UNBALANCED, "a cell's face flows do not balance within balance_tol");
    }
    add_live(g);
    *out = g;
    return PT_OK;
}

int pt_load_quad_grid(const pt_quad_desc* d, void* hip_stream, pt_grid** out) {
    g_err.clear();
    if (!out) return fail(PT_ERR_INVALID_ARG, "out must not be NULL");
    *out = nullptr;
    if (!d) return fail(PT_ERR_INVALID_ARG, "desc must not be NULL");
    if (d->mem != PT_MEM_HOST) return fail(PT_ERR_UNSUPPORTED, "quadtree grids are loaded from host memory");
    if (d->ncell < 1 || d->nsub < 0) return fail(PT_ERR_INVALID_ARG, "ncell must be >= 1 and nsub >= 0");
    if (!d->box || !d->sub_off) return fail(PT_ERR_INVALID_ARG, "box and sub_off must not be NULL");
    if (d->nsub > 0 && (!d->sub_nb || !d->sub_q || !d->sub_lo || !d->sub_hi))
        return fail(PT_ERR_INVALID_ARG, "the subface arrays must not be NULL");
    if (!d->porosity && (!(d->porosity_scalar > 0) || !is_fin(d->porosity_scalar)))
        return fail(PT_ERR_INVALID_ARG, "porosity_scalar must be finite and > 0 when porosity is NULL");
    if (std::isnan(d->balance_tol)) return fail(PT_ERR_INVALID_ARG, "balance_tol is NaN");
    const int64_t ncell = d->ncell, nsub = d->nsub;
    if (d->sub_off[0] != 0 || d->sub_off[6 * ncell] != nsub)
        return fail(PT_ERR_INVALID_ARG, "sub_off must start at 0 and end at nsub");
    for (int64_t q = 0; q < 6 * ncell; ++q) {
        const int64_t cnt = (int64_t)d->sub_off[q + 1] - d->sub_off[q];
        if (cnt < 0) return fail(PT_ERR_INVALID_ARG, "sub_off must be non-decreasing");
        if (cnt > kMaxSubPerFace) return fail(PT_ERR_UNSUPPORTED, "more than 31 subfaces on one face");
    }
    for (int64_t c = 0; c < ncell; ++c)
        for (int a = 0; a < 3; ++a) {
            const double lo = d->box[6 * c + a], h = d->box[6 * c + 3 + a];
            if (!is_fin(lo) || !is_fin(h) || !(h > 0)) return fail(PT_ERR_INVALID_ARG, "box of cell %lld", (long long)c);
        }
    std::vector<double4> rect((size_t)std::max<int64_t>(1, nsub));
    for (int64_t q = 0; q < nsub; ++q) {
        if (d->sub_nb[q] < -1 || d->sub_nb[q] >= d->ncell)
            return fail(PT_ERR_INVALID_ARG, "sub_nb[%lld] out of range", (long long)q);
        const double lu = d->sub_lo[2 * q], lv = d->sub_lo[2 * q + 1];
        const double hu = d->sub_hi[2 * q], hv = d->sub_hi[2 * q + 1];
        if (!(0.0 <= lu && lu <= hu && hu <= 1.0) || !(0.0 <= lv && lv <= hv && hv <= 1.0))
            return fail(PT_ERR_INVALID_ARG, "subface %lld extent must satisfy 0 <= lo <= hi <= 1", (long long)q);
        rect[q] = make_double4(lu, lv, hu, hv);
    }
    int dev = 0;
    int rc = current_device(&dev, nullptr);
    if (rc != PT_OK) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    pt_grid* g = new pt_grid();
    g->magic = kGridMagic;
    g->device = dev;
    g->quad = true;
    auto alloc = [&](size_t bytes, void** ptr) -> hipError_t {
        hipError_t e = hipMalloc(ptr, bytes);
        if (e == hipSuccess) g->allocs.push_back(*ptr);
        return e;
    };
    const size_t n_sub = (size_t)std::max<int64_t>(1, nsub);
    void *box, *off, *nb, *sq, *sr, *por = nullptr, *flags, *rec, *err;
    hipError_t e = alloc(sizeof(QuadBox) * ncell, &box);
    if (e == hipSuccess) e = alloc(sizeof(int32_t) * (6 * ncell + 1), &off);
    if (e == hipSuccess) e = alloc(sizeof(int32_t) * n_sub, &nb);
    if (e == hipSuccess) e = alloc(sizeof(double) * n_sub, &sq);
    if (e == hipSuccess) e = alloc(sizeof(double4) * n_sub, &sr);
    if (e == hipSuccess && d->porosity) e = alloc(sizeof(double) * ncell, &por);
    if (e == hipSuccess) e = alloc(sizeof(int32_t) * ncell, &flags);
    if (e == hipSuccess) e = alloc(sizeof(QuadRec) * ncell, &rec);
    if (e == hipSuccess) e = alloc(4 * sizeof(int), &err);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_grid(g);
        return fail(hip_code(e), "grid allocation failed: %s", hipGetErrorString(e));
    }
    std::vector<int32_t> ones;
    if (!d->flags) ones.assign((size_t)ncell, PT_CELL_ACTIVE);
    const hipMemcpyKind h2d = hipMemcpyHostToDevice;
    e = hipMemcpyAsync(box, d->box, sizeof(QuadBox) * ncell, h2d, s);
    if (e == hipSuccess) e = hipMemcpyAsync(off, d->sub_off, sizeof(int32_t) * (6 * ncell + 1), h2d, s);
    if (e == hipSuccess && nsub) e = hipMemcpyAsync(nb, d->sub_nb, sizeof(int32_t) * nsub, h2d, s);
    if (e == hipSuccess && nsub) e = hipMemcpyAsync(sq, d->sub_q, sizeof(double) * nsub, h2d, s);
    if (e == hipSuccess) e = hipMemcpyAsync(sr, rect.data(), sizeof(double4) * n_sub, h2d, s);
    if (e == hipSuccess && d->porosity) e = hipMemcpyAsync(por, d->porosity, sizeof(double) * ncell, h2d, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(flags, d->flags ? d->flags : ones.data(), sizeof(int32_t) * ncell, h2d, s);
    if (e == hipSuccess) e = hipMemsetAsync(err, 0, 4 * sizeof(int), s);
    BuildQuadParams B;
    std::memset(&B, 0, sizeof B);
    B.ncell = ncell;
    B.box = static_cast<const QuadBox*>(box);
    B.sub_off = static_cast<const int32_t*>(off);
    B.sub_q = static_cast<const double*>(sq);
    B.por = static_cast<const double*>(por);
    B.por_scalar = d->porosity ? 0.0 : d->porosity_scalar;
    B.flags = static_cast<const int32_t*>(flags);
    B.rec = static_cast<QuadRec*>(rec);
    B.balance_tol = d->balance_tol;
    B.err = static_cast<int*>(err);
    if (e == hipSuccess)
        e = launch(build_quad_kernel(), dim3((unsigned)((ncell + 255) / 256)), dim3(256), &B, 0, s);
    int herr[4] = {0, 0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(herr, err, sizeof herr, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_grid(g);
        return fail(hip_code(e), "grid upload failed: %s", hipGetErrorString(e));
    }
    if (herr[0] || herr[1] || herr[2] || herr[3]) {
        free_grid(g);
        if (herr[0]) return fail(PT_ERR_INVALID_ARG, "a subface flow is not finite");
        if (herr[1]) return fail(PT_ERR_INVALID_ARG, "a porosity is not finite and > 0");
        if (herr[2]) return fail(PT_ERR_INVALID_ARG, "a cell flag has unknown bits");
        return fail(PT_ERR_UNBALANCED, "a cell's face flows do not balance within balance_tol");
    }
    GridDev& gd = g->gd;
    std::memset(&gd, 0, sizeof gd);
    gd.rec64 = reinterpret_cast<const CellRec64*>(rec);   // QuadRec shares the record prefix
    gd.por = static_cast<double*>(por);
    gd.flags = static_cast<int32_t*>(flags);
    gd.por_scalar = B.por_scalar;
    gd.nx = d->ncell;
    gd.ny = 1;
    gd.nz = 1;
    gd.plane = 1;
    gd.qbox = static_cast<const QuadBox*>(box);
    gd.sub_nb = static_cast<const int32_t*>(nb);
    gd.sub_rect = static_cast<const double4*>(sr);
    add_live(g);
    *out = g;
    return PT_OK;
}

int pt_track(const pt_grid* const* grids, int32_t n_grids, const pt_particles* p, const pt_track_opts* o,
             void* hip_stream, pt_run** out) {
    g_err.clear();
    if (!out) return fail(PT_ERR_INVALID_ARG, "out must not be NULL");
    *out = nullptr;
    int dev = 0, n_cu = 0;
    int rc = check_track_args(grids, n_grids, p, o, &dev, &n_cu);
    if (rc != PT_OK) return rc;
    Plan PL;
    rc = make_plan(grids, n_grids, p, o, n_cu, SIZE_MAX, kRecheckTracksMax, &PL);
    if (rc != PT_OK) return rc;

    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    pt_run* r = nullptr;
    rc = new_run(dev, &r);
    if (rc != PT_OK) return rc;
    r->stream = s;
    r->sched = PL.key.sched == S_STATIC ? PT_SCHED_STATIC : PT_SCHED_PERSISTENT;
    r->layout = PL.key.layout == L_FACES ? PT_LAYOUT_FACES : PT_LAYOUT_CELL;   // quadtree: its packed records
    r->block = PL.block;
    r->grid = PL.grid;
    r->path_pass = PL.path ? (PL.path_count ? 1 : 2) : 0;

    // per-run tables: grid views, group table, snapshot times
    if (PL.tables) {
        rc = ensure_tables(r, PL.tables);
        if (rc != PT_OK) {
            destroy_run(r);
            return rc;
        }
        // the previous use of this pinned buffer has completed: runs are reused only after
        // pt_release, which waits for them
        unsigned char* h = static_cast<unsigned char*>(r->h_tables);
        write_tables(PL, grids, n_grids, p, o,
                     [&](size_t off, const void* src, size_t bytes) { std::memcpy(h + off, src, bytes); });
        hipError_t e = hipMemcpyAsync(r->d_tables, r->h_tables, PL.tables, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            destroy_run(r);
            return fail(hip_code(e), "table upload failed: %s", hipGetErrorString(e));
        }
    }
    if (PL.path_count) {
        rc = ensure_scan(r, PL.scan_bytes);
        if (rc != PT_OK) {
            destroy_run(r);
            return rc;
        }
    }
    if (PL.sort) {
        rc = ensure_sort(r, PL.sort_bytes);
        if (rc != PT_OK) {
            destroy_run(r);
            return rc;
        }
    }
    if (PL.recheck_bytes) {
        rc = ensure_recheck(r, PL.recheck_bytes);
        if (rc != PT_OK) {
            destroy_run(r);
            return rc;
        }
    }
    TrackParams P;
    SortParams SP;
    ScanParams SC;
    bind_params(PL, grids, n_grids, p, o, static_cast<unsigned char*>(r->d_tables),
                static_cast<unsigned char*>(r->d_sort), static_cast<int64_t*>(r->d_scan),
                static_cast<unsigned char*>(r->d_recheck), r->d_counters, P, SP, SC);
    Counters* cptr = r->d_counters;
    LaunchSeq seq;
    build_seq(PL, p->n, &cptr, &P, &SP, &SC, seq);

    hipError_t e = hipEventRecord(r->ev0, s);
    if (e == hipSuccess) {
        if (o->use_graph) {
            // key: every launch's function, shape, dynamic LDS and argument bytes
            std::vector<unsigned char> gkey;
            for (int q = 0; q < seq.n; ++q) {
                const Launch& L = seq.v[q];
                const unsigned char* a = static_cast<const unsigned char*>(L.arg);
                const unsigned char* f = reinterpret_cast<const unsigned char*>(&L.fn);
                gkey.insert(gkey.end(), f, f + sizeof L.fn);
                const unsigned dims[3] = {L.grid.x, L.block.x, (unsigned)L.lds};
                const unsigned char* d = reinterpret_cast<const unsigned char*>(dims);
                gkey.insert(gkey.end(), d, d + sizeof dims);
                gkey.insert(gkey.end(), a, a + L.bytes);
            }
            if (!r->exec || r->graph_key != gkey) {
                if (r->exec) {
                    (void)hipGraphExecDestroy(r->exec);
                    (void)hipGraphDestroy(r->graph);
                    r->exec = nullptr;
                    r->graph = nullptr;
                }
                hipGraph_t gr = nullptr;
                e = hipGraphCreate(&gr, 0);
                hipGraphNode_t prev = nullptr;
                for (int q = 0; e == hipSuccess && q < seq.n; ++q) {
                    if (q == seq.track_at) {   // event nodes around the tracking kernel
                        hipGraphNode_t ev = nullptr;
                        e = hipGraphAddEventRecordNode(&ev, gr, prev ? &prev : nullptr, prev ? 1 : 0, r->evk0);
                        prev = ev;
                        if (e != hipSuccess) break;
                    }
                    void* args[] = {seq.v[q].arg};
                    hipKernelNodeParams kp;
                    std::memset(&kp, 0, sizeof kp);
                    kp.func = const_cast<void*>(seq.v[q].fn);
                    kp.gridDim = seq.v[q].grid;
                    kp.blockDim = seq.v[q].block;
                    kp.kernelParams = args;
                    kp.sharedMemBytes = (unsigned)seq.v[q].lds;
                    hipGraphNode_t node = nullptr;
                    e = hipGraphAddKernelNode(&node, gr, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
                    prev = node;
                    if (e == hipSuccess && q == seq.track_at) {
                        hipGraphNode_t ev = nullptr;
                        e = hipGraphAddEventRecordNode(&ev, gr, &prev, 1, r->evk1);
                        prev = ev;
                    }
                }
                // no tracking kernel (no particles): both events at the end, track_ms = 0
                for (int q = 0; e == hipSuccess && seq.track_at < 0 && q < 2; ++q) {
                    hipGraphNode_t ev = nullptr;
                    e = hipGraphAddEventRecordNode(&ev, gr, prev ? &prev : nullptr, prev ? 1 : 0, q ? r->evk1 : r->evk0);
                    prev = ev;
                }
                if (e == hipSuccess) e = hipGraphInstantiate(&r->exec, gr, nullptr, nullptr, 0);
                if (e == hipSuccess) {
                    r->graph = gr;
                    r->graph_key = gkey;
                } else if (gr) {
                    (void)hipGraphDestroy(gr);
                    r->exec = nullptr;
                }
            }
            if (e == hipSuccess) e = hipGraphLaunch(r->exec, s);
        } else {
            for (int q = 0; e == hipSuccess && q < seq.n; ++q) {
                if (q == seq.track_at) e = hipEventRecord(r->evk0, s);
                if (e == hipSuccess) e = launch(seq.v[q].fn, seq.v[q].grid, seq.v[q].block, seq.v[q].arg, seq.v[q].lds, s);
                if (e == hipSuccess && q == seq.track_at) e = hipEventRecord(r->evk1, s);
            }
            if (e == hipSuccess && seq.track_at < 0) e = hipEventRecord(r->evk0, s);
            if (e == hipSuccess && seq.track_at < 0) e = hipEventRecord(r->evk1, s);
        }
    }
    if (e == hipSuccess) e = hipEventRecord(r->ev1, s);
    if (e == hipSuccess) e = hipMemcpyAsync(r->h_counters, r->d_counters, sizeof(Counters), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(r->ev_done, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(s);
        destroy_run(r);
        return fail(hip_code(e), "launch failed: %s", hipGetErrorString(e));
    }
    r->launched = true;
    add_live(r);
    *out = r;
    return PT_OK;
}

int pt_track_noalloc(const pt_grid* const* grids, int32_t n_grids, const pt_particles* p,
                     const pt_track_opts* o, void* hip_stream, int64_t* counts) {
    g_err.clear();
    if (!counts) return fail(PT_ERR_INVALID_ARG, "counts must not be NULL");
    int dev = 0, n_cu = 0;
    int rc = check_track_args(grids, n_grids, p, o, &dev, &n_cu);
    if (rc != PT_OK) return rc;
    Plan PL;
    rc = make_plan(grids, n_grids, p, o, n_cu, kScratchBytes - kScratchSort, kScratchRecheckTracks, &PL);
    if (rc != PT_OK) return rc;
    if (PL.tables > kScratchTablesMax)
        return fail(PT_ERR_UNSUPPORTED, "the call's tables (grid views, groups, snapshot times, time steps) take %zu "
                    "bytes, above the %zu of the allocation-free scratch", PL.tables, kScratchTablesMax);
    if (PL.scan_bytes > kScratchScanMax)
        return fail(PT_ERR_UNSUPPORTED, "a pathline count pass over %lld particles needs %zu bytes of scan "
                    "scratch, above the %zu available", (long long)p->n, PL.scan_bytes, kScratchScanMax);
    unsigned char* base = nullptr;
    rc = scratch_of(dev, &base);
    if (rc != PT_OK) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    Counters* cptr = reinterpret_cast<Counters*>(base + kScratchCounters);
    TrackParams P;
    SortParams SP;
    ScanParams SC;
    bind_params(PL, grids, n_grids, p, o, base + kScratchTables, base + kScratchSort,
                reinterpret_cast<int64_t*>(base + kScratchScan), base + kScratchRecheck, cptr, P, SP, SC);
    TableFill tf;
    tf.dst = base + kScratchTables;
    tf.A.nbytes = 0;
    tf.s = s;
    write_tables(PL, grids, n_grids, p, o, [&](size_t off, const void* src, size_t bytes) { tf.put(off, src, bytes); });
    tf.flush();
    hipError_t e = tf.err;
    LaunchSeq seq;
    build_seq(PL, p->n, &cptr, &P, &SP, &SC, seq);
    CountsParams CP;
    CP.c = cptr;
    CP.out = counts;
    CP.path_pass = PL.path ? (PL.path_count ? 1 : 2) : 0;
    seq.push(counts_kernel(), dim3(1), dim3(64), &CP, sizeof CP);
    for (int q = 0; e == hipSuccess && q < seq.n; ++q)
        e = launch(seq.v[q].fn, seq.v[q].grid, seq.v[q].block, seq.v[q].arg, seq.v[q].lds, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(hip_code(e), "launch failed: %s", hipGetErrorString(e));
    }
    return PT_OK;
}

int pt_results(pt_run* r, pt_summary* out) {
    g_err.clear();
    if (!r || !is_live(r, kRunMagic)) return fail(PT_ERR_BAD_HANDLE, "not a live run handle");
    if (!out) return fail(PT_ERR_INVALID_ARG, "out must not be NULL");
    HIP_TRY(hipEventSynchronize(r->ev_done));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, r->ev0, r->ev1));
    float kms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&kms, r->evk0, r->evk1));
    std::memset(out, 0, sizeof *out);
    const Counters& c = *r->h_counters;
    out->crossings = (int64_t)c.crossings;
    int64_t tracked = 0;
    for (int q = 0; q < PT_N_STATUS; ++q) {
        out->status_count[q] = (int64_t)c.status[q];
        tracked += (int64_t)c.status[q];
    }
    out->n_tracked = tracked;
    out->kernel_ms = ms;
    out->track_ms = kms;
    out->schedule = r->sched;
    out->layout = r->layout;
    out->block = r->block;
    out->grid = r->grid;
    out->cr_ambiguous = (int64_t)c.cr_ambiguous;
    out->recheck_tracks = (int64_t)c.recheck_tracks;
    if (r->path_pass == 1) out->path_records = out->crossings;
    if (r->path_pass == 2) {
        out->path_dropped = (int64_t)c.path_dropped;
        out->path_records = out->crossings - out->path_dropped;
    }
    return PT_OK;
}

int pt_shutdown(void) {
    g_err.clear();
    std::vector<void*> live;
    std::vector<pt_run*> pool;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        live.assign(g_live.begin(), g_live.end());
        g_live.clear();
        pool.swap(g_pool);
    }
    // wait for every device this library has work or memory on, then free everything
    std::vector<int> devs;
    auto note = [&](int d) {
        if (std::find(devs.begin(), devs.end(), d) == devs.end()) devs.push_back(d);
    };
    for (void* h : live) note(*reinterpret_cast<uint32_t*>(h) == kGridMagic ? static_cast<pt_grid*>(h)->device
                                                                             : static_cast<pt_run*>(h)->device);
    for (pt_run* r : pool) note(r->device);
    int cur = 0;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    int rc = PT_OK;
    for (int d : devs) {
        hipError_t e = hipSetDevice(d);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            (void)hipGetLastError();
            rc = fail(hip_code(e), "device %d failed before shutdown: %s", d, hipGetErrorString(e));
        }
    }
    for (void* h : live) {
        if (*reinterpret_cast<uint32_t*>(h) == kGridMagic) {
            pt_grid* g = static_cast<pt_grid*>(h);
            (void)hipSetDevice(g->device);
            free_grid(g);
        } else {
            pt_run* r = static_cast<pt_run*>(h);
            (void)hipSetDevice(r->device);
            destroy_run(r);
        }
    }
    for (pt_run* r : pool) {
        (void)hipSetDevice(r->device);
        destroy_run(r);
    }
    if (have_cur) (void)hipSetDevice(cur);
    (void)hipGetLastError();
    return rc;
}

int pt_release(void* h) {
    g_err.clear();
    if (!h) return PT_OK;
    uint32_t magic = 0;
    if (!take_handle(h, &magic)) return fail(PT_ERR_BAD_HANDLE, "not a live handle (released twice?)");
    if (magic == kGridMagic) {
        pt_grid* g = static_cast<pt_grid*>(h);
        (void)hipDeviceSynchronize();  // no run may still read it
        free_grid(g);
        return PT_OK;
    }
    pt_run* r = static_cast<pt_run*>(h);
    hipError_t e = hipEventSynchronize(r->ev_done);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        destroy_run(r);
        return fail(hip_code(e), "run failed on the device: %s", hipGetErrorString(e));
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_pool.size() < kPoolMax) g_pool.push_back(r);
    else destroy_run(r);
    return PT_OK;
}

}  // extern "C"
