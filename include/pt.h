/*
 * pt.h -- C ABI of the MI355X (gfx950) particle tracker.
 *
 * Semi-analytical advective particle tracking through a steady, structured,
 * cell-by-cell face-flow field.  The paper (Introduction; Methods, "MODPATH")
 * describes the problem this library solves: a flow model provides the flow
 * through every cell face; each particle is moved in a single step to the
 * interface of its cell, handed to the neighbour across it, and this repeats
 * until a stopping condition (a boundary face, the maximum tracking time, or
 * a cell with sink flows); particles are independent of one another.  The
 * simulation type and stop time come from the run configuration; outputs are
 * indexed by particle (Methods, "MODPATH" and "Multiprocessing").
 *
 * Every call returns an int32 status: PT_OK (0) or a negative PT_ERR_* code.
 * No exception crosses the ABI.  After a failing call, pt_last_error()
 * returns a message for the calling thread.  Every argument is validated
 * before any device work; a call that fails validation launches nothing.
 * Device-side faults are reported by pt_results() of the run they belong to.
 *
 * Geometry and units.  Cells are indexed (i, j, k) with linear id
 * c = (k*ny + j)*nx + i.  Face flows are positive in the +i / +j / +k
 * direction, in volume per time (e.g. m^3/d).  Inside a cell a particle is
 * located by local coordinates (xi, eta, zeta) in [0,1]^3 along i, j, k; its
 * global position is x = x0 + (i + xi)*dx, y = y0 + (j + eta)*dy,
 * z = z0 + (k + zeta)*dz.
 *
 * Per-cell motion (Pollock's semi-analytical step, to which the paper
 * defers): each velocity component is interpolated linearly between the two
 * face velocities u = Q / (n * (dx*dy*dz)) of its axis, u(xi) = u1 + A*xi with
 * A = u2 - u1.  The components separate, so the particle reaches face xi_e
 * (velocity u_e) after ln(u_e/u_p)/A (or (xi_e - xi)/u_p when A = 0), and
 * xi(tau) = xi + u_p * (exp(A*tau) - 1)/A.  The earliest reachable face ends
 * the step; exact ties go to the lowest axis (i, then j, then k).
 */
#ifndef PT_H
#define PT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes --------------------------------------------------------------------- */
#define PT_OK 0
#define PT_ERR_INVALID_ARG (-1)  /* a pointer, size, enum or value is not acceptable            */
#define PT_ERR_BAD_HANDLE (-2)   /* not a live handle of this library (e.g. released twice)     */
#define PT_ERR_OOM (-3)          /* device or pinned host memory could not be allocated         */
#define PT_ERR_NO_DEVICE (-4)    /* no usable HIP device                                        */
#define PT_ERR_DEVICE (-5)       /* a HIP call or a kernel failed                               */
#define PT_ERR_UNBALANCED (-6)   /* a cell's face flows do not balance within balance_tol       */
#define PT_ERR_UNSUPPORTED (-7)  /* valid but not supported by this build (sizes, layouts)      */

/* ---- particle statuses (int32, in/out) ------------------------------------------------ */
#define PT_ACTIVE 0            /* to be tracked (a fresh release)                              */
#define PT_BOUNDARY 1          /* left the domain through a boundary face                      */
#define PT_SINK 2              /* entered (or was released in) a sink cell                     */
#define PT_MAX_TIME 3          /* reached t_max; tracked again (resumed) by a later call       */
#define PT_STEP_CAP 4          /* made max_steps crossings                                     */
#define PT_STRANDED 5          /* no face of the current cell can be reached                   */
#define PT_INVALID_START 6     /* bad cell, inactive cell, coordinate outside [0,1] or NaN t    */
#define PT_INACTIVE_NEIGHBOR 7 /* the exit face leads into an inactive cell (bad flow field)   */
#define PT_N_STATUS 8

/* ---- cell flags ----------------------------------------------------------------------- */
#define PT_CELL_ACTIVE 1       /* bit 0: the cell takes part in the flow model                 */
#define PT_CELL_SINK 2         /* bit 1: the cell has sink flows (a well)                      */

/* ---- enumerations --------------------------------------------------------------------- */
#define PT_MEM_HOST 0
#define PT_MEM_DEVICE 1

#define PT_ENDPOINT 0          /* final state only                                             */
#define PT_TIMESERIES 1        /* plus positions at the snapshot times                         */
#define PT_PATHLINE 2          /* plus one record per cell crossing (the particle's pathline:   *
                                * the paper's third simulation type, Methods "MODPATH")        */

#define PT_FP64 0              /* all arithmetic in FP64                                       */
#define PT_MIXED 1             /* in-cell arithmetic in FP32; time, global position and the    *
                                * near-zero-gradient branch in FP64                            */

#define PT_SCHED_AUTO 0
#define PT_SCHED_STATIC 1      /* one thread per particle for its whole track                 */
#define PT_SCHED_PERSISTENT 2  /* resident waves pull particles from a device work queue and   *
                                * refill finished lanes (wave-level compaction)               */

#define PT_SORT_AUTO 0         /* order the work by starting cell when n >= 65536              */
#define PT_SORT_NONE 1         /* process particles in index order                            */
#define PT_SORT_CELL 2         /* order the work by starting cell (counting sort on device)   */

#define PT_LAYOUT_AUTO 0
#define PT_LAYOUT_FACES 1      /* face-flow arrays + porosity + flags; velocities per step    */
#define PT_LAYOUT_CELL 2       /* one packed record of six face velocities + flags per cell   */

typedef struct pt_grid pt_grid; /* opaque: a flow field resident in device memory */
typedef struct pt_run pt_run;   /* opaque: one enqueued tracking call            */

/* ---- grid ----------------------------------------------------------------------------- */
typedef struct {
    int32_t nx, ny, nz;           /* cells along i, j, k; each >= 1, nx*ny*nz < 2^31            */
    double dx, dy, dz;            /* cell sizes, finite and > 0                                  */
    double x0, y0, z0;            /* global coordinates of the corner of cell (0,0,0)            */
    const double* qx;             /* [nz][ny][nx+1] flow through the i faces, + = +i             */
    const double* qy;             /* [nz][ny+1][nx] flow through the j faces, + = +j             */
    const double* qz;             /* [nz+1][ny][nx] flow through the k faces, + = +k             */
    const double* porosity;       /* [nz][ny][nx] in (0, inf), or NULL -> porosity_scalar        */
    double porosity_scalar;       /* used when porosity == NULL; finite and > 0                  */
    const int32_t* flags;         /* [nz][ny][nx] PT_CELL_* bits; NULL -> every cell active      */
    int32_t mem;                  /* PT_MEM_HOST or PT_MEM_DEVICE for all the pointers above     */
    double balance_tol;           /* < 0: no check.  Else every active non-sink cell must satisfy *
                                   * |inflow - outflow| <= balance_tol * (sum of |face flows|),  *
                                   * otherwise PT_ERR_UNBALANCED                                 */
} pt_grid_desc;

/*
 * Copy a flow field to the device and build its device layouts (velocity
 * records for FP64 and FP32, and the face arrays).  Validates the
 * description first (sizes, finite flows, porosity > 0, known flag bits,
 * optional balance).  The input arrays are read during the call only; the
 * caller may free them on return.  `hip_stream` (a hipStream_t, NULL = the
 * default stream) orders the copies; the call returns after they complete.
 * On success *out owns the device copy until pt_release(*out).
 */
int pt_load_grid(const pt_grid_desc* desc, void* hip_stream, pt_grid** out);

/* ---- quadtree grid ---------------------------------------------------------------------- */
/*
 * A rectangular unstructured (quadtree) grid: the paper's second test case refines its grid
 * with a quadtree (Methods "Synthetic test cases"; "Grid complexity" in Results).  Cells are
 * boxes; a face f = 2*axis + side (side 1 = high face) may be split into subfaces, each shared
 * with one neighbour or the domain boundary, listed in order.  Tracking in such a cell is the
 * structured step with the face's total flow (its subfaces' flows summed in order) as the flow
 * of that face.  A particle leaving through a face enters the neighbour of the subface holding
 * its exit point (the first in order when the point is on an edge between two); in the
 * neighbour, a face coordinate carries over when both cells span the same range on that axis,
 * otherwise it is mapped through the global coordinate and clamped to [0, 1].  Because the
 * velocity of a split face is an average, face velocities can circulate around a point where
 * cells meet; a particle handed round such a point in 16 zero-time crossings in a row stops
 * there as PT_STRANDED.  Quadtree grids are tracked in FP64, one grid per call, steady flow,
 * with the packed layout (PT_LAYOUT_AUTO or PT_LAYOUT_CELL); every output mode is supported.
 */
typedef struct {
    int32_t ncell;                /* cells, >= 1                                                 */
    int32_t nsub;                 /* subfaces, >= 0                                              */
    const double* box;            /* [ncell][6] x_lo, y_lo, z_lo, hx, hy, hz (h finite, > 0)     */
    const int32_t* sub_off;       /* [ncell*6 + 1]: the subfaces of face f of cell c are          *
                                   * sub_off[6c+f] .. sub_off[6c+f+1]-1; non-decreasing from 0   *
                                   * to nsub, at most 31 per face                                */
    const int32_t* sub_nb;        /* [nsub] neighbour cell, or -1 for the domain boundary        */
    const double* sub_q;          /* [nsub] flow through the subface, + = +axis                  */
    const double* sub_lo;         /* [nsub][2] extent of the subface in the face's two           */
    const double* sub_hi;         /* [nsub][2] tangential local coordinates (x-face: eta, zeta;  *
                                   * y-face: xi, zeta; z-face: xi, eta), 0 <= lo <= hi <= 1      */
    const double* porosity;       /* [ncell] in (0, inf), or NULL -> porosity_scalar             */
    double porosity_scalar;
    const int32_t* flags;         /* [ncell] PT_CELL_* bits; NULL -> every cell active           */
    int32_t mem;                  /* PT_MEM_HOST only (the description is checked on the host)   */
    double balance_tol;           /* as in pt_grid_desc                                          */
} pt_quad_desc;

/* Copy a quadtree grid to the device and build its records; validation and ownership as in
 * pt_load_grid (PT_ERR_UNSUPPORTED for device-resident descriptions). */
int pt_load_quad_grid(const pt_quad_desc* desc, void* hip_stream, pt_grid** out);

/* ---- particles -------------------------------------------------------------------------- */
typedef struct {
    int64_t n;                    /* number of particles, 0 <= n < 2^31 (0: an empty run)         */
    int32_t* cell;                /* [n] linear cell id                      device, in/out      */
    double* xi;                   /* [n] local coordinates in [0,1]          device, in/out      */
    double* eta;
    double* zeta;
    double* t;                    /* [n] release time in, final time out     device, in/out      */
    int32_t* status;              /* [n] PT_ACTIVE / PT_MAX_TIME are tracked, device, in/out     *
                                   * any other status is left untouched                         */
    int32_t* ncross;              /* [n] cell crossings so far               device, in/out      */
    uint64_t* path_hash;          /* [n] FNV-1a style hash of the cells left device, in/out      *
                                   * (start at 0xcbf29ce484222325 for a fresh particle): at each *
                                   * crossing h = (h ^ (uint32)cell) * 0x100000001b3            */
    int32_t n_groups;             /* 0: every particle uses grids[0].  Else particles            *
                                   * [group_offsets[g], group_offsets[g+1]) use                  *
                                   * grids[group_grid[g]]                                       */
    const int64_t* group_offsets; /* host [n_groups+1], 0 = first <= ... <= last = n             */
    const int32_t* group_grid;    /* host [n_groups], each in [0, n_grids)                       */
} pt_particles;

/* ---- pathline record (PT_PATHLINE) ----------------------------------------------------- */
typedef struct {
    double t;                     /* time of the crossing                                        */
    double x, y, z;               /* global position on the crossed face                         */
    int32_t cell;                 /* cell left                                                   */
    int32_t face;                 /* face crossed: 2*axis + 1 for the high face (axis 0 = i,     *
                                   * 1 = j, 2 = k)                                              */
} pt_path_record;                 /* 40 bytes, 8-byte aligned                                    */

/* ---- options ---------------------------------------------------------------------------- */
typedef struct {
    int32_t mode;                 /* PT_ENDPOINT | PT_TIMESERIES | PT_PATHLINE                   */
    int32_t precision;            /* PT_FP64 | PT_MIXED                                          */
    int32_t schedule;             /* PT_SCHED_*                                                  */
    int32_t layout;               /* PT_LAYOUT_* (PT_MIXED requires CELL or AUTO)                */
    int32_t direction;            /* +1 forward, -1 backward (all face flows negated)            */
    int32_t stop_at_sink;         /* 1: stop on entering/release in a sink cell; 0: pass through */
    double t_max;                 /* tracking time limit, not NaN (+inf allowed); a face reached *
                                   * exactly at t_max is still crossed                          */
    int64_t max_steps;            /* crossing cap per particle (counted over all calls), >= 1    */
    const double* snap_times;     /* host [n_snap], non-decreasing, finite (PT_TIMESERIES)       */
    int32_t n_snap;               /* >= 1 for PT_TIMESERIES                                      */
    double* snap_xyz;             /* device [n][n_snap][3] global positions (PT_TIMESERIES):     *
                                   * for a tracked particle, snapshot s gets its position if it  *
                                   * was moving at s (release <= s, and s < termination time,    *
                                   * or s <= t_max for MAX_TIME / STRANDED), NaN otherwise;      *
                                   * a resumed (PT_MAX_TIME) particle keeps snapshots before its *
                                   * current time                                               */
    double* out_xyz;              /* device [n][3] final global position, or NULL; NaN for       *
                                   * PT_INVALID_START                                           */
    int32_t use_graph;            /* 1: launch through a cached hipGraph (replayed when the      *
                                   * same arguments come again)                                 */
    int32_t block;                /* threads per block, 0 = default; multiple of 64, <= 1024      */
    int32_t blocks_per_cu;        /* persistent grid size per compute unit, 0 = default          */
    int32_t refill;               /* persistent: refill a wave's idle lanes once at least this    *
                                   * many are idle, 1..64, 0 = default (1)                      */
    int32_t steps_per_refill;     /* persistent: crossings per lane between refill points, 0 = 1 */
    int32_t chunk;                /* persistent: particles a wave claims from the device queue  *
                                   * per atomic, >= 1, 0 = default (64)                          */
    int32_t sort;                 /* PT_SORT_*: processing order (never changes a result); the   *
                                   * static kernel deals the ordered work to the dies in chunks  *
                                   * of consecutive blocks                                      */
    /* PT_PATHLINE.  A pathline is the release point (the input state), one record per cell
     * crossing made in this call, in crossing order, and the final state.  Records are stored
     * particle by particle (CSR): those of particle p fill path_records[path_offsets[p] ..
     * path_offsets[p+1]).  Two calls with the same inputs produce them:
     *   1. path_count_only = 1 (count pass): a dry run.  The particle arrays and out_xyz are
     *      left untouched and no record is written; path_offsets[0] = 0 and path_offsets[p+1]
     *      = the crossings particles 0..p make (exclusive scan of the per-particle counts), so
     *      path_offsets[n] is the number of records.  pt_summary.path_records reports it.
     *   2. path_count_only = 0 (record pass): tracks and writes the records.  Tracking is
     *      deterministic, so particle p makes exactly path_offsets[p+1] - path_offsets[p]
     *      crossings.  A record whose slot is not in [path_offsets[p], path_offsets[p+1]) or not
     *      in [0, path_cap) is not written and is counted in pt_summary.path_dropped. */
    int64_t* path_offsets;        /* device [n+1] int64: written by the count pass, read by the  *
                                   * record pass                                                */
    int32_t path_count_only;      /* 1: count pass, 0: record pass                               */
    int64_t path_cap;             /* records path_records can hold (record pass), >= 0           */
    pt_path_record* path_records; /* device [path_cap] (record pass; may be NULL if path_cap = 0) */
    /* Transient flow (the paper's outermost loop over the flow model's time steps, Methods
     * "MODPATH": once the end of the current flow conditions is reached, the flow arrays are
     * updated).  With n_tsteps >= 1, grids[s] holds the face flows of time step s, valid until
     * tstep_end[s]; n_grids must equal n_tsteps, every grid must have the same geometry, there
     * are no particle groups, and direction must be +1.  A particle is tracked in the field of
     * the step containing its time (a time equal to a step end belongs to the next step).
     * When its next exit would come after the end of its step, it is advanced analytically to
     * that end and continues in the next step's field from the same cell and position; if the
     * cell is inactive there it stops (PT_INACTIVE_NEIGHBOR), if it is a sink it stops when
     * stop_at_sink = 1 (PT_SINK).  The end of the last step acts as a time limit (PT_MAX_TIME,
     * or PT_STRANDED when no face is reachable), like t_max. */
    int32_t n_tsteps;             /* 0: steady flow                                              */
    const double* tstep_end;      /* host [n_tsteps]: strictly increasing, not NaN; the last may *
                                   * be +inf                                                    */
} pt_track_opts;

/* Fill *o with the defaults: endpoint, FP64, auto schedule and layout, forward,
 * stop at sinks, t_max = +inf, max_steps = 2^20, no snapshots. */
void pt_default_opts(pt_track_opts* o);

/*
 * Enqueue tracking of every particle on `hip_stream` and return at once.
 * grids[0 .. n_grids) are handles from pt_load_grid (n_grids >= 1).  All
 * particle and output pointers are device memory owned by the caller, which
 * must keep them alive and untouched until pt_results() of the returned run.
 * On success *out is a run handle: pass it to pt_results() and then to
 * pt_release().
 */
int pt_track(const pt_grid* const* grids, int32_t n_grids, const pt_particles* p,
             const pt_track_opts* o, void* hip_stream, pt_run** out);

typedef struct {
    int64_t crossings;            /* cell crossings made in this call (all particles)            */
    int64_t n_tracked;            /* particles with status ACTIVE or MAX_TIME at the start       */
    int64_t status_count[PT_N_STATUS]; /* final status of the tracked particles                  */
    double kernel_ms;             /* device time between the run's start and end events          */
    int32_t schedule;             /* the schedule that ran (PT_SCHED_STATIC / _PERSISTENT)       */
    int32_t layout;               /* the layout that ran                                         */
    int32_t block, grid;          /* launch shape of the tracking kernel                         */
    int64_t cr_ambiguous;         /* FP64 log1p/expm1/log evaluations whose correct rounding     *
                                   * was not decided: the nearest double of a 2^-96-accurate     *
                                   * value was used.  Expected 0.  (See recheck_*.)              */
    int64_t path_records;         /* PT_PATHLINE: records counted (count pass) or written        */
    int64_t path_dropped;         /* PT_PATHLINE record pass: records outside their slot range   */
    int64_t recheck_tracks;       /* FP64: particles whose tracking (or snapshots) met an        *
                                   * evaluation within 2^-96 of a rounding boundary (structured  *
                                   * inputs: arguments near 2^-53 .. 2^-50 with regular bit      *
                                   * patterns); each was tracked again from its input state by a *
                                   * careful pass that decides such arguments exactly.  Beyond   *
                                   * 2^20 per call (2^18 for pt_track_noalloc) the rest keep     *
                                   * their first results and count in cr_ambiguous.              */
    double track_ms;              /* device time of the tracking kernel alone (events recorded   *
                                   * just before and after its launch; kernel_ms also encloses   *
                                   * the counter reset, the ordering sort and the careful pass)  */
} pt_summary;

/* Wait for the run, then fill *out.  Reports asynchronous device errors of
 * the run as PT_ERR_DEVICE.  May be called more than once. */
int pt_results(pt_run* run, pt_summary* out);

/* Release a pt_grid* or pt_run* (waits for a run still in flight).  NULL is a
 * no-op.  A pointer that is not a live handle gives PT_ERR_BAD_HANDLE. */
int pt_release(void* handle);

/* ---- allocation-free tracking ----------------------------------------------------------- */
/*
 * For callers that cannot allocate memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  pt_track_noalloc enqueues the same kernels as pt_track,
 * with the same arguments, validation and results, but calls no hipMalloc, hipFree or other
 * allocating routine, host or device, and creates no run handle, event or graph.  Its scratch
 * (the counter block, the per-call tables, the ordering buffers, the pathline offset scan's
 * tile sums and the careful pass's particle list) is one array of PT_NOALLOC_SCRATCH_BYTES in the library's device code, one copy
 * per GPU, held until the process ends.  Limits (PT_ERR_UNSUPPORTED beyond them): the tables of
 * one call -- a 160-byte view per grid for batched or transient runs, the group table, the
 * snapshot times, the time-step ends -- at most 64 KiB; a pathline count pass at most 2^26
 * particles; ordering by starting cell (PT_SORT_CELL) only while its buffers -- 16 bytes per
 * particle plus 4 bytes per tile of 4096 particles and super-bucket (at most 256 super-buckets up
 * to 2.1e6 cells) -- fit in the remaining ~30.9 MiB (PT_SORT_AUTO then simply does not order).
 *
 * The run's counts are written, once its kernels have run, to `counts` (device memory owned by
 * the caller, PT_COUNTS_WORDS int64): PT_COUNT_CROSSINGS, PT_COUNT_TRACKED,
 * PT_COUNT_STATUS + s for each status s, PT_COUNT_CR_AMBIGUOUS, PT_COUNT_PATH_RECORDS,
 * PT_COUNT_PATH_DROPPED, PT_COUNT_RECHECK_TRACKS (the fields of pt_summary, see there), the
 * remaining words 0.
 * Synchronise `hip_stream` before reading them or the particle outputs.  use_graph is ignored
 * (the kernels are launched directly; a capturing caller records them).
 *
 * Every call on one GPU uses that GPU's single scratch array, which keeps the last call's
 * contents: calls whose work overlaps on one GPU (other streams or threads, before the previous
 * call's kernels finished) race and give wrong results.  Calls on one stream are ordered and safe.
 * The call clears what must start at zero (the counters) with kernels, not
 * memsets.  Errors: as pt_track; PT_ERR_INVALID_ARG for counts == NULL.
 */
#define PT_NOALLOC_SCRATCH_BYTES (32 << 20)
#define PT_COUNTS_WORDS 16
#define PT_COUNT_CROSSINGS 0
#define PT_COUNT_TRACKED 1
#define PT_COUNT_STATUS 2
#define PT_COUNT_CR_AMBIGUOUS 10
#define PT_COUNT_PATH_RECORDS 11
#define PT_COUNT_PATH_DROPPED 12
#define PT_COUNT_RECHECK_TRACKS 13
int pt_track_noalloc(const pt_grid* const* grids, int32_t n_grids, const pt_particles* p,
                     const pt_track_opts* o, void* hip_stream, int64_t* counts);

/* Release everything the library holds: every live grid and run handle (waiting for the
 * devices they use first) and the released runs kept for reuse, with their cached hipGraphs,
 * events and device and pinned buffers.  Afterwards every earlier handle is invalid
 * (PT_ERR_BAD_HANDLE), and the library can be used again from scratch.  Call it when no other
 * call of this library is in progress, before the HIP runtime is torn down at process exit
 * (the Python binding registers it with atexit), so that no HIP object of the library outlives
 * the runtime.  Returns PT_ERR_DEVICE if a device reported an asynchronous fault while it was
 * drained; the resources are released in any case. */
int pt_shutdown(void);

/* Message of the last failing call on this thread ("" if none). */
const char* pt_last_error(void);

/* ABI version: 100 * major + minor. */
int pt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PT_H */
