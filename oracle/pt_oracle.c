/*
 * ORACLE -- test infrastructure, not part of the product.
 *
 * A plain, slow, scalar FP64 tracker used only to check the GPU path: only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may build,
 * load or call it.  It shares no code, header, table or constant with the HIP
 * library; the two are written independently from the same description.
 *
 * What it computes (the paper, Introduction and Methods "MODPATH"): each
 * particle is displaced through the flow-model cells one cell at a time, a
 * whole cell in a single semi-analytical step up to a cell interface, and is
 * then handed to the neighbour across that interface, until a stopping
 * condition is met (a boundary face, the maximum tracking time, or a cell with
 * sink flows).  Particles are independent of one another.  The paper defers
 * the per-cell mathematics to Pollock's semi-analytical method; it is written
 * out here from the ODE it solves exactly:
 *
 *   inside a cell, each velocity component is the linear interpolation between
 *   its two face velocities, u(xi) = u1 + A*xi with u = Q / (n * V) in local
 *   units (1/d) and A = u2 - u1.  The components separate, so
 *   dxi/dt = u1 + A*xi has the closed-form solution
 *      xi(tau) = xi + u_p * tau * psi(A*tau),  psi(y) = expm1(y)/y, psi(0) = 1,
 *   and the time to reach face xi_e (velocity u_e) is
 *      dt = ln(u_e / u_p) / A = (D/u_p) * phi(A*D/u_p),  D = xi_e - xi,
 *      phi(x) = log1p(x)/x, phi(0) = 1   (dt = D/u_p when A = 0).
 *
 * Steps per particle, in order (state: cell c, local xi/eta/zeta, time t):
 *   S0 release checks; S1 cell velocities; S2 per-axis exit feasibility;
 *   S3 per-axis exit time; S4 earliest face; S5 time limit; S6 advance;
 *   S7 transfer to the neighbour and stop checks; S8 timeseries positions.
 *
 * Transient flow (Methods "MODPATH": the outermost loop runs over the flow
 * model's time steps, and once the maximum time of the current flow
 * conditions is reached the flow arrays are updated): the field of time step
 * s holds until step_end[s].  A particle is tracked in the field of the step
 * containing its time; when its next exit would come after the end of the
 * step, it is advanced analytically to that end (as at the tracking time
 * limit) and continues from the same cell and local position in the next
 * step's field.
 * Readings where the paper is silent (tie-break, clamping, sink and time-limit
 * semantics, snapshot semantics, path hash) are stated next to each step.
 *
 * Statuses: 0 ACTIVE, 1 BOUNDARY, 2 SINK, 3 MAX_TIME, 4 STEP_CAP, 5 STRANDED,
 * 6 INVALID_START, 7 INACTIVE_NEIGHBOR.
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off (no FMA contraction), -lquadmath.
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stddef.h>

#define ST_ACTIVE 0
#define ST_BOUNDARY 1
#define ST_SINK 2
#define ST_MAX_TIME 3
#define ST_STEP_CAP 4
#define ST_STRANDED 5
#define ST_INVALID_START 6
#define ST_INACTIVE_NEIGHBOR 7

#define CELL_ACTIVE 1
#define CELL_SINK 2

typedef struct {
    int32_t nx, ny, nz;
    double dx, dy, dz, x0, y0, z0;
    const double* qx;        /* [nz][ny][nx+1], + = +i */
    const double* qy;        /* [nz][ny+1][nx], + = +j */
    const double* qz;        /* [nz+1][ny][nx], + = +k */
    const double* porosity;  /* [nz][ny][nx] or NULL */
    double porosity_scalar;
    const int32_t* flags;    /* [nz][ny][nx] */
} oracle_grid;

typedef struct {
    int32_t direction;       /* +1 forward, -1 backward */
    double t_max;
    int64_t max_steps;
    int32_t stop_at_sink;
    const double* snap_times;  /* ascending, or NULL */
    int32_t n_snap;
    double* snap_xyz;          /* [n][n_snap][3] or NULL */
    double* out_xyz;           /* [n][3] or NULL */
    int32_t path_cap;          /* per-particle capacity of the path record, 0 = none */
    int32_t* path_cell;        /* [n][path_cap] cell left at each crossing */
    int32_t* path_face;        /* [n][path_cap] 2*axis + (1 if the high face) */
    double* path_t;            /* [n][path_cap] time at the crossing */
    double* path_xyz;          /* [n][path_cap][3] global position on the face */
    int32_t n_threads;
} oracle_opts;

/*
 * Elementary functions, correctly rounded: evaluated in 113-bit quad precision and
 * rounded once to double, i.e. the double nearest to the exact value (except for a
 * quad value within 2^-112 of a rounding boundary).  The method's result is the exact
 * solution of the cell ODE; the nearest double to each exact function value is the
 * plainest FP64 reading of it, and it does not depend on a libm's last-bit choices.
 */
static double cr_log1p(double x) { return (double)log1pq((__float128)x); }
static double cr_expm1(double x) { return (double)expm1q((__float128)x); }
static double cr_log(double x) { return (double)logq((__float128)x); }

/* One axis of the cell: face velocities u1 (low face) and u2 (high face). */
typedef struct {
    double u1, u2;
} axis_vel;

/* S6 formula: position along one axis after time tau, clamped to [0,1]. */
static double advance(axis_vel v, double xi, double tau) {
    double A = v.u2 - v.u1;
    double up = v.u1 + A * xi;
    if (up == 0.0) return xi;
    double y = A * tau;
    double psi = (y == 0.0) ? 1.0 : cr_expm1(y) / y;
    double xn = xi + (up * tau) * psi;
    if (xn < 0.0) xn = 0.0;
    if (xn > 1.0) xn = 1.0;
    return xn;
}

/*
 * S2 + S3: time for one axis to reach its exit face, +INFINITY if it cannot.
 * The candidate face is the one the velocity points to; it is reached only
 * if the face velocity has the same strict sign as the particle velocity
 * (a linear u cannot change sign without passing through zero, and a face
 * with zero or opposite velocity is approached asymptotically).
 */
static double axis_exit_time(axis_vel v, double xi, double* xi_exit) {
    double A = v.u2 - v.u1;
    double up = v.u1 + A * xi;
    double ue;
    if (up > 0.0) {
        *xi_exit = 1.0;
        ue = v.u2;
        if (!(ue > 0.0)) return INFINITY;
    } else if (up < 0.0) {
        *xi_exit = 0.0;
        ue = v.u1;
        if (!(ue < 0.0)) return INFINITY;
    } else {
        return INFINITY;
    }
    double D = *xi_exit - xi;
    double r = D / up;
    double x = A * r;
    double dt;
    if (x == 0.0) {
        dt = r;
    } else if (x < -0.5) {
        /* strongly decelerating: the ratio u_e/u_p is formed exactly enough,
         * 1 + x would lose digits */
        dt = cr_log(ue / up) / A;
    } else {
        dt = r * (cr_log1p(x) / x);
    }
    if (dt < 0.0) dt = 0.0;
    return dt;
}

/* S2-S4: the earliest reachable face over the three axes; exact ties go to the lowest axis.
 * Returns the time (+INFINITY and *axis = -1 when no face can be reached). */
static double earliest_exit(const axis_vel* v, const double* loc, int* axis, double* xe) {
    double dt = INFINITY;
    *axis = -1;
    *xe = 0.0;
    for (int a = 0; a < 3; ++a) {
        double e = 0.0;
        double ta = axis_exit_time(v[a], loc[a], &e);
        if (ta < dt) {
            dt = ta;
            *axis = a;
            *xe = e;
        }
    }
    return dt;
}

/* Path identity: FNV-1a style over the cells left. */
static uint64_t hash_step(uint64_t h, int64_t c) { return (h ^ (uint64_t)(uint32_t)c) * 0x100000001b3ULL; }

static double cell_porosity(const double* porosity, double scalar, int64_t c) {
    return porosity ? porosity[c] : scalar;
}

static double direction_sign(const oracle_opts* o) { return o->direction < 0 ? -1.0 : 1.0; }

static void global_xyz(const oracle_grid* g, int64_t c, double xi, double eta, double zeta,
                       double* out) {
    int64_t plane = (int64_t)g->nx * g->ny;
    int64_t k = c / plane;
    int64_t rem = c - k * plane;
    int64_t j = rem / g->nx;
    int64_t i = rem - j * g->nx;
    out[0] = g->x0 + ((double)i + xi) * g->dx;
    out[1] = g->y0 + ((double)j + eta) * g->dy;
    out[2] = g->z0 + ((double)k + zeta) * g->dz;
}

static void put_nan3(double* p) {
    p[0] = NAN;
    p[1] = NAN;
    p[2] = NAN;
}

/*
 * S8: positions at every snapshot time s with from <= s < to (or s <= to
 * when closed), evaluated from the state at the start of the current step
 * (time t, coordinates loc) with tau = s - t.  *next is the first snapshot
 * not yet written.
 */
typedef struct oracle_quad oracle_quad;
static void quad_xyz(const oracle_quad* g, int64_t c, const double* loc, double* out);

/* Snapshot positions in a structured grid (g) or a quadtree grid (qg, when g is NULL). */
static void snapshots_in(const oracle_grid* g, const oracle_quad* qg, const oracle_opts* o, double* row,
                         int32_t* next, int64_t c, const axis_vel* v, const double* loc, double t, double to,
                         int closed) {
    while (*next < o->n_snap) {
        double s = o->snap_times[*next];
        if (closed ? !(s <= to) : !(s < to)) break;
        double tau = s - t;
        double l2[3];
        for (int a = 0; a < 3; ++a) l2[a] = advance(v[a], loc[a], tau);
        if (g)
            global_xyz(g, c, l2[0], l2[1], l2[2], row + 3 * (int64_t)(*next));
        else
            quad_xyz(qg, c, l2, row + 3 * (int64_t)(*next));
        ++*next;
    }
}

static void snapshots(const oracle_grid* g, const oracle_opts* o, double* row, int32_t* next,
                      int64_t c, const axis_vel* v, const double* loc, double t, double to,
                      int closed) {
    snapshots_in(g, NULL, o, row, next, c, v, loc, t, to, closed);
}

static void snapshots_nan(const oracle_opts* o, double* row, int32_t* next) {
    while (*next < o->n_snap) {
        put_nan3(row + 3 * (int64_t)(*next));
        ++*next;
    }
}

/* grids[0 .. n_steps): the field of each time step (n_steps = 1, step_end = NULL: steady). */
static void track_one(const oracle_grid* grids, int32_t n_steps, const double* step_end,
                      const oracle_opts* o, int64_t p, int32_t* cell_, double* xi_, double* eta_,
                      double* zeta_, double* t_, int32_t* status_, int32_t* ncross_, uint64_t* hash_) {
    const oracle_grid* g = grids;
    const int64_t ncell = (int64_t)g->nx * g->ny * g->nz;
    const int64_t plane = (int64_t)g->nx * g->ny;
    double* row = (o->snap_xyz && o->n_snap > 0) ? o->snap_xyz + (int64_t)p * o->n_snap * 3 : NULL;
    int32_t st = status_[p];
    if (st != ST_ACTIVE && st != ST_MAX_TIME) return; /* already terminated: left as is */
    const int fresh = (st == ST_ACTIVE);

    int64_t c = cell_[p];
    double loc[3] = {xi_[p], eta_[p], zeta_[p]};
    double t = t_[p];
    int32_t ncross = ncross_[p];
    uint64_t hash = hash_[p];
    int32_t npath = 0;

    /* S0: release checks, in the field of the time step containing t (the last one
     * when t is at or after every step end) */
    int32_t s = 0;
    if (step_end) {
        while (s < n_steps - 1 && !(t < step_end[s])) ++s;
        g = &grids[s];
    }
    int bad = (c < 0 || c >= ncell);
    if (!bad) bad = !(g->flags[c] & CELL_ACTIVE);
    for (int a = 0; a < 3; ++a)
        if (!(loc[a] >= 0.0 && loc[a] <= 1.0)) bad = 1;
    if (!(t == t) || isinf(t)) bad = 1;
    if (bad) {
        status_[p] = ST_INVALID_START;
        if (row) {
            int32_t k0 = 0;
            snapshots_nan(o, row, &k0);
        }
        return;
    }
    int32_t next = 0;
    if (row) {
        /* snapshots before the release of a fresh particle are undefined;
         * a resumed particle keeps what earlier calls wrote */
        while (next < o->n_snap && o->snap_times[next] < t) {
            if (fresh) put_nan3(row + 3 * (int64_t)next);
            ++next;
        }
    }
    if ((g->flags[c] & CELL_SINK) && o->stop_at_sink) {
        status_[p] = ST_SINK;
        if (row) snapshots_nan(o, row, &next);
        return;
    }
    if (t > o->t_max || (step_end && t > step_end[n_steps - 1])) {
        status_[p] = ST_MAX_TIME;
        if (row) snapshots_nan(o, row, &next);
        return;
    }

    const double V = (g->dx * g->dy) * g->dz;
    const double sgn = direction_sign(o);
    for (;;) {
        /* S1: cell initialisation -- face flows to face velocities */
        int64_t k = c / plane;
        int64_t rem = c - k * plane;
        int64_t j = rem / g->nx;
        int64_t i = rem - j * g->nx;
        double n_c = cell_porosity(g->porosity, g->porosity_scalar, c);
        double d = n_c * V;
        double qxl = g->qx[(k * g->ny + j) * (g->nx + 1) + i];
        double qxh = g->qx[(k * g->ny + j) * (g->nx + 1) + i + 1];
        double qyl = g->qy[(k * (g->ny + 1) + j) * g->nx + i];
        double qyh = g->qy[(k * (g->ny + 1) + j + 1) * g->nx + i];
        double qzl = g->qz[(k * g->ny + j) * g->nx + i];
        double qzh = g->qz[((k + 1) * g->ny + j) * g->nx + i];
        axis_vel v[3];
        v[0].u1 = (sgn * qxl) / d;
        v[0].u2 = (sgn * qxh) / d;
        v[1].u1 = (sgn * qyl) / d;
        v[1].u2 = (sgn * qyh) / d;
        v[2].u1 = (sgn * qzl) / d;
        v[2].u2 = (sgn * qzh) / d;

        /* S2-S4: earliest feasible face; exact ties go to the lowest axis */
        int axis;
        double xe;
        double dt = earliest_exit(v, loc, &axis, &xe);

        /* S5: time limit (strict: a face reached exactly at the limit is crossed).  The
         * limit is t_max, or the end of the current time step when that comes first; at
         * the end of a step that is not the last the particle moves on to the next step. */
        double lim = o->t_max;
        int next_step = 0;
        if (step_end && step_end[s] < lim) {
            lim = step_end[s];
            next_step = (s + 1 < n_steps);
        }
        if (axis < 0 && isinf(lim)) {
            status_[p] = ST_STRANDED;
            if (row) snapshots(g, o, row, &next, c, v, loc, t, INFINITY, 1);
            break;
        }
        double t_exit = t + dt;
        if (t_exit > lim) {
            double tau = lim - t;
            if (row) snapshots(g, o, row, &next, c, v, loc, t, lim, 1);
            for (int a = 0; a < 3; ++a) loc[a] = advance(v[a], loc[a], tau);
            t = lim;
            if (next_step) {
                /* the flow arrays of the next time step; the cell must still be active
                 * in them (else the particle stops as at an inactive cell), and a sink
                 * there stops it as on entry */
                ++s;
                g = &grids[s];
                if (!(g->flags[c] & CELL_ACTIVE)) {
                    status_[p] = ST_INACTIVE_NEIGHBOR;
                    break;
                }
                if ((g->flags[c] & CELL_SINK) && o->stop_at_sink) {
                    status_[p] = ST_SINK;
                    break;
                }
                continue;
            }
            status_[p] = axis < 0 ? ST_STRANDED : ST_MAX_TIME;
            if (row) snapshots_nan(o, row, &next);
            break;
        }

        /* S6: advance to the exit face */
        if (row) snapshots(g, o, row, &next, c, v, loc, t, t_exit, 0);
        for (int a = 0; a < 3; ++a)
            loc[a] = (a == axis) ? xe : advance(v[a], loc[a], dt);
        t = t_exit;
        ncross += 1;
        hash = hash_step(hash, c);
        if (o->path_cap > 0 && npath < o->path_cap) {
            int64_t q = (int64_t)p * o->path_cap + npath;
            o->path_cell[q] = (int32_t)c;
            o->path_face[q] = 2 * axis + (xe == 1.0 ? 1 : 0);
            o->path_t[q] = t;
            global_xyz(g, c, loc[0], loc[1], loc[2], o->path_xyz + 3 * q);
            ++npath;
        }

        /* S7: transfer to the neighbour across the exit face */
        int64_t ii = i, jj = j, kk = k;
        int step = (xe == 1.0) ? 1 : -1;
        if (axis == 0) ii += step;
        else if (axis == 1) jj += step;
        else kk += step;
        if (ii < 0 || ii >= g->nx || jj < 0 || jj >= g->ny || kk < 0 || kk >= g->nz) {
            status_[p] = ST_BOUNDARY;
            break;
        }
        int64_t cn = (kk * g->ny + jj) * g->nx + ii;
        if (!(g->flags[cn] & CELL_ACTIVE)) {
            status_[p] = ST_INACTIVE_NEIGHBOR;
            break;
        }
        c = cn;
        loc[axis] = 1.0 - xe;
        if ((g->flags[c] & CELL_SINK) && o->stop_at_sink) {
            status_[p] = ST_SINK;
            break;
        }
        if (ncross >= o->max_steps) {
            status_[p] = ST_STEP_CAP;
            break;
        }
    }
    int32_t fs = status_[p];
    if (row && (fs == ST_BOUNDARY || fs == ST_SINK || fs == ST_STEP_CAP || fs == ST_INACTIVE_NEIGHBOR))
        snapshots_nan(o, row, &next);

    cell_[p] = (int32_t)c;
    xi_[p] = loc[0];
    eta_[p] = loc[1];
    zeta_[p] = loc[2];
    t_[p] = t;
    ncross_[p] = ncross;
    hash_[p] = hash;
}

/* Track particles [0, n) in place.  Returns 0, or -1 on a bad argument. */
int oracle_track(const oracle_grid* g, const oracle_opts* o, int64_t n, int32_t* cell, double* xi,
                 double* eta, double* zeta, double* t, int32_t* status, int32_t* ncross,
                 uint64_t* hash) {
    if (!g || !o || n < 0 || g->nx <= 0 || g->ny <= 0 || g->nz <= 0) return -1;
    if (n == 0) return 0;
    if (!cell || !xi || !eta || !zeta || !t || !status || !ncross || !hash) return -1;
    if (o->snap_xyz && (o->n_snap < 0 || (o->n_snap > 0 && !o->snap_times))) return -1;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) num_threads(o->n_threads > 0 ? o->n_threads : 1)
#endif
    for (int64_t p = 0; p < n; ++p) {
        track_one(g, 1, NULL, o, p, cell, xi, eta, zeta, t, status, ncross, hash);
        if (o->out_xyz) {
            int64_t c = cell[p];
            if (status[p] == ST_INVALID_START || c < 0 || c >= (int64_t)g->nx * g->ny * g->nz)
                put_nan3(o->out_xyz + 3 * p);
            else
                global_xyz(g, c, xi[p], eta[p], zeta[p], o->out_xyz + 3 * p);
        }
    }
    return 0;
}

/* Transient flow: grids[s] is the field of time step s, valid up to step_end[s] (strictly
 * increasing, the last may be +inf); every grid has the same geometry.  Forward only. */
int oracle_track_transient(const oracle_grid* grids, int32_t n_steps, const double* step_end,
                           const oracle_opts* o, int64_t n, int32_t* cell, double* xi, double* eta,
                           double* zeta, double* t, int32_t* status, int32_t* ncross, uint64_t* hash) {
    if (!grids || !step_end || n_steps < 1 || !o || n < 0 || o->direction != 1) return -1;
    for (int32_t q = 0; q < n_steps; ++q) {
        const oracle_grid* a = &grids[q];
        if (a->nx != grids[0].nx || a->ny != grids[0].ny || a->nz != grids[0].nz || a->nx <= 0 ||
            a->ny <= 0 || a->nz <= 0)
            return -1;
        if (isnan(step_end[q]) || (q > 0 && !(step_end[q] > step_end[q - 1]))) return -1;
    }
    if (n == 0) return 0;
    if (!cell || !xi || !eta || !zeta || !t || !status || !ncross || !hash) return -1;
    if (o->snap_xyz && (o->n_snap < 0 || (o->n_snap > 0 && !o->snap_times))) return -1;
    const oracle_grid* g = grids;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) num_threads(o->n_threads > 0 ? o->n_threads : 1)
#endif
    for (int64_t p = 0; p < n; ++p) {
        track_one(grids, n_steps, step_end, o, p, cell, xi, eta, zeta, t, status, ncross, hash);
        if (o->out_xyz) {
            int64_t c = cell[p];
            if (status[p] == ST_INVALID_START || c < 0 || c >= (int64_t)g->nx * g->ny * g->nz)
                put_nan3(o->out_xyz + 3 * p);
            else
                global_xyz(g, c, xi[p], eta[p], zeta[p], o->out_xyz + 3 * p);
        }
    }
    return 0;
}

/* ============================================================================================
 * Quadtree (rectangular unstructured) grids.  The paper's second test case refines its grid
 * with a quadtree (Methods "Synthetic test cases") and defers the tracking to MODPATH; the
 * per-cell step is unchanged, only the geometry and the neighbour lookup differ.  Readings:
 *   - a cell is a box [x_lo, x_lo + hx] x [y_lo, y_lo + hy] x [z_lo, z_lo + hz]; local
 *     coordinates are (x - x_lo)/hx etc.;
 *   - a face may be split into subfaces, each shared with one neighbour (or the domain
 *     boundary); the face velocity of the linear interpolation is the face's total flow
 *     (the sum of its subfaces' flows, in their order) over n V of the cell;
 *   - a particle leaving through a face enters the neighbour of the subface that contains
 *     its exit point (the first one in order when the point is on an edge between two);
 *   - in the neighbour, the coordinate along the exit axis is that of the entry face; a
 *     coordinate along a face axis carries over unchanged when both cells span the same
 *     range on that axis, otherwise it is mapped through the global coordinate (and clamped
 *     to [0, 1]).
 * ============================================================================================ */
struct oracle_quad {
    int32_t ncell;
    const double* box;        /* [ncell][6]: x_lo, y_lo, z_lo, hx, hy, hz */
    const int32_t* sub_off;   /* [ncell*6 + 1]: subfaces of face f = 2*axis + side of cell c */
    const int32_t* sub_nb;    /* [nsub] neighbour cell, -1 = domain boundary */
    const double* sub_q;      /* [nsub] flow, + = +axis */
    const double* sub_lo;     /* [nsub][2] extent in the face's tangential local coordinates */
    const double* sub_hi;     /* [nsub][2] (x-face: eta, zeta; y-face: xi, zeta; z-face: xi, eta) */
    const double* porosity;   /* [ncell] or NULL */
    double porosity_scalar;
    const int32_t* flags;     /* [ncell] */
};

static void quad_xyz(const oracle_quad* g, int64_t c, const double* loc, double* out) {
    const double* b = g->box + 6 * c;
    out[0] = b[0] + loc[0] * b[3];
    out[1] = b[1] + loc[1] * b[4];
    out[2] = b[2] + loc[2] * b[5];
}

static void quad_snapshots(const oracle_quad* g, const oracle_opts* o, double* row, int32_t* next, int64_t c,
                           const axis_vel* v, const double* loc, double t, double to, int closed) {
    snapshots_in(NULL, g, o, row, next, c, v, loc, t, to, closed);
}

#define QUAD_ZERO_RUN 16

/* snapshots after a particle stopped on a circuit of zero-time crossings: it stays put */
static void quad_snapshots_fixed(const oracle_quad* g, const oracle_opts* o, double* row, int32_t* next,
                                 int64_t c, const double* loc) {
    while (*next < o->n_snap && o->snap_times[*next] <= o->t_max) {
        quad_xyz(g, c, loc, row + 3 * (int64_t)(*next));
        ++*next;
    }
    snapshots_nan(o, row, next);
}

static void track_one_quad(const oracle_quad* g, const oracle_opts* o, int64_t p, int32_t* cell_,
                           double* xi_, double* eta_, double* zeta_, double* t_, int32_t* status_,
                           int32_t* ncross_, uint64_t* hash_) {
    double* row = (o->snap_xyz && o->n_snap > 0) ? o->snap_xyz + (int64_t)p * o->n_snap * 3 : NULL;
    int32_t st = status_[p];
    if (st != ST_ACTIVE && st != ST_MAX_TIME) return;
    const int fresh = (st == ST_ACTIVE);
    int64_t c = cell_[p];
    double loc[3] = {xi_[p], eta_[p], zeta_[p]};
    double t = t_[p];
    int32_t ncross = ncross_[p];
    uint64_t hash = hash_[p];
    int32_t npath = 0;
    int32_t zero_run = 0;

    /* S0 */
    int bad = (c < 0 || c >= g->ncell);
    if (!bad) bad = !(g->flags[c] & CELL_ACTIVE);
    for (int a = 0; a < 3; ++a)
        if (!(loc[a] >= 0.0 && loc[a] <= 1.0)) bad = 1;
    if (!(t == t) || isinf(t)) bad = 1;
    if (bad) {
        status_[p] = ST_INVALID_START;
        if (row) {
            int32_t k0 = 0;
            snapshots_nan(o, row, &k0);
        }
        return;
    }
    int32_t next = 0;
    if (row) {
        while (next < o->n_snap && o->snap_times[next] < t) {
            if (fresh) put_nan3(row + 3 * (int64_t)next);
            ++next;
        }
    }
    if ((g->flags[c] & CELL_SINK) && o->stop_at_sink) {
        status_[p] = ST_SINK;
        if (row) snapshots_nan(o, row, &next);
        return;
    }
    if (t > o->t_max) {
        status_[p] = ST_MAX_TIME;
        if (row) snapshots_nan(o, row, &next);
        return;
    }
    const double sgn = direction_sign(o);
    for (;;) {
        /* S1: face velocities from the total flow of each face */
        const double* b = g->box + 6 * c;
        const double V = (b[3] * b[4]) * b[5];
        const double n_c = cell_porosity(g->porosity, g->porosity_scalar, c);
        const double d = n_c * V;
        double face_u[6];
        for (int f = 0; f < 6; ++f) {
            double Q = 0.0;
            for (int32_t q = g->sub_off[6 * c + f]; q < g->sub_off[6 * c + f + 1]; ++q) Q += g->sub_q[q];
            face_u[f] = (sgn * Q) / d;
        }
        axis_vel v[3];
        for (int a = 0; a < 3; ++a) {
            v[a].u1 = face_u[2 * a];
            v[a].u2 = face_u[2 * a + 1];
        }

        /* S2-S4 */
        int axis;
        double xe;
        double dt = earliest_exit(v, loc, &axis, &xe);

        /* S5 */
        if (axis < 0 && isinf(o->t_max)) {
            status_[p] = ST_STRANDED;
            if (row) quad_snapshots(g, o, row, &next, c, v, loc, t, INFINITY, 1);
            break;
        }
        double t_exit = t + dt;
        if (t_exit > o->t_max) {
            double tau = o->t_max - t;
            if (row) quad_snapshots(g, o, row, &next, c, v, loc, t, o->t_max, 1);
            for (int a = 0; a < 3; ++a) loc[a] = advance(v[a], loc[a], tau);
            t = o->t_max;
            status_[p] = axis < 0 ? ST_STRANDED : ST_MAX_TIME;
            if (row) snapshots_nan(o, row, &next);
            break;
        }

        /* S6 */
        if (row) quad_snapshots(g, o, row, &next, c, v, loc, t, t_exit, 0);
        for (int a = 0; a < 3; ++a)
            loc[a] = (a == axis) ? xe : advance(v[a], loc[a], dt);
        t = t_exit;
        ncross += 1;
        hash = hash_step(hash, c);
        const int face = 2 * axis + (xe == 1.0 ? 1 : 0);
        if (o->path_cap > 0 && npath < o->path_cap) {
            int64_t q = (int64_t)p * o->path_cap + npath;
            o->path_cell[q] = (int32_t)c;
            o->path_face[q] = face;
            o->path_t[q] = t;
            quad_xyz(g, c, loc, o->path_xyz + 3 * q);
            ++npath;
        }

        /* S7: the subface holding the exit point (the first in order when the point is on an
         * edge between two), then the neighbour's coordinates */
        const int ta1 = (axis == 0) ? 1 : 0;          /* the face's two tangential axes */
        const int ta2 = (axis == 2) ? 1 : 2;
        const int32_t q0 = g->sub_off[6 * c + face], q1 = g->sub_off[6 * c + face + 1];
        int32_t hit = q1 - 1;
        for (int32_t q = q0; q < q1; ++q) {
            const double* lo = g->sub_lo + 2 * q;
            const double* hi = g->sub_hi + 2 * q;
            if (lo[0] <= loc[ta1] && loc[ta1] <= hi[0] && lo[1] <= loc[ta2] && loc[ta2] <= hi[1]) {
                hit = q;
                break;
            }
        }
        const int64_t cn = (q1 > q0) ? g->sub_nb[hit] : -1;
        if (cn < 0) {
            status_[p] = ST_BOUNDARY;
            break;
        }
        if (!(g->flags[cn] & CELL_ACTIVE)) {
            status_[p] = ST_INACTIVE_NEIGHBOR;
            break;
        }
        const double* bn = g->box + 6 * cn;
        const int tang[2] = {ta1, ta2};
        for (int m = 0; m < 2; ++m) {
            const int a = tang[m];
            if (bn[a] == b[a] && bn[3 + a] == b[3 + a]) continue;   /* same span: unchanged */
            const double x = b[a] + loc[a] * b[3 + a];
            double l = (x - bn[a]) / bn[3 + a];
            if (l < 0.0) l = 0.0;
            if (l > 1.0) l = 1.0;
            loc[a] = l;
        }
        loc[axis] = 1.0 - xe;
        c = cn;
        if ((g->flags[c] & CELL_SINK) && o->stop_at_sink) {
            status_[p] = ST_SINK;
            break;
        }
        if (ncross >= o->max_steps) {
            status_[p] = ST_STEP_CAP;
            break;
        }
        /* The face velocities of a cell whose face is split are averages over the subfaces, so
         * around a point where cells meet the velocities can hand a particle on in a closed
         * circuit of zero-time crossings.  After QUAD_ZERO_RUN of them in a row it is stopped
         * there as stranded. */
        if (dt == 0.0) {
            if (++zero_run >= QUAD_ZERO_RUN) {
                status_[p] = ST_STRANDED;
                break;
            }
        } else {
            zero_run = 0;
        }
    }
    int32_t fs = status_[p];
    if (row && (fs == ST_BOUNDARY || fs == ST_SINK || fs == ST_STEP_CAP || fs == ST_INACTIVE_NEIGHBOR))
        snapshots_nan(o, row, &next);
    if (row && fs == ST_STRANDED && zero_run >= QUAD_ZERO_RUN) {
        /* stranded on a circuit: the position holds for every later snapshot */
        quad_snapshots_fixed(g, o, row, &next, c, loc);
    }
    cell_[p] = (int32_t)c;
    xi_[p] = loc[0];
    eta_[p] = loc[1];
    zeta_[p] = loc[2];
    t_[p] = t;
    ncross_[p] = ncross;
    hash_[p] = hash;
}

int oracle_track_quad(const oracle_quad* g, const oracle_opts* o, int64_t n, int32_t* cell, double* xi,
                      double* eta, double* zeta, double* t, int32_t* status, int32_t* ncross, uint64_t* hash) {
    if (!g || !o || n < 0 || g->ncell <= 0 || !g->box || !g->sub_off || !g->flags) return -1;
    if (n == 0) return 0;
    if (!cell || !xi || !eta || !zeta || !t || !status || !ncross || !hash) return -1;
    if (o->snap_xyz && (o->n_snap < 0 || (o->n_snap > 0 && !o->snap_times))) return -1;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) num_threads(o->n_threads > 0 ? o->n_threads : 1)
#endif
    for (int64_t p = 0; p < n; ++p) {
        track_one_quad(g, o, p, cell, xi, eta, zeta, t, status, ncross, hash);
        if (o->out_xyz) {
            int64_t c = cell[p];
            if (status[p] == ST_INVALID_START || c < 0 || c >= g->ncell) {
                put_nan3(o->out_xyz + 3 * p);
            } else {
                const double loc[3] = {xi[p], eta[p], zeta[p]};
                quad_xyz(g, c, loc, o->out_xyz + 3 * p);
            }
        }
    }
    return 0;
}

