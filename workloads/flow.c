/*
 * Steady groundwater-flow solve that produces the cell-by-cell face flows a
 * particle tracker consumes.  It stands in for the MODFLOW model the paper
 * post-processes (Introduction; Methods, "MODPATH"): the tracker only ever
 * sees face flows, so how they were computed does not enter the tracking.
 *
 * Discretisation: 7-point block-centred finite volumes on a uniform grid,
 * harmonic-mean face conductances, fixed heads on the west (i = 0) and east
 * (i = nx) domain faces with half-cell conductance 2*K*area/d, no flow on the
 * other domain faces except a recharge inflow R*dx*dy through the top face of
 * layer k = 0 (flow in +k), and optional per-cell source terms (wells,
 * negative = extraction).  Face flows are positive in the +i / +j / +k
 * direction, m^3/d.
 *
 * Solver: conjugate gradients in FP64, preconditioned by exact solves of the
 * vertical (k) line of each column (the vertical coupling dominates for flat
 * cells).  Dot products are accumulated in fixed chunks and summed in a fixed
 * order so the result does not depend on the number of threads.
 *
 * Input generation only: this file holds none of the tracking arithmetic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define CHUNK 4096

static double hm2(double a, double b) { return (a > 0.0 && b > 0.0) ? 2.0 * a * b / (a + b) : 0.0; }

typedef struct {
    int nx, ny, nz;
    int64_t n;
    double *cx, *cy, *cz;   /* face conductances, sizes (nx+1)ny nz, nx(ny+1)nz, nx ny(nz+1) */
    double *diag;
    double *lu_d, *lu_u;    /* Thomas factors of each vertical line */
    double *part;           /* per-chunk partial sums */
    int64_t nchunk;
} sys_t;

#define IX(i, j, k) (((int64_t)(k) * s->ny + (j)) * s->nx + (i))
#define FX(i, j, k) (((int64_t)(k) * s->ny + (j)) * (s->nx + 1) + (i))
#define FY(i, j, k) (((int64_t)(k) * (s->ny + 1) + (j)) * s->nx + (i))
#define FZ(i, j, k) (((int64_t)(k) * s->ny + (j)) * s->nx + (i))

static void matvec(const sys_t* s, const double* x, double* y) {
    const int nx = s->nx, ny = s->ny, nz = s->nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t c = IX(i, j, k);
                double v = s->diag[c] * x[c];
                if (i > 0) v -= s->cx[FX(i, j, k)] * x[c - 1];
                if (i < nx - 1) v -= s->cx[FX(i + 1, j, k)] * x[c + 1];
                if (j > 0) v -= s->cy[FY(i, j, k)] * x[c - nx];
                if (j < ny - 1) v -= s->cy[FY(i, j + 1, k)] * x[c + nx];
                if (k > 0) v -= s->cz[FZ(i, j, k)] * x[c - (int64_t)nx * ny];
                if (k < nz - 1) v -= s->cz[FZ(i, j, k + 1)] * x[c + (int64_t)nx * ny];
                y[c] = v;
            }
}

static double dot(const sys_t* s, const double* a, const double* b) {
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < s->nchunk; ++q) {
        int64_t lo = q * CHUNK, hi = lo + CHUNK < s->n ? lo + CHUNK : s->n;
        double acc = 0.0;
        for (int64_t c = lo; c < hi; ++c) acc += a[c] * b[c];
        s->part[q] = acc;
    }
    double t = 0.0;
    for (int64_t q = 0; q < s->nchunk; ++q) t += s->part[q];
    return t;
}

/* Factor the tridiagonal vertical line of every column once. */
static void line_factor(sys_t* s) {
    const int nx = s->nx, ny = s->ny, nz = s->nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double prev_u = 0.0;
            for (int k = 0; k < nz; ++k) {
                int64_t c = IX(i, j, k);
                double lower = k > 0 ? -s->cz[FZ(i, j, k)] : 0.0;
                double d = s->diag[c] - lower * prev_u;
                double upper = k < nz - 1 ? -s->cz[FZ(i, j, k + 1)] : 0.0;
                s->lu_d[c] = d;
                s->lu_u[c] = upper / d;
                prev_u = s->lu_u[c];
            }
        }
}

static void line_solve(const sys_t* s, const double* r, double* z) {
    const int nx = s->nx, ny = s->ny, nz = s->nz;
    const int64_t plane = (int64_t)nx * ny;
#pragma omp parallel for collapse(2) schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double prev = 0.0;
            for (int k = 0; k < nz; ++k) {
                int64_t c = IX(i, j, k);
                double lower = k > 0 ? -s->cz[FZ(i, j, k)] : 0.0;
                prev = (r[c] - lower * prev) / s->lu_d[c];
                z[c] = prev;
            }
            for (int k = nz - 2; k >= 0; --k) {
                int64_t c = IX(i, j, k);
                z[c] -= s->lu_u[c] * z[c + plane];
            }
        }
}

/*
 * Returns 0 on convergence, 1 if max_iter was reached, -1 on bad input.
 * head [nz][ny][nx]; qx [nz][ny][nx+1]; qy [nz][ny+1][nx]; qz [nz+1][ny][nx].
 */
int flow_solve(int nx, int ny, int nz, double dx, double dy, double dz, const double* K,
               double h_west, double h_east, double recharge, const double* source, double rtol,
               int max_iter, int nthreads, double* head, double* qx, double* qy, double* qz,
               double* out_relres, int* out_iters) {
    if (nx <= 0 || ny <= 0 || nz <= 0 || !(dx > 0) || !(dy > 0) || !(dz > 0) || !K || !head || !qx ||
        !qy || !qz)
        return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    sys_t S, *s = &S;
    s->nx = nx; s->ny = ny; s->nz = nz;
    s->n = (int64_t)nx * ny * nz;
    s->nchunk = (s->n + CHUNK - 1) / CHUNK;
    int64_t nfx = (int64_t)(nx + 1) * ny * nz, nfy = (int64_t)nx * (ny + 1) * nz,
            nfz = (int64_t)nx * ny * (nz + 1);
    s->cx = calloc(nfx, sizeof(double));
    s->cy = calloc(nfy, sizeof(double));
    s->cz = calloc(nfz, sizeof(double));
    s->diag = calloc(s->n, sizeof(double));
    s->lu_d = calloc(s->n, sizeof(double));
    s->lu_u = calloc(s->n, sizeof(double));
    s->part = calloc(s->nchunk, sizeof(double));
    double* b = calloc(s->n, sizeof(double));
    double* r = calloc(s->n, sizeof(double));
    double* z = calloc(s->n, sizeof(double));
    double* p = calloc(s->n, sizeof(double));
    double* q = calloc(s->n, sizeof(double));
    const double ax = dy * dz, ay = dx * dz, az = dx * dy;

    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j) {
            for (int i = 0; i <= nx; ++i) {
                double c;
                if (i == 0) c = 2.0 * K[IX(0, j, k)] * ax / dx;
                else if (i == nx) c = 2.0 * K[IX(nx - 1, j, k)] * ax / dx;
                else c = hm2(K[IX(i - 1, j, k)], K[IX(i, j, k)]) * ax / dx;
                s->cx[FX(i, j, k)] = c;
            }
        }
    for (int k = 0; k < nz; ++k)
        for (int j = 1; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                s->cy[FY(i, j, k)] = hm2(K[IX(i, j - 1, k)], K[IX(i, j, k)]) * ay / dy;
    for (int k = 1; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                s->cz[FZ(i, j, k)] = hm2(K[IX(i, j, k - 1)], K[IX(i, j, k)]) * az / dz;

    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t c = IX(i, j, k);
                double d = s->cx[FX(i, j, k)] + s->cx[FX(i + 1, j, k)];
                if (j > 0) d += s->cy[FY(i, j, k)];
                if (j < ny - 1) d += s->cy[FY(i, j + 1, k)];
                if (k > 0) d += s->cz[FZ(i, j, k)];
                if (k < nz - 1) d += s->cz[FZ(i, j, k + 1)];
                s->diag[c] = d;
                double rhs = source ? source[c] : 0.0;
                if (i == 0) rhs += s->cx[FX(0, j, k)] * h_west;
                if (i == nx - 1) rhs += s->cx[FX(nx, j, k)] * h_east;
                if (k == 0) rhs += recharge * az;
                b[c] = rhs;
            }
    line_factor(s);

    /* initial guess: linear west-east head */
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                head[IX(i, j, k)] = h_west + (h_east - h_west) * ((i + 0.5) / nx);

    matvec(s, head, q);
    for (int64_t c = 0; c < s->n; ++c) r[c] = b[c] - q[c];
    double bnorm = sqrt(dot(s, b, b));
    if (bnorm == 0.0) bnorm = 1.0;
    line_solve(s, r, z);
    memcpy(p, z, s->n * sizeof(double));
    double rz = dot(s, r, z);
    double rel = sqrt(dot(s, r, r)) / bnorm;
    int it = 0;
    while (rel > rtol && it < max_iter) {
        matvec(s, p, q);
        double pq = dot(s, p, q);
        if (!(pq > 0.0) || !(rz > 0.0)) break; /* breakdown at the rounding floor */
        double alpha = rz / pq;
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < s->n; ++c) {
            head[c] += alpha * p[c];
            r[c] -= alpha * q[c];
        }
        ++it;
        /* refresh the true residual now and then to avoid drift */
        if (it % 200 == 0) {
            matvec(s, head, q);
            for (int64_t c = 0; c < s->n; ++c) r[c] = b[c] - q[c];
        }
        rel = sqrt(dot(s, r, r)) / bnorm;
        if (rel <= rtol) {
            /* confirm with the true residual; restart the recurrence if it drifted */
            matvec(s, head, q);
            for (int64_t c = 0; c < s->n; ++c) r[c] = b[c] - q[c];
            rel = sqrt(dot(s, r, r)) / bnorm;
            if (rel <= rtol) break;
            line_solve(s, r, z);
            memcpy(p, z, s->n * sizeof(double));
            rz = dot(s, r, z);
            continue;
        }
        line_solve(s, r, z);
        double rz_new = dot(s, r, z);
        double beta = rz_new / rz;
        rz = rz_new;
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < s->n; ++c) p[c] = z[c] + beta * p[c];
    }
    /* true residual */
    matvec(s, head, q);
    for (int64_t c = 0; c < s->n; ++c) r[c] = b[c] - q[c];
    rel = sqrt(dot(s, r, r)) / bnorm;

    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                double c = s->cx[FX(i, j, k)];
                double v;
                if (i == 0) v = c * (h_west - head[IX(0, j, k)]);
                else if (i == nx) v = c * (head[IX(nx - 1, j, k)] - h_east);
                else v = c * (head[IX(i - 1, j, k)] - head[IX(i, j, k)]);
                qx[FX(i, j, k)] = v;
            }
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double v = 0.0;
                if (j > 0 && j < ny) v = s->cy[FY(i, j, k)] * (head[IX(i, j - 1, k)] - head[IX(i, j, k)]);
                qy[FY(i, j, k)] = v;
            }
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double v = 0.0;
                if (k == 0) v = recharge * az;
                else if (k < nz) v = s->cz[FZ(i, j, k)] * (head[IX(i, j, k - 1)] - head[IX(i, j, k)]);
                qz[FZ(i, j, k)] = v;
            }

    if (out_relres) *out_relres = rel;
    if (out_iters) *out_iters = it;
    free(s->cx); free(s->cy); free(s->cz); free(s->diag); free(s->lu_d); free(s->lu_u);
    free(s->part); free(b); free(r); free(z); free(p); free(q);
    return rel <= rtol ? 0 : 1;
}
