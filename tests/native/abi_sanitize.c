/* Host AddressSanitizer / UndefinedBehaviorSanitizer run of libpt's argument validation (the
 * library built with the sanitizers on its host code only).  Every call here fails validation,
 * finds no device, or is a no-op, so no device work is done: bad pointers and sizes, non-finite
 * and unbalanced host flows read over exactly sized arrays, quadtree descriptions with bad
 * offsets and extents, forged and released handles.  Exits 0 when every call returns the
 * expected code; any sanitizer report fails the calling test. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pt.h"

static int failures = 0;

static void expect(int got, int want, const char* what) {
    if (got != want) {
        fprintf(stderr, "%s: got %d, want %d (%s)\n", what, got, want, pt_last_error());
        ++failures;
    }
}

/* an exactly sized host grid (malloc'd: the sanitizer sees reads past its end) */
typedef struct {
    pt_grid_desc d;
    double *qx, *qy, *qz, *por;
    int32_t* flags;
} host_grid;

static void make_grid(host_grid* g, int nx, int ny, int nz) {
    memset(g, 0, sizeof *g);
    const size_t nfx = (size_t)(nx + 1) * ny * nz, nfy = (size_t)nx * (ny + 1) * nz, nfz = (size_t)nx * ny * (nz + 1);
    const size_t nc = (size_t)nx * ny * nz;
    g->qx = malloc(sizeof(double) * nfx);
    g->qy = malloc(sizeof(double) * nfy);
    g->qz = malloc(sizeof(double) * nfz);
    g->por = malloc(sizeof(double) * nc);
    g->flags = malloc(sizeof(int32_t) * nc);
    for (size_t q = 0; q < nfx; ++q) g->qx[q] = 1.0;   /* uniform flow along i: balanced */
    for (size_t q = 0; q < nfy; ++q) g->qy[q] = 0.0;
    for (size_t q = 0; q < nfz; ++q) g->qz[q] = 0.0;
    for (size_t c = 0; c < nc; ++c) {
        g->por[c] = 0.3;
        g->flags[c] = PT_CELL_ACTIVE;
    }
    pt_grid_desc d = {nx, ny, nz, 10.0, 10.0, 2.0, 0.0, 0.0, 0.0, g->qx, g->qy, g->qz, g->por, 0.3, g->flags,
                      PT_MEM_HOST, 1e-9};
    g->d = d;
}

static void free_grid(host_grid* g) {
    free(g->qx);
    free(g->qy);
    free(g->qz);
    free(g->por);
    free(g->flags);
}

int main(void) {
    pt_grid* out = NULL;
    expect(pt_version() >= 100, 1, "version");
    pt_track_opts o;
    pt_default_opts(&o);
    pt_default_opts(NULL);
    expect(pt_load_grid(NULL, NULL, &out), PT_ERR_INVALID_ARG, "NULL desc");
    host_grid g;
    make_grid(&g, 5, 4, 3);
    expect(pt_load_grid(&g.d, NULL, NULL), PT_ERR_INVALID_ARG, "NULL out");
    pt_grid_desc d = g.d;
    d.nx = 0;
    expect(pt_load_grid(&d, NULL, &out), PT_ERR_INVALID_ARG, "nx = 0");
    d = g.d;
    d.dy = NAN;
    expect(pt_load_grid(&d, NULL, &out), PT_ERR_INVALID_ARG, "dy NaN");
    d = g.d;
    d.qz = NULL;
    expect(pt_load_grid(&d, NULL, &out), PT_ERR_INVALID_ARG, "qz NULL");
    d = g.d;
    d.porosity = NULL;
    d.porosity_scalar = -1.0;
    expect(pt_load_grid(&d, NULL, &out), PT_ERR_INVALID_ARG, "porosity scalar");
    d = g.d;
    d.mem = 7;
    expect(pt_load_grid(&d, NULL, &out), PT_ERR_INVALID_ARG, "mem");
    d = g.d;
    d.balance_tol = NAN;
    expect(pt_load_grid(&d, NULL, &out), PT_ERR_INVALID_ARG, "balance NaN");
    d = g.d;
    d.nx = 1 << 16;
    d.ny = 1 << 16;
    expect(pt_load_grid(&d, NULL, &out), PT_ERR_UNSUPPORTED, "too large");
    /* the last element of each host array is read and rejected */
    g.qz[5 * 4 * 4 - 1] = INFINITY;
    expect(pt_load_grid(&g.d, NULL, &out), PT_ERR_INVALID_ARG, "qz last inf");
    g.qz[5 * 4 * 4 - 1] = 0.0;
    g.por[5 * 4 * 3 - 1] = 0.0;
    expect(pt_load_grid(&g.d, NULL, &out), PT_ERR_INVALID_ARG, "porosity last 0");
    g.por[5 * 4 * 3 - 1] = 0.3;
    g.flags[5 * 4 * 3 - 1] = 8;
    expect(pt_load_grid(&g.d, NULL, &out), PT_ERR_INVALID_ARG, "flags last");
    g.flags[5 * 4 * 3 - 1] = PT_CELL_ACTIVE;
    g.qy[5 * 5 * 3 - 1] = 0.5;   /* the last j face of the last cell: that cell no longer balances */
    expect(pt_load_grid(&g.d, NULL, &out), PT_ERR_UNBALANCED, "unbalanced last cell");
    g.qy[5 * 5 * 3 - 1] = 0.0;
    /* a valid host grid: validation passes, then no device */
    expect(pt_load_grid(&g.d, NULL, &out), PT_ERR_NO_DEVICE, "valid grid, no device");
    free_grid(&g);

    /* quadtree descriptions */
    double box[6] = {0, 0, 0, 1, 1, 1};
    int32_t off[7] = {0, 0, 0, 0, 0, 0, 0};
    pt_quad_desc q = {1, 0, box, off, NULL, NULL, NULL, NULL, NULL, 0.3, NULL, PT_MEM_HOST, -1.0};
    expect(pt_load_quad_grid(&q, NULL, NULL), PT_ERR_INVALID_ARG, "quad NULL out");
    expect(pt_load_quad_grid(NULL, NULL, &out), PT_ERR_INVALID_ARG, "quad NULL desc");
    q.mem = PT_MEM_DEVICE;
    expect(pt_load_quad_grid(&q, NULL, &out), PT_ERR_UNSUPPORTED, "quad device");
    q.mem = PT_MEM_HOST;
    off[6] = 1;
    expect(pt_load_quad_grid(&q, NULL, &out), PT_ERR_INVALID_ARG, "quad offsets end");
    off[6] = 0;
    int32_t* nb = malloc(sizeof(int32_t));
    double* sq = malloc(sizeof(double));
    double* lo = malloc(2 * sizeof(double));
    double* hi = malloc(2 * sizeof(double));
    nb[0] = 5;
    sq[0] = 1.0;
    lo[0] = lo[1] = 0.0;
    hi[0] = hi[1] = 1.0;
    int32_t off1[7] = {0, 0, 1, 1, 1, 1, 1};
    pt_quad_desc q1 = {1, 1, box, off1, nb, sq, lo, hi, NULL, 0.3, NULL, PT_MEM_HOST, -1.0};
    expect(pt_load_quad_grid(&q1, NULL, &out), PT_ERR_INVALID_ARG, "quad neighbour out of range");
    nb[0] = -1;
    hi[1] = 1.5;
    expect(pt_load_quad_grid(&q1, NULL, &out), PT_ERR_INVALID_ARG, "quad extent");
    hi[1] = 1.0;
    box[4] = 0.0;
    expect(pt_load_quad_grid(&q1, NULL, &out), PT_ERR_INVALID_ARG, "quad box");
    box[4] = 1.0;
    expect(pt_load_quad_grid(&q1, NULL, &out), PT_ERR_NO_DEVICE, "quad valid, no device");
    free(nb);
    free(sq);
    free(lo);
    free(hi);

    /* handles */
    pt_particles p;
    memset(&p, 0, sizeof p);
    pt_run* run = NULL;
    expect(pt_track(NULL, 1, &p, &o, NULL, &run), PT_ERR_INVALID_ARG, "track NULL grids");
    void* forged = malloc(64);
    memset(forged, 0x44, 64);
    const pt_grid* gl[1] = {(const pt_grid*)forged};
    expect(pt_track(gl, 1, &p, &o, NULL, &run), PT_ERR_BAD_HANDLE, "track forged grid");
    expect(pt_track(gl, 1, &p, &o, NULL, NULL), PT_ERR_INVALID_ARG, "track NULL out");
    expect(pt_release(NULL), PT_OK, "release NULL");
    expect(pt_release(forged), PT_ERR_BAD_HANDLE, "release forged");
    pt_summary s;
    expect(pt_results((pt_run*)forged, &s), PT_ERR_BAD_HANDLE, "results forged");
    int64_t counts[PT_COUNTS_WORDS];
    expect(pt_track_noalloc(gl, 1, &p, &o, NULL, NULL), PT_ERR_INVALID_ARG, "noalloc NULL counts");
    expect(pt_track_noalloc(gl, 1, &p, &o, NULL, counts), PT_ERR_BAD_HANDLE, "noalloc forged grid");
    free(forged);
    expect(pt_shutdown(), PT_OK, "shutdown");
    if (failures) return 1;
    printf("libpt sanitize run ok\n");
    return 0;
}
