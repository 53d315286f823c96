/* Host AddressSanitizer / UndefinedBehaviorSanitizer run of the oracle (built into this one
 * translation unit): small grids with random and degenerate flows, every kind of start, stop and
 * output (endpoint, snapshots, pathline records with small capacities, transient steps, a
 * quadtree grid with split faces).  Exits 0; any sanitizer report fails the calling test. */
#include "../../oracle/pt_oracle.c"

#include <stdio.h>
#include <stdlib.h>

static double urand(uint64_t* s) {
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(*s >> 11) * 0x1p-53;
}

static void fill_flows(double* q, int64_t m, uint64_t* s, double scale) {
    for (int64_t i = 0; i < m; ++i) {
        const double r = urand(s);
        q[i] = r < 0.05 ? 0.0 : scale * (urand(s) - 0.3);
    }
}

int main(void) {
    uint64_t seed = 12345;
    const int nx = 7, ny = 5, nz = 3;
    const int64_t ncell = (int64_t)nx * ny * nz;
    double* qx = malloc(sizeof(double) * (nx + 1) * ny * nz);
    double* qy = malloc(sizeof(double) * nx * (ny + 1) * nz);
    double* qz = malloc(sizeof(double) * nx * ny * (nz + 1));
    double* por = malloc(sizeof(double) * ncell);
    int32_t* flags = malloc(sizeof(int32_t) * ncell);
    fill_flows(qx, (int64_t)(nx + 1) * ny * nz, &seed, 4.0);
    fill_flows(qy, (int64_t)nx * (ny + 1) * nz, &seed, 2.0);
    fill_flows(qz, (int64_t)nx * ny * (nz + 1), &seed, 0.5);
    for (int64_t c = 0; c < ncell; ++c) {
        por[c] = 0.2 + 0.2 * urand(&seed);
        flags[c] = 1 | (urand(&seed) < 0.05 ? 2 : 0);
    }
    flags[5] = 0;   /* an inactive cell */
    oracle_grid g = {nx, ny, nz, 3.0, 2.0, 1.0, 10.0, -5.0, 2.0, qx, qy, qz, por, 0.3, flags};
    const int64_t n = 400;
    int32_t* cell = malloc(sizeof(int32_t) * n);
    double *xi = malloc(sizeof(double) * n), *eta = malloc(sizeof(double) * n), *zeta = malloc(sizeof(double) * n);
    double* t = malloc(sizeof(double) * n);
    int32_t *status = malloc(sizeof(int32_t) * n), *ncross = malloc(sizeof(int32_t) * n);
    uint64_t* hash = malloc(sizeof(uint64_t) * n);
    const int n_snap = 9;
    double snaps[9] = {0.0, 0.5, 1.0, 2.0, 5.0, 10.0, 20.0, 50.0, 100.0};
    double* snap_xyz = malloc(sizeof(double) * n * n_snap * 3);
    double* out_xyz = malloc(sizeof(double) * n * 3);
    const int cap = 5;
    int32_t *pc = malloc(sizeof(int32_t) * n * cap), *pf = malloc(sizeof(int32_t) * n * cap);
    double *pt = malloc(sizeof(double) * n * cap), *px = malloc(sizeof(double) * n * cap * 3);
    for (int rep = 0; rep < 6; ++rep) {
        for (int64_t p = 0; p < n; ++p) {
            cell[p] = (int32_t)(urand(&seed) * ncell);
            xi[p] = urand(&seed);
            eta[p] = urand(&seed);
            zeta[p] = urand(&seed);
            t[p] = (p % 7 == 0) ? 3.0 : 0.0;
            status[p] = (p % 31 == 0) ? 3 : 0;
            ncross[p] = 0;
            hash[p] = 0xcbf29ce484222325ull;
        }
        cell[0] = -3;            /* invalid starts */
        cell[1] = (int32_t)ncell;
        xi[2] = 1.5;
        eta[3] = __builtin_nan("");
        t[4] = __builtin_inf();
        xi[6] = 1.0;             /* on a face */
        oracle_opts o = {rep % 2 ? -1 : 1, rep % 3 ? 60.0 : __builtin_inf(), rep == 2 ? 3 : 2000, rep % 2,
                         snaps, n_snap, snap_xyz, out_xyz, cap, pc, pf, pt, px, rep % 2 ? 2 : 1};
        if (oracle_track(&g, &o, n, cell, xi, eta, zeta, t, status, ncross, hash) != 0) return 2;
        const double ends[3] = {4.0, 30.0, __builtin_inf()};
        oracle_grid gs[3] = {g, g, g};
        o.direction = 1;
        for (int64_t p = 0; p < n; ++p) status[p] = 0;
        if (oracle_track_transient(gs, 3, ends, &o, n, cell, xi, eta, zeta, t, status, ncross, hash) != 0) return 3;
    }
    /* a quadtree: two cells of width 1 next to one of width 2 (split face) */
    const double box[18] = {0, 0, 0, 1, 1, 1, 0, 1, 0, 1, 1, 1, 1, 0, 0, 2, 2, 1};
    int32_t off[19];
    int32_t nb[6];
    double sq[6], lo[12], hi[12];
    int32_t ns = 0;
    for (int c = 0; c < 3; ++c)
        for (int f = 0; f < 6; ++f) {
            off[6 * c + f] = ns;
            const int want = (c < 2 && f == 1) || (c == 2 && f == 0 ? 2 : 0);
            if (c < 2 && f == 1) {
                nb[ns] = 2; sq[ns] = 1.0;
                lo[2 * ns] = 0; lo[2 * ns + 1] = 0; hi[2 * ns] = 1; hi[2 * ns + 1] = 1;
                ++ns;
            } else if (c == 2 && f == 0) {
                for (int h = 0; h < 2; ++h) {
                    nb[ns] = h; sq[ns] = 1.0;
                    lo[2 * ns] = 0.5 * h; lo[2 * ns + 1] = 0; hi[2 * ns] = 0.5 * h + 0.5; hi[2 * ns + 1] = 1;
                    ++ns;
                }
            } else if (c == 2 && f == 1) {
                nb[ns] = -1; sq[ns] = 2.0;
                lo[2 * ns] = 0; lo[2 * ns + 1] = 0; hi[2 * ns] = 1; hi[2 * ns + 1] = 1;
                ++ns;
            }
            (void)want;
        }
    off[18] = ns;
    int32_t qflags[3] = {1, 1, 1};
    oracle_quad q = {3, box, off, nb, sq, lo, hi, NULL, 0.25, qflags};
    for (int64_t p = 0; p < n; ++p) {
        cell[p] = p % 3;
        xi[p] = urand(&seed);
        eta[p] = urand(&seed);
        zeta[p] = urand(&seed);
        t[p] = 0.0;
        status[p] = 0;
        ncross[p] = 0;
        hash[p] = 0xcbf29ce484222325ull;
    }
    oracle_opts oq = {1, __builtin_inf(), 1 << 20, 1, snaps, n_snap, snap_xyz, out_xyz, cap, pc, pf, pt, px, 1};
    if (oracle_track_quad(&q, &oq, n, cell, xi, eta, zeta, t, status, ncross, hash) != 0) return 4;
    free(qx); free(qy); free(qz); free(por); free(flags); free(cell); free(xi); free(eta); free(zeta); free(t);
    free(status); free(ncross); free(hash); free(snap_xyz); free(out_xyz); free(pc); free(pf); free(pt); free(px);
    printf("oracle sanitize run ok\n");
    return 0;
}
