/* Prints sizeof and field offsets of the structs in include/pt.h, for the ABI test. */
#include <stddef.h>
#include <stdio.h>

#include "pt.h"

#define F(T, f) printf("%s.%s %zu\n", #T, #f, offsetof(T, f))
#define S(T) printf("%s.sizeof %zu\n", #T, sizeof(T))

int main(void) {
    S(pt_grid_desc);
    F(pt_grid_desc, nx); F(pt_grid_desc, ny); F(pt_grid_desc, nz); F(pt_grid_desc, dx);
    F(pt_grid_desc, dy); F(pt_grid_desc, dz); F(pt_grid_desc, x0); F(pt_grid_desc, y0);
    F(pt_grid_desc, z0); F(pt_grid_desc, qx); F(pt_grid_desc, qy); F(pt_grid_desc, qz);
    F(pt_grid_desc, porosity); F(pt_grid_desc, porosity_scalar); F(pt_grid_desc, flags);
    F(pt_grid_desc, mem); F(pt_grid_desc, balance_tol);
    S(pt_quad_desc);
    F(pt_quad_desc, ncell); F(pt_quad_desc, nsub); F(pt_quad_desc, box); F(pt_quad_desc, sub_off);
    F(pt_quad_desc, sub_nb); F(pt_quad_desc, sub_q); F(pt_quad_desc, sub_lo); F(pt_quad_desc, sub_hi);
    F(pt_quad_desc, porosity); F(pt_quad_desc, porosity_scalar); F(pt_quad_desc, flags);
    F(pt_quad_desc, mem); F(pt_quad_desc, balance_tol);
    S(pt_particles);
    F(pt_particles, n); F(pt_particles, cell); F(pt_particles, xi); F(pt_particles, eta);
    F(pt_particles, zeta); F(pt_particles, t); F(pt_particles, status); F(pt_particles, ncross);
    F(pt_particles, path_hash); F(pt_particles, n_groups); F(pt_particles, group_offsets);
    F(pt_particles, group_grid);
    S(pt_track_opts);
    F(pt_track_opts, mode); F(pt_track_opts, precision); F(pt_track_opts, schedule);
    F(pt_track_opts, layout); F(pt_track_opts, direction); F(pt_track_opts, stop_at_sink);
    F(pt_track_opts, t_max); F(pt_track_opts, max_steps); F(pt_track_opts, snap_times);
    F(pt_track_opts, n_snap); F(pt_track_opts, snap_xyz); F(pt_track_opts, out_xyz);
    F(pt_track_opts, use_graph); F(pt_track_opts, block); F(pt_track_opts, blocks_per_cu);
    F(pt_track_opts, refill); F(pt_track_opts, steps_per_refill); F(pt_track_opts, chunk);
    F(pt_track_opts, sort); F(pt_track_opts, path_offsets); F(pt_track_opts, path_count_only);
    F(pt_track_opts, path_cap); F(pt_track_opts, path_records); F(pt_track_opts, n_tsteps);
    F(pt_track_opts, tstep_end);
    S(pt_path_record);
    F(pt_path_record, t); F(pt_path_record, x); F(pt_path_record, y); F(pt_path_record, z);
    F(pt_path_record, cell); F(pt_path_record, face);
    S(pt_summary);
    F(pt_summary, crossings); F(pt_summary, n_tracked); F(pt_summary, status_count);
    F(pt_summary, kernel_ms); F(pt_summary, schedule); F(pt_summary, layout); F(pt_summary, block);
    F(pt_summary, grid); F(pt_summary, cr_ambiguous); F(pt_summary, path_records);
    F(pt_summary, path_dropped); F(pt_summary, recheck_tracks); F(pt_summary, track_ms);
    return 0;
}
