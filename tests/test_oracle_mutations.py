"""Sensitivity of the oracle pins: every planted mistake must make at least one pin fail.

Each mutant is a copy of the oracle source with one plausible error (a dropped
term, a swapped index, a wrong sign or comparison), compiled on the CPU into a
temporary library.  The real oracle is never modified.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

from oracle import oracle as O

from . import oracle_pins as P

MUTANTS = {
    "drop_gradient_term": ("    double up = v.u1 + A * xi;\n    double ue;",
                           "    double up = v.u1;\n    double ue;"),
    "swap_y_faces": ("v[1].u1 = (sgn * qyl) / d;", "v[1].u1 = (sgn * qyh) / d;"),
    "wrong_z_high_face": ("double qzh = g->qz[((k + 1) * g->ny + j) * g->nx + i];",
                          "double qzh = g->qz[(k * g->ny + j) * g->nx + i];"),
    "tie_to_last_axis": ("if (ta < dt) {", "if (ta <= dt) {"),
    "ignore_direction": ("return o->direction < 0 ? -1.0 : 1.0;", "return 1.0;"),
    "no_flip_on_transfer": ("        c = cn;\n        loc[axis] = 1.0 - xe;", "        c = cn;\n        loc[axis] = xe;"),
    "quad_no_flip_on_transfer": ("        loc[axis] = 1.0 - xe;\n        c = cn;", "        loc[axis] = xe;\n        c = cn;"),
    "y_scaled_by_dz": ("out[1] = g->y0 + ((double)j + eta) * g->dy;",
                       "out[1] = g->y0 + ((double)j + eta) * g->dz;"),
    "exit_time_without_log": ("dt = r * (cr_log1p(x) / x);", "dt = r;"),
    "no_ratio_branch": ("} else if (x < -0.5) {", "} else if (x < -2.0) {"),
    "non_strict_time_limit": ("if (t_exit > lim) {", "if (t_exit >= lim) {"),
    "scalar_porosity_only": ("return porosity ? porosity[c] : scalar;", "return scalar;"),
    "wrong_hash_prime": ("0x100000001b3ULL", "0x100000001b5ULL"),
    "transposed_neighbour": ("int64_t cn = (kk * g->ny + jj) * g->nx + ii;",
                             "int64_t cn = (kk * g->nx + jj) * g->ny + ii;"),
    "advance_without_exp": ("double psi = (y == 0.0) ? 1.0 : cr_expm1(y) / y;", "double psi = 1.0;"),
    "snapshot_from_zero": ("double tau = s - t;", "double tau = s;"),
    "no_sink_stop_on_entry": ("        loc[axis] = 1.0 - xe;\n        if ((g->flags[c] & CELL_SINK) && o->stop_at_sink) {\n"
                              "            status_[p] = ST_SINK;\n            break;\n        }\n",
                              "        loc[axis] = 1.0 - xe;\n"),
    "quad_no_sink_stop_on_entry": ("        c = cn;\n        if ((g->flags[c] & CELL_SINK) && o->stop_at_sink) {\n"
                                   "            status_[p] = ST_SINK;\n            break;\n        }\n",
                                   "        c = cn;\n"),
    "no_clamp_high": ("    if (xn > 1.0) xn = 1.0;\n", ""),
    "transient_field_not_switched": ("                ++s;\n                g = &grids[s];\n",
                                     "                ++s;\n"),
    "transient_step_end_ignored": ("if (step_end && step_end[s] < lim) {", "if (0) {"),
    "transient_release_in_first_step": ("while (s < n_steps - 1 && !(t < step_end[s])) ++s;",
                                        "while (0) ++s;"),
    "transient_release_at_end_stays": ("while (s < n_steps - 1 && !(t < step_end[s])) ++s;",
                                       "while (s < n_steps - 1 && t > step_end[s]) ++s;"),
    "transient_no_sink_on_switch": ("                if ((g->flags[c] & CELL_SINK) && o->stop_at_sink) {\n"
                                    "                    status_[p] = ST_SINK;\n                    break;\n"
                                    "                }\n", ""),
    "transient_stranded_at_step_end": ("        if (axis < 0 && isinf(lim)) {", "        if (axis < 0) {"),
    "quad_always_first_subface": ("            if (lo[0] <= loc[ta1] && loc[ta1] <= hi[0] && lo[1] <= loc[ta2] && loc[ta2] <= hi[1]) {",
                                  "            if (1) {"),
    "quad_face_flow_first_subface": ("for (int32_t q = g->sub_off[6 * c + f]; q < g->sub_off[6 * c + f + 1]; ++q) Q += g->sub_q[q];",
                                     "Q = g->sub_q[g->sub_off[6 * c + f]];"),
    "quad_tangent_never_mapped": ("            if (bn[a] == b[a] && bn[3 + a] == b[3 + a]) continue;   /* same span: unchanged */",
                                  "            continue;"),
    "quad_tangent_always_mapped": ("            if (bn[a] == b[a] && bn[3 + a] == b[3 + a]) continue;   /* same span: unchanged */",
                                   ""),
    "quad_volume_square": ("const double V = (b[3] * b[4]) * b[5];", "const double V = (b[3] * b[3]) * b[5];"),
    "quad_no_circuit_guard": ("            if (++zero_run >= QUAD_ZERO_RUN) {", "            if (0) {"),
    "quad_position_from_wrong_extent": ("    out[1] = b[1] + loc[1] * b[4];", "    out[1] = b[1] + loc[1] * b[3];"),
}


@pytest.fixture(scope="module")
def tmpdir_mod():
    d = tempfile.mkdtemp(prefix="oracle_mut_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmpdir_mod):
    old, new = MUTANTS[name]
    src = open(O._SRC).read()
    assert src.count(old) == 1, "mutation anchor not unique: %s" % name
    path = os.path.join(tmpdir_mod, name + ".c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    so = os.path.join(tmpdir_mod, name + ".so")
    O.build(force=True, src=path, out=so)
    lib = O.load(so)
    caught = []
    for pin in P.ALL_PINS:
        try:
            pin(lib)
        except (AssertionError, IndexError, ValueError, RuntimeError) as e:
            caught.append(pin.__name__)
            break
    assert caught, "no pin detects mutant %s" % name
