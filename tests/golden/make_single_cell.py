"""Write single_cell.json: exit times and in-cell positions of the linear-velocity ODE.

Each case is one cell with face flows on one axis only.  The face velocities are
formed as the tracker forms them (u = Q / (n * ((dx*dy)*dz)), IEEE double), then
the exact solution of dxi/dt = u1 + (u2 - u1) xi is evaluated in 60-digit decimal
arithmetic:
    exit time   t = ln(u_e / u_p) / A        (t = (xi_e - xi)/u_p when A = 0)
    position    xi(tau) = xi + u_p (exp(A tau) - 1) / A
This is the semi-analytical cell step of Pollock's method that the paper uses for
every particle displacement (Introduction; Methods, "MODPATH").  No tracker code
is called.  Run:  python tests/golden/make_single_cell.py
"""
import decimal
import json
import os

D = decimal.Decimal
decimal.getcontext().prec = 60

GEOM = dict(dx=7.0, dy=3.0, dz=2.0, porosity=0.25)


def vel(q):
    V = (GEOM["dx"] * GEOM["dy"]) * GEOM["dz"]
    return q / (GEOM["porosity"] * V)


def exit_time(u1, u2, xi):
    a1, a2, x = D(u1), D(u2), D(xi)
    A = a2 - a1
    up = a1 + A * x
    if up > 0:
        if not a2 > 0:
            return None
        ue, xe = a2, D(1)
    elif up < 0:
        if not a1 < 0:
            return None
        ue, xe = a1, D(0)
    else:
        return None
    if A == 0:
        return (xe - x) / up
    return (ue / up).ln() / A


def position(u1, u2, xi, tau):
    a1, a2, x, t = D(u1), D(u2), D(xi), D(tau)
    A = a2 - a1
    up = a1 + A * x
    v = x + up * t if A == 0 else x + up * ((A * t).exp() - 1) / A
    return min(max(v, D(0)), D(1))


# (name, Q_low_face, Q_high_face, xi) -- flows in m^3/d along one axis
EXIT_CASES = [
    ("uniform", 4.2, 4.2, 0.25),
    ("uniform_negative", -4.2, -4.2, 0.6),
    ("accelerating", 1.0, 3.0, 0.2),
    ("decelerating", 3.0, 1.0, 0.5),
    ("strong_deceleration", 10.0, 1e-8, 0.0),
    ("very_strong_deceleration", 10.0, 1e-15, 0.0),
    ("tiny_gradient", 1.0, 1.0 + 1e-12, 0.3),
    ("tiny_gradient_2", 0.5, 0.5 - 3e-16, 0.9),
    ("negative_accelerating", -0.5, -2.0, 0.7),
    ("negative_decelerating", -2.0, -0.5, 0.7),
    ("divergent_high", -1.0, 2.0, 0.5),
    ("divergent_low", -1.0, 2.0, 0.2),
    ("convergent", 1.0, -1.0, 0.4),
    ("stagnant_exit_face", 2.0, 0.0, 0.1),
    ("start_on_exit_face", 1.5, 1.5, 1.0),
    ("strong_acceleration", 1e-6, 10.0, 0.0),
    ("near_linear_regime", 1.0, 1.6, 0.0),
]

# (name, Q_low, Q_high, xi, tau) -- position after tau days inside the cell
POSITION_CASES = [
    ("uniform", 4.2, 4.2, 0.25, 1.5),
    ("convergent_towards_stagnation", 1.0, -1.0, 0.1, 40.0),
    ("convergent_long", 1.0, -1.0, 0.9, 500.0),
    ("divergent", -1.0, 2.0, 0.34, 2.0),
    ("decelerating", 3.0, 1.0, 0.05, 2.0),
    ("tiny_gradient", 1.0, 1.0 + 1e-12, 0.3, 5.0),
]


def main():
    out = {"citation": "Pollock semi-analytical cell step (paper: Introduction; Methods, MODPATH)",
           "geometry": GEOM, "exit": [], "position": []}
    for name, ql, qh, xi in EXIT_CASES:
        t = exit_time(vel(ql), vel(qh), xi)
        out["exit"].append(dict(name=name, q_low=ql, q_high=qh, xi=xi,
                                t=None if t is None else str(t)))
    for name, ql, qh, xi, tau in POSITION_CASES:
        out["position"].append(dict(name=name, q_low=ql, q_high=qh, xi=xi, tau=tau,
                                    xi_tau=str(position(vel(ql), vel(qh), xi, tau))))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "single_cell.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
