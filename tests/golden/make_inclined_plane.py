"""Writes inclined_plane.json: closed-form one-step solutions of a particle on
an inclined plane (a pin for the converged contact solve; the paper's own
sliding-box validation compares against the same kind of analytic solution,
Sec. V-B).  Pure formulas, no solver: the particle of mass m starts at rest on a
plane with normal (sin a, 0, cos a) under gravity g; after one step of size h
it sticks (v = 0) iff mu >= tan(a), else it slides downhill with speed
h g (sin a - mu cos a)."""
import json
import math
import os


def case(alpha, mu, m=1.5, h=0.01, g=9.81):
    if mu >= math.tan(alpha):
        v = [0.0, 0.0, 0.0]
        mode = "stick"
    else:
        s = h * g * (math.sin(alpha) - mu * math.cos(alpha))
        v = [s * math.cos(alpha), 0.0, -s * math.sin(alpha)]
        mode = "slip"
    return {"alpha": alpha, "mu": mu, "mass": m, "h": h, "g": g, "v_next": v, "mode": mode,
            "lambda_n": m * h * g * math.cos(alpha)}


if __name__ == "__main__":
    cases = []
    for a in (0.1, 0.35, 0.6, 0.9, 1.2):
        t = math.tan(a)
        cases += [case(a, t - 1e-6), case(a, t + 1e-6), case(a, 0.5 * t), case(a, 2.0 * t)]
    out = {"source": "closed form, particle on an inclined plane from rest (one step)", "cases": cases}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "inclined_plane.json"), "w") as f:
        json.dump(out, f, indent=1)
