"""Small hand-built systems shared by the CPU pin tests (inputs only, no method arithmetic)."""
import math

import numpy as np


def quat_axis_angle(axis, angle):
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    return np.concatenate([[math.cos(angle / 2)], math.sin(angle / 2) * axis])


def qmul(a, b):
    a0, av = a[0], np.asarray(a[1:])
    b0, bv = b[0], np.asarray(b[1:])
    return np.concatenate([[a0 * b0 - av @ bv], a0 * bv + b0 * av + np.cross(av, bv)])


def single_site_model(kind, param, pos=(0.0, 0.0, 0.0), axis=(0.0, 0.0, 1.0), rc=6.0, eps_rf=1.0):
    s = {"kind": kind, "pos": list(pos)}
    if kind in ("dipole", "quadrupole"):
        s["dir"] = list(axis)
    s.update({"charge": {"q": param}, "dipole": {"mu": param}, "quadrupole": {"Q": param}}.get(kind, {}))
    if kind == "lj":
        s.update({"eps": param[0], "sigma": param[1]})
    return {"sites": [s], "mass": 1.0, "inertia": [0.1, 0.1, 0.1]}


def charge_construction(kind, m, pos, axis, d):
    """Point charges standing in for a point dipole (+-q at +-d/2 along axis, mu = q d) or a
    linear quadrupole (q, -2q, q at -d, 0, +d along axis, Q = 2 q d^2)."""
    pos = np.asarray(pos, dtype=np.float64)
    e = np.asarray(axis, dtype=np.float64)
    if kind == "charge":
        return [{"kind": "charge", "pos": list(pos), "q": m}]
    if kind == "dipole":
        q = m / d
        return [{"kind": "charge", "pos": list(pos + 0.5 * d * e), "q": q},
                {"kind": "charge", "pos": list(pos - 0.5 * d * e), "q": -q}]
    q = m / (2 * d * d)
    return [{"kind": "charge", "pos": list(pos + d * e), "q": q},
            {"kind": "charge", "pos": list(pos), "q": -2 * q},
            {"kind": "charge", "pos": list(pos - d * e), "q": q}]


def two_body(compA, compB, rc=6.0, eps_rf=1.0, shift=False, box=20.0):
    return {"components": [compA, compB], "xi": None, "eta": None, "rc": rc, "eps_rf": eps_rf, "lj_shift": shift}
