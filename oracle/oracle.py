"""ctypes wrapper around ``oracle.c``, the plain FP64 brute-force reference.

TEST INFRASTRUCTURE ONLY: the product library never imports this module.  Only the test suite,
the smoke check and the CPU-baseline leg of the benchmark use it.

Model descriptions are the plain dictionaries produced by the workload generators (see
``paper_1408_4599_amd.workloads``): a list of components, each a list of sites with body-frame
offsets and parameters, plus the cutoff, the reaction-field permittivity and the LJTS flag.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

KIND = {"lj": 0, "charge": 1, "dipole": 2, "quadrupole": 3}
SITE_STRIDE = 10


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               _SRC, "-o", _LIB, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


class _Model(ctypes.Structure):
    _fields_ = [
        ("ncomp", ctypes.c_int32),
        ("site_start", ctypes.POINTER(ctypes.c_int32)),
        ("sites", ctypes.POINTER(ctypes.c_double)),
        ("xi", ctypes.POINTER(ctypes.c_double)),
        ("eta", ctypes.POINTER(ctypes.c_double)),
        ("rc", ctypes.c_double),
        ("eps_rf", ctypes.c_double),
        ("lj_shift", ctypes.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lp = ctypes.POINTER(ctypes.c_int64)
        mp = ctypes.POINTER(_Model)
        L.oracle_ncells.argtypes = [dp, ctypes.c_double, ip]
        L.oracle_ncells.restype = ctypes.c_int
        L.oracle_bin.argtypes = [dp, ctypes.c_int64, dp, ctypes.c_double, ip, dp]
        L.oracle_bin.restype = ctypes.c_int64
        L.oracle_half_cells.argtypes = [dp, ctypes.c_int64, dp, ctypes.c_double, ip]
        L.oracle_half_cells.restype = ctypes.c_int64
        L.oracle_rows.argtypes = [mp, dp, dp, ip, ctypes.c_int64, dp, lp, ctypes.c_int64,
                                  dp, dp, dp, dp, dp, lp, dp]
        L.oracle_rows.restype = ctypes.c_int
        L.oracle_all.argtypes = [mp, dp, dp, ip, ctypes.c_int64, dp, dp, dp, dp, dp, dp, lp]
        L.oracle_all.restype = ctypes.c_int
        L.oracle_step.argtypes = [mp, dp, dp, dp, dp, dp, dp, ip, ctypes.c_int64, dp, ctypes.c_double,
                                  ctypes.c_int64, ctypes.c_double, dp]
        L.oracle_step.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _lp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


class OracleModel:
    """Flat site table built from a model description dictionary."""

    def __init__(self, model: dict):
        comps = model["components"]
        nc = len(comps)
        starts = [0]
        recs = []
        for c in comps:
            for s in c["sites"]:
                rec = [0.0] * SITE_STRIDE
                rec[0] = float(KIND[s["kind"]])
                rec[1:4] = [float(v) for v in s["pos"]]
                if s["kind"] in ("dipole", "quadrupole"):
                    rec[4:7] = [float(v) for v in s["dir"]]
                if s["kind"] == "lj":
                    rec[7], rec[8] = float(s["eps"]), float(s["sigma"])
                elif s["kind"] == "charge":
                    rec[7] = float(s["q"])
                elif s["kind"] == "dipole":
                    rec[7] = float(s["mu"])
                else:
                    rec[7] = float(s["Q"])
                recs.append(rec)
            starts.append(len(recs))
        self.site_start = np.asarray(starts, dtype=np.int32)
        self.sites = np.ascontiguousarray(np.asarray(recs, dtype=np.float64).reshape(-1, SITE_STRIDE))
        xi = model.get("xi")
        eta = model.get("eta")
        self.xi = np.ascontiguousarray(np.ones((nc, nc)) if xi is None else np.asarray(xi, dtype=np.float64))
        self.eta = np.ascontiguousarray(np.ones((nc, nc)) if eta is None else np.asarray(eta, dtype=np.float64))
        self.mass = np.asarray([float(c["mass"]) for c in comps], dtype=np.float64)
        self.inertia = np.ascontiguousarray(np.asarray([c["inertia"] for c in comps], dtype=np.float64).reshape(nc, 3))
        eps_rf = model.get("eps_rf", math.inf)
        self.struct = _Model(nc, _ip(self.site_start), _dp(self.sites), _dp(self.xi), _dp(self.eta),
                             float(model["rc"]), float(eps_rf), int(bool(model.get("lj_shift", False))))
        self.rc = float(model["rc"])


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def ncells(box, rc):
    nc = np.zeros(3, dtype=np.int32)
    ok = lib().oracle_ncells(_dp(_f64(box, 3)), float(rc), _ip(nc))
    return tuple(int(v) for v in nc) if ok else None


def bin_cells(pos, box, rc):
    """Wrap + bin: returns (cell_of int32[N], pos_wrapped float64[N,3], ncell)."""
    pos = _f64(pos, (-1, 3))
    N = pos.shape[0]
    cell_of = np.zeros(N, dtype=np.int32)
    pw = np.zeros((N, 3))
    n = lib().oracle_bin(_dp(pos), N, _dp(_f64(box, 3)), float(rc), _ip(cell_of), _dp(pw))
    if n < 0:
        raise ValueError("box smaller than three cells per axis")
    return cell_of, pw, int(n)


def half_cells(pos, box, rc):
    """Half-edge (r_c/2) cell coordinates of every molecule: int32[N, 3] (x, y, z), after the wrap
    of ``bin_cells``."""
    pos = _f64(pos, (-1, 3))
    N = pos.shape[0]
    half = np.zeros((N, 3), dtype=np.int32)
    n = lib().oracle_half_cells(_dp(pos), N, _dp(_f64(box, 3)), float(rc), _ip(half))
    if n < 0:
        raise ValueError("box smaller than three cells per axis")
    return half


def subcell_order(pos, box, rc):
    """The stable order of molecules by r_c cell, then by half-edge cell inside it (octant
    4 z + 2 y + x of the half indices' low bits), then by original index; also each molecule's
    key 8 * cell + octant."""
    cell_of, _, _ = bin_cells(pos, box, rc)
    half = half_cells(pos, box, rc).astype(np.int64)
    octant = 4 * (half[:, 2] & 1) + 2 * (half[:, 1] & 1) + (half[:, 0] & 1)
    key = 8 * cell_of.astype(np.int64) + octant
    return np.lexsort((np.arange(len(key)), key)), key


def _system(model, pos, quat, comp):
    om = model if isinstance(model, OracleModel) else OracleModel(model)
    pos = _f64(pos, (-1, 3))
    N = pos.shape[0]
    quat = None if quat is None else _f64(quat, (N, 4))
    comp = np.zeros(N, dtype=np.int32) if comp is None else np.ascontiguousarray(np.asarray(comp, dtype=np.int32))
    return om, pos, quat, comp, N


def rows(model, pos, quat, comp, box, idx=None, want_dquat=False):
    """Per-molecule sums for the molecules in idx (all if None).  Returns a dict of arrays."""
    om, pos, quat, comp, N = _system(model, pos, quat, comp)
    idx_arr = None if idx is None else np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    n = N if idx_arr is None else idx_arr.shape[0]
    out = dict(F=np.zeros((n, 3)), T=np.zeros((n, 3)), u=np.zeros(n), w=np.zeros(n), wd=np.zeros((n, 3)),
               nnb=np.zeros(n, dtype=np.int64))
    dq = np.zeros((n, 4)) if want_dquat else None
    rc = lib().oracle_rows(ctypes.byref(om.struct), _dp(pos), _dp(quat), _ip(comp), N, _dp(_f64(box, 3)),
                           _lp(idx_arr), n, _dp(out["F"]), _dp(out["T"]), _dp(out["u"]), _dp(out["w"]),
                           _dp(out["wd"]), _lp(out["nnb"]), _dp(dq))
    if rc != 0:
        raise RuntimeError(f"oracle_rows failed ({rc})")
    if want_dquat:
        out["dquat"] = dq
    return out


def forces(model, pos, quat, comp, box):
    """Whole-system evaluation.  Returns dict with F, T, u, w, U, W, Wd (3), npairs."""
    om, pos, quat, comp, N = _system(model, pos, quat, comp)
    F = np.zeros((N, 3))
    T = np.zeros((N, 3))
    u = np.zeros(N)
    w = np.zeros(N)
    glob = np.zeros(5)
    npairs = np.zeros(1, dtype=np.int64)
    rc = lib().oracle_all(ctypes.byref(om.struct), _dp(pos), _dp(quat), _ip(comp), N, _dp(_f64(box, 3)),
                          _dp(F), _dp(T), _dp(u), _dp(w), _dp(glob), _lp(npairs))
    if rc != 0:
        raise RuntimeError(f"oracle_all failed ({rc})")
    return dict(F=F, T=T, u=u, w=w, U=glob[0], W=glob[1], Wd=glob[2:5].copy(), npairs=int(npairs[0]))


def step(model, pos, vel, quat, angmom, comp, box, dt, nsteps, T_target=0.0):
    """Leapfrog nsteps on copies of the state (with velocity rescaling to the kinetic temperature
    T_target after each step when T_target > 0).  Returns (pos, vel, quat, angmom, energies[n,4])."""
    om, pos, quat, comp, N = _system(model, pos, quat, comp)
    pos = pos.copy()
    vel = _f64(vel, (N, 3)).copy()
    quat = None if quat is None else quat.copy()
    angmom = None if angmom is None else _f64(angmom, (N, 3)).copy()
    en = np.zeros((nsteps, 4))
    rc = lib().oracle_step(ctypes.byref(om.struct), _dp(om.mass), _dp(om.inertia), _dp(pos), _dp(vel), _dp(quat),
                           _dp(angmom), _ip(comp), N, _dp(_f64(box, 3)), float(dt), int(nsteps), float(T_target),
                           _dp(en))
    if rc != 0:
        raise RuntimeError(f"oracle_step failed ({rc})")
    return pos, vel, quat, angmom, en


def long_range_correction(model, counts, box):
    """Isotropic cut-off corrections of energy and virial (Sec. 3: the long-range part of the
    dispersive interaction is approximated by a mean-field integral beyond r_c).  Reading: every
    pair of LJ sites (a of component A, b of component B) contributes the tail of the full
    LJ 12-6 potential beyond r_c as if the sites sat at the molecular centres (the cutoff acts on
    the centre distance), with a uniform pair density N_A N_B / V:
        U_lrc = sum_{A,B} sum_{a,b} 2 pi N_A N_B / V * int_rc^inf r^2 u_ab(r) dr
              = sum 2 pi N_A N_B / V * 4 eps_ab (sigma_ab^12 / (9 rc^9) - sigma_ab^6 / (3 rc^3)),
        W_lrc = sum 2 pi N_A N_B / V * int_rc^inf r^2 (-r u_ab'(r)) dr
              = sum 2 pi N_A N_B / V * 4 eps_ab (4 sigma_ab^12 / (3 rc^9) - 2 sigma_ab^6 / rc^3),
    (A, B ordered, so each unlike pair of components enters twice and N_A N_B / 2 pairs of like
    ones once), eps_ab = xi_AB sqrt(eps_a eps_b), sigma_ab = eta_AB (sigma_a + sigma_b) / 2.  The
    truncated and shifted potential (lj_shift) is the model itself: no correction.  The reaction
    field already accounts for the dipolar far field; charges and quadrupoles get none.
    Returns (U_lrc, W_lrc)."""
    if model.get("lj_shift", False):
        return 0.0, 0.0
    comps = model["components"]
    nc = len(comps)
    xi = np.ones((nc, nc)) if model.get("xi") is None else np.asarray(model["xi"], dtype=np.float64)
    eta = np.ones((nc, nc)) if model.get("eta") is None else np.asarray(model["eta"], dtype=np.float64)
    rc = float(model["rc"])
    V = float(np.prod(np.asarray(box, dtype=np.float64)))
    U = W = 0.0
    for A in range(nc):
        for B in range(nc):
            dens = 2.0 * math.pi * float(counts[A]) * float(counts[B]) / V
            for sa in [s for s in comps[A]["sites"] if s["kind"] == "lj"]:
                for sb in [s for s in comps[B]["sites"] if s["kind"] == "lj"]:
                    eps = xi[A, B] * math.sqrt(sa["eps"] * sb["eps"])
                    sig = eta[A, B] * 0.5 * (sa["sigma"] + sb["sigma"])
                    s3 = sig ** 3 / rc ** 3
                    U += dens * 4.0 * eps * sig ** 3 * (s3 ** 3 / 9.0 - s3 / 3.0)
                    W += dens * 4.0 * eps * sig ** 3 * (4.0 * s3 ** 3 / 3.0 - 2.0 * s3)
    return U, W


def num_threads() -> int:
    return int(lib().oracle_num_threads())
