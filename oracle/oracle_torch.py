"""Plain FP64 PyTorch (CPU) energy function for small systems, differentiated by autograd.

TEST INFRASTRUCTURE ONLY: the product library never imports this module.

It is a second, independent writing of the same definition as ``oracle.c``: the total potential
energy U = sum over unordered molecule pairs i < j whose minimum-image COM distance is below r_c
of the sum over their site pairs (LJ 12-6 with Lorentz-Berthelot mixing and optional LJTS shift,
Sec. 2; charge / dipole / linear-quadrupole multipole terms with k_C = 1; reaction field on
dipole pairs, Sec. 3).  Autograd then gives dU/d(positions), dU/d(raw quaternion components) and
dU/d(epsilon, sigma, site offsets, charges, dipole moments, quadrupole moments) -- the reference
for the adjoint kernel.  The cutoff mask is taken without gradient (U is piecewise smooth; test
systems keep every COM distance away from r_c).
"""
from __future__ import annotations

import math

import numpy as np
import torch

KINDS = ("lj", "charge", "dipole", "quadrupole")


def params_from_model(model, requires_grad=True):
    """Per-component parameter tensors (FP64), grouped by site kind in table order."""
    out = []
    for comp in model["components"]:
        d = {}
        for kind in KINDS:
            sites = [s for s in comp["sites"] if s["kind"] == kind]
            d[kind + "_pos"] = torch.tensor([s["pos"] for s in sites], dtype=torch.float64).reshape(-1, 3)
            if kind in ("dipole", "quadrupole"):
                d[kind + "_dir"] = torch.tensor([s["dir"] for s in sites], dtype=torch.float64).reshape(-1, 3)
            if kind == "lj":
                d["lj_eps"] = torch.tensor([s["eps"] for s in sites], dtype=torch.float64)
                d["lj_sigma"] = torch.tensor([s["sigma"] for s in sites], dtype=torch.float64)
            elif kind == "charge":
                d["charge_m"] = torch.tensor([s["q"] for s in sites], dtype=torch.float64)
            elif kind == "dipole":
                d["dipole_m"] = torch.tensor([s["mu"] for s in sites], dtype=torch.float64)
            else:
                d["quadrupole_m"] = torch.tensor([s["Q"] for s in sites], dtype=torch.float64)
        if requires_grad:
            for k, v in d.items():
                if not k.endswith("_dir"):
                    v.requires_grad_(True)
        out.append(d)
    return out


def rotmat(q):
    """Body-to-space matrices of raw quaternions q[..., 4] = (w, x, y, z), polynomial form."""
    w, x, y, z = q.unbind(-1)
    r0 = torch.stack([w * w + x * x - y * y - z * z, 2 * (x * y - w * z), 2 * (x * z + w * y)], -1)
    r1 = torch.stack([2 * (x * y + w * z), w * w - x * x + y * y - z * z, 2 * (y * z - w * x)], -1)
    r2 = torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), w * w - x * x - y * y + z * z], -1)
    return torch.stack([r0, r1, r2], -2)


def _elec(ka, kb, ma, mb, r, ci, cj, cij, kappa, rc):
    """Energy of one electrostatic site-pair kind, vectorised over pairs (k_C = 1)."""
    if ka == "charge" and kb == "charge":
        return ma * mb / r
    if ka == "charge" and kb == "dipole":
        return ma * mb * cj / r ** 2
    if ka == "dipole" and kb == "charge":
        return -ma * mb * ci / r ** 2
    if ka == "charge" and kb == "quadrupole":
        return ma * mb * (3 * cj ** 2 - 1) / (2 * r ** 3)
    if ka == "quadrupole" and kb == "charge":
        return ma * mb * (3 * ci ** 2 - 1) / (2 * r ** 3)
    if ka == "dipole" and kb == "dipole":
        return ma * mb * (cij - 3 * ci * cj) / r ** 3 - kappa * ma * mb * cij / rc ** 3
    if ka == "dipole" and kb == "quadrupole":
        return 1.5 * ma * mb * (ci - 5 * ci * cj ** 2 + 2 * cj * cij) / r ** 4
    if ka == "quadrupole" and kb == "dipole":
        return -1.5 * ma * mb * (cj - 5 * cj * ci ** 2 + 2 * ci * cij) / r ** 4
    if ka == "quadrupole" and kb == "quadrupole":
        s = cij - 5 * ci * cj
        return 0.75 * ma * mb * (1 - 5 * ci ** 2 - 5 * cj ** 2 - 15 * ci ** 2 * cj ** 2 + 2 * s ** 2) / r ** 5
    raise ValueError((ka, kb))


def pair_list(pos, box, rc):
    """Unordered pairs i < j with minimum-image COM distance < r_c (numpy, no gradient)."""
    pos = np.asarray(pos, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    N = pos.shape[0]
    ii, jj = np.triu_indices(N, k=1)
    d = pos[ii] - pos[jj]
    d -= box * np.round(d / box)
    r2 = (d * d).sum(1)
    m = r2 < rc * rc
    return ii[m], jj[m]


def energy(model, pos, quat, comp, box, params, pairs=None):
    """Total potential energy U (0-dim FP64 tensor) of the system; differentiable in pos, quat
    and every tensor of params."""
    box_t = torch.as_tensor(np.asarray(box, dtype=np.float64))
    rc = float(model["rc"])
    eps_rf = float(model.get("eps_rf", math.inf))
    kappa = 1.0 if math.isinf(eps_rf) else 2 * (eps_rf - 1) / (2 * eps_rf + 1)
    ncomp = len(model["components"])
    xi = np.ones((ncomp, ncomp)) if model.get("xi") is None else np.asarray(model["xi"], dtype=np.float64)
    eta = np.ones((ncomp, ncomp)) if model.get("eta") is None else np.asarray(model["eta"], dtype=np.float64)
    comp = np.zeros(pos.shape[0], dtype=np.int64) if comp is None else np.asarray(comp, dtype=np.int64)
    if pairs is None:
        pairs = pair_list(pos.detach().numpy(), box, rc)
    ii_all, jj_all = pairs
    A = rotmat(quat) if quat is not None else None
    U = torch.zeros((), dtype=torch.float64)
    for ca in range(ncomp):
        for cb in range(ncomp):
            sel = (comp[ii_all] == ca) & (comp[jj_all] == cb)
            if not sel.any():
                continue
            ii = torch.as_tensor(ii_all[sel])
            jj = torch.as_tensor(jj_all[sel])
            d = pos[ii] - pos[jj]
            shift = torch.round(d.detach() / box_t) * box_t
            dc = d - shift  # minimum-image COM separation (i minus image of j)
            Pa, Pb = params[ca], params[cb]
            for ka in KINDS:
                for kb in KINDS:
                    if (ka == "lj") != (kb == "lj"):
                        continue
                    na, nb = Pa[ka + "_pos"].shape[0], Pb[kb + "_pos"].shape[0]
                    for a in range(na):
                        for b in range(nb):
                            if A is not None:
                                oa = A[ii] @ Pa[ka + "_pos"][a]
                                ob = A[jj] @ Pb[kb + "_pos"][b]
                            else:
                                oa = Pa[ka + "_pos"][a].expand_as(dc)
                                ob = Pb[kb + "_pos"][b].expand_as(dc)
                            R = dc + oa - ob
                            r2 = (R * R).sum(-1)
                            if ka == "lj":
                                eps = xi[ca, cb] * torch.sqrt(Pa["lj_eps"][a] * Pb["lj_eps"][b])
                                sig = eta[ca, cb] * 0.5 * (Pa["lj_sigma"][a] + Pb["lj_sigma"][b])
                                s6 = (sig * sig / r2) ** 3
                                u = 4 * eps * (s6 * s6 - s6)
                                if model.get("lj_shift", False):
                                    c6 = (sig * sig / (rc * rc)) ** 3
                                    u = u - 4 * eps * (c6 * c6 - c6)
                            else:
                                r = torch.sqrt(r2)
                                rh = R / r[:, None]
                                ea = eb = None
                                if ka in ("dipole", "quadrupole"):
                                    ea = A[ii] @ Pa[ka + "_dir"][a] if A is not None else Pa[ka + "_dir"][a].expand_as(dc)
                                if kb in ("dipole", "quadrupole"):
                                    eb = A[jj] @ Pb[kb + "_dir"][b] if A is not None else Pb[kb + "_dir"][b].expand_as(dc)
                                ci = (ea * rh).sum(-1) if ea is not None else None
                                cj = (eb * rh).sum(-1) if eb is not None else None
                                cij = (ea * eb).sum(-1) if (ea is not None and eb is not None) else None
                                u = _elec(ka, kb, Pa[ka + "_m"][a], Pb[kb + "_m"][b], r, ci, cj, cij, kappa, rc)
                            U = U + u.sum()
    return U


def gradients(model, pos, quat, comp, box):
    """U and its autograd gradients: returns dict(U, dpos[N,3], dquat[N,4] or None, params=list
    of per-component dicts of gradients keyed like params_from_model)."""
    pos_t = torch.tensor(np.asarray(pos, dtype=np.float64), requires_grad=True)
    quat_t = None if quat is None else torch.tensor(np.asarray(quat, dtype=np.float64), requires_grad=True)
    params = params_from_model(model)
    U = energy(model, pos_t, quat_t, comp, box, params)
    leaves = [pos_t] + ([quat_t] if quat_t is not None else [])
    names = []
    for c, d in enumerate(params):
        for k, v in d.items():
            if v.requires_grad:
                leaves.append(v)
                names.append((c, k))
    grads = torch.autograd.grad(U, leaves, allow_unused=True)
    out = {"U": float(U.detach()), "dpos": grads[0].numpy()}
    off = 1
    if quat_t is not None:
        out["dquat"] = grads[1].numpy()
        off = 2
    else:
        out["dquat"] = None
    pg = [dict() for _ in params]
    for (c, k), g in zip(names, grads[off:]):
        pg[c][k] = np.zeros(tuple(params[c][k].shape)) if g is None else g.numpy()
    out["params"] = pg
    return out
