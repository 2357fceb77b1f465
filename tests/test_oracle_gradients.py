"""Pins of the autograd gradient reference (oracle/oracle_torch.py): it is a second writing of the
energy, so it must reproduce the C oracle's energy, forces and quaternion gradient; its
parameter gradients must match central finite differences of the C oracle's energy and the
Euler homogeneity identities of the model."""
import copy
import math

import numpy as np
import pytest

from paper_1408_4599_amd import workloads as W

KEYMAP = {"lj_eps": ("lj", "eps"), "lj_sigma": ("lj", "sigma"), "charge_m": ("charge", "q"),
          "dipole_m": ("dipole", "mu"), "quadrupole_m": ("quadrupole", "Q")}


@pytest.fixture(scope="module")
def OT():
    from oracle import oracle_torch
    return oracle_torch


def _small_cluster(n=10, seed=3):
    m = dict(W.mixture_model(rc=3.5, eps_rf=20.0), rc=6.0)
    rng = np.random.default_rng(seed)
    while True:
        pos = 7.0 + rng.uniform(0, 4.0, size=(n, 3))
        d = np.linalg.norm(pos[:, None] - pos[None], axis=-1)
        iu = np.triu_indices(n, 1)
        if d[iu].min() > 1.3 and np.abs(d[iu] - m["rc"]).min() > 0.05:
            break
    return {"model": m, "pos": pos, "quat": W.random_quaternions(rng, n), "comp": (np.arange(n) % 2).astype(np.int32),
            "box": np.array([20.0, 20.0, 20.0])}


@pytest.mark.parametrize("name", ["c4_small", "c5_small", "mixture_small"])
def test_energy_forces_quaternion_gradient_agree_with_c_oracle(oracle, OT, name):
    c = W.make(name)
    g = OT.gradients(c["model"], c["pos"], c["quat"], c["comp"], c["box"])
    r = oracle.rows(c["model"], c["pos"], c["quat"], c["comp"], c["box"], want_dquat=True)
    U = r["u"].sum()
    assert g["U"] == pytest.approx(U, rel=1e-12)
    scale = np.abs(r["F"]).max()
    np.testing.assert_allclose(-g["dpos"], r["F"], rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(g["dquat"], r["dquat"], rtol=0, atol=1e-12 * np.abs(r["dquat"]).max())


def _set_param(model, comp, kind, idx, field, value):
    sites = [s for s in model["components"][comp]["sites"] if s["kind"] == kind]
    if field == "pos":
        sites[idx]["pos"] = list(value)
    else:
        sites[idx][field] = value


def _get_param(model, comp, kind, idx, field):
    return [s for s in model["components"][comp]["sites"] if s["kind"] == kind][idx][field]


@pytest.mark.parametrize("which", ["cluster", "c5_small"])
def test_parameter_gradients_match_finite_differences(oracle, OT, which):
    c = _small_cluster() if which == "cluster" else W.make("c5_small")
    model = c["model"]
    g = OT.gradients(model, c["pos"], c["quat"], c["comp"], c["box"])

    def U(m):
        return oracle.forces(m, c["pos"], c["quat"], c["comp"], c["box"])["U"]

    checked = 0
    for ci, pg in enumerate(g["params"]):
        for key, grad in pg.items():
            if key.endswith("_pos"):
                kind, field = key[:-4], "pos"
            else:
                kind, field = KEYMAP[key]
            for idx in range(grad.shape[0]):
                comps = range(3) if field == "pos" else [None]
                for k in comps:
                    base = _get_param(model, ci, kind, idx, field)
                    h = 1e-6
                    mp, mm = copy.deepcopy(model), copy.deepcopy(model)
                    if k is None:
                        _set_param(mp, ci, kind, idx, field, base + h)
                        _set_param(mm, ci, kind, idx, field, base - h)
                        ref = grad[idx]
                    else:
                        bp, bm = list(base), list(base)
                        bp[k] += h
                        bm[k] -= h
                        _set_param(mp, ci, kind, idx, field, bp)
                        _set_param(mm, ci, kind, idx, field, bm)
                        ref = grad[idx, k]
                    fd = (U(mp) - U(mm)) / (2 * h)
                    assert ref == pytest.approx(fd, rel=2e-6, abs=2e-6 * max(1.0, abs(g["U"]) / 1e3)), (ci, key, idx, k)
                    checked += 1
    assert checked >= 19


def test_euler_homogeneity_identities(oracle, OT):
    """U_LJ is homogeneous of degree 1 in the site epsilons (geometric-mean mixing):
    sum_a eps_a dU/deps_a = U_LJ.  Dipole terms (incl. reaction field) are bilinear in the
    moments: sum_a mu_a dU/dmu_a = 2 U_dipolar."""
    c = W.make("c5_small")
    m = c["model"]
    g = OT.gradients(m, c["pos"], c["quat"], c["comp"], c["box"])
    nodip = copy.deepcopy(m)
    _set_param(nodip, 0, "dipole", 0, "mu", 0.0)
    U = oracle.forces(m, c["pos"], c["quat"], None, c["box"])["U"]
    U_lj = oracle.forces(nodip, c["pos"], c["quat"], None, c["box"])["U"]
    p = g["params"][0]
    eps = np.array([s["eps"] for s in m["components"][0]["sites"] if s["kind"] == "lj"])
    assert (eps * p["lj_eps"]).sum() == pytest.approx(U_lj, rel=1e-12)
    assert math.sqrt(3.0) * p["dipole_m"][0] == pytest.approx(2 * (U - U_lj), rel=1e-11)
