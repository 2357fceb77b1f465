"""Parity at the full benchmark sizes, in the launch configuration the benchmark times.

* Sampled molecules: the oracle computes the full O(N) rows of 256 seeded molecules; partner
  counts must match bit for bit, forces / torques / energies / virials within the FP64 and FP32
  bars.
* Global sums: interacting-pair count, U and W against tests/golden/full_size.json (written by
  tests/golden/make_full_size.py from the brute-force oracle over all N^2 pairs).
* Properties that hold at any size: sum of u_mol = U, sum of w_mol = W, adjoint dU/dr = -F, and
  the Euler identities of the parameter gradients (U_LJ is homogeneous of degree 1 in the site
  epsilons; dipole and quadrupole energies of degree 2 in their moments)."""
import json
import math
import os

import numpy as np
import pytest
import torch

from tests._gpu import assert_close, dev, elem_err, rel_rms
from paper_1408_4599_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size.json")
NAMES = ["c2_lj_1m", "c3_lj_slab_2m", "c4_2cljq_500k", "c5_4site_200k"]


@pytest.fixture(scope="module")
def md():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1408_4599_amd import md as _md
    _md.lib()
    return _md


@pytest.fixture(scope="module")
def golden():
    return json.load(open(GOLDEN)) if os.path.exists(GOLDEN) else {}


@pytest.mark.parametrize("name", NAMES)
def test_full_size_sampled_and_global(md, oracle, golden, name):
    cfg = W.make(name)
    N = cfg["pos"].shape[0]
    print(f"{name}: N={N}", flush=True)
    m = md.Model(cfg["model"])
    cells = md.Cells()
    md.build_cells(m, cells, dev(cfg["pos"]), dev(cfg["quat"]), None, cfg["box"])
    r = {p: {k: v.cpu().numpy() for k, v in md.forces(m, cells, p).items()} for p in ("fp64", "fp32")}
    idx = np.sort(np.random.default_rng(99).choice(N, size=256, replace=False))
    ref = oracle.rows(cfg["model"], cfg["pos"], cfg["quat"], cfg["comp"], cfg["box"], idx)
    multi = cfg["quat"] is not None
    for p, bar in (("fp64", 1e-11), ("fp32", 1e-5)):
        g = r[p]
        np.testing.assert_array_equal(g["nnb"][idx], ref["nnb"])
        eF, mF = rel_rms(g["force"][idx], ref["F"]), elem_err(g["force"][idx], ref["F"])
        eu, mu = rel_rms(g["u_mol"][idx], ref["u"]), elem_err(g["u_mol"][idx], ref["u"])
        print(f"  {p}: sampled eps_F {eF:.2e} (max per molecule {mF:.2e}) eps_u {eu:.2e} (max {mu:.2e})",
              flush=True)
        assert eF < bar and mF < 10 * bar
        ubar = 1e-11 if p == "fp64" else 1e-6
        assert eu < ubar and mu < 10 * ubar
        assert_close(g["w_mol"][idx], ref["w"], ubar, "w_mol")
        if multi:
            assert_close(g["torque"][idx], ref["T"], bar, "torque")
        U, Wv = g["uw"][0], g["uw"][1]
        assert g["u_mol"].sum() == pytest.approx(U, rel=1e-10)
        assert g["w_mol"].sum() == pytest.approx(Wv, rel=1e-10)
    assert r["fp64"]["npairs"][0] == r["fp32"]["npairs"][0] == r["fp64"]["nnb"].sum() // 2
    if name in golden:
        gd = golden[name]
        assert int(r["fp64"]["npairs"][0]) == gd["npairs"]
        assert r["fp64"]["uw"][0] == pytest.approx(gd["U"], rel=1e-11)
        assert r["fp64"]["uw"][1] == pytest.approx(gd["W"], rel=1e-11)
        np.testing.assert_allclose(r["fp64"]["uw"][2:5], gd["Wd"], rtol=1e-11)
        eU32 = abs(r["fp32"]["uw"][0] - gd["U"]) / abs(gd["U"])
        print(f"  fp32 vs golden: eps_U {eU32:.2e}", flush=True)
        assert eU32 < 1e-9
    else:
        print(f"  (no golden value for {name} yet)", flush=True)


@pytest.mark.parametrize("name", ["c4_2cljq_500k", "c5_4site_200k", "c2_lj_1m"])
def test_full_size_adjoint_properties(md, name):
    cfg = W.make(name)
    m = md.Model(cfg["model"])
    cells = md.Cells()
    md.build_cells(m, cells, dev(cfg["pos"]), dev(cfg["quat"]), None, cfg["box"])
    f = md.forces(m, cells, "fp64", per_molecule=False)
    U = float(f["uw"][0])
    for prec, bar in (("fp64", 1e-10), ("fp32", 1e-6)):
        g = md.forces_adjoint(m, cells, prec, 1.0, want_quat=cfg["quat"] is not None)
        dpos = g["dpos"].cpu().numpy()
        assert_close(dpos, -f["force"].cpu().numpy(), 1e-12 if prec == "fp64" else 1e-5, "dpos")
        par = g["dparams"].cpu().numpy()
        comp = cfg["model"]["components"][0]
        # Euler: sum_a eps_a dU/deps_a + 1/2 sum_moments m dU/dm = U (LJ degree 1 in eps, shift
        # included; dipole-dipole (+ reaction field) and quadrupole-quadrupole degree 2 in moments)
        col, acc = 0, 0.0
        for s in [s for s in comp["sites"] if s["kind"] == "lj"]:
            acc += s["eps"] * par[col]
            col += 5
        for kind, key in (("charge", "q"), ("dipole", "mu"), ("quadrupole", "Q")):
            for s in [s for s in comp["sites"] if s["kind"] == kind]:
                acc += 0.5 * s[key] * par[col]
                col += 4
        assert col == par.shape[0]
        print(f"{name} {prec}: Euler identity rel err {abs(acc - U) / abs(U):.2e}", flush=True)
        assert acc == pytest.approx(U, rel=bar)


def test_fcc_lattice_beyond_32_bit_component_indices(md):
    """Maximum size: a perfect FCC LJTS crystal of 4 x 565^3 = 721 448 500 molecules (3 N passes
    2^31, so per-molecule outputs need 64-bit addressing), generated on the device.  Every
    molecule must feel zero force, count the 54 lattice neighbours inside r_c and carry the
    per-molecule energy of the integer lattice-vector sum, in both precisions."""
    if torch.cuda.get_device_properties(0).total_memory < 150 * 2 ** 30:
        pytest.skip("needs ~90 GiB of device memory")
    n, rho, rc = 565, 0.8, 2.5
    a = (4.0 / rho) ** (1.0 / 3.0)
    N = 4 * n ** 3
    assert 3 * N > 2 ** 31
    # expected: half the LJTS energies over the lattice vectors (a/2)(h, k, l), h + k + l even
    u_expected, nn = 0.0, 0
    shift = 4.0 * (rc ** -12 - rc ** -6)
    for h in range(-4, 5):
        for k in range(-4, 5):
            for l in range(-4, 5):
                if (h + k + l) % 2 or (h, k, l) == (0, 0, 0):
                    continue
                r = 0.5 * a * math.sqrt(h * h + k * k + l * l)
                if r < rc:
                    u_expected += 0.5 * (4.0 * (r ** -12 - r ** -6) - shift)
                    nn += 1
    assert nn == 54
    pos = torch.empty((N, 3), dtype=torch.float64, device="cuda")
    cell = torch.arange(n ** 3, dtype=torch.int64, device="cuda")
    ijk = torch.stack((cell % n, (cell // n) % n, cell // (n * n)), dim=1).to(torch.float64)
    del cell
    view = pos.view(n ** 3, 4, 3)
    for b, off in enumerate(((0.0, 0.0, 0.0), (0.5, 0.5, 0.0), (0.5, 0.0, 0.5), (0.0, 0.5, 0.5))):
        view[:, b, :] = (ijk + torch.tensor(off, dtype=torch.float64, device="cuda")) * a
    del ijk, view
    box = [n * a] * 3
    m = md.Model(W.lj_model(rc, shift=True))
    cells = md.Cells()
    md.build_cells(m, cells, pos, None, None, box)
    del pos
    for prec, fbar in (("fp64", 1e-9), ("fp32", 1e-5)):
        f = md.forces(m, cells, prec, torque=False, per_molecule=True)
        fmax = float(f["force"].abs().max())
        umin, umax = float(f["u_mol"].min()), float(f["u_mol"].max())
        nmin, nmax = int(f["nnb"].min()), int(f["nnb"].max())
        print(f"{prec}: N={N} |F|max {fmax:.2e} u in [{umin:.15f}, {umax:.15f}] expected {u_expected:.15f} "
              f"nnb in [{nmin}, {nmax}]", flush=True)
        assert nmin == nmax == nn
        assert int(f["npairs"][0]) == N * nn // 2
        assert fmax < fbar
        assert abs(umin - u_expected) < 1e-9 * abs(u_expected) and abs(umax - u_expected) < 1e-9 * abs(u_expected)
        assert float(f["uw"][0]) == pytest.approx(N * u_expected, rel=1e-9)
        del f
