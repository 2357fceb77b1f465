"""GPU checks specific to the half-shell multi-site pair kernel (Newton's third law, Fig. 1).

Each molecule pair is evaluated once; the partner receives -F and -tau - d x F, summed exactly
(fixed-point integers in LDS, rows summed in a fixed order), and rows whose terms exceed the
fixed-point range are formed again in FP64 by the fix-up kernel.  Checked here against the FP64
oracle: grids of three cells per axis (the half stencil wraps on both sides of every cell),
overlapping molecules that take the fix-up in both precisions, and
the conservation laws of an isolated cluster."""
import numpy as np
import pytest

from tests._gpu import assert_close, dev, elem_err, rel_rms, run_forces
from tests.test_gpu_parity import _ms_cluster
from paper_1408_4599_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def md():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1408_4599_amd import md as _md
    _md.lib()
    return _md


SMALL_GRIDS = {
    # r_c = 4 (3.5 for the mixture): three cells along most axes, the fewest the grid allows, so that
    # the half stencil reaches across the periodic boundary on both sides of every cell
    "four_site_3x3x4": lambda: W.random_gas(180, [12.3, 12.5, 16.6], W.four_site_model(), seed=51, dmin=1.0),
    "four_site_3x3x3_dense": lambda: W.random_gas(540, [12.2, 12.4, 12.6], W.four_site_model(), seed=52, dmin=0.9),
    "2cljq_3x4x3": lambda: W.random_gas(290, [12.2, 16.6, 12.4], W.twoclj_q_model(), seed=53, dmin=1.0),
    "mixture_3x3x4": lambda: W.random_gas(450, [10.6, 10.8, 14.2], W.mixture_model(), seed=54, dmin=1.0),
}


# FP32 energy bar: 1e-9, the stated target, for every case.  The dilute quadrupolar gas is the
# hard one: its quadrupole-quadrupole energies of both signs cancel to a small U, so the kernel
# forms the direction cosines and angular factors of the energy in FP64.
FP32_U_BAR = 1e-9


def _check(md, oracle, cfg, prec, bar, ubar=1e-9):
    ref = oracle.rows(cfg["model"], cfg["pos"], cfg["quat"], cfg["comp"], cfg["box"])
    got, m, _ = run_forces(md, cfg, prec)
    np.testing.assert_array_equal(got["nnb"], ref["nnb"])
    assert got["npairs"] == ref["nnb"].sum() // 2
    eF, eT = rel_rms(got["force"], ref["F"]), rel_rms(got["torque"], ref["T"])
    mF, mT = elem_err(got["force"], ref["F"]), elem_err(got["torque"], ref["T"])
    eu = rel_rms(got["u_mol"], ref["u"])
    eU = abs(got["U"] - ref["u"].sum()) / abs(ref["u"].sum())
    print(f"  {prec}: eps_F {eF:.2e} (max {mF:.2e}) eps_T {eT:.2e} (max {mT:.2e}) eps_u {eu:.2e} eps_U {eU:.2e}",
          flush=True)
    assert eF < bar and eT < bar
    assert mF < 10 * bar and mT < 10 * bar
    assert_close(got["u_mol"], ref["u"], 1e-11 if prec == "fp64" else 1e-6, "u_mol")
    assert eU < (1e-12 if prec == "fp64" else ubar)
    assert m.status() == 0
    return got


@pytest.mark.parametrize("name", list(SMALL_GRIDS))
def test_small_grids_match_oracle(md, oracle, name):
    cfg = SMALL_GRIDS[name]()
    print(f"{name}: N={len(cfg['pos'])}", flush=True)
    _check(md, oracle, cfg, "fp64", 1e-11)
    _check(md, oracle, cfg, "fp32", 1e-5, FP32_U_BAR)


@pytest.mark.parametrize("args", [(150, 100, 23), (300, 160, 29)], ids=["w1", "w4"])
def test_overlapping_molecules_take_the_fp64_fixup(md, oracle, args):
    """Sites 0.45 apart: pair forces far beyond the fixed-point ranges (2^22 for FP32 terms, 2^50
    for FP64 ones).  The affected partner rows come from the fix-up and match the oracle; the
    status word stays clear and the results are bitwise reproducible."""
    cfg = _ms_cluster(*args)
    ref = oracle.rows(cfg["model"], cfg["pos"], cfg["quat"], cfg["comp"], cfg["box"])
    print(f"max |F| component {np.abs(ref['F']).max():.3e}", flush=True)
    assert np.abs(ref["F"]).max() > 2.0 ** 50
    for prec, bar in (("fp64", 1e-11), ("fp32", 1e-5)):
        a, m, _ = run_forces(md, cfg, prec)
        b, _, _ = run_forces(md, cfg, prec)
        for k in ("force", "torque", "u_mol", "w_mol", "nnb"):
            np.testing.assert_array_equal(a[k], b[k])
        assert np.all(np.isfinite(a["force"])) and np.all(np.isfinite(a["torque"]))
        np.testing.assert_array_equal(a["nnb"], ref["nnb"])
        eF, eT = rel_rms(a["force"], ref["F"]), rel_rms(a["torque"], ref["T"])
        mF, mT = elem_err(a["force"], ref["F"]), elem_err(a["torque"], ref["T"])
        print(f"  {prec}: eps_F {eF:.2e} (max {mF:.2e}) eps_T {eT:.2e} (max {mT:.2e})", flush=True)
        assert eF < bar and eT < bar
        assert mF < 10 * bar and mT < 10 * bar
        assert m.status() == 0


def test_isolated_cluster_conserves_momentum_and_angular_momentum(md):
    """A cluster far from every box face has no periodic partners: the pair forces sum to zero
    and so do the torques about the origin, sum_i (tau_i + r_i x F_i).  Both hold term by term
    for the partner forces and torques of the half shell, up to rounding."""
    c = W.random_gas(400, [9.0, 9.0, 9.0], W.four_site_model(), seed=57, dmin=1.0)
    c["pos"] = c["pos"] + 10.0
    c["box"] = np.array([30.0, 30.0, 30.0])
    got, _, _ = run_forces(md, c, "fp64")
    F, T = got["force"], got["torque"]
    scale_F = np.abs(F).sum()
    assert got["npairs"] > 1000
    assert np.all(np.abs(F.sum(0)) < 1e-13 * scale_F)
    L = T.sum(0) + np.cross(c["pos"], F).sum(0)
    scale_L = np.abs(T).sum() + np.abs(np.cross(c["pos"], F)).sum()
    assert np.all(np.abs(L) < 1e-13 * scale_L)


def test_fixup_list_overflow_sets_status(md):
    """More partner sums out of the fixed-point range than the fix-up list holds (65 536 rows):
    32 768 four-site molecules on a 0.3-spaced grid with r_c = 1.5 (about 97 000 such rows).  The
    call completes, the status word gets MD_DEV_RANGE, the rows beyond the list give NaN and the
    others stay finite."""
    n = 32
    g = np.stack(np.meshgrid(*[np.arange(n)] * 3, indexing="ij"), -1).reshape(-1, 3)
    pos = 2.0 + 0.3 * g
    cfg = {"model": W.four_site_model(rc=1.5), "pos": pos, "quat": W.random_quaternions(W.rng_for(61), len(pos)),
           "comp": np.zeros(len(pos), dtype=np.int32), "box": np.array([30.0, 30.0, 30.0])}
    got, m, _ = run_forces(md, cfg, "fp32")
    st = m.status()
    bad = ~np.isfinite(got["force"]).all(axis=1)
    print(f"status {st:#x}, molecules with a NaN force {int(bad.sum())} of {len(pos)}", flush=True)
    assert st & md.MD_DEV_RANGE
    assert 0 < bad.sum() < len(pos)


# ---------------------------------------------------------------- single-site models, MD_HALF_SHELL
from tests.test_gpu_parity import _force_cfg  # noqa: E402

LJ_CASES = ["c1_ljts_4000", "c3_small", "gas_ragged", "dense_lj", "one_cell"]


@pytest.mark.parametrize("name", LJ_CASES)
def test_single_site_half_shell_matches_oracle(md, oracle, name):
    """MD_HALF_SHELL on single-site LJ fluids (homogeneous, the slab, a ragged gas, dense cells,
    one overfull cell): pair set bit for bit, FP64 within 1e-11, FP32 within the stated errors,
    zero torques."""
    cfg = _force_cfg(name)
    ref = oracle.rows(cfg["model"], cfg["pos"], cfg["quat"], cfg["comp"], cfg["box"])
    U = ref["u"].sum()
    for prec, fbar, ubar in (("fp64", 1e-11, 1e-12), ("fp32", 1e-5, 1e-9)):
        got, m, _ = run_forces(md, cfg, prec, half_shell=True)
        np.testing.assert_array_equal(got["nnb"], ref["nnb"])
        assert got["npairs"] == ref["nnb"].sum() // 2
        eF, eU = rel_rms(got["force"], ref["F"]), abs(got["U"] - U) / abs(U)
        mF = elem_err(got["force"], ref["F"])
        print(f"{name} {prec}: eps_F {eF:.2e} (max {mF:.2e}) eps_U {eU:.2e}", flush=True)
        assert eF < fbar and eU < ubar and mF < 10 * fbar
        assert np.all(got["torque"] == 0.0)
        if prec == "fp64":
            assert got["W"] == pytest.approx(ref["w"].sum(), rel=1e-12)
            assert_close(got["u_mol"], ref["u"], 1e-11, "u_mol")
            assert_close(got["w_mol"], ref["w"], 1e-11, "w_mol")
        assert m.status() == 0


def test_single_site_half_shell_tiny_systems(md, oracle):
    """N = 2 in a large box and N = 1 through the half-shell kernel."""
    mdl = W.lj_model(2.5, shift=False)
    cfg = {"model": mdl, "pos": np.array([[1.0, 1.0, 1.0], [2.2, 1.3, 0.9]]), "quat": None,
           "comp": np.zeros(2, np.int32), "box": np.array([12.0, 13.0, 14.0])}
    got, _, _ = run_forces(md, cfg, "fp64", half_shell=True)
    ref = oracle.forces(mdl, cfg["pos"], None, None, cfg["box"])
    assert got["npairs"] == 1
    np.testing.assert_allclose(got["force"], ref["F"], rtol=1e-13)
    cfg["pos"], cfg["comp"] = cfg["pos"][:1], cfg["comp"][:1]
    got, _, _ = run_forces(md, cfg, "fp64", half_shell=True)
    assert got["npairs"] == 0 and np.all(got["force"] == 0) and got["U"] == 0.0


def test_single_site_half_shell_steps_follow_the_default_kernel(md):
    """md_step with MD_HALF_SHELL and with the default kernel from the same state: the same
    energies to rounding over 20 FP64 steps."""
    import torch
    cfg = W.make("c1_ljts_4000")
    rows = []
    for hs in (False, True):
        m = md.Model(cfg["model"], half_shell=hs)
        cells = md.Cells()
        pos, vel = dev(cfg["pos"]), dev(cfg["vel"])
        en = torch.empty((20, 4), dtype=torch.float64, device="cuda")
        md.step(m, cells, pos, vel, None, None, None, cfg["box"], cfg["dt"], 20, "fp64", en)
        torch.cuda.synchronize()
        rows.append(en.cpu().numpy())
    np.testing.assert_allclose(rows[1], rows[0], rtol=1e-9)
