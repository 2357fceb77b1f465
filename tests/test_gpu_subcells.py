"""Half-edge (r_c/2) cells on the GPU (Sec. 3, the r_c/2 cell variant), against the oracle.

With MD_SUBCELLS the build sorts each cell's molecules by half-edge cell (then by original index)
and the single-site kernel skips the far z-half of the cell layers above and below each
molecule's own z-half.  Bars: cell ids, half-cell starts, the permutation, per-molecule partner
counts and the pair count bit for bit (the pair set must not change); FP64 forces within 1e-11
relative RMS and energies within 1e-12 relative; FP32 within the stated targets (force 1e-5
relative RMS, energy 1e-9 relative), each with the per-molecule bound of ``assert_close``."""
import numpy as np
import pytest

from tests._gpu import assert_close, dev, elem_err, rel_rms, run_forces
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


def _cfg(name):
    if name == "gas_ragged":
        return W.random_gas(1000, [9.1, 11.7, 14.2], W.lj_model(2.5), seed=7, dmin=0.75)
    if name == "outside_box":
        c = W.random_gas(1000, [10.0, 12.5, 15.0], W.lj_model(2.5), seed=9, dmin=0.75)
        c["pos"] = c["pos"] * 3.0 - 7.0
        return c
    if name == "one_cell":  # 200 molecules in one cell: the chunked path for that home cell
        rng = W.rng_for(43)
        c = W.random_gas(10, [8.0, 8.0, 8.0], W.lj_model(2.5, shift=False), seed=41)
        g = np.stack(np.meshgrid(*[np.arange(6)] * 3, indexing="ij"), -1).reshape(-1, 3)[:200]
        c["pos"] = 0.2 + 0.45 * g + rng.uniform(-0.02, 0.02, size=(200, 3))
        c["comp"] = np.zeros(200, dtype=np.int32)
        return c
    if name == "dense_lj":  # ~40 molecules per cell: tiles beyond the LDS tile take the window
        return W.random_gas(2600, [12.0, 12.0, 12.0], W.lj_model(2.5), seed=33, dmin=0.7)
    if name == "faces":  # many z and y coordinates on, or one rounding off, a half-cell face
        c = W.random_gas(1500, [11.0, 12.0, 13.0], W.lj_model(2.5), seed=51, dmin=0.6)
        box = np.asarray(c["box"])
        hh = box / (2 * np.floor(box / 2.5))
        rng = W.rng_for(52)
        pos = c["pos"].copy()
        for k in (1, 2):
            sel = rng.uniform(size=len(pos)) < 0.4
            pos[sel, k] = np.round(pos[sel, k] / hh[k]) * hh[k] * (1 + rng.choice([-2e-16, 0.0, 2e-16], size=sel.sum()))
        # drop molecules that snapping brought closer than 0.6 to an earlier one
        d = pos[:, None, :] - pos[None, :, :]
        d -= box * np.round(d / box)
        close = np.tril((d * d).sum(-1) < 0.36, -1).any(1)
        c["pos"] = np.ascontiguousarray(pos[~close])
        c["comp"] = np.zeros(len(c["pos"]), dtype=np.int32)
        return c
    return W.make(name)


CASES = ["c1_ljts_4000", "c3_small", "gas_ragged", "outside_box", "one_cell", "dense_lj", "faces"]


def _check_cells(v, oracle, pos, box, rc):
    order, key = oracle.subcell_order(pos, box, rc)
    cell_of, _, ncell = oracle.bin_cells(pos, box, rc)
    assert v["ncell"] == ncell
    np.testing.assert_array_equal(v["cell_of"].cpu().numpy(), cell_of)
    np.testing.assert_array_equal(v["perm"].cpu().numpy(), order)
    sub = v["sub_start"].cpu().numpy()
    np.testing.assert_array_equal(np.diff(sub), np.bincount(key, minlength=8 * ncell))
    assert sub[0] == 0 and sub[-1] == len(pos)
    np.testing.assert_array_equal(v["cell_start"].cpu().numpy(), sub[::8])


@pytest.mark.parametrize("name", CASES)
def test_subcell_order_bit_exact(md, oracle, name):
    cfg = _cfg(name)
    _, m, cells = run_forces(md, cfg, "fp64", subcells=True)
    _check_cells(cells.view(), oracle, cfg["pos"], cfg["box"], cfg["model"]["rc"])


def test_subcell_rebuild_in_previous_order(md, oracle):
    """A rebuild of the same cells object visits molecules in the previous sorted order; the
    half-cell order must still be the oracle's."""
    cfg = W.make("c1_ljts_4000")
    moved = cfg["pos"] + W.rng_for(78).uniform(-0.6, 0.6, size=cfg["pos"].shape)
    m = md.Model(cfg["model"], subcells=True)
    cells = md.Cells()
    md.build_cells(m, cells, dev(cfg["pos"]), None, None, cfg["box"])
    md.build_cells(m, cells, dev(moved), None, None, cfg["box"])
    _check_cells(cells.view(), oracle, moved, cfg["box"], cfg["model"]["rc"])


@pytest.mark.parametrize("subcells,ncell_axis", [(True, 85), (False, 162)])
def test_cell_starts_over_many_scan_chunks(md, oracle, subcells, ncell_axis):
    """A sparse grid with more than 4 M bins (half-edge cells: 85^3 cells x 8; plain: 162^3 cells):
    the scan of the tile totals runs over several chunks, and every start must still be the
    oracle's (cell ids, starts and the stable order bit for bit)."""
    rng = W.rng_for(91 + int(subcells))
    N = 150_000
    box = [ncell_axis * 2.5 + 0.01] * 3
    pos = rng.uniform(0.0, box[0], size=(N, 3))
    m = md.Model(W.lj_model(2.5), subcells=subcells)
    cells = md.Cells()
    md.build_cells(m, cells, dev(pos), None, None, box)
    v = cells.view()
    assert v["ncell"] == ncell_axis ** 3 and (8 if subcells else 1) * v["ncell"] > 4096 * 1024
    if subcells:
        _check_cells(v, oracle, pos, box, 2.5)
    else:
        ref_cell, _, ncell = oracle.bin_cells(pos, box, 2.5)
        np.testing.assert_array_equal(v["cell_of"].cpu().numpy(), ref_cell)
        start = v["cell_start"].cpu().numpy()
        np.testing.assert_array_equal(np.diff(start), np.bincount(ref_cell, minlength=ncell))
        assert start[0] == 0 and start[-1] == N
        np.testing.assert_array_equal(v["perm"].cpu().numpy(), np.lexsort((np.arange(N), ref_cell)))


def test_one_cells_object_switches_models(md, oracle):
    """One cells object built alternately for a model with and one without half-edge cells: each
    build carries its own order."""
    cfg = W.make("c1_ljts_4000")
    a, b = md.Model(cfg["model"], subcells=True), md.Model(cfg["model"])
    cells = md.Cells()
    for m, sub in ((a, True), (b, False), (a, True)):
        md.build_cells(m, cells, dev(cfg["pos"]), None, None, cfg["box"])
        v = cells.view()
        if sub:
            _check_cells(v, oracle, cfg["pos"], cfg["box"], cfg["model"]["rc"])
        else:
            assert v["sub_start"] is None
            ref_cell, _, _ = oracle.bin_cells(cfg["pos"], cfg["box"], cfg["model"]["rc"])
            np.testing.assert_array_equal(v["perm"].cpu().numpy(), np.lexsort((np.arange(len(ref_cell)), ref_cell)))
        out = md.forces(m, cells, "fp64")
        assert int(out["npairs"][0]) > 0


@pytest.mark.parametrize("name", CASES)
def test_subcell_forces_fp64_match_oracle(md, oracle, name):
    cfg = _cfg(name)
    ref = oracle.rows(cfg["model"], cfg["pos"], None, None, cfg["box"])
    got, _, _ = run_forces(md, cfg, "fp64", subcells=True)
    np.testing.assert_array_equal(got["nnb"], ref["nnb"])
    assert got["npairs"] == ref["nnb"].sum() // 2
    assert_close(got["force"], ref["F"], 1e-11, "force")
    assert got["U"] == pytest.approx(ref["u"].sum(), rel=1e-12)
    assert got["W"] == pytest.approx(ref["w"].sum(), rel=1e-12)
    np.testing.assert_allclose(got["Wd"], ref["wd"].sum(0), rtol=1e-12)
    assert_close(got["u_mol"], ref["u"], 1e-11, "u_mol")
    assert_close(got["w_mol"], ref["w"], 1e-11, "w_mol")


@pytest.mark.parametrize("name", CASES)
def test_subcell_forces_fp32_within_stated_error(md, oracle, name):
    cfg = _cfg(name)
    ref = oracle.rows(cfg["model"], cfg["pos"], None, None, cfg["box"])
    got, _, _ = run_forces(md, cfg, "fp32", subcells=True)
    np.testing.assert_array_equal(got["nnb"], ref["nnb"])
    eF, mF = rel_rms(got["force"], ref["F"]), elem_err(got["force"], ref["F"])
    eU = abs(got["U"] - ref["u"].sum()) / abs(ref["u"].sum())
    print(f"{name}: half-edge cells fp32 eps_F {eF:.2e} (max per molecule {mF:.2e}) eps_U {eU:.2e}", flush=True)
    assert eF < 1e-5 and mF < 1e-4
    assert eU < 1e-9
    assert_close(got["u_mol"], ref["u"], 1e-6, "u_mol")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_subcells_equal_default_kernel(md, precision):
    """Same configuration with and without half-edge cells: identical partner counts, forces equal
    to rounding (the summation order of a molecule's partners differs)."""
    cfg = W.make("c3_small")
    a, _, _ = run_forces(md, cfg, precision)
    b, _, _ = run_forces(md, cfg, precision, subcells=True)
    np.testing.assert_array_equal(a["nnb"], b["nnb"])
    bar = 1e-13 if precision == "fp64" else 1e-6
    assert_close(b["force"], a["force"], bar, "force")
    assert b["U"] == pytest.approx(a["U"], rel=1e-12 if precision == "fp64" else 1e-10)


def test_subcells_step_matches_default(md):
    """md_step with half-edge cells (rebuilt every step) follows the default kernel's trajectory to
    rounding over 20 FP64 steps."""
    import torch
    cfg = W.make("c1_ljts_4000")
    out = []
    for sub in (False, True):
        m = md.Model(cfg["model"], subcells=sub)
        cells = md.Cells()
        pos, vel = dev(cfg["pos"]), dev(cfg["vel"])
        en = md.step(m, cells, pos, vel, None, None, None, cfg["box"], cfg["dt"], 20, "fp64")
        torch.cuda.synchronize()
        out.append((pos.cpu().numpy(), en.cpu().numpy()))
    np.testing.assert_allclose(out[1][0], out[0][0], rtol=0, atol=1e-10)
    np.testing.assert_allclose(out[1][1], out[0][1], rtol=1e-10)


def _min_image(d, box):
    return d - box * np.round(d / box)


@pytest.mark.parametrize("prec,nsteps", [("fp64", 30), ("fp32", 10)])
def test_subcell_step_matches_oracle_trajectory(md, oracle, prec, nsteps):
    """md_step with half-edge cells (the benchmarked path) against the oracle's integrator on C1:
    FP64 at the default kernel's FP64 bars (positions 1e-9, velocities 1e-6, energies 1e-9), FP32
    at those of its FP32 trajectory test (positions 1e-7 absolute, velocities 1e-5, per-step U
    1e-9, K 1e-8, W 1e-6)."""
    import torch
    cfg = W.make("c1_ljts_4000")
    p_ref, v_ref, _, _, e_ref = oracle.step(cfg["model"], cfg["pos"], cfg["vel"], None, None, cfg["comp"],
                                            cfg["box"], cfg["dt"], nsteps)
    m = md.Model(cfg["model"], subcells=True)
    cells = md.Cells()
    pos, vel = dev(cfg["pos"]), dev(cfg["vel"])
    en = md.step(m, cells, pos, vel, None, None, None, cfg["box"], cfg["dt"], nsteps, prec)
    torch.cuda.synchronize()
    p, v, e = pos.cpu().numpy(), vel.cpu().numpy(), en.cpu().numpy()
    dp = np.abs(_min_image(p - p_ref, cfg["box"])).max()
    dv = np.abs(v - v_ref).max()
    rel = np.abs(e - e_ref) / np.abs(e_ref).max(axis=0).clip(1e-300)
    print(f"{prec}: max |dpos| {dp:.2e} |dvel| {dv:.2e} U {rel[:, 0].max():.2e} K {rel[:, 1].max():.2e} "
          f"W {rel[:, 3].max():.2e}", flush=True)
    if prec == "fp64":  # the default kernel's FP64 trajectory bars
        assert dp < 1e-9 and dv < 1e-6 and rel.max() < 1e-9
    else:
        assert dp < 1e-7 and dv < 1e-5
        assert rel[:, 0].max() < 1e-9 and rel[:, 1].max() < 1e-8 and rel[:, 3].max() < 1e-6


def test_subcell_nonfinite_molecules_take_no_part(md, oracle):
    """Non-finite molecules go to half-cell 0 of cell (index mod ncell), take part in no pair, and
    the others match the oracle for the system without them."""
    cfg = W.make("c1_ljts_4000")
    pos = cfg["pos"].copy()
    N = len(pos)
    bad = np.sort(np.random.default_rng(15).choice(N, N // 10, replace=False))
    pos[bad[::2], 0] = np.nan
    pos[bad[1::2], 2] = -np.inf
    keep = np.setdiff1d(np.arange(N), bad)
    ref = oracle.rows(cfg["model"], pos[keep], None, None, cfg["box"])
    for prec, bar in (("fp64", 1e-11), ("fp32", 1e-5)):
        got, m, cells = run_forces(md, cfg, prec, pos=pos, subcells=True)
        assert m.status() & md.MD_DEV_NONFINITE
        assert np.all(got["nnb"][bad] == 0) and np.all(got["force"][bad] == 0)
        np.testing.assert_array_equal(got["nnb"][keep], ref["nnb"])
        assert_close(got["force"][keep], ref["F"], bar, f"{prec} force")
    v = cells.view()
    ncell = v["ncell"]
    np.testing.assert_array_equal(v["cell_of"].cpu().numpy()[bad], bad % ncell)
    sub = v["sub_start"].cpu().numpy()
    perm = v["perm"].cpu().numpy()
    slot = np.empty(N, dtype=np.int64)
    slot[perm] = np.arange(N)
    # each non-finite molecule sits in half-cell 0 (octant 0) of its cell
    for i in bad[:20]:
        c = i % ncell
        assert sub[8 * c] <= slot[i] < sub[8 * c + 1]


def test_subcell_tiny_systems(md, oracle):
    """N = 2 in a large box (almost every cell empty) and N = 1 (no pairs)."""
    mdl = W.lj_model(2.5, shift=False)
    cfg = {"model": mdl, "pos": np.array([[1.0, 1.0, 1.0], [2.2, 1.3, 0.9]]), "quat": None,
           "comp": np.zeros(2, np.int32), "box": np.array([12.0, 13.0, 14.0])}
    got, _, _ = run_forces(md, cfg, "fp64", subcells=True)
    ref = oracle.forces(mdl, cfg["pos"], None, None, cfg["box"])
    assert got["npairs"] == 1
    np.testing.assert_allclose(got["force"], ref["F"], rtol=1e-13)
    cfg["pos"], cfg["comp"] = cfg["pos"][:1], cfg["comp"][:1]
    got, _, _ = run_forces(md, cfg, "fp32", subcells=True)
    assert got["npairs"] == 0 and np.all(got["force"] == 0) and got["U"] == 0.0


@pytest.mark.parametrize("box", [[7.6, 8.0, 9.9], [7.6, 12.6, 7.7]])
def test_subcell_three_cell_grids(md, oracle, box):
    """Three cells along some axes: the tile of a block holds the same cell twice (two images),
    and the half-layer walk wraps on both sides."""
    cfg = W.random_gas(int(0.7 * np.prod(box)), box, W.lj_model(2.5), seed=61, dmin=0.8)
    ref = oracle.rows(cfg["model"], cfg["pos"], None, None, cfg["box"])
    for prec, bar in (("fp64", 1e-11), ("fp32", 1e-5)):
        got, _, cells = run_forces(md, cfg, prec, subcells=True)
        np.testing.assert_array_equal(got["nnb"], ref["nnb"])
        assert_close(got["force"], ref["F"], bar, f"{prec} force")
        assert got["U"] == pytest.approx(ref["u"].sum(), rel=1e-12 if prec == "fp64" else 1e-9)
    _check_cells(cells.view(), oracle, cfg["pos"], cfg["box"], 2.5)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_subcell_adjoint_and_noalloc_equal_default(md, prec):
    """The adjoint and the allocation-free entry point on cells built with half-edge cells: the
    adjoint equals the default one to rounding, md_forces_noalloc equals md_forces bit for bit."""
    import torch
    cfg = W.make("c1_ljts_4000")
    out = []
    for sub in (False, True):
        m = md.Model(cfg["model"], subcells=sub)
        cells = md.Cells()
        md.build_cells(m, cells, dev(cfg["pos"]), None, None, cfg["box"])
        g = md.forces_adjoint(m, cells, prec, 1.0, want_quat=False)
        torch.cuda.synchronize()
        out.append((g["dpos"].cpu().numpy(), g["dparams"].cpu().numpy()))
        if sub:
            N = len(cfg["pos"])
            mk = lambda v: {"force": torch.full((N, 3), v, dtype=torch.float64, device="cuda"),
                            "uw": torch.full((5,), v, dtype=torch.float64, device="cuda"),
                            "npairs": torch.full((1,), -3, dtype=torch.int64, device="cuda")}
            a, b = mk(1.0), mk(-2.0)
            md.forces_into(m, cells, prec, a)
            md.forces_into_noalloc(m, cells, prec, b)
            torch.cuda.synchronize()
            for k in a:
                np.testing.assert_array_equal(b[k].cpu().numpy(), a[k].cpu().numpy())
    bar = 1e-12 if prec == "fp64" else 1e-6
    assert_close(out[1][0], out[0][0], bar, "dpos")
    np.testing.assert_allclose(out[1][1], out[0][1], rtol=bar, atol=bar * np.abs(out[0][1]).max())
