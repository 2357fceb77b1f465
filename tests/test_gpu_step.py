"""GPU md_step (leapfrog translation + quaternion rotation, cell rebuild every step) against the
FP64 oracle's integrator on the same seeded states.  Trajectories are compared after a short run
(rounding differences grow chaotically, so the bars are loose absolute position tolerances well
below any physical scale) and the per-step energies term by term."""
import numpy as np
import pytest
import torch

from tests._gpu import assert_close, dev
from paper_1408_4599_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def md():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1408_4599_amd import md as _md
    _md.lib()
    return _md


def _run_gpu(md, cfg, nsteps, precision="fp64", dt=None, T_target=0.0):
    m = md.Model(cfg["model"])
    if T_target:
        m.set_thermostat(T_target)
    cells = md.Cells()
    pos, vel = dev(cfg["pos"]), dev(cfg["vel"])
    quat, ang = dev(cfg["quat"]), dev(cfg["angmom"])
    ncomp = len(cfg["model"]["components"])
    comp = dev(cfg["comp"], torch.int32) if ncomp > 1 else None
    en = md.step(m, cells, pos, vel, quat, ang, comp, cfg["box"], dt or cfg["dt"], nsteps, precision)
    torch.cuda.synchronize()
    return (pos.cpu().numpy(), vel.cpu().numpy(), None if quat is None else quat.cpu().numpy(),
            None if ang is None else ang.cpu().numpy(), en.cpu().numpy())


def _min_image(d, box):
    return d - box * np.round(d / box)


@pytest.mark.parametrize("name,nsteps,tol", [("c1_ljts_4000", 100, 1e-9), ("c4_small", 20, 1e-9),
                                             ("mixture_small", 20, 1e-9)])
def test_step_fp64_matches_oracle_trajectory(md, oracle, name, nsteps, tol):
    cfg = W.make(name)
    p_ref, v_ref, q_ref, j_ref, e_ref = oracle.step(cfg["model"], cfg["pos"], cfg["vel"], cfg["quat"], cfg["angmom"],
                                                    cfg["comp"], cfg["box"], cfg["dt"], nsteps)
    p, v, q, j, e = _run_gpu(md, cfg, nsteps)
    assert np.abs(_min_image(p - p_ref, cfg["box"])).max() < tol
    assert np.abs(v - v_ref).max() < 1e3 * tol
    if q is not None:
        assert np.abs(q - q_ref).max() < 1e3 * tol
        assert np.abs(j - j_ref).max() < 1e3 * tol
    # U, K_trans, K_rot, W per step
    np.testing.assert_allclose(e, e_ref, rtol=1e-9, atol=1e-9 * np.abs(e_ref).max())


@pytest.mark.parametrize("name,nsteps,tol", [("c1_ljts_4000", 50, 1e-9), ("c4_small", 20, 1e-9),
                                             ("mixture_small", 20, 1e-9)])
def test_step_nvt_matches_oracle_trajectory(md, oracle, name, nsteps, tol):
    """NVT by velocity rescaling (md_set_thermostat): the trajectory and energies of the oracle's
    rescaled leapfrog, with a target temperature away from the start state's; the kinetic
    temperature must approach the target."""
    cfg = W.make(name)
    T_target = 0.7
    p_ref, v_ref, q_ref, j_ref, e_ref = oracle.step(cfg["model"], cfg["pos"], cfg["vel"], cfg["quat"], cfg["angmom"],
                                                    cfg["comp"], cfg["box"], cfg["dt"], nsteps, T_target=T_target)
    p, v, q, j, e = _run_gpu(md, cfg, nsteps, T_target=T_target)
    assert np.abs(_min_image(p - p_ref, cfg["box"])).max() < tol
    assert np.abs(v - v_ref).max() < 1e3 * tol
    if q is not None:
        assert np.abs(q - q_ref).max() < 1e3 * tol
        assert np.abs(j - j_ref).max() < 1e3 * tol
    np.testing.assert_allclose(e, e_ref, rtol=1e-9, atol=1e-9 * np.abs(e_ref).max())
    N = cfg["pos"].shape[0]
    comps = cfg["model"]["components"]
    comp = np.zeros(N, dtype=np.int64) if cfg["comp"] is None else cfg["comp"]
    f = 3 * N + (0 if cfg["quat"] is None else sum(int(np.sum(np.asarray(comps[c]["inertia"]) > 0)) for c in comp))
    T = 2.0 * (e[:, 1] + e[:, 2]) / f
    assert abs(T[-1] - T_target) < abs(T[0] - T_target)


@pytest.mark.parametrize("name", ["c1_ljts_4000", "c4_small"])
def test_step_fp32_matches_oracle_trajectory(md, oracle, name):
    """The FP32 md_step (the path behind the benchmark's step rate) against the FP64 oracle's
    integrator over 10 steps.  The FP32 force error (below 1e-5 relative) moves a molecule by
    about (10 dt)^2 |dF| / 2 m, some 1e-8 here, so positions are held to 1e-7 absolute, velocities
    and angular momenta to 1e-5 and quaternions to 1e-6.  Per step: U at the FP32 energy bar
    (1e-9 relative), K_trans and K_rot at 1e-8 (velocity errors of 1e-7 relative average out
    over the molecules), W at 1e-6 (it carries the FP32 force scalars)."""
    cfg = W.make(name)
    nsteps = 10
    p_ref, v_ref, q_ref, j_ref, e_ref = oracle.step(cfg["model"], cfg["pos"], cfg["vel"], cfg["quat"], cfg["angmom"],
                                                    cfg["comp"], cfg["box"], cfg["dt"], nsteps)
    p, v, q, j, e = _run_gpu(md, cfg, nsteps, "fp32")
    dp = np.abs(_min_image(p - p_ref, cfg["box"])).max()
    dv = np.abs(v - v_ref).max()
    print(f"{name}: max |dpos| {dp:.2e} max |dvel| {dv:.2e}", flush=True)
    assert dp < 1e-7 and dv < 1e-5
    if q is not None:
        dq, dj = np.abs(q - q_ref).max(), np.abs(j - j_ref).max()
        print(f"  max |dquat| {dq:.2e} max |dangmom| {dj:.2e}", flush=True)
        assert dq < 1e-6 and dj < 1e-5
    rel = np.abs(e - e_ref) / np.abs(e_ref).max(axis=0).clip(1e-300)
    print(f"  per-step relative errors U {rel[:, 0].max():.2e} K_trans {rel[:, 1].max():.2e} "
          f"K_rot {rel[:, 2].max():.2e} W {rel[:, 3].max():.2e}", flush=True)
    assert rel[:, 0].max() < 1e-9
    assert rel[:, 1].max() < 1e-8
    if q is not None:
        assert rel[:, 2].max() < 1e-8
    assert rel[:, 3].max() < 1e-6


def test_step_nve_fp32_energy_conservation(md):
    """FP32 path over 200 steps of C1: the total energy stays within the band of the FP64 path."""
    cfg = W.make("c1_ljts_4000")
    *_, e32 = _run_gpu(md, cfg, 200, "fp32")
    *_, e64 = _run_gpu(md, cfg, 200, "fp64")
    E32, E64 = e32[:, :3].sum(1), e64[:, :3].sum(1)
    s32 = np.abs(E32 - E32[0]).max() / abs(E32[0])
    s64 = np.abs(E64 - E64[0]).max() / abs(E64[0])
    assert s64 < 2e-4
    assert s32 < 1.5 * s64 + 1e-6


@pytest.mark.parametrize("name", ["c4_small", "c5_small"])
def test_step_nve_fp32_energy_conservation_multisite(md, name):
    """Multi-site models (half shell: partner forces and torques summed in fixed point on the
    FP32 path) over 200 steps: the total energy, rotation included, stays within the band of the
    FP64 path."""
    cfg = W.make(name)
    *_, e32 = _run_gpu(md, cfg, 200, "fp32")
    *_, e64 = _run_gpu(md, cfg, 200, "fp64")
    E32, E64 = e32[:, :3].sum(1), e64[:, :3].sum(1)
    s32 = np.abs(E32 - E32[0]).max() / abs(E32[0])
    s64 = np.abs(E64 - E64[0]).max() / abs(E64[0])
    print(f"{name}: relative energy band fp64 {s64:.2e} fp32 {s32:.2e}", flush=True)
    assert s32 < 1.5 * s64 + 1e-6


def test_step_checkpoint_resume_is_bitwise(md):
    """100 steps equal 50 steps, copy the state out (checkpoint), then 50 more from the copy."""
    cfg = W.make("c4_small")
    a = _run_gpu(md, cfg, 40)
    half = _run_gpu(md, cfg, 20)
    cfg2 = dict(cfg, pos=half[0], vel=half[1], quat=half[2], angmom=half[3])
    b = _run_gpu(md, cfg2, 20)
    for x, y in zip(a[:4], b[:4]):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(a[4][20:], b[4])


@pytest.mark.parametrize("name", ["c1_ljts_4000", "c4_small"])
def test_step_energies_on_the_side_stream_equal_single_steps(md, name):
    """One call of 6 steps with an energies row reduces each step on the model's side stream,
    overlapping the next step; six one-step calls reduce on the caller's stream.  Energies rows
    and final state agree bit for bit."""
    cfg = W.make(name)
    a = _run_gpu(md, cfg, 6)
    m = md.Model(cfg["model"])
    cells = md.Cells()
    pos, vel = dev(cfg["pos"]), dev(cfg["vel"])
    quat, ang = dev(cfg["quat"]), dev(cfg["angmom"])
    rows = [md.step(m, cells, pos, vel, quat, ang, None, cfg["box"], cfg["dt"], 1, "fp64").cpu().numpy()[0]
            for _ in range(6)]
    np.testing.assert_array_equal(np.array(rows), a[4])
    np.testing.assert_array_equal(pos.cpu().numpy(), a[0])
    np.testing.assert_array_equal(vel.cpu().numpy(), a[1])


@pytest.mark.parametrize("name", ["c1_ljts_4000", "c4_small"])
def test_step_nvt_without_energies_row_is_bitwise_the_same(md, name):
    """md_step with energies = NULL still reduces K(t) for the thermostat: the final state equals
    the run that also writes the energies row, bit for bit."""
    cfg = W.make(name)
    a = _run_gpu(md, cfg, 15, T_target=0.7)
    m = md.Model(cfg["model"])
    m.set_thermostat(0.7)
    cells = md.Cells()
    pos, vel = dev(cfg["pos"]), dev(cfg["vel"])
    quat, ang = dev(cfg["quat"]), dev(cfg["angmom"])
    boxa = np.ascontiguousarray(np.asarray(cfg["box"], dtype=np.float64))
    md._check(md.lib().md_step(m.handle, cells.handle, md._ptr(pos), md._ptr(vel), md._ptr(quat), md._ptr(ang), None,
                               pos.shape[0], boxa.ctypes.data_as(md._dp), float(cfg["dt"]), 15, md.PRECISION["fp64"],
                               None, md._stream()))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(pos.cpu().numpy(), a[0])
    np.testing.assert_array_equal(vel.cpu().numpy(), a[1])
    if quat is not None:
        np.testing.assert_array_equal(quat.cpu().numpy(), a[2])
        np.testing.assert_array_equal(ang.cpu().numpy(), a[3])


def test_step_same_objects_across_sizes(md):
    """One model and one cells object driven through systems of different N and box (larger,
    smaller, then the first again): each run equals a run on fresh objects, bit for bit."""
    base = W.make("c1_ljts_4000")
    small = W.random_gas(2500, [15.0, 16.0, 17.0], base["model"], seed=21, dmin=0.9)
    small["vel"] = W.maxwell_velocities(np.random.default_rng(5), np.ones(2500), 1.0)
    big = W.random_gas(6000, [20.0, 21.0, 22.0], base["model"], seed=22, dmin=0.9)
    big["vel"] = W.maxwell_velocities(np.random.default_rng(6), np.ones(6000), 1.0)
    m = md.Model(base["model"])
    cells = md.Cells()
    for cfg in (base, big, small, base):
        pos, vel = dev(cfg["pos"]), dev(cfg["vel"])
        en = md.step(m, cells, pos, vel, None, None, None, cfg["box"], base["dt"], 5, "fp64")
        torch.cuda.synchronize()
        ref = _run_gpu(md, dict(cfg, quat=None, angmom=None, comp=None), 5, dt=base["dt"])
        np.testing.assert_array_equal(pos.cpu().numpy(), ref[0])
        np.testing.assert_array_equal(vel.cpu().numpy(), ref[1])
        np.testing.assert_array_equal(en.cpu().numpy(), ref[4])
