"""GPU adjoint (md_forces_adjoint: recomputation backward, no stored pair list) against the FP64
autograd reference of oracle/oracle_torch.py: dU/d(positions), dU/d(raw quaternions) and
dU/d(epsilon, sigma, site offsets, charges, dipole and quadrupole moments)."""
import numpy as np
import pytest
import torch

from tests._gpu import assert_close, dev, elem_err, rel_rms
from paper_1408_4599_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def md():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1408_4599_amd import md as _md
    _md.lib()
    return _md


def _abi_params(model, pg):
    """Autograd parameter gradients laid out like md_forces_adjoint's dparams."""
    out = []
    for c, comp in enumerate(model["components"]):
        g = pg[c]
        for kind, key in (("lj", None), ("charge", "charge_m"), ("dipole", "dipole_m"), ("quadrupole", "quadrupole_m")):
            n = sum(1 for s in comp["sites"] if s["kind"] == kind)
            for a in range(n):
                if kind == "lj":
                    out += [g["lj_eps"][a], g["lj_sigma"][a]]
                else:
                    out += [g[key][a]]
                out += list(g[kind + "_pos"][a])
    return np.array(out)


def _cfg(name):
    if name == "c5_dilute":  # about 11 molecules per cell: one wavefront per home cell
        return W.random_gas(400, [14.0, 15.0, 16.5], W.four_site_model(), seed=17, T=1.2, dmin=1.0)
    if name == "c1_sub":
        c = W.make("c1_ljts_4000")
        c["pos"], c["vel"], c["comp"] = c["pos"][:1200], c["vel"][:1200], c["comp"][:1200]
        return c
    return W.make(name)


@pytest.fixture(scope="module")
def refs():
    from oracle import oracle_torch as OT
    out = {}
    for name in ("c1_sub", "c4_small", "c5_small", "mixture_small", "c5_dilute", "mixture4_small"):
        c = _cfg(name)
        out[name] = (c, OT.gradients(c["model"], c["pos"], c["quat"], c["comp"], c["box"]))
    return out


BARS = {"fp64": (1e-10, 1e-10, 1e-10), "fp32": (1e-5, 1e-5, 1e-5)}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["c1_sub", "c4_small", "c5_small", "mixture_small", "c5_dilute", "mixture4_small"])
def test_adjoint_matches_autograd_reference(md, refs, name, prec):
    c, ref = refs[name]
    m = md.Model(c["model"])
    cells = md.Cells()
    ncomp = len(c["model"]["components"])
    md.build_cells(m, cells, dev(c["pos"]), dev(c["quat"]), dev(c["comp"], torch.int32) if ncomp > 1 else None, c["box"])
    gU = 0.75
    g = md.forces_adjoint(m, cells, prec, gU, want_quat=c["quat"] is not None)
    torch.cuda.synchronize()
    bp, bq, bpar = BARS[prec]
    dpos = g["dpos"].cpu().numpy()
    e_pos, m_pos = rel_rms(dpos, gU * ref["dpos"]), elem_err(dpos, gU * ref["dpos"])
    msg = f"{name} {prec}: dpos {e_pos:.2e} (max per molecule {m_pos:.2e})"
    assert e_pos < bp and m_pos < 10 * bp, msg
    if c["quat"] is not None:
        dq = g["dquat"].cpu().numpy()
        e_q, m_q = rel_rms(dq, gU * ref["dquat"]), elem_err(dq, gU * ref["dquat"])
        msg += f" dquat {e_q:.2e} (max {m_q:.2e})"
        assert e_q < bq and m_q < 10 * bq, msg
    par = g["dparams"].cpu().numpy()
    want = gU * _abi_params(c["model"], ref["params"])
    assert par.shape == want.shape
    # offsets of a single-site model sum to ~0 (Newton's third law): compare against the scale
    scale = np.abs(want).max()
    e_par = np.abs(par - want).max() / scale
    msg += f" params {e_par:.2e}"
    print(msg, flush=True)
    assert e_par < bpar, msg


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["c1_sub", "c4_small", "c5_small", "mixture_small", "c5_dilute", "mixture4_small"])
def test_adjoint_without_parameters(md, refs, name, prec):
    """dpos and dquat only (no dparams): the kernels without the parameter partials must meet the
    same bars against the autograd reference and agree with the full call to rounding (the
    position and axis gradients are the same arithmetic)."""
    c, ref = refs[name]
    m = md.Model(c["model"])
    cells = md.Cells()
    ncomp = len(c["model"]["components"])
    md.build_cells(m, cells, dev(c["pos"]), dev(c["quat"]), dev(c["comp"], torch.int32) if ncomp > 1 else None, c["box"])
    gU = 0.75
    multi = c["quat"] is not None
    full = md.forces_adjoint(m, cells, prec, gU, want_quat=multi)
    part = md.forces_adjoint(m, cells, prec, gU, want_quat=multi, want_params=False)
    torch.cuda.synchronize()
    assert part["dparams"] is None
    bp, bq, _ = BARS[prec]
    tight = 1e-13 if prec == "fp64" else 1e-6
    dpos = part["dpos"].cpu().numpy()
    assert rel_rms(dpos, gU * ref["dpos"]) < bp and elem_err(dpos, gU * ref["dpos"]) < 10 * bp
    assert elem_err(dpos, full["dpos"].cpu().numpy()) < tight
    if multi:
        dq = part["dquat"].cpu().numpy()
        assert rel_rms(dq, gU * ref["dquat"]) < bq and elem_err(dq, gU * ref["dquat"]) < 10 * bq
        assert elem_err(dq, full["dquat"].cpu().numpy()) < tight


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("half_shell", [False, True])
def test_single_site_adjoint_through_the_force_kernels(md, refs, prec, half_shell):
    """Single-site models take the adjoint from one force evaluation (dU/dr = -F; eps and sigma
    gradients from U, W and the pair count): through the full-shell and the half-shell force
    kernel alike, against the autograd reference, with and without parameter gradients, at two
    values of gU."""
    c, ref = refs["c1_sub"]
    m = md.Model(c["model"], half_shell=half_shell)
    cells = md.Cells()
    md.build_cells(m, cells, dev(c["pos"]), None, None, c["box"])
    bp, _, bpar = BARS[prec]
    want = _abi_params(c["model"], ref["params"])
    for gU in (0.75, -2.0):
        g = md.forces_adjoint(m, cells, prec, gU, want_quat=False)
        h = md.forces_adjoint(m, cells, prec, gU, want_quat=False, want_params=False)
        torch.cuda.synchronize()
        for d in (g["dpos"], h["dpos"]):
            dpos = d.cpu().numpy()
            assert rel_rms(dpos, gU * ref["dpos"]) < bp and elem_err(dpos, gU * ref["dpos"]) < 10 * bp
        par = g["dparams"].cpu().numpy()
        assert par.shape == want.shape
        assert np.abs(par - gU * want).max() / np.abs(gU * want).max() < bpar


def test_energy_autograd_function(md, refs):
    """EnergyFn: forward = md_forces energy, backward = md_forces_adjoint (gradients w.r.t. the
    position and quaternion tensors), chained through further torch operations."""
    c, ref = refs["c5_small"]
    m = md.Model(c["model"])
    cells = md.Cells()
    pos = dev(c["pos"]).requires_grad_(True)
    quat = dev(c["quat"]).requires_grad_(True)
    U = md.energy(pos, quat, m, cells, c["box"])
    assert float(U) == pytest.approx(ref["U"], rel=1e-12)
    (3.0 * U).backward()
    assert_close(pos.grad.cpu().numpy(), 3.0 * ref["dpos"], 1e-10, "dpos")
    assert_close(quat.grad.cpu().numpy(), 3.0 * ref["dquat"], 1e-10, "dquat")


def _perturbed(model, scale_eps=1.1, scale_sig=0.97, shift_off=0.01, scale_m=0.9):
    """A copy of the model with every site parameter changed (inputs only)."""
    import copy
    m = copy.deepcopy(model)
    for comp in m["components"]:
        for s in comp["sites"]:
            if s["kind"] == "lj":
                s["eps"] *= scale_eps
                s["sigma"] *= scale_sig
            for key in ("q", "mu", "Q"):
                if key in s:
                    s[key] *= scale_m
            if len(comp["sites"]) > 1:
                s["pos"] = [v + shift_off for v in s["pos"]]
    return m


@pytest.mark.parametrize("name", ["c5_small", "mixture_small", "c1_sub"])
def test_energy_fn_parameter_gradients(md, name):
    """EnergyFn(pos, quat, params): the parameter vector is a differentiable input.  With every
    parameter moved away from the model's own values, U and the gradients with respect to pos,
    quat and params equal the FP64 autograd reference of the perturbed model at 1e-10."""
    from oracle import oracle_torch as OT
    c = _cfg(name)
    pm = _perturbed(c["model"])
    ref = OT.gradients(pm, c["pos"], c["quat"], c["comp"], c["box"])
    m = md.Model(c["model"])
    cells = md.Cells()
    ncomp = len(c["model"]["components"])
    comp = dev(c["comp"], torch.int32) if ncomp > 1 else None
    as_np = lambda model: [{k: v.numpy() for k, v in d.items()}
                           for d in OT.params_from_model(model, requires_grad=False)]
    want_params = _abi_params(pm, as_np(pm))
    np.testing.assert_array_equal(m.params(), _abi_params(c["model"], as_np(c["model"])))
    params = torch.tensor(want_params, dtype=torch.float64).requires_grad_(True)
    pos = dev(c["pos"]).requires_grad_(True)
    quat = None if c["quat"] is None else dev(c["quat"]).requires_grad_(True)
    U = md.energy(pos, quat, m, cells, c["box"], comp, params=params)
    np.testing.assert_array_equal(m.params(), want_params)
    assert float(U) == pytest.approx(ref["U"], rel=1e-12)
    (2.0 * U).backward()
    assert_close(pos.grad.cpu().numpy(), 2.0 * ref["dpos"], 1e-10, "dpos")
    if quat is not None:
        assert_close(quat.grad.cpu().numpy(), 2.0 * ref["dquat"], 1e-10, "dquat")
    want = 2.0 * _abi_params(pm, ref["params"])
    got = params.grad.numpy()
    e = np.abs(got - want).max() / np.abs(want).max()
    print(f"{name}: params grad max rel err {e:.2e}", flush=True)
    assert e < 1e-10


def test_energy_fn_parameter_errors(md):
    m = md.Model(W.four_site_model())
    p = m.params()
    bad = p.copy()
    bad[0] = -1.0  # epsilon of the first LJ site
    with pytest.raises(md.MDError) as e:
        m.set_params(bad)
    assert e.value.code == md.MD_EINVAL
    np.testing.assert_array_equal(m.params(), p)
    bad[0] = np.nan
    with pytest.raises(md.MDError) as e:
        m.set_params(bad)
    assert e.value.code == md.MD_ENONFINITE
    lj = md.Model(W.lj_model(2.5))
    q = lj.params()
    q[2] = 0.1  # the single site's offset
    with pytest.raises(md.MDError) as e:
        lj.set_params(q)
    assert e.value.code == md.MD_EINVAL


def test_energy_fn_non_contiguous_quaternions(md, refs):
    """Quaternions as a strided view into an N x 7 state tensor: the copies made for the library
    stay valid through backward, and the gradient lands in the view."""
    c, ref = refs["c5_small"]
    m = md.Model(c["model"])
    cells = md.Cells()
    state = torch.cat([dev(c["pos"]), dev(c["quat"])], dim=1).requires_grad_(True)
    pos, quat = state[:, :3], state[:, 3:]
    assert not quat.is_contiguous()
    U = md.energy(pos, quat, m, cells, c["box"])
    # churn the caching allocator between forward and backward
    junk = [torch.empty_like(quat).fill_(7.0) for _ in range(4)]
    U.backward()
    del junk
    g = state.grad.cpu().numpy()
    assert_close(g[:, :3], ref["dpos"], 1e-10, "dpos")
    assert_close(g[:, 3:], ref["dquat"], 1e-10, "dquat")


def test_adjoint_after_step_uses_the_built_copy(md):
    """After md_step the cells hold the configuration at the start of the last step: the adjoint
    equals, bit for bit, the adjoint of a fresh build from that configuration, although the
    caller's arrays have moved on (and are overwritten here)."""
    c = W.make("c4_small")
    m = md.Model(c["model"])
    cells = md.Cells()
    pos, vel, quat, ang = dev(c["pos"]), dev(c["vel"]), dev(c["quat"]), dev(c["angmom"])
    p0, q0 = pos.clone(), quat.clone()
    md.step(m, cells, pos, vel, quat, ang, None, c["box"], c["dt"], 1, "fp64")
    quat.fill_(0.5)
    pos.fill_(1.0)
    a = md.forces_adjoint(m, cells, "fp64", 1.0)
    m2 = md.Model(c["model"])
    cells2 = md.Cells()
    md.build_cells(m2, cells2, p0, q0, None, c["box"])
    b = md.forces_adjoint(m2, cells2, "fp64", 1.0)
    torch.cuda.synchronize()
    for k in ("dpos", "dquat", "dparams"):
        np.testing.assert_array_equal(a[k].cpu().numpy(), b[k].cpu().numpy())
