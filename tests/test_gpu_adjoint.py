"""GPU adjoint (md_forces_adjoint: recomputation backward, no stored pair list) against the FP64
autograd reference of oracle/oracle_torch.py: dU/d(positions), dU/d(raw quaternions) and
dU/d(epsilon, sigma, site offsets, charges, dipole and quadrupole moments)."""
import numpy as np
import pytest
import torch

from tests._gpu import dev, rel_rms
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
    e_pos = rel_rms(dpos, gU * ref["dpos"])
    msg = f"{name} {prec}: dpos {e_pos:.2e}"
    assert e_pos < bp, msg
    if c["quat"] is not None:
        e_q = rel_rms(g["dquat"].cpu().numpy(), gU * ref["dquat"])
        msg += f" dquat {e_q:.2e}"
        assert e_q < bq, msg
    par = g["dparams"].cpu().numpy()
    want = gU * _abi_params(c["model"], ref["params"])
    assert par.shape == want.shape
    # offsets of a single-site model sum to ~0 (Newton's third law): compare against the scale
    scale = np.abs(want).max()
    e_par = np.abs(par - want).max() / scale
    msg += f" params {e_par:.2e}"
    print(msg, flush=True)
    assert e_par < bpar, msg


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
    assert rel_rms(pos.grad.cpu().numpy(), 3.0 * ref["dpos"]) < 1e-10
    assert rel_rms(quat.grad.cpu().numpy(), 3.0 * ref["dquat"]) < 1e-10
