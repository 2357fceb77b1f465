"""Helpers for the GPU tests: move generator arrays onto the device and run the library."""
import numpy as np
import torch


def dev(a, dtype=torch.float64):
    if a is None:
        return None
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def run_forces(md, cfg, precision="fp64", pos=None, quat=None, comp=None, model=None, check=False, half_shell=False,
               subcells=False):
    """Build cells and evaluate forces; returns (numpy dict, Model, Cells)."""
    pos = cfg["pos"] if pos is None else pos
    quat = cfg["quat"] if quat is None else quat
    comp = cfg["comp"] if comp is None else comp
    m = md.Model(cfg["model"] if model is None else model, check=check, half_shell=half_shell, subcells=subcells)
    cells = md.Cells()
    ncomp = len((cfg["model"] if model is None else model)["components"])
    md.build_cells(m, cells, dev(pos), dev(quat), dev(comp, torch.int32) if ncomp > 1 else None, cfg["box"])
    r = md.forces(m, cells, precision)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in r.items()}
    out["U"] = float(out["uw"][0])
    out["W"] = float(out["uw"][1])
    out["Wd"] = out["uw"][2:5]
    out["npairs"] = int(out["npairs"][0])
    return out, m, cells


def rel_rms(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def elem_err(a, b):
    """Largest per-molecule error, max_i |a_i - b_i| (Euclidean norm over molecule i's row), over
    the RMS per-molecule magnitude of b.  A bound on every molecule, so that an error confined to
    a few molecules (one tile path, one fix-up row) cannot hide inside a global RMS."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    if a.ndim == 1:
        a, b = a[:, None], b[:, None]
    scale = np.sqrt(np.mean(np.sum(b * b, axis=1)))
    return float(np.linalg.norm(a - b, axis=1).max() / max(scale, 1e-300))


def assert_close(a, b, rms_bar, what="", elem_bar=None):
    """Global relative RMS below rms_bar and every molecule's error below elem_bar (default
    10 rms_bar) times the RMS magnitude; returns both errors."""
    elem_bar = 10.0 * rms_bar if elem_bar is None else elem_bar
    e, m = rel_rms(a, b), elem_err(a, b)
    assert e < rms_bar and m < elem_bar, f"{what}: rel RMS {e:.2e} (bar {rms_bar:.0e}), max per molecule {m:.2e} (bar {elem_bar:.0e})"
    return e, m
