"""ctypes binding of libmdcell (include/md.h).  Argument marshalling only: every step of the
force path runs in the library's HIP kernels.  PyTorch supplies device memory (CUDA tensors on
ROCm) and the current stream.  There is no CPU fallback: without the built library or a GPU every
call raises.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdcell.so")

MD_OK, MD_EINVAL, MD_EBOX, MD_ECOMP, MD_ENONFINITE, MD_EHIP, MD_ENOMEM, MD_EDEVICE = 0, -1, -2, -3, -4, -5, -6, -7
MD_LJ_SHIFT, MD_CHECK, MD_HALF_SHELL, MD_SUBCELLS = 0x1, 0x2, 0x4, 0x8
MD_FP64, MD_FP32 = 0, 1
# device status word bits (Model.status)
MD_DEV_NONFINITE, MD_DEV_COMP, MD_DEV_QUAT, MD_DEV_CAPACITY, MD_DEV_RANGE = 0x1, 0x2, 0x4, 0x8, 0x10
PRECISION = {"fp64": MD_FP64, "fp32": MD_FP32, MD_FP64: MD_FP64, MD_FP32: MD_FP32}
MAX_COMP, MAX_LJ, MAX_CHG, MAX_DIP, MAX_QUAD = 4, 4, 4, 2, 2


class MDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libmdcell error {code}: {msg}")
        self.code = code


_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_lp = ctypes.POINTER(ctypes.c_int64)


class ComponentDesc(ctypes.Structure):
    _fields_ = [("n_lj", ctypes.c_int32), ("n_chg", ctypes.c_int32), ("n_dip", ctypes.c_int32),
                ("n_quad", ctypes.c_int32), ("lj_pos", _dp), ("lj_eps", _dp), ("lj_sigma", _dp),
                ("chg_pos", _dp), ("chg_q", _dp), ("dip_pos", _dp), ("dip_dir", _dp), ("dip_mu", _dp),
                ("quad_pos", _dp), ("quad_dir", _dp), ("quad_Q", _dp), ("mass", ctypes.c_double),
                ("inertia", ctypes.c_double * 3)]


class CellsInfo(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("ncell", ctypes.c_int64), ("nc", ctypes.c_int32 * 3),
                ("box", ctypes.c_double * 3), ("cell_of", ctypes.c_void_p), ("cell_start", ctypes.c_void_p),
                ("perm", ctypes.c_void_p), ("sub_start", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libmdcell.so (built in-tree by ``paper_1408_4599_amd.build``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libmdcell.so not built ({LIB_PATH}); run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    L.md_last_error.restype = ctypes.c_char_p
    L.md_last_error.argtypes = []
    L.md_model_create.argtypes = [ctypes.POINTER(ComponentDesc), ctypes.c_int32, _dp, _dp, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_uint32, ctypes.POINTER(vp)]
    L.md_model_destroy.argtypes = [vp]
    L.md_param_count.argtypes = [vp]
    L.md_param_count.restype = ctypes.c_int64
    L.md_cells_create.argtypes = [ctypes.POINTER(vp)]
    L.md_cells_destroy.argtypes = [vp]
    L.md_cells_view.argtypes = [vp, ctypes.POINTER(CellsInfo)]
    L.md_build_cells.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int64, _dp, vp]
    L.md_forces.argtypes = [vp, vp, ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, vp]
    L.md_forces_noalloc.argtypes = [vp, vp, ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, vp]
    L.md_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.c_int64, _dp, ctypes.c_double, ctypes.c_int64,
                          ctypes.c_int, vp, vp]
    L.md_forces_adjoint.argtypes = [vp, vp, ctypes.c_int, ctypes.c_double, vp, vp, vp, vp]
    L.md_status.argtypes = [vp, _ip]
    L.md_profile.argtypes = [vp, ctypes.c_int]
    L.md_profile_read.argtypes = [vp, ctypes.c_char_p, _dp, _lp]
    L.md_set_thermostat.argtypes = [vp, ctypes.c_double]
    L.md_model_get_params.argtypes = [vp, _dp]
    L.md_model_set_params.argtypes = [vp, _dp]
    L.md_long_range_correction.argtypes = [ctypes.POINTER(ComponentDesc), ctypes.c_int32, _dp, _dp, ctypes.c_double,
                                           ctypes.c_uint32, _lp, _dp, _dp, _dp]
    for name in ("md_model_create", "md_model_destroy", "md_cells_create", "md_cells_destroy", "md_cells_view",
                 "md_build_cells", "md_forces", "md_forces_noalloc", "md_step", "md_forces_adjoint", "md_status",
                 "md_profile",
                 "md_profile_read", "md_set_thermostat", "md_long_range_correction", "md_model_get_params",
                 "md_model_set_params"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc):
    if rc != MD_OK:
        raise MDError(rc, lib().md_last_error().decode(errors="replace"))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, dtype, shape, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (ROCm) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _arr(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
    return a


def _component_descs(model: dict):
    """md_component_desc array (host) for a model dictionary, and the arrays it points into."""
    comps = model["components"]
    nc = len(comps)
    descs = (ComponentDesc * nc)()
    keep = []
    for d, comp in zip(descs, comps):
        by = {k: [s for s in comp["sites"] if s["kind"] == k] for k in ("lj", "charge", "dipole", "quadrupole")}
        d.n_lj, d.n_chg, d.n_dip, d.n_quad = (len(by[k]) for k in ("lj", "charge", "dipole", "quadrupole"))

        def put(vals):
            a = _arr(vals) if len(vals) else np.zeros(1)
            keep.append(a)
            return a.ctypes.data_as(_dp)

        d.lj_pos = put([s["pos"] for s in by["lj"]])
        d.lj_eps = put([s["eps"] for s in by["lj"]])
        d.lj_sigma = put([s["sigma"] for s in by["lj"]])
        d.chg_pos = put([s["pos"] for s in by["charge"]])
        d.chg_q = put([s["q"] for s in by["charge"]])
        d.dip_pos = put([s["pos"] for s in by["dipole"]])
        d.dip_dir = put([s["dir"] for s in by["dipole"]])
        d.dip_mu = put([s["mu"] for s in by["dipole"]])
        d.quad_pos = put([s["pos"] for s in by["quadrupole"]])
        d.quad_dir = put([s["dir"] for s in by["quadrupole"]])
        d.quad_Q = put([s["Q"] for s in by["quadrupole"]])
        d.mass = float(comp["mass"])
        for k in range(3):
            d.inertia[k] = float(comp["inertia"][k])
    xi = None if model.get("xi") is None else _arr(model["xi"])
    eta = None if model.get("eta") is None else _arr(model["eta"])
    keep += [xi, eta]
    return descs, keep, xi, eta


def long_range_correction(model: dict, counts, box):
    """(U_lrc, W_lrc): isotropic cut-off corrections of energy and virial (md_long_range_correction;
    host only, no device needed).  counts: molecules per component."""
    descs, keep, xi, eta = _component_descs(model)
    cnt = np.ascontiguousarray(np.asarray(counts, dtype=np.int64).reshape(-1))
    if cnt.shape[0] != len(model["components"]):
        raise ValueError("counts must have one entry per component")
    b = _arr(box)
    u, w = ctypes.c_double(0.0), ctypes.c_double(0.0)
    flags = MD_LJ_SHIFT if model.get("lj_shift") else 0
    _check(lib().md_long_range_correction(descs, len(model["components"]),
                                          None if xi is None else xi.ctypes.data_as(_dp),
                                          None if eta is None else eta.ctypes.data_as(_dp), float(model["rc"]), flags,
                                          cnt.ctypes.data_as(_lp), b.ctypes.data_as(_dp), ctypes.byref(u),
                                          ctypes.byref(w)))
    return u.value, w.value


class Model:
    """A molecule model (component site tables, mixing, cutoff, reaction field) on the device.
    Built from the model dictionaries of ``workloads``.  ``half_shell`` selects the half-shell
    pair kernel for a single-site model (MD_HALF_SHELL); ``subcells`` the half-edge cell order and
    culling of the single-site kernel (MD_SUBCELLS)."""

    def __init__(self, model: dict, check: bool = False, half_shell: bool = False, subcells: bool = False):
        comps = model["components"]
        nc = len(comps)
        descs, self._keep, xi, eta = _component_descs(model)
        flags = ((MD_LJ_SHIFT if model.get("lj_shift") else 0) | (MD_CHECK if check else 0) |
                 (MD_HALF_SHELL if half_shell else 0) | (MD_SUBCELLS if subcells else 0))
        h = ctypes.c_void_p()
        _check(lib().md_model_create(descs, nc, None if xi is None else xi.ctypes.data_as(_dp),
                                     None if eta is None else eta.ctypes.data_as(_dp), float(model["rc"]),
                                     float(model.get("eps_rf", math.inf)), flags, ctypes.byref(h)))
        self.handle = h
        self.model = model
        self.ncomp = nc
        self.single_site = (nc == 1 and len(comps[0]["sites"]) == 1 and comps[0]["sites"][0]["kind"] == "lj"
                            and all(v == 0 for v in comps[0]["sites"][0]["pos"]))
        self.nparam = int(lib().md_param_count(h))

    def close(self):
        if getattr(self, "handle", None):
            lib().md_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def status(self) -> int:
        v = ctypes.c_int32(0)
        _check(lib().md_status(self.handle, ctypes.byref(v)))
        return int(v.value)

    def set_thermostat(self, T_target: float):
        """NVT by velocity rescaling to the kinetic temperature T_target in later md_step calls
        (0: NVE); md_set_thermostat."""
        _check(lib().md_set_thermostat(self.handle, float(T_target)))

    def profile(self, enable: bool):
        _check(lib().md_profile(self.handle, int(enable)))

    def profile_read(self, group: str):
        ms = ctypes.c_double(0)
        n = ctypes.c_int64(0)
        _check(lib().md_profile_read(self.handle, group.encode(), ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)

    def params(self) -> np.ndarray:
        """The differentiable parameters (md_model_get_params), host FP64 [nparam] in the layout
        of md_forces_adjoint's dparams."""
        out = np.zeros(max(1, self.nparam), dtype=np.float64)
        _check(lib().md_model_get_params(self.handle, out.ctypes.data_as(_dp)))
        return out[:self.nparam]

    def set_params(self, params):
        """Replace the differentiable parameters (md_model_set_params; syncs the device)."""
        a = np.ascontiguousarray(np.asarray(params.detach().cpu() if isinstance(params, torch.Tensor) else params,
                                            dtype=np.float64).reshape(-1))
        if a.shape[0] != self.nparam:
            raise ValueError(f"params: expected {self.nparam} values, got {a.shape[0]}")
        _check(lib().md_model_set_params(self.handle, a.ctypes.data_as(_dp)))

    def param_layout(self):
        """List of (component, kind, index, names) in the order of md_forces_adjoint's dparams."""
        out = []
        for c, comp in enumerate(self.model["components"]):
            for kind, names in (("lj", ("eps", "sigma", "x", "y", "z")), ("charge", ("q", "x", "y", "z")),
                                ("dipole", ("mu", "x", "y", "z")), ("quadrupole", ("Q", "x", "y", "z"))):
                for i, _ in enumerate([s for s in comp["sites"] if s["kind"] == kind]):
                    out.append((c, kind, i, names))
        return out


class Cells:
    """A linked-cell grid with molecules sorted into it (library-owned device buffers)."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(lib().md_cells_create(ctypes.byref(h)))
        self.handle = h
        self.N = 0

    def close(self):
        if getattr(self, "handle", None):
            lib().md_cells_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def view(self):
        """Device copies of cell_of [N], cell_start [ncell+1], perm [N] and, for half-edge cells,
        sub_start [8 ncell + 1] (int32 CUDA tensors; None otherwise), plus the grid shape."""
        info = CellsInfo()
        _check(lib().md_cells_view(self.handle, ctypes.byref(info)))
        N, nc = int(info.N), int(info.ncell)

        def copy(ptr, n):
            out = torch.empty(n, dtype=torch.int32, device="cuda")
            _hip_copy(out.data_ptr(), ptr, 4 * n)
            return out

        return {"N": N, "ncell": nc, "nc": tuple(info.nc), "box": tuple(info.box),
                "cell_of": copy(info.cell_of, N), "cell_start": copy(info.cell_start, nc + 1),
                "perm": copy(info.perm, N),
                "sub_start": copy(info.sub_start, 8 * nc + 1) if info.sub_start else None}


_hiprt = None


def _hip_copy(dst, src, nbytes):
    """Device-to-device copy on the current stream through the HIP runtime (plumbing only)."""
    global _hiprt
    if _hiprt is None:
        _hiprt = ctypes.CDLL("libamdhip64.so")
        _hiprt.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                          ctypes.c_void_p]
        _hiprt.hipMemcpyAsync.restype = ctypes.c_int
    err = _hiprt.hipMemcpyAsync(ctypes.c_void_p(dst), ctypes.c_void_p(src), nbytes, 3, _stream())
    if err != 0:
        raise RuntimeError(f"hipMemcpyAsync failed ({err})")


def build_cells(model: Model, cells: Cells, pos, quat, comp, box):
    N = pos.shape[0]
    _need(pos, torch.float64, (N, 3), "pos")
    if quat is not None:
        _need(quat, torch.float64, (N, 4), "quat")
    if comp is not None:
        _need(comp, torch.int32, (N,), "comp")
    boxa = _arr(box)
    _check(lib().md_build_cells(model.handle, cells.handle, _ptr(pos), _ptr(quat), _ptr(comp), N,
                                boxa.ctypes.data_as(_dp), _stream()))
    cells.N = N


def forces(model: Model, cells: Cells, precision="fp64", torque=True, per_molecule=True):
    """Returns dict of CUDA tensors: force [N,3], torque [N,3] (if requested), u_mol, w_mol,
    nnb (if per_molecule), uw [5] = (U, W, Wxx, Wyy, Wzz), npairs [1]."""
    N = cells.N
    dev = "cuda"
    out = {"force": torch.empty((N, 3), dtype=torch.float64, device=dev),
           "uw": torch.empty(5, dtype=torch.float64, device=dev),
           "npairs": torch.empty(1, dtype=torch.int64, device=dev)}
    if torque:
        out["torque"] = torch.empty((N, 3), dtype=torch.float64, device=dev)
    if per_molecule:
        out["u_mol"] = torch.empty(N, dtype=torch.float64, device=dev)
        out["w_mol"] = torch.empty(N, dtype=torch.float64, device=dev)
        out["nnb"] = torch.empty(N, dtype=torch.int32, device=dev)
    forces_into(model, cells, precision, out)
    return out


def forces_into(model: Model, cells: Cells, precision, out: dict):
    """md_forces into preallocated tensors (keys as ``forces``; optional ones may be absent)."""
    _check(lib().md_forces(model.handle, cells.handle, PRECISION[precision], _ptr(out["force"]),
                           _ptr(out.get("torque")), _ptr(out.get("u_mol")), _ptr(out.get("w_mol")),
                           _ptr(out.get("nnb")), _ptr(out["uw"]), _ptr(out.get("npairs")), _stream()))


def forces_into_noalloc(model: Model, cells: Cells, precision, out: dict):
    """md_forces_noalloc into preallocated tensors (keys as ``forces``): the same results with the
    per-call scratch in the library's static device array (no device allocation)."""
    _check(lib().md_forces_noalloc(model.handle, cells.handle, PRECISION[precision], _ptr(out["force"]),
                                   _ptr(out.get("torque")), _ptr(out.get("u_mol")), _ptr(out.get("w_mol")),
                                   _ptr(out.get("nnb")), _ptr(out["uw"]), _ptr(out.get("npairs")), _stream()))


def step(model: Model, cells: Cells, pos, vel, quat, angmom, comp, box, dt, nsteps, precision="fp64",
         energies=None):
    """nsteps leapfrog steps in place on (pos, vel, quat, angmom); returns energies [nsteps, 4]
    (U, K_trans, K_rot, W) as a CUDA tensor."""
    N = pos.shape[0]
    _need(pos, torch.float64, (N, 3), "pos")
    _need(vel, torch.float64, (N, 3), "vel")
    if quat is not None:
        _need(quat, torch.float64, (N, 4), "quat")
        _need(angmom, torch.float64, (N, 3), "angmom")
    if comp is not None:
        _need(comp, torch.int32, (N,), "comp")
    if energies is None:
        energies = torch.empty((max(1, nsteps), 4), dtype=torch.float64, device="cuda")
    boxa = _arr(box)
    _check(lib().md_step(model.handle, cells.handle, _ptr(pos), _ptr(vel), _ptr(quat), _ptr(angmom), _ptr(comp), N,
                         boxa.ctypes.data_as(_dp), float(dt), int(nsteps), PRECISION[precision], _ptr(energies),
                         _stream()))
    cells.N = N
    return energies[:nsteps]


def forces_adjoint(model: Model, cells: Cells, precision="fp64", gU=1.0, want_quat=True, want_params=True):
    """gU * dU/d(pos, quat, parameters) by the recomputing adjoint kernel."""
    N = cells.N
    out = {"dpos": torch.empty((N, 3), dtype=torch.float64, device="cuda")}
    out["dquat"] = torch.empty((N, 4), dtype=torch.float64, device="cuda") if want_quat else None
    out["dparams"] = (torch.empty(max(1, model.nparam), dtype=torch.float64, device="cuda")
                      if (want_params and model.nparam > 0) else None)
    _check(lib().md_forces_adjoint(model.handle, cells.handle, PRECISION[precision], float(gU), _ptr(out["dpos"]),
                                   _ptr(out["dquat"]), _ptr(out["dparams"]), _stream()))
    return out


class EnergyFn(torch.autograd.Function):
    """U(pos, quat, params) as a differentiable FP64 scalar.  Forward sets the model's parameters
    from ``params`` (when given: a FP64 tensor in the layout of ``Model.params()``), then runs
    md_build_cells + md_forces; backward re-traverses the cells with md_forces_adjoint
    (recomputation, no stored pair list) and returns gradients for pos, quat and params.  The
    contiguous copies handed to the library live until the adjoint has run."""

    @staticmethod
    def forward(ctx, pos, quat, params, model, cells, box, comp, precision):
        if params is not None:
            model.set_params(params)
        pos_c = pos.detach().contiguous()
        quat_c = None if quat is None else quat.detach().contiguous()
        build_cells(model, cells, pos_c, quat_c, comp, box)
        r = forces(model, cells, precision, torque=False, per_molecule=False)
        ctx.model, ctx.cells, ctx.precision = model, cells, precision
        ctx.has_quat = quat is not None
        ctx.has_params = params is not None
        empty = torch.empty(0, device=pos.device)
        ctx.save_for_backward(pos, quat if quat is not None else empty, comp if comp is not None else empty,
                              params.detach() if params is not None else empty)
        ctx.box = box
        return r["uw"][0].clone()

    @staticmethod
    def backward(ctx, gU):
        pos, quat, comp, params = ctx.saved_tensors
        comp_t = comp if comp.numel() else None
        if ctx.has_params:  # another forward may have changed the model since
            ctx.model.set_params(params)
        pos_c = pos.detach().contiguous()
        quat_c = quat.detach().contiguous() if ctx.has_quat else None
        build_cells(ctx.model, ctx.cells, pos_c, quat_c, comp_t, ctx.box)
        want_params = ctx.has_params and ctx.needs_input_grad[2]
        g = forces_adjoint(ctx.model, ctx.cells, ctx.precision, float(gU.item()), want_quat=ctx.has_quat,
                           want_params=want_params)
        dparams = None
        if want_params:
            dparams = (g["dparams"][:ctx.model.nparam].to(params.device) if ctx.model.nparam > 0
                       else torch.zeros_like(params))
        return g["dpos"], (g["dquat"] if ctx.has_quat else None), dparams, None, None, None, None, None


def energy(pos, quat, model, cells, box, comp=None, precision="fp64", params=None):
    """U through EnergyFn; ``params`` (optional FP64 tensor, layout of ``Model.params()``) makes
    the model's parameters differentiable inputs."""
    return EnergyFn.apply(pos, quat, params, model, cells, box, comp, precision)
