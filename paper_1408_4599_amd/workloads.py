"""Seeded synthetic scenario generators (the role of the paper's internal scenario generators,
Sec. 1, which create the initial configuration directly in memory).

This module produces inputs only -- molecule models, positions, velocities, orientations and
angular momenta -- and holds none of the force, cell or integrator arithmetic.  Both the GPU
library and the CPU reference consume exactly these arrays.

State points follow the paper's scenario families: a homogeneous Lennard-Jones fluid, a planar
vapour-liquid interface of the LJTS fluid (Sec. 5.2, scenario list) and rigid multi-centre
molecules with LJ sites plus point polarities (Sec. 2).  The ethylene-oxide parameters the paper
cites are not given in it, so the four-site molecule here is a synthetic stand-in of the same
shape (three LJ sites and one point dipole).

Model dictionaries:
    {"components": [{"sites": [...], "mass": m, "inertia": [Ix, Iy, Iz]}, ...],
     "xi": ncomp x ncomp or None, "eta": ncomp x ncomp or None,
     "rc": r_c, "eps_rf": permittivity (inf allowed), "lj_shift": bool}
Sites (body frame, COM at the origin, principal axes = body axes), grouped by kind in the order
LJ, charge, dipole, quadrupole:
    {"kind": "lj", "pos": [x,y,z], "eps": e, "sigma": s}
    {"kind": "charge", "pos": [...], "q": q}
    {"kind": "dipole", "pos": [...], "dir": unit [..], "mu": mu}
    {"kind": "quadrupole", "pos": [...], "dir": unit [..], "Q": Q}
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 14084599
KIND_ORDER = ("lj", "charge", "dipole", "quadrupole")


# ----------------------------------------------------------------------------- molecule models

def lj_model(rc=2.5, shift=True):
    """Single-site LJ 12-6 (LJTS when shift is set), epsilon = sigma = m = 1."""
    comp = {"sites": [{"kind": "lj", "pos": [0.0, 0.0, 0.0], "eps": 1.0, "sigma": 1.0}],
            "mass": 1.0, "inertia": [0.0, 0.0, 0.0]}
    return {"components": [comp], "xi": None, "eta": None, "rc": float(rc), "eps_rf": math.inf,
            "lj_shift": bool(shift)}


def twoclj_q_model(elong=0.5, q2=2.0, rc=4.0, eps_rf=math.inf, shift=False):
    """Rigid two-centre LJ plus a point quadrupole on the axis (2CLJQ): LJ sites at +-elong/2 on
    body z, epsilon = sigma = 1, quadrupole Q = sqrt(q2) at the COM along z, total mass 1 split
    over the two sites; linear molecule, so I_z = 0."""
    h = 0.5 * elong
    comp = {"sites": [{"kind": "lj", "pos": [0.0, 0.0, -h], "eps": 1.0, "sigma": 1.0},
                      {"kind": "lj", "pos": [0.0, 0.0, h], "eps": 1.0, "sigma": 1.0},
                      {"kind": "quadrupole", "pos": [0.0, 0.0, 0.0], "dir": [0.0, 0.0, 1.0], "Q": math.sqrt(q2)}],
            "mass": 1.0, "inertia": [2 * 0.5 * h * h, 2 * 0.5 * h * h, 0.0]}
    return {"components": [comp], "xi": None, "eta": None, "rc": float(rc), "eps_rf": float(eps_rf),
            "lj_shift": bool(shift)}


def four_site_model(mu2=3.0, rc=4.0, eps_rf=math.inf, shift=False):
    """Synthetic three-LJ-site + point-dipole molecule (stand-in for the ethylene-oxide shape):
    LJ sites (-0.4,0,-0.2), (0.4,0,-0.2), (0,0,0.4) with sigma (1,1,0.9), epsilon (1,1,1.5), mass
    1/3 each (COM at the origin, principal axes = body axes), dipole mu = sqrt(mu2) at the COM
    along +z."""
    pos = [[-0.4, 0.0, -0.2], [0.4, 0.0, -0.2], [0.0, 0.0, 0.4]]
    m = 1.0 / 3.0
    I = [sum(m * (p[1] ** 2 + p[2] ** 2) for p in pos), sum(m * (p[0] ** 2 + p[2] ** 2) for p in pos),
         sum(m * (p[0] ** 2 + p[1] ** 2) for p in pos)]
    sig = [1.0, 1.0, 0.9]
    eps = [1.0, 1.0, 1.5]
    sites = [{"kind": "lj", "pos": p, "eps": e, "sigma": s} for p, e, s in zip(pos, eps, sig)]
    sites.append({"kind": "dipole", "pos": [0.0, 0.0, 0.0], "dir": [0.0, 0.0, 1.0], "mu": math.sqrt(mu2)})
    comp = {"sites": sites, "mass": 1.0, "inertia": I}
    return {"components": [comp], "xi": None, "eta": None, "rc": float(rc), "eps_rf": float(eps_rf),
            "lj_shift": bool(shift)}


def mixture_model(rc=3.5, eps_rf=20.0, shift=True):
    """Two-component mixture exercising every site kind and every electrostatic pairing.
    A: two LJ sites, a +-q charge pair, an off-centre dipole.  B: one LJ site, a charge, an
    off-axis dipole and an off-centre quadrupole.  Binary parameters xi, eta differ from 1."""
    a = {"sites": [{"kind": "lj", "pos": [0.0, 0.0, -0.3], "eps": 1.0, "sigma": 1.0},
                   {"kind": "lj", "pos": [0.0, 0.0, 0.3], "eps": 0.8, "sigma": 0.9},
                   {"kind": "charge", "pos": [0.2, 0.0, 0.1], "q": 0.6},
                   {"kind": "charge", "pos": [-0.2, 0.0, 0.1], "q": -0.6},
                   {"kind": "dipole", "pos": [0.0, 0.1, 0.0], "dir": [0.0, 0.6, 0.8], "mu": 0.9}],
         "mass": 1.3, "inertia": [0.2, 0.25, 0.05]}
    b = {"sites": [{"kind": "lj", "pos": [0.0, 0.0, 0.0], "eps": 1.2, "sigma": 1.05},
                   {"kind": "charge", "pos": [0.0, 0.15, 0.0], "q": 0.3},
                   {"kind": "dipole", "pos": [0.1, 0.0, 0.0], "dir": [1.0, 0.0, 0.0], "mu": 0.7},
                   {"kind": "quadrupole", "pos": [0.0, 0.0, 0.12], "dir": [0.0, 0.0, 1.0], "Q": 0.8}],
         "mass": 0.9, "inertia": [0.1, 0.1, 0.12]}
    return {"components": [a, b], "xi": [[1.0, 0.95], [0.95, 1.0]], "eta": [[1.0, 1.02], [1.02, 1.0]],
            "rc": float(rc), "eps_rf": float(eps_rf), "lj_shift": bool(shift)}


def mixture4_model(rc=3.5, eps_rf=20.0, shift=True):
    """Four components (the most a model may hold): the two of mixture_model, a linear two-centre
    LJ + quadrupole molecule (one principal moment zero) and a plain LJ atom (no rotation);
    binary parameters xi, eta differ from 1."""
    m = mixture_model(rc, eps_rf, shift)
    c = {"sites": [{"kind": "lj", "pos": [0.0, 0.0, -0.25], "eps": 0.9, "sigma": 1.0},
                   {"kind": "lj", "pos": [0.0, 0.0, 0.25], "eps": 0.9, "sigma": 1.0},
                   {"kind": "quadrupole", "pos": [0.0, 0.0, 0.0], "dir": [0.0, 0.0, 1.0], "Q": 1.1}],
         "mass": 1.0, "inertia": [0.0625, 0.0625, 0.0]}
    d = {"sites": [{"kind": "lj", "pos": [0.0, 0.0, 0.0], "eps": 0.7, "sigma": 1.1}],
         "mass": 0.8, "inertia": [0.0, 0.0, 0.0]}
    xi = [[1.0, 0.95, 0.9, 1.05], [0.95, 1.0, 0.97, 1.0], [0.9, 0.97, 1.0, 0.93], [1.05, 1.0, 0.93, 1.0]]
    eta = [[1.0, 1.02, 0.98, 1.0], [1.02, 1.0, 1.01, 0.99], [0.98, 1.01, 1.0, 1.03], [1.0, 0.99, 1.03, 1.0]]
    m["components"] = m["components"] + [c, d]
    m["xi"], m["eta"] = xi, eta
    return m


def mixture4_small(N=600, seed=27):
    """The four-component mixture as a dilute random gas (minimum COM separation 1), components
    drawn uniformly."""
    c = random_gas(N, [14.0, 15.0, 16.0], mixture4_model(), seed=seed, T=1.5, name="mixture4_small", dmin=1.0)
    c["comp"] = rng_for(seed + 1).integers(0, 4, size=N).astype(np.int32)
    return c


# ----------------------------------------------------------------------------- building blocks

def rng_for(k: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + int(k)))


def fcc_lattice(n: int, a: float) -> np.ndarray:
    """n^3 FCC unit cells of edge a (4 n^3 sites), offset by a/4 so no site lies on a cell face."""
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]], dtype=np.float64)
    g = np.arange(n, dtype=np.float64)
    cells = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    pts = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    return (pts + 0.25) * a


def fcc_positions_device(n: int, rho: float, seed: int, device, amp=0.05):
    """Large inputs made on a torch device: the n^3 FCC cells of fcc_lattice (same site order) at
    density rho with uniform jitter in [-amp, amp) from a seeded torch generator.  Returns
    (pos [4 n^3, 3] float64 tensor, box)."""
    import torch
    N = 4 * n ** 3
    L = (N / rho) ** (1.0 / 3.0)
    a = L / n
    idx = torch.arange(n ** 3, device=device, dtype=torch.int64)
    ijk = torch.stack((idx // (n * n), (idx // n) % n, idx % n), dim=1).to(torch.float64)
    basis = torch.tensor([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]], device=device, dtype=torch.float64)
    pos = ((ijk[:, None, :] + basis[None, :, :]).reshape(-1, 3) + 0.25) * a
    del ijk, idx
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    pos += (torch.rand(pos.shape, generator=g, device=device, dtype=torch.float64) * 2.0 - 1.0) * amp
    return pos, [L, L, L]


def jitter(rng, pos, amp=0.05):
    return pos + rng.uniform(-amp, amp, size=pos.shape)


def maxwell_velocities(rng, masses, T):
    """N(0, T/m) per component, zero total momentum, rescaled to exactly T over 3N - 3 DOF."""
    N = masses.shape[0]
    v = rng.normal(0.0, 1.0, size=(N, 3)) * np.sqrt(T / masses)[:, None]
    p = (masses[:, None] * v).sum(axis=0) / masses.sum()
    v -= p
    Tin = (masses[:, None] * v * v).sum() / (3 * N - 3)
    return v * math.sqrt(T / Tin)


def random_quaternions(rng, N):
    """Four i.i.d. normals, normalised: uniform on SO(3); scalar-first (w, x, y, z)."""
    q = rng.normal(size=(N, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def angular_momenta(rng, quat, inertia, T):
    """Body-frame j_k ~ N(0, T I_k) for I_k > 0 (0 otherwise), returned in the space frame."""
    from scipy.spatial.transform import Rotation
    I = np.asarray(inertia, dtype=np.float64)
    jb = rng.normal(size=(quat.shape[0], 3)) * np.sqrt(T * I)[None, :]
    rot = Rotation.from_quat(np.concatenate([quat[:, 1:], quat[:, :1]], axis=1))  # scalar-last
    return rot.apply(jb)


def orientations_without_overlap(rng, pos, box, site_pos, dmin, max_rounds=200):
    """Random orientations (uniform on SO(3)) such that no two sites of different molecules are
    closer than dmin (minimum image): in every round, one molecule of each clashing pair, picked
    at random, draws a new orientation, until no clash is left."""
    from scipy.spatial import cKDTree
    N, box = pos.shape[0], np.asarray(box, dtype=np.float64)
    site_pos = np.asarray(site_pos, dtype=np.float64)
    mol = np.repeat(np.arange(N), site_pos.shape[0])
    quat = random_quaternions(rng, N)
    for _ in range(max_rounds):
        w, x, y, z = quat.T
        A = np.stack([np.stack([w * w + x * x - y * y - z * z, 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
                      np.stack([2 * (x * y + w * z), w * w - x * x + y * y - z * z, 2 * (y * z - w * x)], -1),
                      np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), w * w - x * x - y * y + z * z], -1)], -2)
        sites = (pos[:, None, :] + np.einsum("nij,sj->nsi", A, site_pos)).reshape(-1, 3) % box
        sites = np.where(sites >= box, sites - box, sites)
        pairs = cKDTree(sites, boxsize=box).query_pairs(dmin, output_type="ndarray")
        mp = mol[pairs]
        mp = mp[mp[:, 0] != mp[:, 1]]
        if len(mp) == 0:
            return quat
        bad = np.unique(mp[np.arange(len(mp)), rng.integers(0, 2, size=len(mp))])
        quat[bad] = random_quaternions(rng, len(bad))
    raise RuntimeError("orientations_without_overlap: no arrangement found")


def _system(name, model, pos, box, T, rng, dt, nsteps, comp=None, rotate=True, note="", quat=None):
    N = pos.shape[0]
    comp = np.zeros(N, dtype=np.int32) if comp is None else np.asarray(comp, dtype=np.int32)
    masses = np.asarray([model["components"][c]["mass"] for c in comp], dtype=np.float64)
    vel = maxwell_velocities(rng, masses, T)
    multi = any(len(c["sites"]) > 1 or c["sites"][0]["kind"] != "lj" or any(v != 0 for v in c["sites"][0]["pos"])
                for c in model["components"])
    angmom = None
    if not (multi and rotate):
        quat = None
    else:
        quat = random_quaternions(rng, N) if quat is None else quat
        angmom = np.zeros((N, 3))
        for c, cm in enumerate(model["components"]):
            sel = comp == c
            if sel.any():
                angmom[sel] = angular_momenta(rng, quat[sel], cm["inertia"], T)
    return {"name": name, "model": model, "pos": np.ascontiguousarray(pos), "vel": vel, "quat": quat,
            "angmom": angmom, "comp": comp, "box": np.asarray(box, dtype=np.float64), "T": float(T),
            "dt": float(dt), "nsteps": int(nsteps), "note": note}


# ----------------------------------------------------------------------------- scenarios

def homogeneous_lj(ncell_fcc, rho, T, rc=2.5, shift=True, seed=0, name="lj", nsteps=100, dt=0.002):
    """Homogeneous LJ(TS) fluid: FCC start at density rho, uniform jitter 0.05 sigma."""
    rng = rng_for(seed)
    N = 4 * ncell_fcc ** 3
    L = (N / rho) ** (1.0 / 3.0)
    pos = jitter(rng, fcc_lattice(ncell_fcc, L / ncell_fcc))
    return _system(name, lj_model(rc, shift), pos, [L, L, L], T, rng, dt, nsteps)


def c1_ljts_4000():
    """LJTS r_c = 2.5, N = 4000 (FCC 10^3), rho = 0.8, T = 1.0; 100 leapfrog steps, dt = 0.002."""
    return homogeneous_lj(10, 0.8, 1.0, rc=2.5, shift=True, seed=1, name="c1_ljts_4000", nsteps=100)


def c2_lj_1m():
    """Homogeneous LJ liquid, N = 1,048,576 (FCC 64^3), rho = 0.75, T = 0.9, r_c = 2.5 (shifted)."""
    return homogeneous_lj(64, 0.75, 0.9, rc=2.5, shift=True, seed=2, name="c2_lj_1m", nsteps=1000)


def c3_lj_slab_2m(N_total=2_000_000, name="c3_lj_slab_2m"):
    """Planar vapour-liquid interface: box 3L x L x L with rho_avg * 3L^3 = N, liquid slab
    (rho = 0.73, FCC with random vacancies) in the middle third along x, vapour (rho = 0.02,
    uniform, no two molecules closer than 1 sigma) elsewhere; T = 0.85, r_c = 3 (shifted)."""
    rng = rng_for(3)
    L = (N_total / 0.77) ** (1.0 / 3.0)
    n_liq = int(round(0.73 * L ** 3))
    n_vap = N_total - n_liq
    nf = int(math.ceil((n_liq / 4) ** (1.0 / 3.0)))
    lat = jitter(rng, fcc_lattice(nf, L / nf))
    keep = rng.choice(lat.shape[0], size=n_liq, replace=False)
    keep.sort()
    liq = lat[keep]
    liq[:, 0] += L
    vap = _vapour(rng, n_vap, L, liq)
    pos = np.concatenate([liq, vap], axis=0)
    perm = rng.permutation(pos.shape[0])
    return _system(name, lj_model(3.0, True), pos[perm], [3 * L, L, L], 0.85, rng, 0.002, 1000)


def c3_small():
    """The slab of c3_lj_slab_2m at N = 12 000 (box 75 x 25 x 25): liquid neighbourhoods hold far
    more molecules than the box average, as in the full-size slab."""
    return c3_lj_slab_2m(12_000, "c3_small")


def _vapour(rng, n, L, liq, dmin=1.0):
    """n uniform points in x in [0, L) U [2L, 3L), y, z in [0, L), none within dmin of another
    point or of a liquid molecule (periodic in all three directions)."""
    from scipy.spatial import cKDTree
    box = np.array([3 * L, L, L])
    face = liq[(liq[:, 0] < L + dmin) | (liq[:, 0] >= 2 * L - dmin)]
    tree = cKDTree(np.mod(face, box), boxsize=box)
    ng = np.floor(box / dmin).astype(np.int64)  # grid cells of edge box/ng >= dmin
    edge = box / ng
    grid = {}
    out = []
    while len(out) < n:
        cand = rng.uniform(0.0, 1.0, size=(4 * (n - len(out)) + 64, 3)) * np.array([2 * L, L, L])
        cand[:, 0] = np.where(cand[:, 0] < L, cand[:, 0], cand[:, 0] + L)
        ok = np.array([len(x) == 0 for x in tree.query_ball_point(cand, dmin)])
        for p in cand[ok]:
            key = np.minimum((p // edge).astype(np.int64), ng - 1)
            clash = False
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        kk = ((key[0] + dx) % ng[0], (key[1] + dy) % ng[1], (key[2] + dz) % ng[2])
                        for q in grid.get(kk, ()):
                            d = p - q
                            d -= box * np.round(d / box)
                            if d @ d < dmin * dmin:
                                clash = True
                                break
                        if clash:
                            break
                    if clash:
                        break
                if clash:
                    break
            if clash:
                continue
            grid.setdefault((key[0], key[1], key[2]), []).append(p)
            out.append(p)
            if len(out) == n:
                break
    return np.asarray(out)


def c4_2cljq(nf=50, rho=0.5, name="c4_2cljq_500k", seed=4):
    """2CLJQ, L* = 0.5, Q*^2 = 2, rho = 0.5 (FCC nf^3, a = (4/rho)^(1/3)), T = 1.5, random
    orientations, r_c = 4 on the COM distance, reaction field set (no dipoles: no effect)."""
    rng = rng_for(seed)
    N = 4 * nf ** 3
    L = nf * (4.0 / rho) ** (1.0 / 3.0)
    if abs(rho - 0.5) < 1e-15:
        L = 2.0 * nf  # a = 2 exactly at rho = 0.5
    pos = jitter(rng, fcc_lattice(nf, L / nf))
    return _system(name, twoclj_q_model(), pos, [L, L, L], 1.5, rng, 0.002, 1000)


def c4_small():
    """2CLJQ at the C4 state point, N = 1372 (FCC 7^3, L = 14)."""
    return c4_2cljq(nf=7, name="c4_small", seed=14)


def c5_four_site(N=200_000, rho=0.4, name="c5_4site_200k", seed=5):
    """Four-site stand-in (3 LJ + dipole mu^2 = 3), rho = 0.4, T = 1.2, random orientations,
    r_c = 4, reaction field eps_RF = infinity: FCC with random vacancies down to N.  The
    elongated molecules on the lattice would put some LJ sites of neighbours almost on top of each
    other; orientations are drawn until no two sites of different molecules are closer than
    0.7 sigma, so that the start state can be integrated at dt = 0.002."""
    rng = rng_for(seed)
    L = (N / rho) ** (1.0 / 3.0)
    nf = int(math.ceil((N / 4) ** (1.0 / 3.0)))
    lat = jitter(rng, fcc_lattice(nf, L / nf))
    keep = np.sort(rng.choice(lat.shape[0], size=N, replace=False))
    model = four_site_model()
    lj = [st["pos"] for st in model["components"][0]["sites"] if st["kind"] == "lj"]
    quat = orientations_without_overlap(rng, lat[keep], [L, L, L], lj, 0.7)
    return _system(name, model, lat[keep], [L, L, L], 1.2, rng, 0.002, 1000, quat=quat)


def c5_small():
    """Four-site model at the C5 state point, N = 864 (FCC 6^3 without vacancies)."""
    return c5_four_site(N=864, name="c5_small", seed=15)


def mixture_small(N=1000, seed=21):
    """Two-component mixture (every site kind), rho = 0.3, T = 1.5, ragged FCC (vacancies),
    non-cubic box 1.0 : 1.15 : 1.3, random orientations."""
    rng = rng_for(seed)
    rho = 0.3
    V = N / rho
    s = (V / (1.0 * 1.15 * 1.3)) ** (1.0 / 3.0)
    box = np.array([1.0, 1.15, 1.3]) * s
    nf = int(math.ceil((N / 4 / 1.0) ** (1.0 / 3.0))) + 1
    a = (4.0 / 0.4) ** (1.0 / 3.0)  # denser lattice, thinned to N below
    lat = fcc_lattice(nf + 2, a)
    lat = lat[(lat[:, 0] < box[0] - 0.3 * a) & (lat[:, 1] < box[1] - 0.3 * a) & (lat[:, 2] < box[2] - 0.3 * a)]
    keep = np.sort(rng.choice(lat.shape[0], size=min(N, lat.shape[0]), replace=False))
    pos = jitter(rng, lat[keep], 0.1)
    comp = (rng.uniform(size=pos.shape[0]) < 0.5).astype(np.int32)
    return _system("mixture_small", mixture_model(), pos, box, 1.5, rng, 0.001, 100, comp=comp)


def random_gas(N, box, model, seed=31, T=1.0, name="random_gas", dmin=0.0):
    """Uniform random COMs (uneven cell occupancy, empty cells), optionally with no two
    molecules closer than dmin (random sequential addition on a periodic grid hash; keep
    N dmin^3 / V well below ~1.5, the jamming density of that process)."""
    rng = rng_for(seed)
    box = np.asarray(box, dtype=np.float64)
    if dmin <= 0.0:
        pos = rng.uniform(size=(N, 3)) * box
    else:
        if N * dmin ** 3 / np.prod(box) > 1.0:
            raise ValueError("random_gas: too dense for the requested minimum separation")
        ng = np.maximum(np.floor(box / dmin).astype(np.int64), 1)
        edge = box / ng
        grid = {}
        pts = []
        while len(pts) < N:
            p = rng.uniform(size=3) * box
            key = np.minimum((p // edge).astype(np.int64), ng - 1)
            ok = True
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        for q in grid.get(((key[0] + dx) % ng[0], (key[1] + dy) % ng[1], (key[2] + dz) % ng[2]), ()):
                            d = p - q
                            d -= box * np.round(d / box)
                            if d @ d < dmin * dmin:
                                ok = False
            if ok:
                grid.setdefault((key[0], key[1], key[2]), []).append(p)
                pts.append(p)
        pos = np.asarray(pts)
    return _system(name, model, pos, box, T, rng, 0.001, 10)


CONFIGS = {
    "c1_ljts_4000": c1_ljts_4000,
    "c2_lj_1m": c2_lj_1m,
    "c3_lj_slab_2m": c3_lj_slab_2m,
    "c4_2cljq_500k": c4_2cljq,
    "c5_4site_200k": c5_four_site,
    "c4_small": c4_small,
    "c5_small": c5_small,
    "c3_small": c3_small,
    "mixture_small": mixture_small,
    "mixture4_small": mixture4_small,
}


def make(name: str) -> dict:
    return CONFIGS[name]()
