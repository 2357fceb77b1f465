"""Pins of the FP64 CPU oracle against facts that do not come from the oracle itself:
closed forms, point-charge constructions of the multipoles, symmetry, conservation laws,
finite differences, an independent library pair counter and integrator error scaling."""
import math

import numpy as np
import pytest

from tests._systems import charge_construction, qmul, quat_axis_angle, single_site_model, two_body
from paper_1408_4599_amd import workloads as W

BOX = np.array([20.0, 20.0, 20.0])


def _two(oracle, model, rA, rB, qA=None, qB=None):
    pos = np.array([rA, rB], dtype=np.float64)
    quat = None if qA is None else np.array([qA, qB], dtype=np.float64)
    return oracle.forces(model, pos, quat, np.array([0, 1], dtype=np.int32), BOX)


# ----------------------------------------------------------------------------- Lennard-Jones

def test_lj_closed_forms(oracle):
    """u(sigma) = 0; u(2^(1/6) sigma) = -epsilon with zero force (LJ equation, Sec. 2)."""
    for eps, sig in [(1.0, 1.0), (2.5, 1.3)]:
        comp = single_site_model("lj", (eps, sig))
        m = two_body(comp, comp, rc=6.0)
        r = _two(oracle, m, [5, 5, 5], [5 + sig, 5, 5])
        assert abs(r["U"]) < 1e-14 * eps
        rmin = 2 ** (1 / 6) * sig
        r = _two(oracle, m, [5, 5, 5], [5, 5 + rmin, 5])
        assert r["U"] == pytest.approx(-eps, rel=1e-14)
        assert np.abs(r["F"]).max() < 1e-12 * eps / sig


def test_ljts_shift_is_constant_per_counted_pair(oracle):
    """LJTS subtracts u(r_c) once per interacting site pair: U_shift - U_plain = -P u(r_c)."""
    c = W.make("c1_ljts_4000")
    plain = dict(c["model"], lj_shift=False)
    a = oracle.forces(c["model"], c["pos"], None, None, c["box"])
    b = oracle.forces(plain, c["pos"], None, None, c["box"])
    rc = c["model"]["rc"]
    urc = 4 * (rc ** -12 - rc ** -6)
    assert a["npairs"] == b["npairs"]
    assert a["U"] - b["U"] == pytest.approx(-a["npairs"] * urc, rel=1e-10)
    assert np.array_equal(a["F"], b["F"])


def test_lorentz_berthelot(oracle):
    """Geometric mean on epsilon, arithmetic mean on sigma (Sec. 2, combination rules): an A-B
    pair equals a single-type pair with epsilon = sqrt(eA eB), sigma = (sA + sB)/2, scaled by
    the binary factors xi (energy) and eta (size)."""
    r = 1.37
    A = single_site_model("lj", (0.7, 0.9))
    B = single_site_model("lj", (2.8, 1.3))
    m = two_body(A, B)
    m["xi"] = [[1.0, 0.9], [0.9, 1.0]]
    m["eta"] = [[1.0, 1.05], [1.05, 1.0]]
    ab = _two(oracle, m, [5, 5, 5], [5, 5, 5 + r])["U"]
    eq = single_site_model("lj", (0.9 * math.sqrt(0.7 * 2.8), 1.05 * 1.1))
    ref = _two(oracle, two_body(eq, eq), [5, 5, 5], [5, 5, 5 + r])["U"]
    assert ab == pytest.approx(ref, rel=1e-13)


def test_two_centre_at_zero_elongation(oracle):
    """A 2CLJ molecule with both sites on the COM is four single-site pairs."""
    two = W.twoclj_q_model(elong=0.0, q2=0.0, rc=6.0)
    one = W.lj_model(rc=6.0, shift=False)
    rng = np.random.default_rng(3)
    pos = rng.uniform(0, 20, size=(40, 3))
    q = W.random_quaternions(rng, 40)
    a = oracle.forces(two, pos, q, None, BOX)
    b = oracle.forces(one, pos, None, None, BOX)
    assert a["U"] == pytest.approx(4 * b["U"], rel=1e-12)
    np.testing.assert_allclose(a["F"], 4 * b["F"], rtol=1e-11, atol=1e-11)


def _fcc_shell_energy(a, rc):
    """Per-molecule FCC lattice energy 1/2 sum_R u(|R|) over lattice vectors |R| < rc, from an
    integer enumeration of the lattice (independent of any pair loop)."""
    prim = 0.5 * a * np.array([[0, 1, 1], [1, 0, 1], [1, 1, 0]], dtype=np.float64)
    n = int(math.ceil(rc / (a / math.sqrt(2)))) + 2
    g = np.arange(-n, n + 1)
    ijk = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    R = ijk @ prim
    r = np.linalg.norm(R, axis=1)
    r = r[(r > 0) & (r < rc)]
    return 0.5 * float(np.sum(4 * (r ** -12 - r ** -6))), int(r.size)


def test_fcc_lattice_zero_force_and_shell_energy(oracle):
    nf, rho, rc = 6, 0.8, 2.5
    a = (4 / rho) ** (1 / 3)
    pos = W.fcc_lattice(nf, a)
    L = nf * a
    r = oracle.forces(W.lj_model(rc, shift=False), pos, None, None, [L, L, L])
    assert np.abs(r["F"]).max() < 1e-12
    e, z = _fcc_shell_energy(a, rc)
    np.testing.assert_allclose(r["u"], e, rtol=1e-12)
    assert r["npairs"] == pos.shape[0] * z // 2


# ----------------------------------------------------------------------------- multipoles

ORIENT = [quat_axis_angle([0.3, -0.5, 0.8], 1.1), quat_axis_angle([-0.7, 0.2, 0.4], 2.3)]
OFFSETS = [[0.12, -0.05, 0.2], [-0.08, 0.15, -0.1]]
AXES = [[0.36, 0.48, 0.8], [0.0, 0.6, -0.8]]
MOMENTS = {"charge": [0.8, -0.55], "dipole": [1.3, 0.9], "quadrupole": [1.1, -0.7]}


def _mp_model(kA, kB, eps_rf=1.0):
    cA = single_site_model(kA, MOMENTS[kA][0], OFFSETS[0], AXES[0])
    cB = single_site_model(kB, MOMENTS[kB][1], OFFSETS[1], AXES[1])
    return two_body(cA, cB, eps_rf=eps_rf)


def _construction_limit(kA, kB, rA, rB):
    """Energy, force on A and torques on A and B of the point-charge constructions of the two
    sites, in 50-digit arithmetic (mpmath), Richardson-extrapolated to d -> 0."""
    import mpmath as mp
    from scipy.spatial.transform import Rotation
    mp.mp.dps = 50

    def world(q, v):
        return Rotation.from_quat([q[1], q[2], q[3], q[0]]).apply(v)

    def eval_d(d):
        d = mp.mpf(d)
        mols = []
        for k, kind, r in ((0, kA, rA), (1, kB, rB)):
            site = [mp.mpf(float(x)) for x in np.asarray(r) + world(ORIENT[k], OFFSETS[k])]
            e = [mp.mpf(float(x)) for x in world(ORIENT[k], AXES[k])]
            m = mp.mpf(MOMENTS[kind][k])
            if kind == "charge":
                ch = [(site, m)]
            elif kind == "dipole":
                q = m / d
                ch = [([s + d / 2 * x for s, x in zip(site, e)], q), ([s - d / 2 * x for s, x in zip(site, e)], -q)]
            else:
                q = m / (2 * d * d)
                ch = [([s + d * x for s, x in zip(site, e)], q), (site, -2 * q), ([s - d * x for s, x in zip(site, e)], q)]
            mols.append(ch)
        U = mp.mpf(0)
        F = [mp.mpf(0)] * 3
        TA = [mp.mpf(0)] * 3
        TB = [mp.mpf(0)] * 3
        cA = [mp.mpf(float(x)) for x in rA]
        cB = [mp.mpf(float(x)) for x in rB]
        for xa, qa in mols[0]:
            for xb, qb in mols[1]:
                R = [a - b for a, b in zip(xa, xb)]
                r = mp.sqrt(sum(x * x for x in R))
                U += qa * qb / r
                f = [qa * qb * x / r ** 3 for x in R]  # force on the A charge
                F = [a + b for a, b in zip(F, f)]
                la = [a - c for a, c in zip(xa, cA)]
                lb = [b - c for b, c in zip(xb, cB)]
                TA = [TA[0] + la[1] * f[2] - la[2] * f[1], TA[1] + la[2] * f[0] - la[0] * f[2], TA[2] + la[0] * f[1] - la[1] * f[0]]
                TB = [TB[0] - (lb[1] * f[2] - lb[2] * f[1]), TB[1] - (lb[2] * f[0] - lb[0] * f[2]), TB[2] - (lb[0] * f[1] - lb[1] * f[0])]
        return [U] + F + TA + TB

    v = [eval_d(d) for d in ("1e-4", "5e-5", "2.5e-5")]
    for p in (1, 2):
        v = [[(4 ** p * b - a) / (4 ** p - 1) for a, b in zip(v[i], v[i + 1])] for i in range(len(v) - 1)]
    return np.array([float(x) for x in v[0]])


@pytest.mark.parametrize("kA,kB", [(a, b) for a in ("charge", "dipole", "quadrupole")
                                   for b in ("charge", "dipole", "quadrupole")])
def test_multipole_against_point_charge_construction(oracle, kA, kB):
    """Every charge/dipole/quadrupole pairing equals the d -> 0 limit of explicit point-charge
    constructions (dipole: +-q at +-d/2; linear quadrupole: q, -2q, q at -d, 0, +d), for energy,
    force and both torques."""
    rA, rB = [6.0, 7.0, 5.5], [8.1, 7.6, 4.9]
    ref = _two(oracle, _mp_model(kA, kB), rA, rB, ORIENT[0], ORIENT[1])
    lim = _construction_limit(kA, kB, rA, rB)
    got = np.concatenate([[ref["U"]], ref["F"][0], ref["T"][0], ref["T"][1]])
    scale = np.abs(got).max()
    np.testing.assert_allclose(got, lim, rtol=0, atol=1e-12 * scale)


def test_textbook_dipole_and_quadrupole_geometries(oracle):
    """Head-to-tail dipoles -2 mu^2/r^3, side-by-side parallel +mu^2/r^3, collinear linear
    quadrupoles +6 Q^2/r^5, T-shaped quadrupoles -3 Q^2/r^5 (identity orientation: axis = z)."""
    mu, Q, r = 1.7, 1.3, 2.2
    idq = [1.0, 0, 0, 0]
    dip = single_site_model("dipole", mu)
    m = two_body(dip, dip)
    assert _two(oracle, m, [5, 5, 5], [5, 5, 5 + r], idq, idq)["U"] == pytest.approx(-2 * mu ** 2 / r ** 3, rel=1e-14)
    assert _two(oracle, m, [5, 5, 5], [5 + r, 5, 5], idq, idq)["U"] == pytest.approx(mu ** 2 / r ** 3, rel=1e-14)
    quad = single_site_model("quadrupole", Q)
    m = two_body(quad, quad)
    assert _two(oracle, m, [5, 5, 5], [5, 5, 5 + r], idq, idq)["U"] == pytest.approx(6 * Q ** 2 / r ** 5, rel=1e-14)
    qy = list(quat_axis_angle([1, 0, 0], math.pi / 2))  # rotates z onto -y
    assert _two(oracle, m, [5, 5, 5], [5, 5, 5 + r], idq, qy)["U"] == pytest.approx(-3 * Q ** 2 / r ** 5, rel=1e-12)


def test_reaction_field_limits(oracle):
    """kappa(eps_RF = 1) = 0 (no reaction field); at eps_RF = inf each dipole pair inside the
    cutoff gains -mu_i.mu_j / r_c^3 and no force."""
    c = W.make("c5_small")
    base = dict(c["model"], eps_rf=1.0)
    full = dict(c["model"], eps_rf=math.inf)
    a = oracle.forces(base, c["pos"], c["quat"], None, c["box"])
    b = oracle.forces(full, c["pos"], c["quat"], None, c["box"])
    rc = c["model"]["rc"]
    # dipole axes in the space frame: third column of the rotation, here via scipy
    from scipy.spatial.transform import Rotation
    q = c["quat"]
    e = Rotation.from_quat(np.concatenate([q[:, 1:], q[:, :1]], 1)).apply([0, 0, 1])
    from oracle.oracle_torch import pair_list
    ii, jj = pair_list(c["pos"], c["box"], rc)
    mu2 = 3.0
    du = -(mu2 * (e[ii] * e[jj]).sum(1)).sum() / rc ** 3
    assert b["U"] - a["U"] == pytest.approx(du, rel=1e-10)
    np.testing.assert_allclose(a["F"], b["F"], rtol=0, atol=1e-9 * np.abs(a["F"]).max())


# ----------------------------------------------------------------------------- derivatives

def _cluster(n=6, seed=5):
    m = W.mixture_model(rc=3.5, eps_rf=20.0)
    rng = np.random.default_rng(seed)
    while True:
        pos = 7.0 + rng.uniform(0, 3.2, size=(n, 3))
        d = np.linalg.norm(pos[:, None] - pos[None], axis=-1)
        iu = np.triu_indices(n, 1)
        if d[iu].min() > 1.4 and np.abs(d[iu] - m["rc"]).min() > 0.05:
            break
    quat = W.random_quaternions(rng, n)
    comp = (np.arange(n) % 2).astype(np.int32)
    return m, pos, quat, comp


def test_forces_and_torques_match_finite_differences(oracle):
    m, pos, quat, comp = _cluster()
    r = oracle.forces(m, pos, quat, comp, BOX)
    h = 1e-5
    for i in range(pos.shape[0]):
        for k in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[i, k] += h
            p2[i, k] -= h
            dU = (oracle.forces(m, p1, quat, comp, BOX)["U"] - oracle.forces(m, p2, quat, comp, BOX)["U"]) / (2 * h)
            assert -dU == pytest.approx(r["F"][i, k], abs=2e-7 * (1 + abs(r["F"][i, k])))
            # rotation by angle h about space axis k: torque_k = -dU/dh
            q1, q2 = quat.copy(), quat.copy()
            q1[i] = qmul(quat_axis_angle(np.eye(3)[k], h), quat[i])
            q2[i] = qmul(quat_axis_angle(np.eye(3)[k], -h), quat[i])
            dU = (oracle.forces(m, pos, q1, comp, BOX)["U"] - oracle.forces(m, pos, q2, comp, BOX)["U"]) / (2 * h)
            assert -dU == pytest.approx(r["T"][i, k], abs=2e-7 * (1 + abs(r["T"][i, k])))


def test_quaternion_gradient_chain_rule(oracle):
    """dU/dq (raw components, no renormalisation) from the oracle's site chain rule equals
    central differences of U."""
    m, pos, quat, comp = _cluster(seed=9)
    rows = oracle.rows(m, pos, quat, comp, BOX, want_dquat=True)
    h = 1e-6
    for i in range(pos.shape[0]):
        for k in range(4):
            q1, q2 = quat.copy(), quat.copy()
            q1[i, k] += h
            q2[i, k] -= h
            dU = (oracle.forces(m, pos, q1, comp, BOX)["U"] - oracle.forces(m, pos, q2, comp, BOX)["U"]) / (2 * h)
            assert dU == pytest.approx(rows["dquat"][i, k], abs=1e-6 * (1 + abs(dU)))


def test_newton_third_law_and_angular_momentum(oracle):
    """Sum of forces vanishes (each pair is evaluated from both ends independently); for an
    isolated cluster the total torque about the origin, sum(tau_i + r_i x F_i), vanishes."""
    c = W.make("mixture_small")
    r = oracle.forces(c["model"], c["pos"], c["quat"], c["comp"], c["box"])
    assert np.abs(r["F"].sum(0)).max() < 1e-12 * np.abs(r["F"]).sum()
    m, pos, quat, comp = _cluster(n=8, seed=2)
    r = oracle.forces(m, pos, quat, comp, BOX)
    L = r["T"].sum(0) + np.cross(pos, r["F"]).sum(0)
    assert np.abs(L).max() < 1e-11 * (np.abs(r["T"]).sum() + np.abs(np.cross(pos, r["F"])).sum())


def test_virial_is_box_scaling_derivative(oracle):
    """W = -dU/d(lambda) when every COM and the box are scaled by lambda at fixed orientations;
    W_aa likewise for scaling axis a only."""
    c = W.make("mixture_small")
    m, pos, quat, comp, box = c["model"], c["pos"], c["quat"], c["comp"], c["box"]
    r = oracle.forces(m, pos, quat, comp, box)
    h = 1e-6

    def U(s):
        return oracle.forces(m, pos * s, quat, comp, box * s)["U"]

    for ax in range(4):
        s1, s2 = np.ones(3), np.ones(3)
        if ax == 3:
            s1 += h
            s2 -= h
            ref = r["W"]
        else:
            s1[ax] += h
            s2[ax] -= h
            ref = r["Wd"][ax]
        assert oracle.forces(m, pos * s1, quat, comp, box * s1)["npairs"] == r["npairs"]
        assert -(U(s1) - U(s2)) / (2 * h) == pytest.approx(ref, rel=1e-6, abs=1e-6)
    assert r["Wd"].sum() == pytest.approx(r["W"], rel=1e-12)
    assert r["u"].sum() == pytest.approx(r["U"], rel=1e-12)


# ----------------------------------------------------------------------------- cells and counts

def test_pair_count_matches_library_kdtree(oracle):
    """Number of unordered pairs with periodic COM distance < r_c equals scipy's cKDTree count."""
    from scipy.spatial import cKDTree
    for cfg in [W.make("c1_ljts_4000"), W.random_gas(3000, [9.1, 11.7, 14.2], W.lj_model(2.5), seed=7)]:
        r = oracle.forces(cfg["model"], cfg["pos"], cfg["quat"], cfg["comp"], cfg["box"])
        pw = np.mod(cfg["pos"], cfg["box"])
        t = cKDTree(pw, boxsize=cfg["box"])
        assert r["npairs"] == len(t.query_pairs(cfg["model"]["rc"]))


def test_binning_invariants(oracle):
    """Wrapped positions lie in [0, L); every molecule's cell is the one whose slab contains it
    (to one rounding at faces); positions at -L, 0, L, 2L - tiny wrap as expected."""
    cfg = W.random_gas(5000, [9.1, 11.7, 14.2], W.lj_model(2.5), seed=8)
    pos = cfg["pos"] * 3.0 - 10.0  # far outside the box on both sides
    box = cfg["box"]
    cell, pw, ncell = oracle.bin_cells(pos, box, 2.5)
    nc = oracle.ncells(box, 2.5)
    assert ncell == nc[0] * nc[1] * nc[2] and nc == (3, 4, 5)
    assert (pw >= 0).all() and (pw < box).all()
    np.testing.assert_allclose(pw, np.mod(pos, box), atol=1e-12)
    cx, cy, cz = cell % nc[0], (cell // nc[0]) % nc[1], cell // (nc[0] * nc[1])
    h = box / np.array(nc)
    for k, ck in enumerate((cx, cy, cz)):
        assert (pw[:, k] >= ck * h[k] - 1e-12).all() and (pw[:, k] < (ck + 1) * h[k] + 1e-12).all()
    edge = np.array([[-box[0], 0.0, box[2]], [2 * box[0] - 1e-300, box[1] * (1 - 2 ** -53), -0.0]])
    cell, pw, _ = oracle.bin_cells(edge, box, 2.5)
    assert (pw >= 0).all() and (pw < box).all()
    assert cell[0] == 0


def test_cells_per_axis_rule(oracle):
    """floor(L / r_c) cells, with the edge kept strictly above r_c; fewer than three refused."""
    assert oracle.ncells([10.0, 10.0, 10.0], 2.5) == (3, 3, 3)
    assert oracle.ncells([10.01, 12.6, 100.0], 2.5) == (4, 5, 39)
    assert oracle.ncells([7.4, 10.0, 10.0], 2.5) is None


def test_half_cells_refine_cells(oracle):
    """Half-edge cells (Sec. 3, r_c/2 variant): every molecule's half-cell coordinates halved are
    its cell coordinates, and its wrapped coordinate lies in the half-cell's slab (to one rounding
    at faces); hand-worked values on a box of 3 cells of edge 10/3 per axis."""
    cfg = W.random_gas(5000, [9.1, 11.7, 14.2], W.lj_model(2.5), seed=18)
    box = np.asarray(cfg["box"])
    nc = np.array(oracle.ncells(box, 2.5))
    hh = box / (2 * nc)
    # random positions far outside the box, plus positions on every half-cell face and at 0, L
    faces = np.stack(np.meshgrid(*[np.arange(2 * n + 1) * h for n, h in zip(nc, hh)], indexing="ij"), -1)
    pos = np.concatenate([cfg["pos"] * 3.0 - 10.0, faces.reshape(-1, 3), faces.reshape(-1, 3) * (1 - 2 ** -52),
                          -faces.reshape(-1, 3)])
    cell, pw, _ = oracle.bin_cells(pos, box, 2.5)
    half = oracle.half_cells(pos, box, 2.5)
    coords = np.stack([cell % nc[0], (cell // nc[0]) % nc[1], cell // (nc[0] * nc[1])], -1)
    np.testing.assert_array_equal(half // 2, coords)
    assert (half >= 0).all() and (half < 2 * nc).all()
    assert (pw >= half * hh - 1e-12).all() and (pw < (half + 1) * hh + 1e-12).all()
    # 3 cells of edge 10/3 (edge 2.5 is refused: it must exceed r_c), half-cells of edge 5/3
    h = oracle.half_cells([[1.7, 5.0, 9.99], [1.6, 3.4, -0.1]], [10.0, 10.0, 10.0], 2.5)
    np.testing.assert_array_equal(h, [[1, 3, 5], [0, 2, 5]])


@pytest.mark.parametrize("seed,rho", [(21, 0.9), (22, 0.3)])
def test_half_cell_culling_keeps_every_pair(oracle, seed, rho):
    """The half-edge-cell culling rule: within the 27 cells around a home cell, a partner whose
    half-cell lies three half-cells away from the home molecule's along any axis (the far half
    of a neighbour cell) is more than one cell edge >= r_c away along that axis, so no pair inside
    the cutoff is ever culled.  Brute force over all pairs of dense and dilute fluids, with
    positions snapped onto half-cell faces."""
    rng = W.rng_for(seed)
    N = 1500
    box = np.array([1.0, 1.2, 1.45]) * (N / rho / 1.74) ** (1 / 3)
    nc = np.array(oracle.ncells(box, 2.5))
    hh = box / (2 * nc)
    pos = rng.uniform(0, 1, size=(N, 3)) * box
    snap = rng.uniform(size=(N, 3)) < 0.3  # a third of the coordinates exactly on a half-cell face
    pos = np.where(snap, np.round(pos / hh) * hh, pos)
    cell, pw, _ = oracle.bin_cells(pos, box, 2.5)
    half = oracle.half_cells(pos, box, 2.5).astype(np.int64)
    c = np.stack([cell % nc[0], (cell // nc[0]) % nc[1], cell // (nc[0] * nc[1])], -1).astype(np.int64)
    d = pw[:, None, :] - pw[None, :, :]
    d -= box * np.round(d / box)
    r2 = (d * d).sum(-1)
    i, j = np.nonzero((r2 < 2.5 ** 2 * (1 + 1e-9)) & ~np.eye(N, dtype=bool))
    assert len(i) > 5 * N * rho
    # image of j next to i: cell offset in {-1, 0, 1} per axis, half-cell offset of that image
    dc = (c[j] - c[i] + 1) % nc - 1
    assert (np.abs(dc) <= 1).all()
    ds = half[j] - half[i] + 2 * (dc - (c[j] - c[i]))
    assert (np.abs(ds) <= 2).all()
    # and the rule does cull: some pairs three half-cells apart exist, all outside the cutoff
    far = np.abs((half[:, None, :] - half[None, :, :] + 2 * ((c[None, :, :] - c[:, None, :] + 1) % nc - 1
                                                             - (c[None, :, :] - c[:, None, :]))))
    culled = (far == 3).any(-1)
    assert culled.sum() > 0 and (r2[culled] >= 2.5 ** 2).all()


# ----------------------------------------------------------------------------- integrator

def _energy_spread(en):
    E = en[:, 0] + en[:, 1] + en[:, 2]
    return np.abs(E - E[0]).max() / abs(E[0])


def test_leapfrog_nve_dt2_scaling(oracle):
    """Translational leapfrog (Sec. 3, Eqs. 2-3): total energy stays within a small band and the
    band shrinks ~4x when dt halves (second-order method)."""
    c = W.make("c1_ljts_4000")
    args = (c["model"], c["pos"], c["vel"], None, None, None, c["box"])
    *_, e1 = oracle.step(*args, 0.004, 50)
    *_, e2 = oracle.step(*args, 0.002, 100)
    s1, s2 = _energy_spread(e1), _energy_spread(e2)
    assert s2 < 2e-4
    assert 2.5 < s1 / s2 < 6.5


@pytest.mark.parametrize("kind", ["mixture", "2cljq"])
def test_rotational_leapfrog_nve(oracle, kind):
    """Rotational leapfrog with quaternions (Sec. 3, Eqs. 4-5) on an isolated cluster whose pairs
    all stay inside the cutoff (so U is smooth): U + K_trans + K_rot is conserved to second
    order in dt, for asymmetric tops and for linear molecules (I_z = 0)."""
    m, pos, quat, comp = _cluster(n=6, seed=4)
    if kind == "2cljq":
        m = W.twoclj_q_model(rc=6.0)
        comp = np.zeros(6, dtype=np.int32)
    else:
        m = dict(m, rc=6.0)
    rng = np.random.default_rng(11)
    masses = np.array([m["components"][c]["mass"] for c in comp])
    vel = W.maxwell_velocities(rng, masses, 1.0)
    angmom = np.zeros((6, 3))
    for i, c in enumerate(comp):
        angmom[i] = W.angular_momenta(rng, quat[i:i + 1], m["components"][c]["inertia"], 1.0)[0]
    spreads = []
    for dt, n in ((0.002, 25), (0.001, 50), (0.0005, 100)):
        _, _, q, _, en = oracle.step(m, pos, vel, quat, angmom, comp, BOX, dt, n)
        spreads.append(_energy_spread(en))
        assert np.all(en[:, 2] > 0)
        np.testing.assert_allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-14)
    assert spreads[2] < 1e-4
    assert 3.0 < spreads[0] / spreads[1] < 5.5 and 3.0 < spreads[1] / spreads[2] < 5.5


def test_free_rotor(oracle):
    """An isolated asymmetric top: angular momentum is constant (no torque) and K_rot stays
    constant to O(dt^2); quaternions stay unit."""
    m = W.four_site_model()
    box = np.array([13.0, 13.0, 13.0])
    pos = np.array([[6.0, 6.0, 6.0]])
    vel = np.zeros((1, 3))
    quat = np.array([quat_axis_angle([0.2, 0.9, -0.3], 0.7)])
    j = np.array([[0.31, -0.22, 0.4]])
    ks = []
    for dt, n in ((0.01, 400), (0.005, 800)):
        _, _, q, jj, en = oracle.step(m, pos, vel, quat, j, None, box, dt, n)
        np.testing.assert_array_equal(jj, j)
        assert abs(np.linalg.norm(q) - 1) < 1e-14
        ks.append(np.abs(en[:, 2] - en[0, 2]).max() / en[0, 2])
    assert ks[1] < 1e-4
    assert ks[0] / ks[1] > 3.0  # at least second order (observed ~8: third order for a free top)


# ----------------------------------------------------------------------------- NVT, cut-off corrections

def _quad_tail(eps, sig, rc, power_weight):
    """int_rc^inf r^2 u(r) dr (power_weight = 0) or int_rc^inf r^2 (-r u'(r)) dr (= 1), by
    adaptive quadrature of the LJ 12-6 potential written out here."""
    from scipy.integrate import quad
    u = lambda r: 4.0 * eps * ((sig / r) ** 12 - (sig / r) ** 6)
    mru = lambda r: 4.0 * eps * (12.0 * (sig / r) ** 12 - 6.0 * (sig / r) ** 6)  # -r u'(r)
    f = (lambda r: r * r * u(r)) if power_weight == 0 else (lambda r: r * r * mru(r))
    val, err = quad(f, rc, np.inf, epsabs=0.0, epsrel=1e-13, limit=200)
    return val


@pytest.mark.parametrize("case", ["lj", "mixture_xi_eta", "2clj"])
def test_long_range_correction_matches_quadrature(oracle, case):
    """Cut-off corrections (Sec. 3: mean-field integral of the dispersive tail) against adaptive
    quadrature of the pair integral 2 pi N_A N_B / V int_rc^inf r^2 u(r) dr per LJ site pair, with
    Lorentz-Berthelot mixing and binary factors; the textbook single-component value
    U/N = 8/3 pi rho eps sigma^3 [(sigma/rc)^9 / 3 - (sigma/rc)^3] is checked as well."""
    box = np.array([11.0, 12.0, 13.0])
    V = float(np.prod(box))
    rc = 3.0
    if case == "lj":
        m = dict(W.lj_model(rc, shift=False))
        counts = [1500]
    elif case == "mixture_xi_eta":
        m = W.mixture_model(rc=rc)
        m = dict(m, lj_shift=False, xi=[[1.0, 0.93], [0.93, 1.0]], eta=[[1.0, 1.07], [1.07, 1.0]])
        counts = [700, 900]
    else:
        m = dict(W.twoclj_q_model(rc=rc), lj_shift=False)
        counts = [1200]
    U, Wv = oracle.long_range_correction(m, counts, box)
    comps = m["components"]
    nc = len(comps)
    xi = np.ones((nc, nc)) if m.get("xi") is None else np.asarray(m["xi"])
    eta = np.ones((nc, nc)) if m.get("eta") is None else np.asarray(m["eta"])
    Uq = Wq = 0.0
    for A in range(nc):
        for B in range(nc):
            for sa in [s for s in comps[A]["sites"] if s["kind"] == "lj"]:
                for sb in [s for s in comps[B]["sites"] if s["kind"] == "lj"]:
                    eps = xi[A, B] * math.sqrt(sa["eps"] * sb["eps"])
                    sig = eta[A, B] * 0.5 * (sa["sigma"] + sb["sigma"])
                    pref = 2.0 * math.pi * counts[A] * counts[B] / V
                    Uq += pref * _quad_tail(eps, sig, rc, 0)
                    Wq += pref * _quad_tail(eps, sig, rc, 1)
    assert U == pytest.approx(Uq, rel=1e-11)
    assert Wv == pytest.approx(Wq, rel=1e-11)
    if case == "lj":
        rho = counts[0] / V
        x = 1.0 / rc
        assert U / counts[0] == pytest.approx(8.0 / 3.0 * math.pi * rho * (x ** 9 / 3.0 - x ** 3), rel=1e-13)
    assert oracle.long_range_correction(dict(m, lj_shift=True), counts, box) == (0.0, 0.0)


@pytest.mark.parametrize("kind", ["ljts", "2cljq", "mixture4"])
def test_velocity_rescaling_thermostat(oracle, kind):
    """NVT by velocity rescaling (Sec. 2): one step with the thermostat equals one step without it
    followed by v <- beta v, j <- beta j with beta = sqrt(T_target / T(t)), where the test forms
    T(t) = 2 K(t) / f itself (k_B = 1; f = 3N + 2 per linear molecule, the 2CLJQ has I_z = 0;
    the four-component mixture mixes asymmetric tops, a linear molecule and a non-rotating one)."""
    if kind == "ljts":
        c = W.random_gas(300, [9.0, 9.0, 9.0], W.lj_model(2.5), seed=5, dmin=0.9)
        m, pos, quat, comp, box = c["model"], c["pos"], None, None, c["box"]
        vel = W.maxwell_velocities(np.random.default_rng(3), np.ones(300), 1.3)
        angmom = None
        f = 3 * 300
    elif kind == "mixture4":
        c = W.make("mixture4_small")
        m, pos, quat, comp, box = c["model"], c["pos"], c["quat"], c["comp"], c["box"]
        vel, angmom = c["vel"], c["angmom"]
        f = 3 * len(pos) + sum(int(np.sum(np.asarray(m["components"][k]["inertia"]) > 0)) for k in comp)
    else:
        m = W.twoclj_q_model(rc=4.0)
        c = W.random_gas(120, [12.5, 12.5, 12.5], m, seed=6, dmin=1.3)
        pos, box = c["pos"], c["box"]
        rng = np.random.default_rng(8)
        quat = W.random_quaternions(rng, 120)
        comp = np.zeros(120, dtype=np.int32)
        vel = W.maxwell_velocities(rng, np.full(120, m["components"][0]["mass"]), 1.3)
        angmom = W.angular_momenta(rng, quat, m["components"][0]["inertia"], 1.3)
        f = 3 * 120 + 2 * 120
    T_target = 0.8
    _, v0, _, j0, e0 = oracle.step(m, pos, vel, quat, angmom, comp, box, 0.002, 1)
    p1, v1, q1, j1, e1 = oracle.step(m, pos, vel, quat, angmom, comp, box, 0.002, 1, T_target=T_target)
    np.testing.assert_array_equal(e0, e1)  # the energies row keeps K(t) before the rescaling
    K = e0[0, 1] + e0[0, 2]
    beta = math.sqrt(T_target / (2.0 * K / f))
    np.testing.assert_allclose(v1, beta * v0, rtol=1e-14, atol=0)
    if angmom is not None:
        rot = np.ones(len(j0), dtype=bool) if comp is None else np.array(
            [np.any(np.asarray(m["components"][k]["inertia"]) > 0) for k in comp])
        np.testing.assert_allclose(j1[rot], beta * j0[rot], rtol=1e-14, atol=0)
        np.testing.assert_array_equal(j1[~rot], j0[~rot])  # molecules without inertia keep j
