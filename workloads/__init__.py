"""Seeded synthetic problem descriptions shared by the oracle and the HIP path.

This module only *describes* problems: grid sizes, boundary-condition codes,
material tables, per-voxel material ids and load steps.  It holds none of the
solver's arithmetic (no transforms, stencils, Green operators or laws), so the
oracle and the product path can both consume it without sharing any of the
method's code.  Every random draw comes from ``numpy.random.default_rng(seed)``.

Conventions
-----------
* Axes: x (paper e1), y (e2), z (e3).  Voxel-centred arrays are shaped
  ``(n3, n2, n1)`` in C order, i.e. x is the fastest-varying index.
* Boundary conditions: ``bc[q][i][a]`` for displacement component q, axis i and
  face a (0 = face through the origin, 1 = opposite face), with codes
  ``P=0`` (periodic), ``D=1`` (Dirichlet), ``N=2`` (Neumann), the per-face,
  per-component choice of the mechanical problem statement (Sec. 2.2).
* Prescribed displacement u* is a quadratic polynomial of the node position
  ``x = (j1 h, j2 h, j3 h)``::

      u*_q(x) = c[q] + sum_l G[q][l] x_l + 1/2 sum_lm H[q][l][m] x_l x_m

  which covers the affine, bending and torsion loadings used here.
* Voigt order for symmetric tensors: xx, yy, zz, yz, xz, xy (tensor shears,
  not engineering shears).
* Stresses in GPa for the polycrystal / J2 / crystal-plasticity workloads.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

P, D, N = 0, 1, 2
HEX1, TETRA2 = 0, 1
GREEN_B0, GREEN_2MU0, GREEN_C0 = 0, 1, 2
FP64, FP32_MIXED = 0, 1

LAW_ISO, LAW_ANISO, LAW_J2, LAW_CP, LAW_SVK, LAW_NEOHOOKE = 0, 1, 2, 3, 4, 5


# --------------------------------------------------------------------------
# Material table entries
# --------------------------------------------------------------------------
def iso_from_E_nu(E: float, nu: float) -> tuple:
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def mat_iso(lam: float, mu: float) -> dict:
    """Isotropic linear elasticity, sigma = 2 mu eps + lam tr(eps) 1."""
    return {"law": LAW_ISO, "lam": float(lam), "mu": float(mu)}


def mat_cubic(C11: float, C12: float, C44: float, quat: Sequence[float]) -> dict:
    """Cubic anisotropic elasticity with crystal axes rotated by ``quat``
    (unit quaternion w, x, y, z mapping crystal to sample frame)."""
    return {"law": LAW_ANISO, "C11": float(C11), "C12": float(C12),
            "C44": float(C44), "quat": [float(v) for v in quat]}


def mat_j2(lam: float, mu: float, sy0: float, H: float) -> dict:
    """Small-strain J2 plasticity, linear isotropic hardening sy = sy0 + H p."""
    return {"law": LAW_J2, "lam": float(lam), "mu": float(mu),
            "sy0": float(sy0), "H": float(H)}


def mat_cp(C11, C12, C44, quat, gdot0, nexp, tau0, taus, theta0) -> dict:
    """Small-strain FCC crystal viscoplasticity: 12 {111}<110> systems,
    power-law rate, Voce isotropic hardening of the common CRSS."""
    return {"law": LAW_CP, "C11": float(C11), "C12": float(C12), "C44": float(C44),
            "quat": [float(v) for v in quat], "gdot0": float(gdot0),
            "n": float(nexp), "tau0": float(tau0), "taus": float(taus),
            "theta0": float(theta0)}


def mat_svk(lam: float, mu: float) -> dict:
    """Finite-strain Saint Venant-Kirchhoff, Pi = lam tr(E) 1 + 2 mu E."""
    return {"law": LAW_SVK, "lam": float(lam), "mu": float(mu)}


def mat_neohooke(mu: float, K: float) -> dict:
    """Finite-strain compressible Neo-Hookean, psi = mu/2 (I1bar - 3) + K/2 (J - 1)^2."""
    return {"law": LAW_NEOHOOKE, "mu": float(mu), "K": float(K)}


# --------------------------------------------------------------------------
# Load steps
# --------------------------------------------------------------------------
@dataclasses.dataclass
class LoadStep:
    c: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))
    G: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((3, 3)))
    H: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((3, 3, 3)))
    # mixed macroscopic control: mask over the 6 Voigt components; where set,
    # the symmetric part of G on that component is adjusted so <sigma> = target
    mixed_mask: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(6, dtype=np.int32))
    mixed_target: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(6))
    dt: float = 1.0
    # applied traction T*[axis i][face a][component q], uniform over the face
    # S_{i a}; non-zero only where u_q is Neumann on that face
    traction: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((3, 2, 3)))
    # optional nodal field added to the polynomial u*: (3, N1, N2, N3), index
    # [q, i, j, k] at node (i h, j h, k h)
    ustar_nodal: Optional[np.ndarray] = None

    def copy(self) -> "LoadStep":
        return LoadStep(self.c.copy(), self.G.copy(), self.H.copy(),
                        self.mixed_mask.copy(), self.mixed_target.copy(), self.dt,
                        self.traction.copy(),
                        None if self.ustar_nodal is None else self.ustar_nodal.copy())


def step_affine(G) -> LoadStep:
    return LoadStep(G=np.array(G, dtype=np.float64))


def step_bending_torsion(kappa: float, twist: float, zc: float, yc: float) -> LoadStep:
    """u* = (k x (z - zc), -t x (z - zc), t x (y - yc) - k x^2 / 2)."""
    s = LoadStep()
    s.G[0, 0] = -kappa * zc
    s.H[0, 0, 2] = s.H[0, 2, 0] = kappa
    s.G[1, 0] = twist * zc
    s.H[1, 0, 2] = s.H[1, 2, 0] = -twist
    s.G[2, 0] = -twist * yc
    s.H[2, 0, 1] = s.H[2, 1, 0] = twist
    s.H[2, 0, 0] = -kappa
    return s


# --------------------------------------------------------------------------
# Problem description
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    n: tuple
    h: float
    bc: np.ndarray                 # int32 [3][3][2]
    scheme: int
    green: int
    lambda0: float
    mu0: float
    materials: List[dict]
    mat_id: np.ndarray             # int32 (n3, n2, n1)
    steps: List[LoadStep]
    tol: float = 1e-8
    max_iter: int = 2000
    aa_depth: int = 4
    aa_period: int = 3
    prec: int = FP64
    name: str = ""
    finite_strain: int = 0       # 1: Lagrangian finite-strain formulation (P = F Pi)

    @property
    def n_vox(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])


def bc_uniform_axes(types_per_axis) -> np.ndarray:
    """Same per-axis BC code on both faces and for all three components."""
    bc = np.zeros((3, 3, 2), dtype=np.int32)
    for i, t in enumerate(types_per_axis):
        bc[:, i, :] = t
    return bc


def random_quats(rng, k: int) -> np.ndarray:
    """Uniform random rotations: normalised 4-D standard normal samples."""
    q = rng.standard_normal((k, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def voxel_centres(n, h=1.0):
    n1, n2, n3 = n
    z, y, x = np.meshgrid((np.arange(n3) + 0.5) * h, (np.arange(n2) + 0.5) * h,
                          (np.arange(n1) + 0.5) * h, indexing="ij")
    return x, y, z


def spheres_to_ids(n, centres, radii, periodic=(False, False, False), h=1.0) -> np.ndarray:
    """Voxel belongs to an inclusion iff its centre lies within a sphere
    (minimum-image distance along periodic axes).  Returns 0/1 ids."""
    n1, n2, n3 = n
    L = np.array([n1, n2, n3], dtype=np.float64) * h
    ids = np.zeros((n3, n2, n1), dtype=np.int32)
    gx = (np.arange(n1) + 0.5) * h
    gy = (np.arange(n2) + 0.5) * h
    gz = (np.arange(n3) + 0.5) * h
    for c, r in zip(centres, radii):
        d = []
        for ax, g in enumerate((gx, gy, gz)):
            dd = g - c[ax]
            if periodic[ax]:
                dd = dd - L[ax] * np.round(dd / L[ax])
            d.append(dd)
        r2 = (d[2][:, None, None] ** 2 + d[1][None, :, None] ** 2 + d[0][None, None, :] ** 2)
        ids[r2 <= r * r] = 1
    return ids


def voronoi_ids(n, seeds, periodic=(False, False, False), h=1.0) -> np.ndarray:
    """Nearest seed to each voxel centre (Euclidean; periodic images along
    periodic axes).  Exact ties have probability zero for continuous seeds."""
    from scipy.spatial import cKDTree
    n1, n2, n3 = n
    L = np.array([n1, n2, n3], dtype=np.float64) * h
    pts = [seeds]
    idx = [np.arange(len(seeds))]
    shifts = [(-1, 0, 1) if periodic[a] else (0,) for a in range(3)]
    for sx in shifts[0]:
        for sy in shifts[1]:
            for sz in shifts[2]:
                if sx == sy == sz == 0:
                    continue
                pts.append(seeds + L * np.array([sx, sy, sz]))
                idx.append(np.arange(len(seeds)))
    tree = cKDTree(np.concatenate(pts))
    allidx = np.concatenate(idx)
    out = np.empty((n3, n2, n1), dtype=np.int32)
    gx = (np.arange(n1) + 0.5) * h
    gy = (np.arange(n2) + 0.5) * h
    X, Y = np.meshgrid(gx, gy, indexing="xy")   # (n2, n1)
    for k in range(n3):
        q = np.stack([X.ravel(), Y.ravel(), np.full(X.size, (k + 0.5) * h)], axis=1)
        _, j = tree.query(q)
        out[k] = allidx[j].reshape(n2, n1)
    return out


# --------------------------------------------------------------------------
# The five workload families
# --------------------------------------------------------------------------
def config_inclusion32(prec=FP64) -> Problem:
    """32^3 two-phase isotropic elasticity, centred sphere R=8 (E 1 / 10,
    nu 0.3), eps_zz = 1e-3 through Dirichlet z faces (all components),
    Neumann x faces, periodic y; HEX1, B0 with the mean phase moduli."""
    n = (32, 32, 32)
    ids = spheres_to_ids(n, [(16.0, 16.0, 16.0)], [8.0])
    m0 = iso_from_E_nu(1.0, 0.3)
    m1 = iso_from_E_nu(10.0, 0.3)
    bc = np.zeros((3, 3, 2), dtype=np.int32)
    bc[:, 0, :] = N
    bc[:, 1, :] = P
    bc[:, 2, :] = D
    G = np.zeros((3, 3)); G[2, 2] = 1e-3
    return Problem(n=n, h=1.0, bc=bc, scheme=HEX1, green=GREEN_B0,
                   lambda0=0.5 * (m0[0] + m1[0]), mu0=0.5 * (m0[1] + m1[1]),
                   materials=[mat_iso(*m0), mat_iso(*m1)], mat_id=ids,
                   steps=[step_affine(G)], tol=1e-8, max_iter=3000, prec=prec,
                   name="inclusion32")


def cubic_reference(C11, C12, C44):
    """Reference medium for cubic phases: lambda0 = C12, mu0 = max(C44, (C11-C12)/2)."""
    return C12, max(C44, 0.5 * (C11 - C12))


def config_polycrystal_bending(nv=256, n_grains=500, seed=2, prec=FP64, kappa=1e-4,
                               tol=1e-6, scheme=TETRA2) -> Problem:
    """Voronoi polycrystal, cubic elasticity (168/121/75 GPa), random
    orientations; bending through Dirichlet x faces (u* = (k x (z-zc), 0,
    -k x^2/2)), Neumann y and z faces; TETRA2, B0 with lambda0 = 121, mu0 = 75."""
    rng = np.random.default_rng(seed)
    n = (nv, nv, nv)
    seeds = rng.uniform(0.0, float(nv), size=(n_grains, 3))
    quats = random_quats(rng, n_grains)
    ids = voronoi_ids(n, seeds)
    mats = [mat_cubic(168.0, 121.0, 75.0, q) for q in quats]
    bc = np.zeros((3, 3, 2), dtype=np.int32)
    bc[:, 0, :] = D
    bc[:, 1, :] = N
    bc[:, 2, :] = N
    step = step_bending_torsion(kappa / 1.0, 0.0, zc=0.5 * nv, yc=0.5 * nv)
    lam0, mu0 = cubic_reference(168.0, 121.0, 75.0)
    return Problem(n=n, h=1.0, bc=bc, scheme=scheme, green=GREEN_B0, lambda0=lam0,
                   mu0=mu0, materials=mats, mat_id=ids, steps=[step], tol=tol,
                   max_iter=3000, prec=prec, name=f"polycrystal{nv}")


def rsa_spheres(rng, n, rmin, rmax, phi, periodic=(True, True, False)):
    """Random sequential addition of non-overlapping spheres (radius ~ U[rmin,
    rmax]); centres keep the sphere inside along non-periodic axes; stop at the
    first sphere that brings the voxel volume fraction to >= phi."""
    L = np.array(n, dtype=np.float64)
    cs, rs = [], []
    ids = np.zeros((n[2], n[1], n[0]), dtype=np.int32)
    tries = 0
    while True:
        tries += 1
        if tries > 200000:
            raise RuntimeError("RSA did not reach the target volume fraction")
        r = rng.uniform(rmin, rmax)
        c = np.empty(3)
        for a in range(3):
            c[a] = rng.uniform(0.0, L[a]) if periodic[a] else rng.uniform(r, L[a] - r)
        ok = True
        for c2, r2 in zip(cs, rs):
            d = c - c2
            for a in range(3):
                if periodic[a]:
                    d[a] -= L[a] * np.round(d[a] / L[a])
            if np.dot(d, d) < (r + r2) ** 2:
                ok = False
                break
        if not ok:
            continue
        cs.append(c); rs.append(r)
        ids |= spheres_to_ids(n, [c], [r], periodic=periodic)
        if ids.mean() >= phi:
            return ids, cs, rs


def config_j2_inclusions(nv=256, seed=3, prec=FP32_MIXED, n_steps=20, eps_final=2e-2,
                         tol=1e-6, phi=0.20, rmin=6.0, rmax=12.0) -> Problem:
    """Elastic spheres (E 400 GPa, nu 0.2) in a J2 matrix (E 70 GPa, nu 0.33,
    sy0 0.1 GPa, H 1 GPa); u_z Dirichlet / u_x,u_y Neumann on the z faces,
    periodic x and y; eps_zz ramps to ``eps_final`` with <sigma_xx> =
    <sigma_yy> = 0; HEX1, B0 with the maximum phase moduli."""
    rng = np.random.default_rng(seed)
    n = (nv, nv, nv)
    ids, _, _ = rsa_spheres(rng, n, rmin, rmax, phi)
    incl = iso_from_E_nu(400.0, 0.2)
    matx = iso_from_E_nu(70.0, 0.33)
    mats = [mat_j2(matx[0], matx[1], 0.1, 1.0), mat_iso(*incl)]
    bc = np.zeros((3, 3, 2), dtype=np.int32)
    bc[:, 0, :] = P
    bc[:, 1, :] = P
    bc[0, 2, :] = N
    bc[1, 2, :] = N
    bc[2, 2, :] = D
    steps = []
    for t in range(1, n_steps + 1):
        s = LoadStep()
        s.G[2, 2] = eps_final * t / n_steps
        s.mixed_mask = np.array([1, 1, 0, 0, 0, 0], dtype=np.int32)
        s.mixed_target = np.zeros(6)
        steps.append(s)
    return Problem(n=n, h=1.0, bc=bc, scheme=HEX1, green=GREEN_B0,
                   lambda0=max(incl[0], matx[0]), mu0=max(incl[1], matx[1]),
                   materials=mats, mat_id=ids, steps=steps, tol=tol, max_iter=3000,
                   prec=prec, name=f"j2_inclusions{nv}")


def random_rve(rng, nv, prec=FP32_MIXED, tol=1e-6) -> Problem:
    """One draw of the batched elastic family: 8-32 spheres of radius
    U[n/16, n/8] (union), stiffness contrast log-uniform in [2, 100], nu 0.3,
    macroscopic strain entries U[-1e-3, 1e-3] (symmetric), per-axis BC type
    uniform over P/D/N for all components and both faces (the all-Neumann draw
    is resampled); HEX1, B0 with the maximum phase moduli."""
    n = (nv, nv, nv)
    while True:
        types = rng.integers(0, 3, size=3)
        if not np.all(types == N):
            break
    k = int(rng.integers(8, 33))
    cs = rng.uniform(0.0, float(nv), size=(k, 3))
    rs = rng.uniform(nv / 16.0, nv / 8.0, size=k)
    periodic = tuple(bool(t == P) for t in types)
    ids = spheres_to_ids(n, cs, rs, periodic=periodic)
    contrast = math.exp(rng.uniform(math.log(2.0), math.log(100.0)))
    m0 = iso_from_E_nu(1.0, 0.3)
    m1 = iso_from_E_nu(contrast, 0.3)
    E = rng.uniform(-1e-3, 1e-3, size=(3, 3))
    E = 0.5 * (E + E.T)
    bc = bc_uniform_axes(types)
    return Problem(n=n, h=1.0, bc=bc, scheme=HEX1, green=GREEN_B0,
                   lambda0=max(m0[0], m1[0]), mu0=max(m0[1], m1[1]),
                   materials=[mat_iso(*m0), mat_iso(*m1)], mat_id=ids,
                   steps=[step_affine(E)], tol=tol, max_iter=3000, prec=prec,
                   name=f"rve{nv}")


def config_batch(count=512, sizes=(32, 48, 64, 96), seed=4, prec=FP32_MIXED, tol=1e-6):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        nv = int(sizes[int(rng.integers(0, len(sizes)))])
        out.append(random_rve(rng, nv, prec=prec, tol=tol))
    return out


CP_PARAMS = dict(gdot0=1e-3, nexp=20.0, tau0=0.050, taus=0.150, theta0=0.300)


def cp_polycrystal(rng, nv, n_grains, prec=FP32_MIXED, n_steps=10, eps_max=5e-3,
                   tol=1e-6, scheme=TETRA2) -> Problem:
    """FCC crystal plasticity polycrystal under torsion-bending: Dirichlet on
    all components of the x faces, Neumann on y and z faces; amplitudes
    kappa = twist = 2 eps_max / n at the last increment (dt = 1 s)."""
    n = (nv, nv, nv)
    seeds = rng.uniform(0.0, float(nv), size=(n_grains, 3))
    quats = random_quats(rng, n_grains)
    ids = voronoi_ids(n, seeds)
    mats = [mat_cp(168.0, 121.0, 75.0, q, CP_PARAMS["gdot0"], CP_PARAMS["nexp"],
                   CP_PARAMS["tau0"], CP_PARAMS["taus"], CP_PARAMS["theta0"])
            for q in quats]
    bc = np.zeros((3, 3, 2), dtype=np.int32)
    bc[:, 0, :] = D
    bc[:, 1, :] = N
    bc[:, 2, :] = N
    amp = 2.0 * eps_max / nv
    steps = []
    for t in range(1, n_steps + 1):
        s = step_bending_torsion(amp * t / n_steps, amp * t / n_steps,
                                 zc=0.5 * nv, yc=0.5 * nv)
        s.dt = 1.0
        steps.append(s)
    lam0, mu0 = cubic_reference(168.0, 121.0, 75.0)
    return Problem(n=n, h=1.0, bc=bc, scheme=scheme, green=GREEN_B0, lambda0=lam0,
                   mu0=mu0, materials=mats, mat_id=ids, steps=steps, tol=tol,
                   max_iter=3000, prec=prec, name=f"cp{nv}")


def cantilever(n=(100, 10, 10), h=1.0, t2=1e-3, scheme=HEX1, n_steps=1, prec=FP64, tol=1e-8) -> Problem:
    """Elastic cantilever (lambda 120, mu 80 GPa) clamped on the face x = 0
    (every component Dirichlet, u* = 0) and loaded on the top face y = n_y h
    by a uniform traction -t2 e_y; every other face is traction-free.  The
    increments scale the load linearly up to t2."""
    bc = np.full((3, 3, 2), N, dtype=np.int32)
    bc[:, 0, 0] = D
    steps = []
    for k in range(1, n_steps + 1):
        s = LoadStep()
        s.traction[1, 1, 1] = -t2 * k / n_steps
        steps.append(s)
    lam, mu = 120.0, 80.0
    return Problem(n=tuple(n), h=h, bc=bc, scheme=scheme, green=GREEN_B0, lambda0=lam, mu0=mu,
                   materials=[mat_iso(lam, mu)], mat_id=np.zeros((n[2], n[1], n[0]), dtype=np.int32),
                   steps=steps, tol=tol, max_iter=20000, prec=prec, name="cantilever")


@dataclasses.dataclass
class Request:
    arrival_s: float
    problem: Problem


def serving_stream(count=500, rate=200.0, sizes=(32, 64, 96, 128, 160, 192), seed=5,
                   prec=FP32_MIXED, grains=(8, 64), n_steps=10):
    """Poisson arrivals (exponential gaps, mean 1/rate) of crystal-plasticity
    torsion-bending solves with uniform grid size and grain count."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += rng.exponential(1.0 / rate)
        nv = int(sizes[int(rng.integers(0, len(sizes)))])
        g = int(rng.integers(grains[0], grains[1] + 1))
        out.append(Request(t, cp_polycrystal(rng, nv, g, prec=prec, n_steps=n_steps)))
    return out


# extension pairs of the normal component along an axis under the C0
# operator's normal-mixed conditions (Eq. SGO_BCs); the tangential components
# take the opposite pair
NORMAL_MIXED_PAIRS = [(P, P), (N, N), (D, D), (N, D), (D, N)]


def normal_mixed_bc(choice) -> np.ndarray:
    """bc[q][i][a] from one pair per axis for the normal component (indices
    into NORMAL_MIXED_PAIRS); tangential components get the opposite condition
    (Dirichlet <-> Neumann), periodic axes stay periodic for all."""
    opp = {P: P, N: D, D: N}
    bc = np.zeros((3, 3, 2), dtype=np.int32)
    for i in range(3):
        l, r = NORMAL_MIXED_PAIRS[int(choice[i])]
        for q in range(3):
            bc[q, i, 0] = l if q == i else opp[l]
            bc[q, i, 1] = r if q == i else opp[r]
    return bc


def random_small_problem(rng, n=(6, 5, 7), scheme=HEX1, law="iso", green=GREEN_B0,
                         bc=None, prec=FP64, tol=1e-10, n_steps=1) -> Problem:
    """Small random two-phase problem for parity tests: random per-face,
    per-component BCs (periodic faces paired), random quadratic load."""
    if bc is None:
        bc = np.zeros((3, 3, 2), dtype=np.int32)
        for q in range(3):
            for i in range(3):
                if rng.random() < 0.3:
                    bc[q, i, :] = P
                else:
                    bc[q, i, 0] = rng.integers(1, 3)
                    bc[q, i, 1] = rng.integers(1, 3)
        # keep at least one Dirichlet face somewhere so the load does something
    ids = (rng.random((n[2], n[1], n[0])) < 0.35).astype(np.int32)
    m0 = iso_from_E_nu(1.0, 0.3)
    m1 = iso_from_E_nu(float(rng.uniform(2.0, 8.0)), 0.25)
    if law == "iso":
        mats = [mat_iso(*m0), mat_iso(*m1)]
        lam0, mu0 = max(m0[0], m1[0]), max(m0[1], m1[1])
    elif law == "cubic":
        qs = random_quats(rng, 2)
        mats = [mat_cubic(1.68, 1.21, 0.75, qs[0]), mat_cubic(1.68, 1.21, 0.75, qs[1])]
        lam0, mu0 = cubic_reference(1.68, 1.21, 0.75)
    elif law == "j2":
        mats = [mat_j2(m0[0], m0[1], 1.5e-3, 0.05), mat_iso(*m1)]
        lam0, mu0 = max(m0[0], m1[0]), max(m0[1], m1[1])
    elif law == "cp":
        qs = random_quats(rng, 2)
        mats = [mat_cp(168.0, 121.0, 75.0, qs[k], **{"gdot0": 1e-3, "nexp": 20.0,
                       "tau0": 0.05, "taus": 0.15, "theta0": 0.3}) for k in range(2)]
        lam0, mu0 = cubic_reference(168.0, 121.0, 75.0)
    else:
        raise ValueError(law)
    steps = []
    G0 = rng.uniform(-1e-3, 1e-3, size=(3, 3))
    H0 = rng.uniform(-1e-4, 1e-4, size=(3, 3, 3))
    H0 = 0.5 * (H0 + H0.transpose(0, 2, 1))
    scale = 1.0 if law != "cp" else 2.0
    for t in range(1, n_steps + 1):
        s = LoadStep(c=np.zeros(3), G=scale * G0 * t, H=scale * H0 * t)
        steps.append(s)
    return Problem(n=tuple(n), h=1.0, bc=bc, scheme=scheme, green=green, lambda0=lam0,
                   mu0=mu0, materials=mats, mat_id=ids, steps=steps, tol=tol,
                   max_iter=5000, prec=prec, name="small")
