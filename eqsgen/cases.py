"""Workload recipes: meshes, materials, Dirichlet data and drives (input data only).

Every workload is the unit cube meshed by the Kuhn split (see ``mesh.py``),
grounded at z = 0 and driven by phi = A sin(2 pi f t + phase) at z = 1, with
natural (zero normal current) conditions on the four side faces. Materials
follow the paper's microvaristor field-grading setting (Sec. I and Sec. V):
a linear polymer host and embedded varistor material whose conductivity
grows as a power of the field strength,
    kappa(|E|) = kappa0 * (1 + (|E| / e_s) ** alpha).
An element takes the material whose region contains its centroid.

Recipes (sizes are n sub-cubes per edge):
  c0  n = 8,   host eps_r = 4, kappa = 1e-12; slab 0.4 < z < 0.6 with
               eps_r = 12, kappa0 = 1e-10, e_s = 0.5, alpha = 10.
               RKC s = 8, 200 steps, tau = 1e-4 s, PCG rel-res 1e-10, FP64.
  c1  n = 64,  host as c0 (no slab); seeded spherical inclusions of radius
               U[0.03, 0.08] up to 5 % of the volume, per sphere
               alpha ~ U[8, 14], eps_r ~ U[8, 15].
               RKC s = 12, 500 steps, PCG rel-res 1e-8, FP64.
  c2  n = 128, same inclusion layout as c1 (same seed), RKC s = 16,
               200 steps, FP32 AMG under FP64 CG, rel-res 1e-8.
  c3  64 independent instances, n ~ U{16, 24, 32, 40, 48}, inclusions with
               eps_r ~ U[2, 15], alpha ~ U[6, 14], drive amplitude ~ U[0.5, 2] V
               and frequency ~ U[25, 100] Hz; seed 3000 + i. s = 8, 200 steps.
  c4  = c2 with a learned start vector.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .mesh import kuhn_cube_mesh, kuhn_cube_mesh_p2

CASE_NAMES = ("c0", "c1", "c2", "c3", "c4", "p2")

HOST = dict(eps_r=4.0, kappa0=1e-12, e_s=1.0, alpha=0.0, nonlinear=0)
VARISTOR_KAPPA0 = 1e-10
VARISTOR_ES = 0.5


@dataclass
class Case:
    name: str
    n: int
    xyz: np.ndarray  # [N, 3] float64
    tets: np.ndarray  # [T, 4] int32
    tet_mat: np.ndarray  # [T] int32
    eps_r: np.ndarray  # [n_mat] float64
    kappa0: np.ndarray  # [n_mat] float64
    e_s: np.ndarray  # [n_mat] float64
    alpha: np.ndarray  # [n_mat] float64
    nonlinear: np.ndarray  # [n_mat] int32
    dir_nodes: np.ndarray  # [n_d] int32
    dir_drive: np.ndarray  # [n_d] int32
    amp: np.ndarray  # [n_drive] float64
    freq: np.ndarray  # [n_drive] float64
    phase: np.ndarray  # [n_drive] float64
    s: int = 8
    steps: int = 200
    tau: float = 1e-4
    rtol: float = 1e-10
    precision: str = "fp64"
    seed: Optional[int] = None
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])

    @property
    def n_mat(self) -> int:
        return int(self.eps_r.shape[0])

    def x0(self) -> np.ndarray:
        """Initial potential phi(0) = 0 on every node."""
        return np.zeros(self.n_nodes, dtype=np.float64)


def _centroids(xyz, tets):
    return xyz[tets[:, :4]].mean(axis=1)  # the vertices (10-node tets list them first)


def _dirichlet_top_bottom(xyz, amp=1.0, freq=50.0, phase=0.0):
    z = xyz[:, 2]
    bottom = np.flatnonzero(z == 0.0)
    top = np.flatnonzero(z == 1.0)
    nodes = np.concatenate([bottom, top]).astype(np.int32)
    drive = np.concatenate([np.zeros(bottom.size, np.int32), np.ones(top.size, np.int32)])
    order = np.argsort(nodes, kind="stable")
    return (
        nodes[order],
        drive[order],
        np.array([0.0, amp]),
        np.array([0.0, freq]),
        np.array([0.0, phase]),
    )


def _material_table(rows):
    return (
        np.array([r["eps_r"] for r in rows], dtype=np.float64),
        np.array([r["kappa0"] for r in rows], dtype=np.float64),
        np.array([r["e_s"] for r in rows], dtype=np.float64),
        np.array([r["alpha"] for r in rows], dtype=np.float64),
        np.array([r["nonlinear"] for r in rows], dtype=np.int32),
    )


def draw_spheres(seed: int, eps_range, alpha_range, vol_frac=0.05, r_range=(0.03, 0.08), max_tries=100000):
    """Non-overlapping spheres inside the unit cube up to a total volume fraction."""
    rng = np.random.default_rng(seed)
    spheres = []  # (cx, cy, cz, r, eps_r, alpha)
    vol = 0.0
    tries = 0
    while vol < vol_frac:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place inclusions")
        r = rng.uniform(*r_range)
        c = rng.uniform(r, 1.0 - r, size=3)
        ok = all(np.linalg.norm(c - np.array(s[:3])) >= r + s[3] for s in spheres)
        if not ok:
            continue
        eps_r = rng.uniform(*eps_range)
        alpha = rng.uniform(*alpha_range)
        spheres.append((c[0], c[1], c[2], r, eps_r, alpha))
        vol += 4.0 / 3.0 * np.pi * r ** 3
    return spheres


def _assign_spheres(cent, spheres):
    """Material id per element: 0 = host, 1 + k = first sphere k containing the centroid."""
    mat = np.zeros(cent.shape[0], dtype=np.int32)
    order = np.argsort(cent[:, 2], kind="stable")
    zs = cent[order, 2]
    for k in range(len(spheres) - 1, -1, -1):  # reverse, so the lowest index wins
        cx, cy, cz, r = spheres[k][:4]
        lo = np.searchsorted(zs, cz - r, side="left")
        hi = np.searchsorted(zs, cz + r, side="right")
        cand = order[lo:hi]
        d2 = ((cent[cand] - np.array([cx, cy, cz])) ** 2).sum(axis=1)
        mat[cand[d2 < r * r]] = k + 1
    return mat


def case_c0(n: int = 8) -> Case:
    xyz, tets = kuhn_cube_mesh(n)
    cz = _centroids(xyz, tets)[:, 2]
    tet_mat = ((cz > 0.4) & (cz < 0.6)).astype(np.int32)
    slab = dict(eps_r=12.0, kappa0=VARISTOR_KAPPA0, e_s=VARISTOR_ES, alpha=10.0, nonlinear=1)
    eps, k0, es, al, nl = _material_table([HOST, slab])
    dn, dd, amp, freq, ph = _dirichlet_top_bottom(xyz)
    return Case("c0", n, xyz, tets, tet_mat, eps, k0, es, al, nl, dn, dd, amp, freq, ph,
                s=8, steps=200, tau=1e-4, rtol=1e-10, precision="fp64")


def _inclusion_case(name, n, seed, eps_range, alpha_range, amp=1.0, freq=50.0, order=1) -> Case:
    xyz, tets = kuhn_cube_mesh(n) if order == 1 else kuhn_cube_mesh_p2(n)
    spheres = draw_spheres(seed, eps_range, alpha_range)
    tet_mat = _assign_spheres(_centroids(xyz, tets), spheres)
    rows = [HOST] + [
        dict(eps_r=s[4], kappa0=VARISTOR_KAPPA0, e_s=VARISTOR_ES, alpha=s[5], nonlinear=1) for s in spheres
    ]
    eps, k0, es, al, nl = _material_table(rows)
    dn, dd, a, f, ph = _dirichlet_top_bottom(xyz, amp=amp, freq=freq)
    c = Case(name, n, xyz, tets, tet_mat, eps, k0, es, al, nl, dn, dd, a, f, ph, seed=seed)
    c.meta["spheres"] = spheres
    c.meta["tet_fraction_in_inclusions"] = float((tet_mat > 0).mean())
    return c


def case_c1(n: int = 64, seed: int = 1) -> Case:
    c = _inclusion_case("c1", n, seed, (8.0, 15.0), (8.0, 14.0))
    c.s, c.steps, c.tau, c.rtol, c.precision = 12, 500, 1e-4, 1e-8, "fp64"
    return c


def case_c2(n: int = 128, seed: int = 1) -> Case:
    c = _inclusion_case("c2", n, seed, (8.0, 15.0), (8.0, 14.0))
    c.s, c.steps, c.tau, c.rtol, c.precision = 16, 200, 1e-4, 1e-8, "fp32"
    return c


def case_p2(n: int = 64, seed: int = 1) -> Case:
    """Second-order (10-node) tets on the n^3 Kuhn mesh: (2n+1)^3 nodes, the
    inclusion layout of c1/c2 (same seed), RKC s = 16, FP32 AMG under FP64 CG,
    rel-res 1e-8. n = 64 has the 2.1M free DOF of c2; n = 128 the 17M of the
    paper's second-order model."""
    c = _inclusion_case("p2", n, seed, (8.0, 15.0), (8.0, 14.0), order=2)
    c.s, c.steps, c.tau, c.rtol, c.precision = 16, 200, 1e-4, 1e-8, "fp32"
    return c


def case_c0_p2(n: int = 8) -> Case:
    """The c0 slab problem on second-order (10-node) tets."""
    c = case_c0(n)
    xyz, tets = kuhn_cube_mesh_p2(n)
    c.xyz, c.tets = xyz, tets
    c.dir_nodes, c.dir_drive, c.amp, c.freq, c.phase = _dirichlet_top_bottom(xyz)
    c.name = "c0p2"
    return c


def case_batch(n_inst: int = 64, base_seed: int = 3000, sizes=(16, 24, 32, 40, 48)) -> List[Case]:
    out = []
    for i in range(n_inst):
        rng = np.random.default_rng(base_seed + i)
        n = int(rng.choice(sizes))
        amp = float(rng.uniform(0.5, 2.0))
        freq = float(rng.uniform(25.0, 100.0))
        c = _inclusion_case("c3", n, base_seed + i, (2.0, 15.0), (6.0, 14.0), amp=amp, freq=freq)
        c.s, c.steps, c.tau, c.rtol, c.precision = 8, 200, 1e-4, 1e-8, "fp32"
        out.append(c)
    return out


def layered_case(n: int, layers, amp: float = 1.0, freq: float = 50.0, phase: float = 0.0, name="layers") -> Case:
    """Cube with mesh-aligned horizontal layers.

    ``layers`` is a list of (z_lo, z_hi, material-dict); an element belongs to
    the first layer whose open z-range contains its centroid, else to the last.
    Material dicts carry eps_r, kappa0, e_s, alpha, nonlinear.
    """
    xyz, tets = kuhn_cube_mesh(n)
    cz = _centroids(xyz, tets)[:, 2]
    tet_mat = np.full(tets.shape[0], len(layers) - 1, dtype=np.int32)
    for k in range(len(layers) - 1, -1, -1):
        lo, hi, _ = layers[k]
        tet_mat[(cz > lo) & (cz < hi)] = k
    eps, k0, es, al, nl = _material_table([m for _, _, m in layers])
    dn, dd, a, f, ph = _dirichlet_top_bottom(xyz, amp=amp, freq=freq, phase=phase)
    return Case(name, n, xyz, tets, tet_mat, eps, k0, es, al, nl, dn, dd, a, f, ph)


def make_case(name: str, n: Optional[int] = None, seed: Optional[int] = None):
    if name == "c0":
        return case_c0(n or 8)
    if name == "c1":
        return case_c1(n or 64, 1 if seed is None else seed)
    if name in ("c2", "c4"):
        c = case_c2(n or 128, 1 if seed is None else seed)
        c.name = name
        return c
    if name == "c3":
        return case_batch()
    if name == "p2":
        return case_p2(n or 64, 1 if seed is None else seed)
    raise ValueError(f"unknown case {name!r}")


def random_state(n_nodes: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded random potentials on all nodes, uniform in [-scale, scale]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, size=n_nodes)


def mlp_init(seed: int = 4, layers=(32, 64, 64, 16)):
    """Seeded Xavier-uniform initial weights (zero biases) of the start-vector
    network, float32: {W1, b1, W2, b2, W3, b3}, W_l of shape [out, in]."""
    rng = np.random.default_rng(seed)
    out = {}
    for l in range(len(layers) - 1):
        fan_in, fan_out = layers[l], layers[l + 1]
        bound = np.sqrt(6.0 / (fan_in + fan_out))
        out[f"W{l + 1}"] = rng.uniform(-bound, bound, size=(fan_out, fan_in)).astype(np.float32)
        out[f"b{l + 1}"] = np.zeros(fan_out, dtype=np.float32)
    return out
