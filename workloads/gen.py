"""Seeded generators for the synthetic VRC workloads.

Every generator takes an explicit seed and draws from
``numpy.random.Generator(PCG64(seed))``.  Values are produced in float64; the
FP32 variants are round-to-nearest copies (``rays_to_f32``).

The paper's own test problems (PWR assembly, criticality-accident room,
reflected Godiva; Sec. 5) need ACE data and benchmark specifications that are
not available, so these synthetic inputs stand in for them.  They keep the
features the estimator is sensitive to: Cartesian meshes with one material per
voxel (Sec. 3), continuous-energy total cross sections tabulated on an energy
grid and interpolated linearly (Sec. 3), optically thick and thin regions,
voids, and rays from uniformly distributed collision points with isotropic
directions.

Layouts (shared by both sides of every comparison):

* mesh: ``lo[3]``, ``h[3]`` (cm), ``n[3]``, and ``mat`` (uint8, x fastest:
  ``mat[i + nx*(j + ny*k)]``).
* cross sections: ``offs[n_mat+1]`` (int64) into concatenated ``energy`` (MeV,
  strictly increasing per material) and ``sigma`` (1/cm) arrays.
* rays: structure of arrays ``ox, oy, oz, ux, uy, uz, e, w``.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

E_MIN_MEV = 1.0e-11
E_MAX_MEV = 20.0


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclasses.dataclass
class Mesh:
    lo: np.ndarray  # (3,) float64, cm
    h: np.ndarray  # (3,) float64, cm
    n: np.ndarray  # (3,) int32
    mat: np.ndarray  # (nx*ny*nz,) uint8, x fastest
    density: Optional[np.ndarray] = None  # (nx*ny*nz,) float64 factors on the material's Sigma, or None

    @property
    def n_voxels(self) -> int:
        return int(np.prod(self.n.astype(np.int64)))

    def check(self) -> None:
        assert self.lo.shape == (3,) and self.h.shape == (3,) and self.n.shape == (3,)
        assert self.mat.dtype == np.uint8 and self.mat.size == self.n_voxels
        assert np.all(self.h > 0) and np.all(self.n > 0)


@dataclasses.dataclass
class RectMesh:
    """Rectilinear mesh: per axis a table of n_a + 1 increasing planes (cm)."""
    planes: list  # 3 arrays of float64
    mat: np.ndarray  # (nx*ny*nz,) uint8, x fastest
    density: Optional[np.ndarray] = None  # per-voxel factors, as for Mesh

    @property
    def n(self) -> np.ndarray:
        return np.array([p.size - 1 for p in self.planes], np.int32)

    @property
    def lo(self) -> np.ndarray:
        return np.array([p[0] for p in self.planes], np.float64)

    @property
    def hi(self) -> np.ndarray:
        return np.array([p[-1] for p in self.planes], np.float64)

    @property
    def n_voxels(self) -> int:
        return int(np.prod(self.n.astype(np.int64)))

    def check(self) -> None:
        assert len(self.planes) == 3
        for p in self.planes:
            assert p.ndim == 1 and p.size >= 2 and np.all(np.diff(p) > 0)
        assert self.mat.dtype == np.uint8 and self.mat.size == self.n_voxels


@dataclasses.dataclass
class RZMesh:
    """R-Z (cylindrical) mesh: a cylinder along z with its axis through centre = (cx, cy), cut into
    shells by radii 0 = radii[0] < ... < radii[nr] and into slabs by planes zpl[0] < ... < zpl[nz].
    Cell (i, k) is r_i <= rho < r_{i+1}, z_k <= z < z_{k+1}, number i + nr k; mat is r fastest."""
    centre: np.ndarray  # (2,) float64, cm
    radii: np.ndarray  # (nr + 1,) float64, cm, radii[0] = 0
    zpl: np.ndarray  # (nz + 1,) float64, cm
    mat: np.ndarray  # (nr * nz,) uint8
    density: Optional[np.ndarray] = None  # per-cell factors on the material's Sigma, or None

    @property
    def nr(self) -> int:
        return int(self.radii.size - 1)

    @property
    def nz(self) -> int:
        return int(self.zpl.size - 1)

    @property
    def n_voxels(self) -> int:
        return self.nr * self.nz

    def check(self) -> None:
        assert self.centre.shape == (2,) and self.radii[0] == 0.0
        assert np.all(np.diff(self.radii) > 0) and np.all(np.diff(self.zpl) > 0)
        assert self.mat.dtype == np.uint8 and self.mat.size == self.n_voxels


def rz_mesh(seed: int, nr: int, nz: int, r_max: float, z_lo: float, z_hi: float, n_mat: int = 3,
            centre=(0.0, 0.0), uneven: bool = True, ring: int = 5, slab: int = 10) -> RZMesh:
    """R-Z mesh: radii uniform in r (with seeded jitter of up to a third of a spacing when uneven), z planes
    uniform, materials drawn per block of `ring` shells x `slab` slabs."""
    rng = _rng(seed)
    radii = np.linspace(0.0, r_max, nr + 1)
    if uneven and nr > 1:
        dr = r_max / nr
        radii[1:-1] += rng.uniform(-dr / 3, dr / 3, nr - 1)
    zpl = np.linspace(z_lo, z_hi, nz + 1)
    blocks = rng.integers(0, n_mat, ((nz + slab - 1) // slab, (nr + ring - 1) // ring)).astype(np.uint8)
    mat = np.repeat(np.repeat(blocks, slab, axis=0)[:nz], ring, axis=1)[:, :nr]
    return RZMesh(np.asarray(centre, np.float64), radii, zpl, mat.reshape(-1).copy())


def rect_mesh(seed: int, n, lo=(0.0, 0.0, 0.0), h_min: float = 0.2, h_max: float = 1.5, n_mat: int = 3,
              slab: int = 4) -> RectMesh:
    """Rectilinear mesh with spacings drawn uniformly in [h_min, h_max] per plane, materials per z slab."""
    rng = _rng(seed)
    planes = [lo[a] + np.concatenate([[0.0], np.cumsum(rng.uniform(h_min, h_max, int(n[a])))]) for a in range(3)]
    nz_slabs = (int(n[2]) + slab - 1) // slab
    slab_mat = rng.integers(0, n_mat, nz_slabs).astype(np.uint8)
    mat = np.repeat(slab_mat, slab)[: int(n[2])]
    vol = np.broadcast_to(mat[:, None, None], (int(n[2]), int(n[1]), int(n[0]))).reshape(-1).copy()
    return RectMesh(planes, vol)


@dataclasses.dataclass
class XSTables:
    offs: np.ndarray  # (n_mat+1,) int64
    energy: np.ndarray  # float64 MeV, concatenated per material
    sigma: np.ndarray  # float64 1/cm, concatenated per material

    @property
    def n_mat(self) -> int:
        return int(self.offs.size - 1)

    def table(self, m: int):
        a, b = int(self.offs[m]), int(self.offs[m + 1])
        return self.energy[a:b], self.sigma[a:b]


@dataclasses.dataclass
class Rays:
    ox: np.ndarray
    oy: np.ndarray
    oz: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    uz: np.ndarray
    e: np.ndarray
    w: np.ndarray

    FIELDS = ("ox", "oy", "oz", "ux", "uy", "uz", "e", "w")

    @property
    def n(self) -> int:
        return int(self.ox.size)

    def arrays(self) -> List[np.ndarray]:
        return [getattr(self, f) for f in self.FIELDS]

    def take(self, idx) -> "Rays":
        return Rays(*[np.ascontiguousarray(a[idx]) for a in self.arrays()])

    def as_f64(self) -> "Rays":
        return Rays(*[np.ascontiguousarray(a, dtype=np.float64) for a in self.arrays()])

    @staticmethod
    def concat(parts: Sequence["Rays"]) -> "Rays":
        return Rays(*[np.concatenate([getattr(p, f) for p in parts]) for f in Rays.FIELDS])


@dataclasses.dataclass
class Workload:
    name: str
    mesh: Mesh
    xs: XSTables
    rays: Optional[Rays]
    ebin_edges: Optional[np.ndarray] = None  # None means a single energy bin
    extra: dict = dataclasses.field(default_factory=dict)


def rays_to_f32(r: Rays) -> Rays:
    """Round-to-nearest FP32 copy of a ray batch (directions rounded from FP64 unit vectors)."""
    return Rays(*[np.ascontiguousarray(a, dtype=np.float32) for a in r.arrays()])


# ----------------------------------------------------------------------------
# directions, energies, weights
# ----------------------------------------------------------------------------

def isotropic_directions(rng: np.random.Generator, n: int):
    mu = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    s = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    return s * np.cos(phi), s * np.sin(phi), mu


def log_uniform_energies(rng: np.random.Generator, n: int, lo=E_MIN_MEV, hi=E_MAX_MEV):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), n))


def log_bin_edges(n_bins: int, lo=E_MIN_MEV, hi=E_MAX_MEV) -> np.ndarray:
    return np.exp(np.linspace(math.log(lo), math.log(hi), n_bins + 1))


# ----------------------------------------------------------------------------
# cross-section tables
# ----------------------------------------------------------------------------

def log_energy_grid(K: int, lo=E_MIN_MEV, hi=E_MAX_MEV) -> np.ndarray:
    k = np.arange(K, dtype=np.float64)
    return lo * (hi / lo) ** (k / (K - 1))


def synthetic_sigma_table(seed: int, K: int, a: float, b: float, clip_lo: float, clip_hi: float,
                          n_peaks: int = 200) -> np.ndarray:
    """Sigma_t(E) on the log grid: a*sqrt(1e-6/E) + b + sum of seeded Lorentzian peaks, clipped.

    Stands in for an NJOY-processed continuous-energy total cross section
    (Sec. 3): a smooth 1/v term plus resonance-like peaks.
    """
    rng = _rng(seed)
    E = log_energy_grid(K)
    Ej = np.exp(rng.uniform(math.log(1e-7), math.log(1e-2), n_peaks))
    Gj = Ej * 10.0 ** rng.uniform(-3.0, -1.5, n_peaks)
    hj = np.exp(rng.uniform(math.log(0.3), math.log(40.0), n_peaks))
    s = a * np.sqrt(1e-6 / E) + b
    for j in range(n_peaks):
        s = s + hj[j] * Gj[j] ** 2 / ((E - Ej[j]) ** 2 + Gj[j] ** 2)
    return np.clip(s, clip_lo, clip_hi)


def constant_sigma_table(value: float):
    """Two-point table of an energy-independent cross section."""
    return np.array([E_MIN_MEV, E_MAX_MEV]), np.array([value, value], dtype=np.float64)


def make_xs(tables) -> XSTables:
    offs = [0]
    es, ss = [], []
    for e, s in tables:
        e = np.asarray(e, dtype=np.float64)
        s = np.asarray(s, dtype=np.float64)
        assert e.size == s.size and e.size >= 1
        assert np.all(np.diff(e) > 0)
        es.append(e)
        ss.append(s)
        offs.append(offs[-1] + e.size)
    return XSTables(np.array(offs, dtype=np.int64), np.concatenate(es), np.concatenate(ss))


_MAT_A = (0.3, 0.1, 0.15)
_MAT_B = (0.1, 0.3, 0.05)


@dataclasses.dataclass
class Mixtures:
    """Materials made of tabulated components: material k takes components
    comp[offs[k]:offs[k+1]] with factors frac[offs[k]:offs[k+1]] (>= 0)."""
    offs: np.ndarray  # (n_mix+1,) int64
    comp: np.ndarray  # int32 component (table) ids
    frac: np.ndarray  # float64 factors

    @property
    def n_mix(self) -> int:
        return int(self.offs.size - 1)


def random_mixtures(seed: int, n_comp: int, n_mix: int, max_comp: int = 3) -> Mixtures:
    """n_mix mixtures of 1..max_comp distinct components with factors in [0.05, 1.5]."""
    rng = _rng(seed)
    offs, comp, frac = [0], [], []
    for _ in range(n_mix):
        k = int(rng.integers(1, min(max_comp, n_comp) + 1))
        c = rng.choice(n_comp, size=k, replace=False)
        comp.extend(int(x) for x in c)
        frac.extend(float(x) for x in rng.uniform(0.05, 1.5, k))
        offs.append(len(comp))
    return Mixtures(np.array(offs, np.int64), np.array(comp, np.int32), np.array(frac, np.float64))


def density_field(seed: int, n_voxels: int, low: float = 0.5, high: float = 2.0, frac_zero: float = 0.0) -> np.ndarray:
    """Per-voxel density factors uniform in [low, high], a fraction frac_zero of them 0 (voids)."""
    rng = _rng(seed)
    rho = rng.uniform(low, high, n_voxels)
    if frac_zero > 0:
        rho[rng.uniform(size=n_voxels) < frac_zero] = 0.0
    return rho


def three_material_xs(seed: int, K: int, clip_lo=0.05, clip_hi=50.0) -> XSTables:
    E = log_energy_grid(K)
    tabs = []
    for m in range(3):
        tabs.append((E, synthetic_sigma_table(seed * 10 + m, K, _MAT_A[m], _MAT_B[m], clip_lo, clip_hi)))
    return make_xs(tabs)


# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------

def slab_mesh(seed: int, n: int, h: float, slab: int = 10, n_mat: int = 3, lo=None) -> Mesh:
    """n^3 mesh with materials assigned per z-slab of ``slab`` voxels, uniformly from {0..n_mat-1}."""
    rng = _rng(seed)
    n_slabs = (n + slab - 1) // slab
    slab_mat = rng.integers(0, n_mat, n_slabs).astype(np.uint8)
    kz = np.arange(n) // slab
    mat = np.broadcast_to(slab_mat[kz][:, None, None], (n, n, n)).reshape(-1).copy()
    lo = np.zeros(3) if lo is None else np.asarray(lo, dtype=np.float64)
    return Mesh(lo, np.full(3, h, dtype=np.float64), np.full(3, n, dtype=np.int32), mat)


def _centres(mesh: Mesh, axis: int) -> np.ndarray:
    return mesh.lo[axis] + (np.arange(mesh.n[axis]) + 0.5) * mesh.h[axis]


def cylinder_spheres_mesh(seed: int, n: int = 256, h: float = 0.2, radius: float = 20.0,
                          n_spheres: int = 8, sphere_mats=(1, 1, 1, 1, 2, 2, 2, 2),
                          r_range=(2.0, 5.0), void_mat: int = 3) -> Mesh:
    """Water-like cylinder along z (material 0) in a void box, with seeded spherical inserts.

    The mesh is centred on the origin.  Voxel materials are set by testing the
    voxel centre.  Spheres do not overlap and lie fully inside the cylinder.
    """
    rng = _rng(seed)
    L = n * h
    lo = np.full(3, -L / 2)
    mesh = Mesh(lo, np.full(3, h), np.full(3, n, dtype=np.int32), np.empty(n ** 3, np.uint8))
    xc, yc, zc = _centres(mesh, 0), _centres(mesh, 1), _centres(mesh, 2)
    spheres = []
    tries = 0
    while len(spheres) < n_spheres:
        tries += 1
        assert tries < 100000
        r = rng.uniform(*r_range)
        rho = radius - r
        ang = rng.uniform(0, 2 * math.pi)
        d = rho * math.sqrt(rng.uniform())
        c = np.array([d * math.cos(ang), d * math.sin(ang), rng.uniform(-L / 2 + r, L / 2 - r)])
        if all(np.linalg.norm(c - c2) > r + r2 for c2, r2 in spheres):
            spheres.append((c, r))
    r2xy = xc[None, :] ** 2 + yc[:, None] ** 2  # (ny, nx)
    inside_cyl = r2xy < radius * radius
    mat = np.where(inside_cyl, 0, void_mat).astype(np.uint8)
    mat = np.broadcast_to(mat[None, :, :], (n, n, n)).copy()  # (nz, ny, nx)
    for (c, r), m in zip(spheres, sphere_mats):
        i0 = max(0, int((c[0] - r - lo[0]) / h) - 1)
        i1 = min(n, int((c[0] + r - lo[0]) / h) + 2)
        j0 = max(0, int((c[1] - r - lo[1]) / h) - 1)
        j1 = min(n, int((c[1] + r - lo[1]) / h) + 2)
        k0 = max(0, int((c[2] - r - lo[2]) / h) - 1)
        k1 = min(n, int((c[2] + r - lo[2]) / h) + 2)
        d2 = ((xc[None, None, i0:i1] - c[0]) ** 2 + (yc[None, j0:j1, None] - c[1]) ** 2
              + (zc[k0:k1, None, None] - c[2]) ** 2)
        sub = mat[k0:k1, j0:j1, i0:i1]
        sub[d2 < r * r] = m
    mesh.mat = mat.reshape(-1)
    mesh.extra_spheres = spheres  # type: ignore[attr-defined]
    return mesh


def sphere_mesh(n: int = 200, h: float = 1.0, radius: float = 50.0, inner_mat: int = 1,
                outer_mat: int = 0) -> Mesh:
    """Cube centred on the origin with a centred sphere of ``inner_mat`` in ``outer_mat``."""
    L = n * h
    mesh = Mesh(np.full(3, -L / 2), np.full(3, h), np.full(3, n, dtype=np.int32), np.empty(n ** 3, np.uint8))
    xc, yc, zc = _centres(mesh, 0), _centres(mesh, 1), _centres(mesh, 2)
    mat = np.empty((n, n, n), np.uint8)
    for k in range(n):
        d2 = xc[None, :] ** 2 + yc[:, None] ** 2 + zc[k] ** 2
        mat[k] = np.where(d2 < radius * radius, inner_mat, outer_mat)
    mesh.mat = mat.reshape(-1)
    return mesh


# ----------------------------------------------------------------------------
# rays
# ----------------------------------------------------------------------------

def _finish_rays(rng, ox, oy, oz, weights: str, w_value: float = 1.0) -> Rays:
    n = ox.size
    ux, uy, uz = isotropic_directions(rng, n)
    e = log_uniform_energies(rng, n)
    if weights == "lognormal":
        w = rng.lognormal(0.0, 0.5, n)
    else:
        w = np.full(n, w_value, dtype=np.float64)
    return Rays(ox, oy, oz, ux, uy, uz, e, w)


def rays_in_box(seed: int, mesh: Mesh, n: int, weights: str = "lognormal", w_value: float = 1.0) -> Rays:
    rng = _rng(seed)
    hi = mesh.hi if isinstance(mesh, RectMesh) else mesh.lo + mesh.n * mesh.h
    o = [rng.uniform(mesh.lo[a], hi[a], n) for a in range(3)]
    return _finish_rays(rng, *o, weights=weights, w_value=w_value)


def rays_in_cylinder(seed: int, mesh: Mesh, n: int, radius: float, weights: str = "lognormal") -> Rays:
    """Origins uniform in the z-aligned cylinder through the mesh centre."""
    rng = _rng(seed)
    c = mesh.lo + 0.5 * mesh.n * mesh.h
    r = radius * np.sqrt(rng.uniform(0.0, 1.0, n))
    th = rng.uniform(0.0, 2.0 * math.pi, n)
    ox = c[0] + r * np.cos(th)
    oy = c[1] + r * np.sin(th)
    oz = rng.uniform(mesh.lo[2], mesh.lo[2] + mesh.n[2] * mesh.h[2], n)
    return _finish_rays(rng, ox, oy, oz, weights=weights)


def rays_in_rz(seed: int, mesh: "RZMesh", n: int, weights: str = "lognormal", r_frac: float = 1.0) -> Rays:
    """Origins uniform in the volume of the R-Z mesh's cylinder (radius r_frac times its outer radius)."""
    rng = _rng(seed)
    r = r_frac * mesh.radii[-1] * np.sqrt(rng.uniform(0.0, 1.0, n))
    th = rng.uniform(0.0, 2.0 * math.pi, n)
    ox = mesh.centre[0] + r * np.cos(th)
    oy = mesh.centre[1] + r * np.sin(th)
    oz = rng.uniform(mesh.zpl[0], mesh.zpl[-1], n)
    return _finish_rays(rng, ox, oy, oz, weights=weights)


def rays_near_faces(seed: int, mesh: Mesh, n: int, frac_face: float = 0.5, weights: str = "lognormal") -> Rays:
    """Half of the origins within one voxel of a random face, the rest uniform in the box."""
    rng = _rng(seed)
    hi = mesh.lo + mesh.n * mesh.h
    o = np.stack([rng.uniform(mesh.lo[a], hi[a], n) for a in range(3)], axis=1)
    near = rng.uniform(size=n) < frac_face
    face = rng.integers(0, 6, n)
    ax = face // 2
    side = face % 2
    d = rng.uniform(0.0, 1.0, n)
    for a in range(3):
        sel = near & (ax == a)
        lo_side = sel & (side == 0)
        hi_side = sel & (side == 1)
        o[lo_side, a] = mesh.lo[a] + d[lo_side] * mesh.h[a]
        o[hi_side, a] = hi[a] - d[hi_side] * mesh.h[a]
    return _finish_rays(rng, o[:, 0].copy(), o[:, 1].copy(), o[:, 2].copy(), weights=weights)


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

def config1_tiny(n_rays: int = 10_000, seed: int = 101) -> Workload:
    """10^3 mesh of 1 cm voxels, one material with Sigma_t = 0.5/cm, unit weights, FP64 tally."""
    mesh = Mesh(np.zeros(3), np.ones(3), np.full(3, 10, dtype=np.int32), np.zeros(1000, np.uint8))
    xs = make_xs([constant_sigma_table(0.5)])
    rays = rays_in_box(seed, mesh, n_rays, weights="const", w_value=1.0) if n_rays else None
    return Workload("tiny-10^3-1mat", mesh, xs, rays)


def config2_multimaterial(n_rays: int = 1_000_000, seed: int = 202, K: int = 20_000, n: int = 100,
                          h: float = 0.5) -> Workload:
    """100^3 mesh of 0.5 cm voxels, 3 materials in 10-voxel z-slabs, 20k-point tables."""
    mesh = slab_mesh(seed, n, h)
    xs = three_material_xs(seed, K)
    rays = rays_in_box(seed + 1, mesh, n_rays) if n_rays else None
    return Workload(f"multimat-{n}^3-{K}pt", mesh, xs, rays)


def config3_precision(n_rays: int = 10_000_000, seed: int = 303, K: int = 50_000, n: int = 256,
                      h: float = 0.2, radius: float = 20.0) -> Workload:
    """256^3 mesh of 0.2 cm voxels: water-like cylinder (0.1-5/cm) with 8 spherical inserts, void outside."""
    mesh = cylinder_spheres_mesh(seed, n, h, radius)
    E = log_energy_grid(K)
    water = synthetic_sigma_table(seed * 10, K, _MAT_A[0], _MAT_B[0], 0.1, 5.0)
    m1 = synthetic_sigma_table(seed * 10 + 1, K, _MAT_A[1], _MAT_B[1], 0.05, 50.0)
    m2 = synthetic_sigma_table(seed * 10 + 2, K, _MAT_A[2], _MAT_B[2], 0.05, 50.0)
    void = constant_sigma_table(0.0)
    xs = make_xs([(E, water), (E, m1), (E, m2), void])
    rays = rays_in_cylinder(seed + 1, mesh, n_rays, radius) if n_rays else None
    return Workload(f"cylinder-{n}^3-{K}pt", mesh, xs, rays, extra={"radius": radius})


def config4_batches(n_batches: int = 2000, seed: int = 404, sizes=(64, 128, 160, 200), h: float = 0.5,
                    K: int = 20_000, median: float = 2e4, sigma: float = 1.3, size_range=(1000, 1_000_000),
                    materialise: bool = True) -> Workload:
    """Several meshes with config-2 materials and uneven ray batches started near faces or inside."""
    rng = _rng(seed)
    meshes = [slab_mesh(seed + 10 + i, s, h) for i, s in enumerate(sizes)]
    xs = three_material_xs(202, K)
    mesh_of = rng.integers(0, len(sizes), n_batches)
    bsz = np.clip(np.round(rng.lognormal(math.log(median), sigma, n_batches)), *size_range).astype(np.int64)
    batches = []
    if materialise:
        for b in range(n_batches):
            batches.append(rays_near_faces(seed * 1000 + b, meshes[mesh_of[b]], int(bsz[b])))
    wl = Workload("batched-uneven", meshes[0], xs, None,
                  extra={"meshes": meshes, "mesh_of": mesh_of, "sizes": bsz, "batches": batches})
    return wl


def config5_serving_geometry(n: int = 200, h: float = 1.0, radius: float = 50.0, n_bins: int = 10) -> Workload:
    """200^3 mesh, sphere of Sigma=1.0/cm in Sigma=0.1/cm, one-group tables, 10 log energy bins."""
    mesh = sphere_mesh(n, h, radius)
    xs = make_xs([constant_sigma_table(0.1), constant_sigma_table(1.0)])
    return Workload("serving-200^3-sphere", mesh, xs, None, ebin_edges=log_bin_edges(n_bins),
                    extra={"p_abs": 0.3, "sigma": (0.1, 1.0), "radius": radius})


# ----------------------------------------------------------------------------
# device-side generation of the large batched workload (benchmark only)
# ----------------------------------------------------------------------------

def config4_batches_device(device, n_batches: int = 2000, seed: int = 404, dtype=None, **kw):
    """The batched workload with its rays drawn on the GPU (torch generator seeded per batch).

    Batch sizes, mesh assignment, meshes and tables come from
    ``config4_batches(materialise=False)``; each batch's rays follow the same
    recipe as ``rays_near_faces`` (half within one voxel of a random face,
    half uniform in the box; isotropic directions; log-uniform energies;
    lognormal(0, 0.5) weights).  Returns (workload, list of 8-tensor lists).
    """
    import torch

    dtype = torch.float32 if dtype is None else dtype
    wl = config4_batches(n_batches=n_batches, seed=seed, materialise=False, **kw)
    out = []
    for b in range(n_batches):
        mesh = wl.extra["meshes"][wl.extra["mesh_of"][b]]
        n = int(wl.extra["sizes"][b])
        g = torch.Generator(device=device)
        g.manual_seed(seed * 1000 + b)
        lo = torch.tensor(mesh.lo, dtype=torch.float64, device=device)
        span = torch.tensor(mesh.n * mesh.h, dtype=torch.float64, device=device)
        hvox = torch.tensor(mesh.h, dtype=torch.float64, device=device)
        o = lo + torch.rand((n, 3), generator=g, device=device, dtype=torch.float64) * span
        near = torch.rand(n, generator=g, device=device, dtype=torch.float64) < 0.5
        face = torch.randint(0, 6, (n,), generator=g, device=device)
        d = torch.rand(n, generator=g, device=device, dtype=torch.float64)
        for a in range(3):
            lo_side = near & (face == 2 * a)
            hi_side = near & (face == 2 * a + 1)
            o[:, a] = torch.where(lo_side, lo[a] + d * hvox[a], o[:, a])
            o[:, a] = torch.where(hi_side, lo[a] + span[a] - d * hvox[a], o[:, a])
        mu = torch.rand(n, generator=g, device=device, dtype=torch.float64) * 2 - 1
        phi = torch.rand(n, generator=g, device=device, dtype=torch.float64) * (2 * math.pi)
        s = torch.sqrt(torch.clamp(1 - mu * mu, min=0))
        e = torch.exp(math.log(E_MIN_MEV) + torch.rand(n, generator=g, device=device, dtype=torch.float64)
                      * (math.log(E_MAX_MEV) - math.log(E_MIN_MEV)))
        w = torch.exp(0.5 * torch.randn(n, generator=g, device=device, dtype=torch.float64))
        cols = [o[:, 0], o[:, 1], o[:, 2], s * torch.cos(phi), s * torch.sin(phi), mu, e, w]
        out.append([c.to(dtype).contiguous() for c in cols])
    return wl, out
