"""Seeded, synthetic inputs for S_N transport problems on uniform Cartesian grids.

This module builds what a caller hands to a transport solver: the mesh, the
per-cell cross sections sigma_t / sigma_s and source q, the angular quadrature
{Omega_d, w_d}, boundary-inflow arrays and detector weights.  It holds none of
the solution method's arithmetic (no sweep, no moment, no diffusion
operator); both the CPU oracle and the GPU library consume its arrays.

Conventions shared by every consumer (they are part of the library's C ABI):

* cells are numbered lexicographically, x fastest: c = (k*ny + j)*nx + i;
* Q1 nodes sit at cell corners, numbered a + 2b (+ 4c) with a, b, c in {0, 1}
  the x-, y- (and z-) node of the corner (0 = low side);
* directions are ordered octant-major, octant o = (mu<0) + 2(eta<0) + 4(xi<0);
  a 2D problem uses the xi > 0 half of a 3D set with doubled weights, so its
  octants are the four quadrants o = 0..3;
* the weights sum to 4*pi and the scalar flux is phi = sum_d w_d psi_d
  (the S_N semi-discrete form, Section 1 of the paper).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "level_symmetric", "Problem", "config", "CONFIG_NAMES", "tile_materials",
    "inflow_size", "unit_inflow_on_face", "patch_source", "fd_cells",
    "crooked_pipe", "PIPE_PROBLEMS", "pipe_regions",
]

# First level cosine of the level-symmetric LQ_N sets.  S4 follows from the
# fourth-moment condition (6 a^2 - 4 a + 0.4 = 0 with a = mu_1^2); S8 and S12
# use the customary tabulated values (the remaining weights are then fixed by
# the even-moment conditions solved below).
_MU1 = {
    4: math.sqrt((4.0 - math.sqrt(16.0 - 9.6)) / 12.0),
    8: 0.2182179,
    12: 0.1672126,
}


def level_symmetric(order: int, dim: int):
    """Level-symmetric LQ_N quadrature, octant-major.

    Levels mu_i^2 = mu_1^2 + (i-1) * 2 (1 - 3 mu_1^2) / (N - 2), i = 1..N/2;
    one octant holds the points (mu_i, mu_j, mu_k) with i + j + k = N/2 + 2.
    Points equivalent under axis permutation share a weight; the class weights
    solve the even-moment conditions sum_p w_p mu_p^(2n) = 1/(2n+1) over one
    octant (weights normalised to 1 per octant, then scaled to pi/2 so that
    the full sphere sums to 4 pi).

    Returns (omega [D,3] float64, w [D] float64).  For dim == 2 only the
    xi > 0 half is kept and its weights are doubled (D = N(N+2)/2).
    """
    if order not in _MU1:
        raise ValueError(f"level-symmetric order {order} not tabulated")
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    n = order
    nl = n // 2
    mu1 = _MU1[n]
    lev = np.sqrt(np.array([mu1 * mu1 + i * 2.0 * (1.0 - 3.0 * mu1 * mu1) / (n - 2)
                            for i in range(nl)]))
    pts = [(i, j, n // 2 + 2 - i - j) for i in range(1, nl + 1) for j in range(1, nl + 1)
           if 1 <= n // 2 + 2 - i - j <= nl]
    classes = sorted({tuple(sorted(p)) for p in pts})
    cls = [classes.index(tuple(sorted(p))) for p in pts]
    # even-moment conditions n = 0 .. nl-1 (n = 1 holds by symmetry but is kept)
    a = np.zeros((nl, len(classes)))
    rhs = np.array([1.0 / (2 * m + 1) for m in range(nl)])
    for p, c in zip(pts, cls):
        for m in range(nl):
            a[m, c] += lev[p[0] - 1] ** (2 * m)
    wc, *_ = np.linalg.lstsq(a, rhs, rcond=None)
    if np.max(np.abs(a @ wc - rhs)) > 1e-12:
        raise RuntimeError(f"LQ{n}: even-moment conditions inconsistent")
    if np.any(wc <= 0):
        raise RuntimeError(f"LQ{n}: non-positive weight")
    base = np.array([[lev[i - 1], lev[j - 1], lev[k - 1]] for (i, j, k) in pts])
    wpt = np.array([wc[c] for c in cls]) * (math.pi / 2.0)
    noct = 4 if dim == 2 else 8
    om, ww = [], []
    for o in range(noct):
        sx = -1.0 if (o & 1) else 1.0
        sy = -1.0 if (o & 2) else 1.0
        sz = -1.0 if (o & 4) else 1.0
        for p, wp in zip(base, wpt):
            om.append([sx * p[0], sy * p[1], sz * p[2]])
            ww.append(wp * (2.0 if dim == 2 else 1.0))
    return np.ascontiguousarray(om, dtype=np.float64), np.ascontiguousarray(ww, dtype=np.float64)


@dataclasses.dataclass
class Problem:
    """One S_N transport problem on a uniform Cartesian grid (vacuum unless inflow given)."""
    name: str
    dim: int
    nx: int
    ny: int
    nz: int
    h: tuple                 # (hx, hy, hz); hz unused in 2D
    sigma_t: np.ndarray      # [ncells] float64
    sigma_s: np.ndarray      # [ncells] float64
    q: np.ndarray            # [ncells] float64, total isotropic source density
    omega: np.ndarray        # [D, 3]
    w: np.ndarray            # [D]
    eta: float = 1.0         # thick threshold: a cell is thick iff sigma_s >= eta
    meta: dict = dataclasses.field(default_factory=dict)
    order: int = 1           # DG order p: Q_p on the (p + 1)^dim Gauss-Lobatto nodes of each cell

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def nn(self) -> int:
        return (self.order + 1) ** self.dim

    @property
    def ndirs(self) -> int:
        return int(self.w.shape[0])

    def thick_mask(self, eta: Optional[float] = None) -> np.ndarray:
        e = self.eta if eta is None else eta
        return self.sigma_s >= e


def tile_materials(dims, tile, seed, mats, frac_void=0.2, frac_thick=0.3):
    """Seeded tile layout: round(0.2 T) void, round(0.3 T) thick, the rest thin.

    Tiles are numbered lexicographically (x fastest); a permutation drawn from
    numpy.random.default_rng(seed) assigns the first round(frac_void*T) tiles
    void, the next round(frac_thick*T) thick.  Returns per-cell arrays
    (sigma_t, sigma_s, kind) with kind 0 void, 1 thin, 2 thick.
    """
    dims = tuple(dims)
    nt = tuple(d // tile for d in dims)
    if any(d % tile for d in dims):
        raise ValueError("grid not divisible by tile size")
    ntiles = int(np.prod(nt))
    nv = int(round(frac_void * ntiles))
    nk = int(round(frac_thick * ntiles))
    perm = np.random.default_rng(seed).permutation(ntiles)
    tkind = np.ones(ntiles, dtype=np.int8)
    tkind[perm[:nv]] = 0
    tkind[perm[nv:nv + nk]] = 2
    # per-cell tile index, lexicographic with x fastest
    idx = [np.arange(d) // tile for d in dims]
    if len(dims) == 2:
        tj, ti = np.meshgrid(idx[1], idx[0], indexing="ij")
        tid = tj * nt[0] + ti
    else:
        tk, tj, ti = np.meshgrid(idx[2], idx[1], idx[0], indexing="ij")
        tid = (tk * nt[1] + tj) * nt[0] + ti
    kind = tkind[tid.ravel()]
    st = np.empty(kind.shape, dtype=np.float64)
    ss = np.empty(kind.shape, dtype=np.float64)
    for k, (a, b) in mats.items():
        st[kind == k] = a
        ss[kind == k] = b
    return st, ss, kind


CONFIG_NAMES = ("c1", "c2", "c3", "c4", "c5")

_MIX = {0: (0.0, 0.0), 1: (1.0, 0.5), 2: (1.0e3, 999.9)}


def config(name: str) -> Problem:
    """The five synthetic workloads (uniform h = 1, vacuum boundaries).

    c1  2D 16x16, S4: background (1, 0.9), thick block cells 4..7 (100, 99.9),
        void block i in 10..13, j in 2..5; q = 1 on cells 1..2 squared.
    c2  2D 256x256, S8, 16x16-cell tiles (seed 0) void/thin/thick 20/50/30 %.
    c3  3D 64^3, S8, 8^3 tiles, same mix.
    c4  2D 128x128, S8, 8x8 tiles, same mix plus lognormal jitter (0.2, seed 1)
        on sigma_t and sigma_s, then sigma_s clipped to sigma_t.
    c5  3D 128^3, S12, 16^3 tiles, same mix.
    Thin tiles carry q = 1; thick tiles (1e3, 999.9); thin (1, 0.5); void (0, 0).
    c2s c2 with pure-scatterer thick tiles (1e3, 1e3): sigma_a = 0 there, so the
        thick-region diffusion operator has no absorption (the regime of the
        sigma_a = 0 rows of the paper's crooked-pipe table).
    """
    name = name.lower()
    if name == "c2s":
        p = config("c2")
        ss = np.where(p.meta["kind"] == 2, p.sigma_t, p.sigma_s)
        return Problem("c2s", 2, p.nx, p.ny, 1, p.h, p.sigma_t, ss, p.q, p.omega, p.w, meta=p.meta)
    if name == "c1":
        n = 16
        om, w = level_symmetric(4, 2)
        st = np.full(n * n, 1.0)
        ss = np.full(n * n, 0.9)
        q = np.zeros(n * n)
        for j in range(n):
            for i in range(n):
                c = j * n + i
                if 4 <= i <= 7 and 4 <= j <= 7:
                    st[c], ss[c] = 100.0, 99.9
                if 10 <= i <= 13 and 2 <= j <= 5:
                    st[c], ss[c] = 0.0, 0.0
                if 1 <= i <= 2 and 1 <= j <= 2:
                    q[c] = 1.0
        return Problem("c1", 2, n, n, 1, (1.0, 1.0, 1.0), st, ss, q, om, w)
    if name in ("c2", "c4"):
        n, tile = (256, 16) if name == "c2" else (128, 8)
        om, w = level_symmetric(8, 2)
        st, ss, kind = tile_materials((n, n), tile, 0, _MIX)
        q = (kind == 1).astype(np.float64)
        meta = {"tile": tile, "kind": kind}
        if name == "c4":
            rng = np.random.default_rng(1)
            zt = rng.standard_normal(n * n)
            zs = rng.standard_normal(n * n)
            st = st * np.exp(0.2 * zt)
            ss = ss * np.exp(0.2 * zs)
            clipped = ss > st
            ss = np.minimum(ss, st)
            meta["clipped"] = clipped
        return Problem(name, 2, n, n, 1, (1.0, 1.0, 1.0), st, ss, q, om, w, meta=meta)
    if name in ("c3", "c5"):
        n, tile, order = (64, 8, 8) if name == "c3" else (128, 16, 12)
        om, w = level_symmetric(order, 3)
        st, ss, kind = tile_materials((n, n, n), tile, 0, _MIX)
        q = (kind == 1).astype(np.float64)
        return Problem(name, 3, n, n, n, (1.0, 1.0, 1.0), st, ss, q, om, w,
                       meta={"tile": tile, "kind": kind})
    raise ValueError(f"unknown config {name!r}")


# Scattering cross sections (pipe, wall, edge, block) of the five heterogeneous
# crooked-pipe problems of Sec. 4.1 (Table problems).
PIPE_PROBLEMS = {
    1: (1e-3, 500.0, 1e-4, 100.0),
    2: (0.1, 200.0, 200.0, 5.0),
    3: (1e-4, 10.0, 500.0, 0.1),
    4: (1e-6, 0.1, 100.0, 1000.0),
    5: (1e-4, 10.0, 500.0, 100.0),
}
PIPE_REGIONS = ("pipe", "wall", "edge", "block")


def pipe_regions(nx: int, ny: int, h: float) -> np.ndarray:
    """Region index per cell (0 pipe, 1 wall, 2 edge, 3 block) of a synthetic
    crooked-pipe geometry on [0, 14] x [0, 10].  The paper's geometry exists
    only as a figure; this stand-in has its four kinds of region with the area
    shares implied by its thin/thick percentages at eta = 1 (pipe 32%, wall
    about 37%, edge 25%, block 7%):

    * pipe: a channel of width 2 entering at x = 0 (y in [1.5, 3.5]), rising
      at x in [2, 4] to y in [6, 8], crossing to x = 12, falling at x in
      [10, 12] to y in [2.5, 4.5] and leaving at x = 14 (44 of 140 units^2);
    * edge: the bands y < 1.25 and y > 8.75 along the bottom and top;
    * block: the rectangle [5, 9] x [3, 5.5] inside the bend;
    * wall: the rest.
    Cell centres decide the region."""
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    Y, X = np.meshgrid(y, x, indexing="ij")
    reg = np.ones((ny, nx), dtype=np.int8)
    reg[(Y < 1.25) | (Y > 8.75)] = 2
    reg[(X > 5.0) & (X < 9.0) & (Y > 3.0) & (Y < 5.5)] = 3
    inside = lambda x0, x1, y0, y1: (X > x0) & (X < x1) & (Y > y0) & (Y < y1)
    pipe = (inside(0.0, 4.0, 1.5, 3.5) | inside(2.0, 4.0, 1.5, 8.0) | inside(2.0, 12.0, 6.0, 8.0) |
            inside(10.0, 12.0, 2.5, 8.0) | inside(10.0, 14.0, 2.5, 4.5))
    reg[pipe] = 0
    return reg.ravel()


def crooked_pipe(sigmas, cdt: Optional[float], cells_per_unit: int = 8, order: int = 8,
                 name: str = "pipe") -> Problem:
    """A crooked-pipe problem (Sec. 4.1): sigma_s piecewise constant over the
    regions of pipe_regions, sigma_t = sigma_s + 1/cdt (cdt None: no
    absorption, sigma_t = sigma_s), S_N of the given order in 2D, vacuum
    boundaries, unit isotropic source in the pipe cells of the inlet unit
    (x < 1).  sigmas: (pipe, wall, edge, block), or a problem number of
    PIPE_PROBLEMS."""
    if isinstance(sigmas, int):
        sigmas = PIPE_PROBLEMS[sigmas]
    h = 1.0 / cells_per_unit
    nx, ny = 14 * cells_per_unit, 10 * cells_per_unit
    reg = pipe_regions(nx, ny, h)
    ss = np.asarray(sigmas, dtype=np.float64)[reg]
    st = ss + (0.0 if cdt is None else 1.0 / cdt)
    xc = (np.arange(nx * ny) % nx + 0.5) * h
    q = ((reg == 0) & (xc < 1.0)).astype(np.float64)
    om, w = level_symmetric(order, 2)
    return Problem(name, 2, nx, ny, 1, (h, h, h), st, ss, q, om, w,
                   meta={"regions": reg, "sigmas": tuple(sigmas), "cdt": cdt})


# Pseudo-scattering thermal radiative transfer (Sec. 4.2): NIF units
TRT_A = 137.199          # radiation constant
TRT_C = 2.9979e4         # speed of light
TRT_DT = 1e-3            # time step (one long step, about 10% of an implosion)
# Table hohlraum_materials: (opacity sigma, heat capacity Cv)
HOHLRAUM_MATERIALS = {"gold": (1e3, 1e5), "helium": (1e-3, 1e-2), "ch": (1e2, 1e3), "hydrogen": (1.0, 1.0)}
HOHLRAUM_T_COLD = 1e-3   # keV: the initial temperature everywhere
HOHLRAUM_T_HOT = 0.4     # keV: the laser-heated parts of the gold wall


def trt_pseudo_scattering(sigma, cv, T, dt=TRT_DT):
    """eq. hohlraum_sigma and eq. hohlraum_q: the pseudo-scattering cross
    section sigma_ps and the gray-body source q_ps of one implicit time step
    (opacity sigma, which is also the absorption opacity, heat capacity Cv,
    temperature T, step dt)."""
    sigma, cv, T = (np.asarray(v, dtype=np.float64) for v in (sigma, cv, T))
    b = 16.0 * np.pi * TRT_A * TRT_C * T ** 3
    den = cv / dt + sigma * b
    sigma_ps = sigma ** 2 * b / den
    q_ps = sigma * TRT_A * TRT_C * T ** 4 - sigma ** 2 * 16.0 * np.pi * TRT_A ** 2 * TRT_C ** 2 * T ** 7 / den
    return sigma_ps, q_ps


HOHLRAUM_REGIONS = ("gold", "gold_hot", "helium", "ch", "hydrogen")


def hohlraum_regions(nx: int, ny: int) -> np.ndarray:
    """Region index per cell (HOHLRAUM_REGIONS, x fastest) of a synthetic 2D
    hohlraum on [0, 2] x [0, 1], decided at cell centres: a gold wall 0.06
    thick along x = 0, 2 and 0.1 thick along y = 0, 1, with laser entrance
    holes |y - 1/2| < 0.2 in the end walls (helium); on the long walls the
    inner half of the thickness is laser-heated for x in [0.55, 0.85] and
    [1.15, 1.45]; helium fill; a capsule of radius 0.25 at the centre, a CH
    shell over 0.2 < r < 0.25 around hydrogen fuel.  Materials left to right
    through the middle: gold (hole), helium, CH, hydrogen, CH, helium, gold."""
    xc = (np.arange(nx) + 0.5) * (2.0 / nx)
    yc = (np.arange(ny) + 0.5) * (1.0 / ny)
    X, Y = np.meshgrid(xc, yc)
    reg = np.full(X.shape, 2, dtype=np.int64)                       # helium
    endwall = ((X < 0.06) | (X > 1.94)) & ~(np.abs(Y - 0.5) < 0.2)
    sidewall = (Y < 0.1) | (Y > 0.9)
    reg[endwall | sidewall] = 0
    hot = ((Y > 0.05) & (Y < 0.1)) | ((Y > 0.9) & (Y < 0.95))
    hot &= ((X > 0.55) & (X < 0.85)) | ((X > 1.15) & (X < 1.45))
    reg[hot] = 1
    r = np.hypot(X - 1.0, Y - 0.5)
    reg[(r < 0.25) & (r >= 0.2)] = 3
    reg[r < 0.2] = 4
    return reg.ravel()


def hohlraum(nx: int, ny: int, sn: int = 8, order: int = 1, name: str = "hohlraum") -> Problem:
    """The hohlraum stand-in (Sec. 4.2) as a transport problem: sigma_t =
    sigma, sigma_s = sigma_ps, and the angular source q_ps in every direction
    (total isotropic density 4 pi q_ps), with sigma_ps and q_ps of
    trt_pseudo_scattering at the cell's temperature: 0.4 keV in the heated
    gold, 1e-3 keV elsewhere.  Vacuum boundaries, S_N of the given order,
    DG order `order`, cells of 2/nx by 1/ny."""
    reg = hohlraum_regions(nx, ny)
    mats = [HOHLRAUM_MATERIALS["gold"], HOHLRAUM_MATERIALS["gold"], HOHLRAUM_MATERIALS["helium"],
            HOHLRAUM_MATERIALS["ch"], HOHLRAUM_MATERIALS["hydrogen"]]
    sig = np.array([mats[k][0] for k in reg])
    cv = np.array([mats[k][1] for k in reg])
    T = np.where(reg == 1, HOHLRAUM_T_HOT, HOHLRAUM_T_COLD)
    sps, qps = trt_pseudo_scattering(sig, cv, T)
    om, w = level_symmetric(sn, 2)
    return Problem(name, 2, nx, ny, 1, (2.0 / nx, 1.0 / ny, 1.0), sig, np.minimum(sps, sig), 4.0 * np.pi * qps,
                   om, w, order=order, meta={"regions": reg})


def inflow_size(dim: int, nx: int, ny: int, nz: int) -> int:
    """Boundary-face nodes per direction in the inflow layout.

    For each direction the inflow faces are, in this order, the upwind x face
    (x = 0 if mu > 0 else x = nx*hx), the upwind y face and (3D) the upwind z
    face.  Node order inside a face: x face ((k*ny + j)*F + (b + 2c)),
    y face ((k*nx + i)*F + (a + 2c)), z face ((j*nx + i)*4 + (a + 2b)),
    F = 2 in 2D and 4 in 3D, node labels in global orientation.
    """
    if dim == 2:
        return 2 * ny + 2 * nx
    return 4 * (ny * nz + nx * nz + nx * ny)


def unit_inflow_on_face(p: Problem, axis: int, high: bool, directions_sign: int) -> np.ndarray:
    """Inflow array [D, nbf]: 1 on every node of the given domain face for the
    directions whose component along `axis` has sign `directions_sign`, else 0.

    Only directions for which that face is upwind receive data; e.g. the face
    x = L (axis 0, high=True) is an inflow face for mu < 0.
    """
    nbf = inflow_size(p.dim, p.nx, p.ny, p.nz)
    out = np.zeros((p.ndirs, nbf))
    F = 2 if p.dim == 2 else 4
    sizes = [p.ny * p.nz * F, p.nx * p.nz * F] + ([p.nx * p.ny * F] if p.dim == 3 else [])
    off = [0, sizes[0], sizes[0] + sizes[1]]
    for d in range(p.ndirs):
        comp = p.omega[d, axis]
        if np.sign(comp) != directions_sign:
            continue
        upwind_is_high = comp < 0
        if upwind_is_high != high:
            continue
        out[d, off[axis]:off[axis] + sizes[axis]] = 1.0
    return out


def patch_source(p: Problem, lo, hi, value: float = 4.0 * math.pi) -> np.ndarray:
    """Per-cell density equal to `value` on the cell box lo <= (i,j[,k]) < hi."""
    q = np.zeros(p.ncells)
    if p.dim == 2:
        for j in range(lo[1], hi[1]):
            for i in range(lo[0], hi[0]):
                q[j * p.nx + i] = value
    else:
        for k in range(lo[2], hi[2]):
            for j in range(lo[1], hi[1]):
                for i in range(lo[0], hi[0]):
                    q[(k * p.ny + j) * p.nx + i] = value
    return q


def fd_cells(p: Problem, count: int = 20, seed: int = 2) -> np.ndarray:
    """Cells for finite-difference checks: non-void cells whose sigma_s <= sigma_t
    clip was inactive, drawn without replacement from default_rng(seed)."""
    ok = p.sigma_t > 0
    if "clipped" in p.meta:
        ok &= ~p.meta["clipped"]
    cand = np.nonzero(ok)[0]
    return np.sort(np.random.default_rng(seed).choice(cand, size=count, replace=False))
