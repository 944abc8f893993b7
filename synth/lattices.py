"""Lattice generators: CSR neighbour lists with per-entry exchange constants.

Conventions (the material description of the paper's "Material building"
section, held as arrays):
  * ``row_ptr`` int64 [n+1], ``col`` int32 [nnz]: both directions of every
    link are stored, with equal constants (``J[p(i->j)] == J[p(j->i)]``).
  * ``k`` float64 [n] uniaxial constants (None = 0 everywhere), ``axis``
    float64 [n, 3] unit anisotropy axes (None = +z), ``ndir`` float64 [n, 3]
    unit field directions (None = +z), ``kc`` float64 [n] cubic constants
    (None = 0), ``norm`` float64 [n] spin norms (None = 1).
  * Bond b is the b-th CSR entry (i, p) with col[p] > i, taken in row-major
    order; ``Lattice.bonds()`` lists them.
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .splitmix import uniform01, normal01, unit_vectors, splitmix64


@dataclass
class Lattice:
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    J: np.ndarray
    k: Optional[np.ndarray] = None
    axis: Optional[np.ndarray] = None
    ndir: Optional[np.ndarray] = None
    pos: Optional[np.ndarray] = None
    site_type: Optional[np.ndarray] = None
    name: str = ""
    meta: dict = field(default_factory=dict)
    kc: Optional[np.ndarray] = None      # [n] cubic anisotropy constants (None = 0)
    norm: Optional[np.ndarray] = None    # [n] spin norms (None = 1)

    @property
    def nnz(self):
        return int(self.row_ptr[-1])

    @property
    def n_bonds(self):
        return self.nnz // 2

    @property
    def degree(self):
        return np.diff(self.row_ptr)

    @property
    def mean_degree(self):
        return self.nnz / max(self.n, 1)

    def rows(self):
        return np.repeat(np.arange(self.n, dtype=np.int64), self.degree)

    def bonds(self):
        """(i, j, J) of every unordered bond, i < j, in row-major CSR order."""
        r = self.rows()
        sel = self.col.astype(np.int64) > r
        return r[sel], self.col[sel].astype(np.int64), self.J[sel]

    def entry_bond_id(self):
        """Bond id of every CSR entry (both directions map to one bond)."""
        r = self.rows()
        c = self.col.astype(np.int64)
        lo = np.minimum(r, c)
        hi = np.maximum(r, c)
        bi, bj, _ = self.bonds()
        key_b = bi * self.n + bj
        key_e = lo * self.n + hi
        order = np.argsort(key_b)
        pos = np.searchsorted(key_b[order], key_e)
        return order[pos].astype(np.int32)

    def with_bond_J(self, Jb):
        """Copy of the lattice with per-bond constants Jb (row-major bond order)."""
        J = np.asarray(Jb, dtype=np.float64)[self.entry_bond_id()]
        return Lattice(self.n, self.row_ptr, self.col, J, self.k, self.axis,
                       self.ndir, self.pos, self.site_type, self.name, dict(self.meta),
                       self.kc, self.norm)


def from_bonds(n, bi, bj, bJ, **kw):
    """CSR from an unordered bond list; entries of a row sorted by column."""
    bi = np.asarray(bi, dtype=np.int64)
    bj = np.asarray(bj, dtype=np.int64)
    bJ = np.asarray(bJ, dtype=np.float64)
    rows = np.concatenate([bi, bj])
    cols = np.concatenate([bj, bi])
    vals = np.concatenate([bJ, bJ])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Lattice(n, row_ptr, cols.astype(np.int32), vals, **kw)


def isolated(n, **kw):
    """n sites without any exchange link (empty CSR rows)."""
    return Lattice(n, np.zeros(n + 1, dtype=np.int64), np.zeros(0, dtype=np.int32),
                   np.zeros(0, dtype=np.float64), name=f"isolated{n}", **kw)


def sc_periodic(Lx, Ly=None, Lz=None, J=1.0, **kw):
    """Periodic simple-cubic lattice, site index x + Lx*(y + Ly*z); each row
    lists its neighbours in the order +x, -x, +y, -y, +z, -z."""
    Ly = Lx if Ly is None else Ly
    Lz = Lx if Lz is None else Lz
    if min(Lx, Ly, Lz) < 3:
        raise ValueError("periodic sides must be >= 3 (no repeated neighbours)")
    n = Lx * Ly * Lz
    i = np.arange(n, dtype=np.int64)
    x, y, z = i % Lx, (i // Lx) % Ly, i // (Lx * Ly)

    def idx(a, b, c):
        return (a % Lx) + Lx * ((b % Ly) + Ly * (c % Lz))
    nb = np.stack([idx(x + 1, y, z), idx(x - 1, y, z), idx(x, y + 1, z),
                   idx(x, y - 1, z), idx(x, y, z + 1), idx(x, y, z - 1)], axis=1)
    row_ptr = np.arange(0, 6 * n + 1, 6, dtype=np.int64)
    col = nb.reshape(-1).astype(np.int32)
    Jv = np.full(6 * n, float(J))
    pos = np.stack([x, y, z], axis=1).astype(np.float64)
    return Lattice(n, row_ptr, col, Jv, pos=pos, name=f"sc{Lx}x{Ly}x{Lz}", **kw)


def open_chain(n, J=1.0):
    """Open chain 0-1-...-(n-1) with uniform constant J."""
    i = np.arange(n - 1)
    return from_bonds(n, i, i + 1, np.full(n - 1, float(J)), name=f"chain{n}")


def random_tree(n, seed, max_degree=8, jmin=-1.5, jmax=1.5):
    """Random tree: node i > 0 links to an earlier node with free degree;
    per-bond constants uniform in [jmin, jmax] (either sign)."""
    u = uniform01(seed, 2 * n, tag=11)
    deg = np.zeros(n, dtype=np.int64)
    bi, bj = [], []
    for i in range(1, n):
        cand = int(u[i] * i)
        while deg[cand] >= max_degree:
            cand = (cand + 1) % i
        bi.append(cand)
        bj.append(i)
        deg[cand] += 1
        deg[i] += 1
    Jb = jmin + (jmax - jmin) * uniform01(seed, n - 1, tag=12)
    return from_bonds(n, bi, bj, Jb, name=f"tree{n}")


def core_shell_ball(R=20, Rc=16, J_core=1.0, J_shell=0.3, J_int=-0.5,
                    k_core=0.01, k_surf=1.0):
    """Sphere cut from a simple-cubic lattice, centred on a site: sites with
    x^2+y^2+z^2 <= R^2; core r <= Rc.  Core-core bonds J_core, shell-shell
    J_shell, core-shell J_int.  Core sites: k_core along +z.  Surface sites
    (fewer than 6 neighbours): k_surf along the radial direction.  Other shell
    sites: k = 0."""
    r = np.arange(-R, R + 1)
    X, Y, Z = np.meshgrid(r, r, r, indexing="ij")
    X, Y, Z = X.ravel(), Y.ravel(), Z.ravel()
    inside = X * X + Y * Y + Z * Z <= R * R
    X, Y, Z = X[inside], Y[inside], Z[inside]
    n = X.size
    side = 2 * R + 1
    key = (X + R) + side * ((Y + R) + side * (Z + R))
    lut = -np.ones(side ** 3, dtype=np.int64)
    lut[key] = np.arange(n)
    bi, bj = [], []
    for dx, dy, dz in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
        X2, Y2, Z2 = X + dx, Y + dy, Z + dz
        ok = (np.abs(X2) <= R) & (np.abs(Y2) <= R) & (np.abs(Z2) <= R)
        j = -np.ones(n, dtype=np.int64)
        j[ok] = lut[(X2[ok] + R) + side * ((Y2[ok] + R) + side * (Z2[ok] + R))]
        sel = j >= 0
        bi.append(np.arange(n)[sel])
        bj.append(j[sel])
    bi = np.concatenate(bi)
    bj = np.concatenate(bj)
    core = X * X + Y * Y + Z * Z <= Rc * Rc
    ci, cj = core[bi], core[bj]
    Jb = np.where(ci & cj, J_core, np.where(~ci & ~cj, J_shell, J_int))
    lat = from_bonds(n, bi, bj, Jb, name=f"ball{R}")
    deg = lat.degree
    surf = deg < 6
    k = np.where(core, k_core, 0.0)
    k = np.where(surf, k_surf, k)
    axis = np.tile(np.array([0.0, 0.0, 1.0]), (n, 1))
    rad = np.stack([X, Y, Z], axis=1).astype(np.float64)
    norm = np.linalg.norm(rad, axis=1)
    axis[surf] = rad[surf] / norm[surf, None]
    lat.k, lat.axis = k, axis
    lat.pos = rad
    lat.site_type = np.where(core, 0, np.where(surf, 2, 1)).astype(np.int32)
    return lat


def diluted_film(L, d, seed, p_vac=0.1, jmin=0.5, jmax=1.5, k=0.05):
    """L x L x d film, periodic in x and y, open in z; every site vacant with
    probability p_vac; per-bond constants uniform in [jmin, jmax]; uniaxial
    constant k along +z."""
    N = L * L * d
    occ = uniform01(seed, N, tag=21) >= p_vac
    i = np.arange(N, dtype=np.int64)
    x, y, z = i % L, (i // L) % L, i // (L * L)
    new = -np.ones(N, dtype=np.int64)
    new[occ] = np.arange(int(occ.sum()))
    bi, bj = [], []
    for nb, ok in (((x + 1) % L + L * (y + L * z), np.ones(N, bool)),
                   (x + L * ((y + 1) % L + L * z), np.ones(N, bool)),
                   (x + L * (y + L * np.minimum(z + 1, d - 1)), z + 1 < d)):
        sel = occ & ok & occ[nb]
        bi.append(new[i[sel]])
        bj.append(new[nb[sel]])
    bi = np.concatenate(bi)
    bj = np.concatenate(bj)
    Jb = jmin + (jmax - jmin) * uniform01(seed, bi.size, tag=22)
    n = int(occ.sum())
    lat = from_bonds(n, bi, bj, Jb, name=f"film{L}x{L}x{d}")
    lat.k = np.full(n, float(k))
    lat.axis = np.tile(np.array([0.0, 0.0, 1.0]), (n, 1))
    lat.pos = np.stack([x[occ], y[occ], z[occ]], axis=1).astype(np.float64)
    return lat


def film_batch(n_films=256, seed=3, Lmin=16, Lmax=128, dmin=2, dmax=10,
               Tmin=0.2, Tmax=2.0):
    """Uneven batch of diluted films: L uniform in {Lmin..Lmax}, d uniform in
    {dmin..dmax}, each film at its own temperature uniform in [Tmin, Tmax]."""
    u = uniform01(seed, 3 * n_films, tag=31)
    Ls = Lmin + np.minimum((u[0::3] * (Lmax - Lmin + 1)).astype(np.int64), Lmax - Lmin)
    ds = dmin + np.minimum((u[1::3] * (dmax - dmin + 1)).astype(np.int64), dmax - dmin)
    Ts = Tmin + (Tmax - Tmin) * u[2::3]
    films = [diluted_film(int(L), int(d), seed=seed * 1000003 + f)
             for f, (L, d) in enumerate(zip(Ls, ds))]
    return films, Ts


def gradient_lattice(L=32, seed=4, J_mean=1.0, J_sd=0.1, k_max=0.2):
    """Periodic simple-cubic lattice with per-bond constants ~ N(J_mean, J_sd),
    per-site k ~ U[0, k_max] and per-site axes uniform on the sphere."""
    lat = sc_periodic(L)
    nb = lat.n_bonds
    Jb = J_mean + J_sd * normal01(seed, nb, tag=41)
    lat = lat.with_bond_J(Jb)
    lat.k = k_max * uniform01(seed, lat.n, tag=42)
    lat.axis = unit_vectors(seed, lat.n, tag=43)
    lat.name = f"grad-sc{L}"
    return lat


def random_spins(seed, n, batch=None, tag=51):
    """Unit spins uniform on the sphere: (n, 3), or (batch, n, 3)."""
    if batch is None:
        return unit_vectors(seed, n, tag)
    return unit_vectors(seed, n * batch, tag).reshape(batch, n, 3)
