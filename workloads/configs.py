"""Seeded, paper-shaped synthetic systems.

Every physical input of the filter path (effective potential at quadrature
points, atom positions, projector channel parameters, the per-atom coupling
matrices Delta_H and Delta_S, the trial vectors and the k-point) is drawn here
from NumPy PCG64 streams.  The shapes follow the paper's workloads: spectral
hexahedral elements of degree p on Gauss-Lobatto-Legendre nodes (FE
discretization section), 18 s/p/d projectors per atom (two radial functions
per angular momentum), blocks of trial vectors, Chebyshev degree m.

Nothing here evaluates a finite-element table, a projector integral or any
step of the filter.  The only numerical work is sampling the synthetic
Gaussian-well potential at the points where the caller asks for it, which is
input synthesis (in the paper this field comes from the SCF loop).

Random streams: ``SeedSequence(26037 + 1000*config_index).spawn(6)`` in the
order wells, atoms, Delta_H, Delta_S, trial vectors, k-point.
"""

from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

# Synthetic potential: each well is -WELL_DEPTH * exp(-|d|^2 / (2 WELL_WIDTH^2)),
# summed over all periodic images, truncated at |d| < WELL_CUTOFF (the
# truncated tail is below 3e-11 Ha).
WELL_DEPTH = 1.0
WELL_WIDTH = 1.0
WELL_CUTOFF = 7.0

# Real solid harmonic channel (l, m) lists.  m runs -l..l in the order
# l=1: y, z, x;  l=2: xy, yz, 3z^2-r^2, xz, x^2-y^2.
_SPD_FIRST8 = [(0, 0), (1, -1), (1, 0), (1, 1), (2, -2), (2, -1), (2, 0), (2, 1)]


@dataclass(frozen=True)
class ConfigSpec:
    name: str
    index: int
    ncell: tuple
    box: tuple
    degree: int
    nq: int
    natoms: int
    atom_mode: str          # "random" (rejection sampled) or "lattice"
    lattice_a: float
    jitter: float
    rcut: float
    channels: str           # "spd8" (8 channels, one radial), "spd18", "spd27", "max32"
    wells: str              # "random2" or "per_atom"
    nstates: int
    block: int
    cheb_degree: int
    iterations: int
    # Coupling scales.  Delta_H = s_H * sym(A_H);
    # Delta_S = s_S * sym(A_S) / ||sym(A_S)||_2, with A ~ N(0,1).
    # Fixed numbers, chosen once so that ||Delta_S|| * lambda_max(<p|p>) ~ 0.5
    # and s_H ~ 1 / lambda_max(<p|p>) for the channel set in use
    # (lambda_max ~ 0.39 for "spd8" at r_c = 1.5, ~ 1.14 for "spd18" at r_c = 2).
    s_H: float
    s_S: float
    is_complex: bool = False


CONFIGS = {
    # Tiny FP64 periodic cube: L=10, 4^3 cells, p=4, 6 Gauss points/dim,
    # 2 wells, 2 atoms x 8 projectors (r_c = 1.5), 16 states, degree 20.
    "tiny": ConfigSpec(
        name="tiny", index=0, ncell=(4, 4, 4), box=(10.0, 10.0, 10.0),
        degree=4, nq=6, natoms=2, atom_mode="random", lattice_a=0.0,
        jitter=0.0, rcut=1.5, channels="spd8", wells="random2",
        nstates=16, block=16, cheb_degree=20, iterations=3,
        s_H=2.5, s_S=1.25,
    ),
    # Paper-scale block: 20^3 cells at p=6 (1,728,000 DOFs), 8 Gauss
    # points/dim, 128 atoms on a jittered simple-cubic lattice, 18
    # projectors each (r_c = 2), 1024 states in blocks of 256, degree 30.
    "paper": ConfigSpec(
        name="paper", index=1, ncell=(20, 20, 20), box=(40.0, 40.0, 40.0),
        degree=6, nq=8, natoms=128, atom_mode="lattice", lattice_a=5.0,
        jitter=0.25, rcut=2.0, channels="spd18", wells="per_atom",
        nstates=1024, block=256, cheb_degree=30, iterations=3,
        s_H=0.9, s_S=0.45,
    ),
    # A mid-size system with the paper-scale element (p=6, 8 Gauss
    # points, 18 projectors, r_c = 2) on a smaller box: used for parity at
    # sizes the oracle finishes in seconds while spanning many cell tiles.
    "mid": ConfigSpec(
        name="mid", index=5, ncell=(5, 4, 3), box=(10.0, 8.0, 6.0),
        degree=6, nq=8, natoms=3, atom_mode="random", lattice_a=0.0,
        jitter=0.0, rcut=2.0, channels="spd18", wells="per_atom",
        nstates=70, block=40, cheb_degree=12, iterations=2,
        s_H=0.9, s_S=0.45,
    ),
}


def config_names():
    return list(CONFIGS)


@dataclass
class System:
    """All inputs of one operator plus the solver parameters.

    Layouts (shared interface of the oracle and the C ABI):
      cell e = i + nx*(j + ny*k); quadrature point q = qx + nq*(qy + nq*qz)
      veff_q[e, q]   effective potential (Ha) at the Gauss points of cell e
      pos[a, :]      atom position (bohr); rcut[a] augmentation radius
      nproj[a]       projectors of atom a; proj_l/proj_m/proj_sigma are the
                     per-projector channel parameters, atom after atom
      dH, dS         the nproj[a]^2 blocks, row-major, atom after atom
    """

    name: str
    ncell: tuple
    box: tuple
    degree: int
    nq: int
    veff_q: np.ndarray
    pos: np.ndarray
    rcut: np.ndarray
    nproj: np.ndarray
    proj_l: np.ndarray
    proj_m: np.ndarray
    proj_sigma: np.ndarray
    dH: np.ndarray
    dS: np.ndarray
    wells: np.ndarray
    kpoint: np.ndarray
    is_complex: bool
    nstates: int
    block: int
    cheb_degree: int
    iterations: int
    x_seed: int
    spec: ConfigSpec = field(repr=False, default=None)
    # graded mesh: per-axis cell boundaries (ncell[d] + 1 each, 0 .. box[d]);
    # None = uniform cells
    xgrid: tuple = None
    # GGA vector field V_GGA at the Gauss points, [E][3][nq^3]; None = no GGA term
    vgga_q: np.ndarray = field(repr=False, default=None)

    @property
    def ndof(self) -> int:
        return int(np.prod(self.ncell)) * self.degree ** 3

    @property
    def ncells(self) -> int:
        return int(np.prod(self.ncell))

    def dH_blocks(self):
        return _unpack(self.dH, self.nproj)

    def dS_blocks(self):
        return _unpack(self.dS, self.nproj)

    def with_veff(self, veff_q):
        return dataclasses.replace(self, veff_q=np.ascontiguousarray(veff_q, dtype=np.float64))

    def with_dH(self, dH):
        return dataclasses.replace(self, dH=np.ascontiguousarray(dH, dtype=np.float64))

    def trial(self, ncols=None, col0=0):
        """Seeded random-normal trial vectors, shape (ndof, ncols)."""
        n = self.nstates if ncols is None else ncols
        return random_block(self.x_seed, self.ndof, col0, n, self.is_complex)


def _unpack(packed, nproj):
    out, off = [], 0
    for n in nproj:
        n = int(n)
        out.append(packed[off:off + n * n].reshape(n, n))
        off += n * n
    return out


def _channels(kind, rcut):
    if kind == "spd8":
        return [(l, m, rcut / 3.0) for (l, m) in _SPD_FIRST8]
    if kind == "spd18":
        ch = []
        for l in range(3):
            for sig in (rcut / 3.0, rcut / 5.0):
                for m in range(-l, l + 1):
                    ch.append((l, m, sig))
        return ch
    if kind in ("spd27", "max32"):
        # (s, p, d) x three radial widths; "max32" adds d at a fourth width
        # (32 channels, the most the library takes per atom)
        ch = []
        for l in range(3):
            for sig in (rcut / 3.0, rcut / 4.0, rcut / 5.0):
                for m in range(-l, l + 1):
                    ch.append((l, m, sig))
        if kind == "max32":
            ch += [(2, m, rcut / 6.0) for m in range(-2, 3)]
        return ch
    raise ValueError(kind)


def _min_image_dist(a, b, box):
    d = np.asarray(a) - np.asarray(b)
    box = np.asarray(box)
    d -= box * np.round(d / box)
    return float(np.sqrt((d * d).sum()))


def _place_atoms(spec, rng):
    box = np.asarray(spec.box, dtype=np.float64)
    need = 2.0 * spec.rcut + 0.5
    if spec.atom_mode == "lattice":
        nsite = [int(round(b / spec.lattice_a)) for b in box]
        sites = np.array([(i, j, k) for k in range(nsite[2]) for j in range(nsite[1])
                          for i in range(nsite[0])], dtype=np.float64)
        pick = rng.choice(len(sites), size=spec.natoms, replace=False)
        pick.sort()
        pos = (sites[pick] + 0.5) * spec.lattice_a
        pos += rng.uniform(-spec.jitter, spec.jitter, size=pos.shape)
        return np.mod(pos, box)
    pos = []
    tries = 0
    while len(pos) < spec.natoms:
        tries += 1
        if tries > 100000:
            raise RuntimeError("atom placement failed")
        p = rng.uniform(0.0, 1.0, size=3) * box
        if all(_min_image_dist(p, q, box) >= need for q in pos):
            pos.append(p)
    return np.array(pos, dtype=np.float64)


def _gauss_legendre(n):
    # Sampling points for the synthetic potential only.
    return np.polynomial.legendre.leggauss(n)[0]


def sample_wells(wells, ncell, box, nq, depth=WELL_DEPTH, width=WELL_WIDTH,
                 cutoff=WELL_CUTOFF):
    """Gaussian wells sampled at the Gauss points of every cell.

    V(x) = -depth * sum_w sum_images exp(-|x - c_w - L_r|^2 / (2 width^2)),
    terms with |x - c_w - L_r| >= cutoff dropped.  Returns (E, nq^3).
    """
    ncell = np.asarray(ncell)
    box = np.asarray(box, dtype=np.float64)
    h = box / ncell
    eta = _gauss_legendre(nq)
    off1 = [(eta + 1.0) * 0.5 * h[d] for d in range(3)]   # (nq,) per dim
    # local point offsets, q = qx + nq*(qy + nq*qz)
    qz, qy, qx = np.meshgrid(np.arange(nq), np.arange(nq), np.arange(nq), indexing="ij")
    loc = np.stack([off1[0][qx.ravel()], off1[1][qy.ravel()], off1[2][qz.ravel()]], axis=1)
    E = int(np.prod(ncell))
    V = np.zeros((E, nq ** 3))
    r2max = cutoff * cutoff
    for c in np.asarray(wells, dtype=np.float64):
        lo = np.floor((c - cutoff) / h).astype(int)
        hi = np.floor((c + cutoff) / h).astype(int)
        iu = np.arange(lo[0], hi[0] + 1)
        ju = np.arange(lo[1], hi[1] + 1)
        ku = np.arange(lo[2], hi[2] + 1)
        KU, JU, IU = np.meshgrid(ku, ju, iu, indexing="ij")
        IU, JU, KU = IU.ravel(), JU.ravel(), KU.ravel()
        # each unwrapped cell is one (cell, periodic image) pair
        org = np.stack([IU * h[0], JU * h[1], KU * h[2]], axis=1)      # (nc, 3)
        e = (np.mod(IU, ncell[0]) + ncell[0] * (np.mod(JU, ncell[1])
             + ncell[1] * np.mod(KU, ncell[2])))
        d = org[:, None, :] + loc[None, :, :] - c[None, None, :]
        r2 = (d * d).sum(axis=2)
        val = np.where(r2 < r2max, -depth * np.exp(-r2 / (2.0 * width * width)), 0.0)
        np.add.at(V, e, val)
    return V


def two_level_grid(ncell, box, pos, r_fine):
    """Per-axis cell boundaries of a two-level mesh: on the uniform grid of
    ncell[d] cells, a cell whose centre lies within r_fine (periodically) of
    some atom coordinate along that axis is fine, the others coarse, and the
    coarse cells are made twice as long as the fine ones (each axis still
    spans box[d] in ncell[d] cells)."""
    out = []
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    for d in range(3):
        n, L = int(ncell[d]), float(box[d])
        centres = (np.arange(n) + 0.5) * L / n
        fine = np.zeros(n, dtype=bool)
        for x in pos[:, d]:
            dist = np.abs(centres - x)
            dist = np.minimum(dist, L - dist)
            fine |= dist < r_fine
        length = np.where(fine, 1.0, 2.0)
        b = np.concatenate([[0.0], np.cumsum(length)]) * (L / length.sum())
        b[-1] = L
        out.append(b)
    return tuple(out)


def _gauss_1d(bounds, L, nq, lo, hi):
    """Gauss points along one axis of every (cell, periodic image) whose
    interval [b_i, b_{i+1}] + s L meets [lo, hi]: (cell indices, points[n, nq])."""
    eta = _gauss_legendre(nq)
    cells, pts = [], []
    for s in range(int(np.floor(lo / L)) - 1, int(np.floor(hi / L)) + 2):
        for i in range(len(bounds) - 1):
            a, b = bounds[i] + s * L, bounds[i + 1] + s * L
            if a <= hi and b >= lo:
                cells.append(i)
                pts.append(a + 0.5 * (eta + 1.0) * (b - a))
    return np.asarray(cells, dtype=np.int64), np.asarray(pts).reshape(-1, nq)


def sample_centred(centres, ncell, box, nq, xgrid, cutoff, fn, ncomp):
    """Sum over centres c and periodic images of fn(d) at every Gauss point x
    (d = x - c - L_r, terms with |d| >= cutoff dropped), on the uniform
    (xgrid None) or graded grid.  fn maps d[..., 3] to [..., ncomp].
    Returns [E][ncomp][nq^3]."""
    ncell = np.asarray(ncell)
    box = np.asarray(box, dtype=np.float64)
    if xgrid is None:
        xgrid = [np.arange(ncell[d] + 1) * (box[d] / ncell[d]) for d in range(3)]
    E = int(np.prod(ncell))
    out = np.zeros((E, ncomp, nq ** 3))
    for c in np.asarray(centres, dtype=np.float64).reshape(-1, 3):
        ax = [_gauss_1d(np.asarray(xgrid[d]), box[d], nq, c[d] - cutoff, c[d] + cutoff) for d in range(3)]
        (ci, xi), (cj, yj), (ck, zk) = ax
        # d[k, j, i, qz, qy, qx, 3]
        dx = (xi - c[0])[None, None, :, None, None, :]
        dy = (yj - c[1])[None, :, None, None, :, None]
        dz = (zk - c[2])[:, None, None, :, None, None]
        shape = (len(ck), len(cj), len(ci), nq, nq, nq)
        d = np.stack(np.broadcast_arrays(dx, dy, dz), axis=-1).reshape(shape + (3,))
        r2 = (d * d).sum(axis=-1)
        val = np.where((r2 < cutoff * cutoff)[..., None], fn(d), 0.0)     # shape + (ncomp,)
        e = (ci[None, None, :] + ncell[0] * (cj[None, :, None] + ncell[1] * ck[:, None, None])).ravel()
        val = val.reshape(len(e), nq ** 3, ncomp).transpose(0, 2, 1)
        np.add.at(out, e, val)
    return out


def sample_wells_graded(wells, ncell, box, nq, xgrid, depth=WELL_DEPTH, width=WELL_WIDTH,
                        cutoff=WELL_CUTOFF):
    """sample_wells on a uniform or graded grid: (E, nq^3)."""
    fn = lambda d: (-depth * np.exp(-(d * d).sum(axis=-1) / (2.0 * width * width)))[..., None]
    return sample_centred(wells, ncell, box, nq, xgrid, cutoff, fn, 1)[:, 0, :]


def sample_gga(centres, ncell, box, nq, xgrid=None, amp=0.05, width=WELL_WIDTH, cutoff=WELL_CUTOFF):
    """Synthetic GGA field (the gradient correction is a vector field): the
    gradient of amp * sum exp(-|d|^2 / (2 width^2)) over centres and images,
    i.e. -amp d / width^2 exp(-|d|^2 / (2 width^2)); [E][3][nq^3]."""
    def fn(d):
        g = np.exp(-(d * d).sum(axis=-1) / (2.0 * width * width))
        return (-amp / (width * width)) * d * g[..., None]
    return sample_centred(centres, ncell, box, nq, xgrid, cutoff, fn, 3)


def with_two_level_gga(system, r_fine=1.0, gga_amp=0.05, graded=True, gga=True):
    """The system on a two-level mesh around its atoms (graded=True) and/or
    with a GGA field centred on its wells (gga=True); the potential is
    resampled at the new Gauss points."""
    xg = two_level_grid(system.ncell, system.box, system.pos, r_fine) if graded else None
    vq = system.veff_q
    if graded and len(system.wells):
        vq = sample_wells_graded(system.wells, system.ncell, system.box, system.nq, xg)
    vg = None
    if gga:
        centres = system.wells if len(system.wells) else system.pos
        vg = np.ascontiguousarray(sample_gga(centres, system.ncell, system.box, system.nq, xg, amp=gga_amp))
    return dataclasses.replace(system, xgrid=xg, veff_q=np.ascontiguousarray(vq), vgga_q=vg)


def random_block(seed, nrows, col0, ncols, is_complex=False):
    """Random-normal columns col0..col0+ncols-1, reproducible per 16-column chunk.

    Chunk j is drawn from PCG64(SeedSequence(seed, spawn_key=(j,))), so any
    column range can be regenerated without drawing the others.
    """
    CH = 16
    out = np.empty((nrows, ncols), dtype=np.complex128 if is_complex else np.float64)
    j0, j1 = col0 // CH, (col0 + ncols - 1) // CH
    for j in range(j0, j1 + 1):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(j,))))
        blk = rng.standard_normal((nrows, CH))
        if is_complex:
            blk = (blk + 1j * rng.standard_normal((nrows, CH))) / np.sqrt(2.0)
        a = max(col0, j * CH)
        b = min(col0 + ncols, (j + 1) * CH)
        out[:, a - col0:b - col0] = blk[:, a - j * CH:b - j * CH]
    return out


def _sym_gaussian(rng, n):
    A = rng.standard_normal((n, n))
    return 0.5 * (A + A.T)


def make_system(name_or_spec, veff=True) -> System:
    spec = CONFIGS[name_or_spec] if isinstance(name_or_spec, str) else name_or_spec
    ss = np.random.SeedSequence(26037 + 1000 * spec.index).spawn(6)
    rng_w, rng_a, rng_h, rng_s, rng_x, rng_k = [np.random.Generator(np.random.PCG64(s)) for s in ss]
    box = np.asarray(spec.box, dtype=np.float64)

    pos = _place_atoms(spec, rng_a)
    if spec.wells == "random2":
        wells = rng_w.uniform(0.0, 1.0, size=(2, 3)) * box
    elif spec.wells == "per_atom":
        wells = pos.copy()
    else:
        raise ValueError(spec.wells)

    ch = _channels(spec.channels, spec.rcut)
    npj = len(ch)
    nproj = np.full(spec.natoms, npj, dtype=np.int32)
    proj_l = np.tile(np.array([c[0] for c in ch], dtype=np.int32), spec.natoms)
    proj_m = np.tile(np.array([c[1] for c in ch], dtype=np.int32), spec.natoms)
    proj_sigma = np.tile(np.array([c[2] for c in ch], dtype=np.float64), spec.natoms)

    dH, dS = [], []
    for _ in range(spec.natoms):
        dH.append((spec.s_H * _sym_gaussian(rng_h, npj)).ravel())
    for _ in range(spec.natoms):
        A = _sym_gaussian(rng_s, npj)
        dS.append((spec.s_S * A / np.linalg.norm(A, 2)).ravel())

    k = np.zeros(3)
    if spec.is_complex:
        k = 2.0 * np.pi * rng_k.uniform(0.0, 0.5, size=3) / box

    E = int(np.prod(spec.ncell))
    vq = (sample_wells(wells, spec.ncell, box, spec.nq) if veff
          else np.zeros((E, spec.nq ** 3)))
    return System(
        name=spec.name, ncell=tuple(spec.ncell), box=tuple(float(b) for b in box),
        degree=spec.degree, nq=spec.nq, veff_q=np.ascontiguousarray(vq),
        pos=pos, rcut=np.full(spec.natoms, spec.rcut), nproj=nproj,
        proj_l=proj_l, proj_m=proj_m, proj_sigma=proj_sigma,
        dH=np.concatenate(dH) if dH else np.zeros(0),
        dS=np.concatenate(dS) if dS else np.zeros(0),
        wells=wells, kpoint=k, is_complex=spec.is_complex,
        nstates=spec.nstates, block=spec.block, cheb_degree=spec.cheb_degree,
        iterations=spec.iterations, x_seed=int(ss[4].generate_state(1)[0]), spec=spec,
    )


def custom_system(ncell, box, degree, nq, pos=(), rcut=1.5, channels="spd8",
                  wells=(), s_H=0.5, s_S=0.5, seed=7, nstates=8, kpoint=(0, 0, 0),
                  is_complex=False) -> System:
    """A small hand-specified system (tests of special cases)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    na = len(pos)
    ch = _channels(channels, rcut)
    npj = len(ch)
    dH = [(s_H * _sym_gaussian(rng, npj)).ravel() for _ in range(na)]
    dS = []
    for _ in range(na):
        A = _sym_gaussian(rng, npj)
        dS.append((s_S * A / np.linalg.norm(A, 2)).ravel())
    E = int(np.prod(ncell))
    wells = np.asarray(wells, dtype=np.float64).reshape(-1, 3)
    vq = sample_wells(wells, ncell, box, nq) if len(wells) else np.zeros((E, nq ** 3))
    return System(
        name="custom", ncell=tuple(ncell), box=tuple(float(b) for b in box),
        degree=degree, nq=nq, veff_q=vq, pos=pos, rcut=np.full(na, float(rcut)),
        nproj=np.full(na, npj, dtype=np.int32),
        proj_l=np.tile(np.array([c[0] for c in ch], dtype=np.int32), na),
        proj_m=np.tile(np.array([c[1] for c in ch], dtype=np.int32), na),
        proj_sigma=np.tile(np.array([c[2] for c in ch]), na),
        dH=np.concatenate(dH) if dH else np.zeros(0),
        dS=np.concatenate(dS) if dS else np.zeros(0),
        wells=wells, kpoint=np.asarray(kpoint, dtype=np.float64), is_complex=is_complex,
        nstates=nstates, block=nstates, cheb_degree=10, iterations=1,
        x_seed=int(rng.integers(1, 2 ** 62)), spec=None,
    )


def batch_systems(count=24, seed=26037 + 4000, small=False, complex_=False):
    """Independent problems of uneven size for the batched filter: cubes of
    6-14 cells of degree-5 elements (7 Gauss points), 8-64 PAW atoms of 18
    projectors on a jittered lattice, 64-384 states (small=True: 2-4 cells
    of degree 2-4, 0-2 atoms, 8-24 states, for parity tests).  complex_=True
    gives complex (k-point) operators with the Bloch vector drawn per problem
    in reduced coordinates kappa in [0, 0.5)^3, k_d = 2 pi kappa_d / L_d
    (drawn after the problem's other inputs).  Seeded; no arithmetic of the
    method here."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    out = []
    for i in range(count):
        if small:
            n = tuple(int(v) for v in rng.integers(2, 5, size=3))
            degree = int(rng.integers(2, 5))
            nq = degree + 2
            h = 1.25
            box = tuple(h * v for v in n)
            na = int(rng.integers(0, 3))
            pos = rng.uniform(0.0, 1.0, size=(na, 3)) * np.asarray(box)
            nst = int(rng.choice([8, 16, 24]))
            s = custom_system(n, box, degree, nq, pos=pos, rcut=1.0, channels="spd8",
                              wells=rng.uniform(0.0, 1.0, size=(2, 3)) * np.asarray(box),
                              s_H=0.5, s_S=0.4, seed=int(rng.integers(1, 2 ** 31)), nstates=nst)
        else:
            c = int(rng.integers(6, 15))
            n = (c, c, c)
            degree, nq = 5, 7
            h = 2.0
            box = tuple(h * v for v in n)
            na = int(rng.integers(8, 65))
            a = (np.prod(box) / na) ** (1.0 / 3.0)
            g = int(np.ceil(na ** (1.0 / 3.0)))
            grid = np.array([(x, y, z) for z in range(g) for y in range(g) for x in range(g)], dtype=np.float64)
            pos = (grid[:na] + 0.5) * (np.asarray(box) / g) + rng.normal(0.0, 0.1 * a, size=(na, 3))
            nst = int(rng.choice([64, 128, 192, 256, 384]))
            s = custom_system(n, box, degree, nq, pos=pos, rcut=1.8, channels="spd18",
                              wells=rng.uniform(0.0, 1.0, size=(4, 3)) * np.asarray(box),
                              s_H=0.9, s_S=0.45, seed=int(rng.integers(1, 2 ** 31)), nstates=nst)
        if complex_:
            kappa = rng.uniform(0.0, 0.5, size=3)
            s = dataclasses.replace(s, kpoint=2.0 * np.pi * kappa / np.asarray(box, dtype=np.float64),
                                    is_complex=True)
        out.append(s)
    return out
