"""Synthetic tight-binding systems (geometry + real-space Slater-Koster blocks).

The paper's structures and SK parameter files are not available, so the
systems here are seeded stand-ins with the same shapes: diamond-lattice
silicon cells (a = 10.26 bohr), amorphous supercells made by a seeded
Gaussian displacement of every atom, an sp3 basis (s, px, py, pz) per atom,
and two-centre hopping integrals that decay as exp(-r/2) up to a strict
10-bohr cutoff.  The overlap uses the same two-centre form scaled by 0.1.

Every real-space block couples the orbitals of atom I (rows) to those of an
image of atom J (columns); its bond vector is d = R_J + L - R_I, the full
vector from atom I to the image of J in lattice cell L.  Both directions
(I, J, L) and (J, I, -L) are listed, so H0(J, I, -L) = H0(I, J, L)^T.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

C_LIGHT = 137.035999084          # speed of light in atomic units
FS_AU = 41.341373335             # one femtosecond in atomic time units
A_SI = 10.26                     # cubic diamond lattice constant (bohr)
R_NN = A_SI * math.sqrt(3.0) / 4.0
CUTOFF = 10.0                    # strict hopping cutoff (bohr)
DECAY = 2.0                      # hopping decay length (bohr)

# Si-like nominal two-centre parameters at the nearest-neighbour distance
# (hartree).  Order: ss-sigma, sp-sigma, pp-sigma, pp-pi.
EPS_S, EPS_P = -0.50, -0.24
V_NOMINAL = np.array([-0.07, 0.09, 0.16, -0.04])
S_SCALE = 0.1

_DIAMOND_BASIS = np.array([
    [0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0],
    [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75], [0.75, 0.75, 0.25],
])


@dataclasses.dataclass
class TBSystem:
    """One periodic tight-binding system, described entirely in real space."""

    name: str
    cell: np.ndarray        # (3, 3) rows are lattice vectors, bohr
    pos: np.ndarray         # (n_atoms, 3) bohr
    norb: int               # orbitals per atom (uniform)
    blk_i: np.ndarray       # (n_blocks,) int32 row atom
    blk_j: np.ndarray       # (n_blocks,) int32 column atom
    blk_d: np.ndarray       # (n_blocks, 3) bond vector R_J + L - R_I
    blk_h0: np.ndarray      # (n_blocks, norb, norb) real
    blk_s: np.ndarray       # (n_blocks, norb, norb) real
    kpts: np.ndarray        # (n_k, 3) cartesian, 1/bohr
    kw: np.ndarray          # (n_k,) weights summing to one
    n_electrons: float      # electrons per k-point (spin-unpolarised, f = 2)
    z_ref: Optional[np.ndarray] = None   # per-atom reference charge; None = ground-state charges
    gamma: Optional[np.ndarray] = None   # (n_atoms, n_atoms) SCC kernel, None = non-SCC
    hubbard_u: float = 0.0
    # (n_blocks, 3, norb, norb) real: dS(d)/dd^alpha, the gradient of each overlap
    # block with respect to the bond vector (= with respect to R_J); zero for the
    # on-site blocks.  Needed by the momentum-matrix coupling; None if not provided.
    blk_ds: Optional[np.ndarray] = None

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_orb(self) -> int:
        return self.n_atoms * self.norb

    @property
    def n_k(self) -> int:
        return int(self.kpts.shape[0])

    @property
    def n_blocks(self) -> int:
        return int(self.blk_i.shape[0])

    @property
    def volume(self) -> float:
        return float(abs(np.linalg.det(self.cell)))

    @property
    def scc(self) -> bool:
        return self.gamma is not None

    def n_pairs(self) -> int:
        """Distinct (I, J) atom pairs, i.e. nonzero blocks of H(k)."""
        return int(np.unique(self.blk_i.astype(np.int64) * self.n_atoms + self.blk_j).size)

    def with_kpts(self, kpts, kw=None) -> "TBSystem":
        kpts = np.ascontiguousarray(np.asarray(kpts, dtype=np.float64).reshape(-1, 3))
        if kw is None:
            kw = np.full(kpts.shape[0], 1.0 / kpts.shape[0])
        return dataclasses.replace(self, kpts=kpts, kw=np.asarray(kw, dtype=np.float64))

    def save(self, path: str) -> None:
        arrays = {f.name: getattr(self, f.name) for f in dataclasses.fields(self)}
        arrays = {k: (np.asarray(v) if v is not None else np.zeros(0)) for k, v in arrays.items()}
        arrays["has_gamma"] = np.asarray(self.gamma is not None)
        arrays["has_z_ref"] = np.asarray(self.z_ref is not None)
        arrays["has_blk_ds"] = np.asarray(self.blk_ds is not None)
        np.savez(path, **arrays)

    @staticmethod
    def load(path: str) -> "TBSystem":
        f = np.load(path, allow_pickle=False)
        kw = {}
        for fld in dataclasses.fields(TBSystem):
            v = f[fld.name]
            kw[fld.name] = v
        kw["name"] = str(kw["name"])
        kw["norb"] = int(kw["norb"])
        kw["n_electrons"] = float(kw["n_electrons"])
        kw["hubbard_u"] = float(kw["hubbard_u"])
        if not bool(f["has_gamma"]):
            kw["gamma"] = None
        if not bool(f["has_z_ref"]):
            kw["z_ref"] = None
        if "has_blk_ds" not in f.files or not bool(f["has_blk_ds"]):
            kw["blk_ds"] = None
        return TBSystem(**kw)


# ---------------------------------------------------------------------------
# Two-centre Slater-Koster blocks (s, px, py, pz), Slater & Koster (1954).
# ---------------------------------------------------------------------------

def sk_block_sp(d: np.ndarray, v: np.ndarray) -> np.ndarray:
    """4x4 block <phi_mu(I)| X |phi_nu(J)> for bond vector d from I to J.

    v = (ss-sigma, sp-sigma, pp-sigma, pp-pi) bond integrals at |d|.
    The s-p element carries the direction cosine of d; the p-s element the
    opposite sign, so the block for -d is the transpose of the block for d.
    """
    r = float(np.linalg.norm(d))
    c = d / r
    vss, vsp, vpps, vppp = v
    b = np.empty((4, 4))
    b[0, 0] = vss
    b[0, 1:] = c * vsp
    b[1:, 0] = -c * vsp
    b[1:, 1:] = np.outer(c, c) * (vpps - vppp) + np.eye(3) * vppp
    return b


def sk_block_sp_grad(d: np.ndarray, v: np.ndarray, dv: np.ndarray) -> np.ndarray:
    """Gradient of sk_block_sp(d, v(|d|)) with respect to d: shape (3, 4, 4).

    v and dv are the bond integrals and their radial derivatives at |d|; with
    c = d / r, dr/dd_a = c_a and dc_i/dd_a = (delta_ia - c_i c_a) / r.
    """
    r = float(np.linalg.norm(d))
    c = d / r
    vss, vsp, vpps, vppp = v
    dss, dsp, dpps, dppp = dv
    dc = (np.eye(3) - np.outer(c, c)) / r            # dc[i, a] = dc_i / dd_a
    g = np.empty((3, 4, 4))
    for a in range(3):
        g[a, 0, 0] = dss * c[a]
        g[a, 0, 1:] = dc[:, a] * vsp + c * dsp * c[a]
        g[a, 1:, 0] = -g[a, 0, 1:]
        dcc = np.outer(dc[:, a], c) + np.outer(c, dc[:, a])
        g[a, 1:, 1:] = dcc * (vpps - vppp) + np.outer(c, c) * (dpps - dppp) * c[a] + np.eye(3) * dppp * c[a]
    return g


def bond_integrals(v0: np.ndarray, r: float) -> np.ndarray:
    """Distance dependence v0 * exp(-(r - R_NN) / DECAY)."""
    return v0 * math.exp(-(r - R_NN) / DECAY)


def bond_integrals_dr(v0: np.ndarray, r: float) -> np.ndarray:
    """Radial derivative of bond_integrals."""
    return -bond_integrals(v0, r) / DECAY


def _images(cell: np.ndarray, reach: float) -> np.ndarray:
    inv = np.linalg.inv(cell)
    heights = 1.0 / np.linalg.norm(inv, axis=0)     # distance between lattice planes
    nmax = [int(math.ceil(reach / h)) + 1 for h in heights]
    rng = [np.arange(-n, n + 1) for n in nmax]
    n = np.stack(np.meshgrid(*rng, indexing="ij"), -1).reshape(-1, 3)
    return n @ cell


def build_blocks(cell, pos, norb, onsite_h, onsite_s, hop_h, hop_s, cutoff=CUTOFF,
                 hop_s_grad=None):
    """List every (I, J, L) with 0 < |d| < cutoff plus the on-site blocks.

    hop_h(d) and hop_s(d) return the norb x norb real blocks for bond d;
    hop_s_grad(d) (optional) the (3, norb, norb) gradient of hop_s, and then a
    sixth array of gradients is returned (zero on site).
    """
    L = _images(cell, cutoff)
    bi, bj, bd, bh, bs, bg = [], [], [], [], [], []
    n = pos.shape[0]
    for i in range(n):
        dvec = (pos[None, :, None, :] + L[None, None, :, :] - pos[i][None, None, None, :])[0]
        r = np.linalg.norm(dvec, axis=-1)                    # (n, n_images)
        for j in range(n):
            for li in np.nonzero(r[j] < cutoff)[0]:
                d = dvec[j, li]
                if r[j, li] < 1e-12:
                    if i != j:
                        raise ValueError("two atoms coincide")
                    bi.append(i); bj.append(j); bd.append(np.zeros(3))
                    bh.append(onsite_h.copy()); bs.append(onsite_s.copy())
                    if hop_s_grad is not None:
                        bg.append(np.zeros((3, norb, norb)))
                else:
                    bi.append(i); bj.append(j); bd.append(d)
                    bh.append(hop_h(d)); bs.append(hop_s(d))
                    if hop_s_grad is not None:
                        bg.append(hop_s_grad(d))
    out = (np.asarray(bi, np.int32), np.asarray(bj, np.int32), np.asarray(bd, np.float64),
           np.asarray(bh, np.float64), np.asarray(bs, np.float64))
    if hop_s_grad is not None:
        out = out + (np.asarray(bg, np.float64).reshape(-1, 3, norb, norb),)
    return out


def gamma_mesh(cell: np.ndarray, mesh) -> tuple:
    """Gamma-centred mesh k = sum_i (n_i / N_i) b_i, n_i = 0..N_i-1, equal weights."""
    recip = 2.0 * math.pi * np.linalg.inv(cell).T           # rows are b_i
    grids = [np.arange(m) / m for m in mesh]
    f = np.stack(np.meshgrid(*grids, indexing="ij"), -1).reshape(-1, 3)
    k = f @ recip
    return np.ascontiguousarray(k), np.full(k.shape[0], 1.0 / k.shape[0])


def min_image_distances(cell: np.ndarray, pos: np.ndarray) -> np.ndarray:
    L = _images(cell, 0.0)
    diff = pos[None, :, None, :] + L[None, None, :, :] - pos[:, None, None, :]
    return np.linalg.norm(diff, axis=-1).min(axis=-1)


def gamma_matrix(cell, pos, u) -> np.ndarray:
    """Ewald-free SCC kernel 1/sqrt(r^2 + U^-2) over minimum-image distances.

    The diagonal (r = 0) equals U, the on-site Hubbard value.
    """
    r = min_image_distances(cell, pos)
    return 1.0 / np.sqrt(r * r + 1.0 / (u * u))


def _sk_params(seed_h, seed_s):
    rh = np.random.default_rng(seed_h)
    rs = np.random.default_rng(seed_s)
    vh = V_NOMINAL * (1.0 + 0.1 * rh.uniform(-1.0, 1.0, 4))
    vs = S_SCALE * np.abs(V_NOMINAL) * (1.0 + 0.1 * rs.uniform(-1.0, 1.0, 4))
    return vh, vs


def _sp_system(name, cell, pos, vh, vs, kmesh, n_electrons, gamma_u=None, cutoff=CUTOFF):
    onsite_h = np.diag([EPS_S, EPS_P, EPS_P, EPS_P])
    onsite_s = np.eye(4)

    def hop_h(d):
        return sk_block_sp(d, bond_integrals(vh, float(np.linalg.norm(d))))

    def hop_s(d):
        return sk_block_sp(d, bond_integrals(vs, float(np.linalg.norm(d))))

    def hop_s_grad(d):
        r = float(np.linalg.norm(d))
        return sk_block_sp_grad(d, bond_integrals(vs, r), bond_integrals_dr(vs, r))

    bi, bj, bd, bh, bs, bg = build_blocks(cell, pos, 4, onsite_h, onsite_s, hop_h, hop_s, cutoff,
                                          hop_s_grad)
    kpts, kw = gamma_mesh(cell, kmesh)
    gam = gamma_matrix(cell, pos, gamma_u) if gamma_u is not None else None
    return TBSystem(name=name, cell=cell, pos=pos, norb=4, blk_i=bi, blk_j=bj, blk_d=bd,
                    blk_h0=bh, blk_s=bs, kpts=kpts, kw=kw, n_electrons=float(n_electrons),
                    z_ref=None, gamma=gam, hubbard_u=float(gamma_u or 0.0), blk_ds=bg)


def diamond_positions(ncell: int) -> tuple:
    cell = np.eye(3) * A_SI * ncell
    shifts = np.stack(np.meshgrid(*[np.arange(ncell)] * 3, indexing="ij"), -1).reshape(-1, 3)
    frac = (shifts[:, None, :] + _DIAMOND_BASIS[None, :, :]).reshape(-1, 3)
    return cell, frac * A_SI


def diamond_supercell(ncell: int, kmesh, n_electrons=None, seed: int = 1001,
                      gamma_u=None, name=None) -> TBSystem:
    ss = np.random.SeedSequence(seed).spawn(3)
    cell, pos = diamond_positions(ncell)
    vh, vs = _sk_params(ss[1], ss[2])
    if n_electrons is None:
        n_electrons = 4 * pos.shape[0]
    return _sp_system(name or f"c-Si{pos.shape[0]}", cell, pos, vh, vs, kmesh, n_electrons, gamma_u)


def amorphous_si(ncell: int, kmesh, sigma: float = 0.3, seed: int = 1002,
                 gamma_u=0.25, n_electrons=None, name=None) -> TBSystem:
    """Diamond supercell with a seeded N(0, sigma^2) displacement per component."""
    ss = np.random.SeedSequence(seed).spawn(3)
    cell, pos = diamond_positions(ncell)
    pos = pos + np.random.default_rng(ss[0]).normal(0.0, sigma, pos.shape)
    vh, vs = _sk_params(ss[1], ss[2])
    if n_electrons is None:
        n_electrons = 4 * pos.shape[0]
    return _sp_system(name or f"a-Si{pos.shape[0]}", cell, pos, vh, vs, kmesh, n_electrons, gamma_u)


def primitive_diamond(vh=None, cutoff: float = 5.0, kmesh=(1, 1, 1)) -> TBSystem:
    """Two-atom fcc primitive cell, nearest neighbours only, S = I (textbook sp3 model)."""
    vh = V_NOMINAL.copy() if vh is None else np.asarray(vh, float)
    a = A_SI
    cell = 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    pos = np.array([[0.0, 0.0, 0.0], [0.25 * a, 0.25 * a, 0.25 * a]])
    onsite_h = np.diag([EPS_S, EPS_P, EPS_P, EPS_P])

    def hop_h(d):
        return sk_block_sp(d, bond_integrals(vh, float(np.linalg.norm(d))))

    def hop_s(d):
        return np.zeros((4, 4))

    bi, bj, bd, bh, bs = build_blocks(cell, pos, 4, onsite_h, np.eye(4), hop_h, hop_s, cutoff)
    kpts, kw = gamma_mesh(cell, kmesh)
    return TBSystem(name="diamond-primitive", cell=cell, pos=pos, norb=4, blk_i=bi, blk_j=bj,
                    blk_d=bd, blk_h0=bh, blk_s=bs, kpts=kpts, kw=kw, n_electrons=8.0)


def linear_chain(n_k: int, a: float = 4.0, eps: float = -0.3, t: float = -0.1,
                 s1: float = 0.0, vacuum: float = 60.0, n_electrons: float = 1.0) -> TBSystem:
    """One s orbital per cell on a line along x; nearest-neighbour hopping t.

    H(k) = eps + 2 t cos(k a) when the overlap hopping s1 is zero.
    """
    cell = np.diag([a, vacuum, vacuum])
    pos = np.zeros((1, 3))

    def hop_h(d):
        return np.array([[t]])

    def hop_s(d):
        return np.array([[s1]])

    bi, bj, bd, bh, bs = build_blocks(cell, pos, 1, np.array([[eps]]), np.array([[1.0]]),
                                      hop_h, hop_s, cutoff=1.5 * a)
    k = np.zeros((n_k, 3))
    k[:, 0] = 2.0 * math.pi * np.arange(n_k) / (a * n_k)
    return TBSystem(name="chain", cell=cell, pos=pos, norb=1, blk_i=bi, blk_j=bj, blk_d=bd,
                    blk_h0=bh, blk_s=bs, kpts=k, kw=np.full(n_k, 1.0 / n_k),
                    n_electrons=float(n_electrons))


# ---------------------------------------------------------------------------
# The named workloads: structure, k-mesh, physics and drive of each.
# ---------------------------------------------------------------------------

CONFIGS = {
    # 8-atom cubic diamond cell, 64 k-points, non-SCC, 16 electrons per cell, x kick.
    "si8_k64": dict(kind="crystal", ncell=1, kmesh=(4, 4, 4), n_electrons=16, scc=False,
                    drive="kick", a0=0.01, dt=0.2, n_steps=1000, seed=1001),
    # 64-atom amorphous cell, 2x2x2 mesh, SCC (U = 0.25), sin^2 pulse.
    "asi64_k8_scc": dict(kind="amorphous", ncell=2, kmesh=(2, 2, 2), n_electrons=None, scc=True,
                         drive="pulse", omega=0.1, t_fs=20.0, a_peak=0.05, dt=0.2,
                         n_steps=5000, seed=1002),
    # 512-atom amorphous cell (2048 orbitals), Gamma plus 7 k-points, SCC, same pulse.
    "asi512_k8_scc": dict(kind="amorphous", ncell=4, kmesh=(2, 2, 2), n_electrons=None, scc=True,
                          drive="pulse", omega=0.1, t_fs=20.0, a_peak=0.05, dt=0.2,
                          n_steps=10000, seed=1003),
    # 216-atom crystal, 6x6x6 mesh, kick.
    "csi216_k216": dict(kind="crystal", ncell=3, kmesh=(6, 6, 6), n_electrons=None, scc=False,
                        drive="kick", a0=0.01, dt=0.2, n_steps=2000, seed=1004),
}


def config_system(name: str) -> TBSystem:
    c = CONFIGS[name]
    u = 0.25 if c["scc"] else None
    if c["kind"] == "crystal":
        return diamond_supercell(c["ncell"], c["kmesh"], c["n_electrons"], c["seed"], u, name)
    return amorphous_si(c["ncell"], c["kmesh"], 0.3, c["seed"], u, c["n_electrons"], name)


def random_cell(n_atoms: int, kmesh=(1, 1, 1), seed: int = 7, gamma_u=None,
                n_electrons=None, min_dist: float = 3.6, name=None) -> TBSystem:
    """n_atoms at seeded random positions in a cubic cell of silicon density.

    Used for ragged sizes (N not a multiple of any tile) and disordered tests.
    """
    ss = np.random.SeedSequence(seed).spawn(3)
    rng = np.random.default_rng(ss[0])
    side = (n_atoms * A_SI ** 3 / 8.0) ** (1.0 / 3.0)
    cell = np.eye(3) * side
    pos = []
    imgs = _images(cell, 0.0)
    while len(pos) < n_atoms:
        p = rng.uniform(0.0, side, 3)
        ok = True
        for q in pos:
            if np.min(np.linalg.norm(p - q + imgs, axis=1)) < min_dist:
                ok = False
                break
        if ok:
            pos.append(p)
    pos = np.asarray(pos)
    vh, vs = _sk_params(ss[1], ss[2])
    if n_electrons is None:
        n_electrons = 4 * n_atoms
    return _sp_system(name or f"random{n_atoms}", cell, pos, vh, vs, kmesh, n_electrons, gamma_u)


def random_hermitian_density(n: int, n_k: int, seed: int = 5, scale: float = 0.05,
                             diag: float = 0.5) -> np.ndarray:
    """Seeded Hermitian matrices (n_k, n, n) shaped like a density: diag + noise.

    Used as a non-stationary starting density where only the equation of
    motion, not the ground state, is being tested.
    """
    rng = np.random.default_rng(seed)
    out = np.empty((n_k, n, n), dtype=np.complex128)
    for k in range(n_k):
        a = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
        out[k] = scale * 0.5 * (a + a.conj().T) + diag * np.eye(n)
    return out
