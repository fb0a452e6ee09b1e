"""Seeded synthetic inputs for the J/K build: molecules, contracted basis sets, densities.

This module draws inputs only. It holds none of the J/K arithmetic: no integrals, no
screening, no digestion. Both the HIP path and the CPU oracle receive what it returns.

Basis layout (shared by every consumer)
---------------------------------------
``shell_atom[ns]``  atom of each shell
``shell_l[ns]``     angular momentum, 0..4
``shell_nprim[ns]`` contraction order K
``shell_off[ns]``   offset of the shell's first primitive in ``prim_exp``/``prim_coef``
``shell_pure[ns]``  0 = Cartesian components, 1 = real solid harmonics (l >= 2 only)
``prim_exp``, ``prim_coef``  exponents and contraction coefficients.

Each coefficient multiplies an unnormalised primitive x^ax y^ay z^az exp(-a r^2)
centred on the shell's atom (paper section 2, the Cartesian primitive Gaussian and the
contraction over K primitives). The coefficients already carry every normalisation
factor: the x^l Cartesian component of each contracted shell has unit norm. With
Racah-normalised solid harmonics (norm 4pi/(2l+1) on the unit sphere, the same as
x^l), every spherical function then has unit norm as well.

Recipes (seed = 240709700 + 10*config + {0: geometry, 1: basis, 2: density})
------------------------------------------------------------------------------
* ``uniform``: atoms uniform in a cube, rejection to a minimum separation.
* ``clusters``: 3-atom clusters (centre atom + two atoms at a bond length along random
  directions at least 60 degrees apart), cluster centres rejection-sampled in a cube of
  side 10.5 * n_clusters^(1/3) bohr at least 8.6 bohr apart.
* exponents: for each l, one even-tempered ladder from the largest to the smallest
  exponent over all primitives of that l; the ladder is cut into contiguous blocks in
  shell order (tightest block first). An l with a single primitive takes the geometric
  mean of the range. Coefficients are U(0.2, 1) before normalisation.
* density: D = 2 C C^T with C (nbf x nocc) the Q factor of an N(0,1) matrix.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 240709700


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def nfunc(l: int, pure: int) -> int:
    return 2 * l + 1 if (pure and l >= 2) else ncart(l)


@dataclass
class Molecule:
    coords: np.ndarray          # (natom, 3) bohr
    shell_atom: np.ndarray      # int32
    shell_l: np.ndarray         # int32
    shell_nprim: np.ndarray     # int32
    shell_off: np.ndarray       # int32
    shell_pure: np.ndarray      # int32
    prim_exp: np.ndarray        # float64
    prim_coef: np.ndarray       # float64
    D: np.ndarray               # (nbf, nbf) float64, symmetric
    thresh: float
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def natom(self) -> int:
        return int(self.coords.shape[0])

    @property
    def nshell(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def nbf(self) -> int:
        return int(sum(nfunc(int(l), int(p)) for l, p in zip(self.shell_l, self.shell_pure)))

    @property
    def nbf_cart(self) -> int:
        return int(sum(ncart(int(l)) for l in self.shell_l))

    def ao_offsets(self) -> np.ndarray:
        n = [nfunc(int(l), int(p)) for l, p in zip(self.shell_l, self.shell_pure)]
        return np.concatenate([[0], np.cumsum(n)]).astype(np.int64)


# --------------------------------------------------------------------------- geometry

def _uniform_cube(rng, natom, side, dmin):
    pts = []
    tries = 0
    while len(pts) < natom:
        p = rng.uniform(0.0, side, size=3)
        tries += 1
        if tries > 1_000_000:
            raise RuntimeError("rejection sampling did not converge")
        if all(np.linalg.norm(p - q) >= dmin for q in pts):
            pts.append(p)
    return np.array(pts)


def _random_unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def _clusters(rng, natom, bond=1.8, centre_sep=8.6):
    ncl = (natom + 2) // 3
    side = 10.5 * ncl ** (1.0 / 3.0)
    centres = []
    tries = 0
    while len(centres) < ncl:
        p = rng.uniform(0.0, side, size=3)
        tries += 1
        if tries > 5_000_000:
            raise RuntimeError("cluster placement did not converge")
        if all(np.linalg.norm(p - q) >= centre_sep for q in centres):
            centres.append(p)
    atoms = []
    for ic, c in enumerate(centres):
        nat = min(3, natom - 3 * ic)
        atoms.append(c)
        if nat >= 2:
            u1 = _random_unit(rng)
            atoms.append(c + bond * u1)
        if nat >= 3:
            while True:
                u2 = _random_unit(rng)
                if float(np.dot(u1, u2)) <= 0.5:      # angle >= 60 degrees
                    break
            atoms.append(c + bond * u2)
    return np.array(atoms[:natom])


# --------------------------------------------------------------------------- basis

def _dfact(n: int) -> float:
    r = 1.0
    while n > 1:
        r *= n
        n -= 2
    return r


def _norm_coefs(l, exps, coefs):
    """Scale coefficients so that the contracted x^l component has unit norm.

    <x^l g_i | x^l g_j> = (2l-1)!! / (2 s)^l * (pi / s)^(3/2) with s = a_i + a_j.
    """
    s = exps[:, None] + exps[None, :]
    ov = _dfact(2 * l - 1) / (2.0 * s) ** l * (math.pi / s) ** 1.5
    n2 = float(coefs @ ov @ coefs)
    return coefs / math.sqrt(n2)


def _atom_basis(rng, shells, amin, amax):
    """shells: list of (l, K). Returns list of (l, exps, coefs) for one atom type."""
    by_l = {}
    for l, k in shells:
        by_l.setdefault(l, []).append(k)
    ladder = {}
    for l, ks in by_l.items():
        ptot = sum(ks)
        if ptot == 1:
            ladder[l] = np.array([math.sqrt(amin * amax)])
        else:
            ladder[l] = amax * (amin / amax) ** (np.arange(ptot) / (ptot - 1))
    used = {l: 0 for l in by_l}
    out = []
    for l, k in shells:
        e = ladder[l][used[l]:used[l] + k].copy()
        used[l] += k
        c = rng.uniform(0.2, 1.0, size=k)
        out.append((l, e, _norm_coefs(l, e, c)))
    return out


def _assemble(coords, atom_basis, pure_from_l, thresh, name, rng_d, nocc):
    sa, sl, sn, so, sp, pe, pc = [], [], [], [], [], [], []
    off = 0
    for ia in range(coords.shape[0]):
        for l, e, c in atom_basis:
            sa.append(ia)
            sl.append(l)
            sn.append(len(e))
            so.append(off)
            sp.append(1 if (l >= 2 and l >= pure_from_l) else 0)
            pe.extend(e.tolist())
            pc.extend(c.tolist())
            off += len(e)
    mol = Molecule(coords=np.ascontiguousarray(coords, dtype=np.float64),
                   shell_atom=np.array(sa, np.int32), shell_l=np.array(sl, np.int32),
                   shell_nprim=np.array(sn, np.int32), shell_off=np.array(so, np.int32),
                   shell_pure=np.array(sp, np.int32), prim_exp=np.array(pe, np.float64),
                   prim_coef=np.array(pc, np.float64), D=None, thresh=thresh, name=name)
    mol.D = random_density(rng_d, mol.nbf, nocc)
    mol.meta["nocc"] = nocc
    return mol


def nuclear_charges(mol: Molecule) -> np.ndarray:
    """Integer nuclear charges that make the molecule neutral with its occupied count: 2 nocc
    electrons spread over the atoms as evenly as integers allow (the first atoms take the
    remainder). The synthetic molecules have no elements; an SCF needs some charges."""
    nel = 2 * int(mol.meta.get("nocc", 1))
    z = np.full(mol.natom, nel // mol.natom, dtype=np.float64)
    z[: nel % mol.natom] += 1.0
    return z


def random_density(rng, nbf, nocc):
    nocc = min(nocc, nbf)
    a = rng.normal(size=(nbf, nocc))
    q, _ = np.linalg.qr(a)
    return np.ascontiguousarray(2.0 * q @ q.T)


# --------------------------------------------------------------------------- configs

BASIS_3S2P1D = [(0, 6), (0, 1), (0, 1), (1, 3), (1, 1), (2, 1)]
BASIS_3S2P1D1F = [(0, 6), (0, 1), (0, 1), (1, 3), (1, 1), (2, 1), (3, 1)]


def make_config(k: int, natom: int | None = None) -> Molecule:
    """Config k (1..4) of the benchmark suite; ``natom`` overrides the atom count
    (same recipe, smaller molecule) for quick parity cases."""
    g = np.random.default_rng(SEED_BASE + 10 * k + 0)
    b = np.random.default_rng(SEED_BASE + 10 * k + 1)
    d = np.random.default_rng(SEED_BASE + 10 * k + 2)
    if k == 1:
        n = natom or 6
        coords = _uniform_cube(g, n, 6.0, 1.8)
        basis = _atom_basis(b, [(0, 3), (0, 3), (0, 3), (1, 2)], 0.1, 10.0)
        return _assemble(coords, basis, 99, 0.0, "cfg1", d, 8 if natom is None else max(1, n + 2))
    if k in (2, 4):
        n = natom or (64 if k == 2 else 256)
        coords = _clusters(g, n)
        basis = _atom_basis(b, BASIS_3S2P1D, 0.15, 3000.0)
        nocc = (160 if k == 2 else 640) if natom is None else max(1, int(round(2.5 * n)))
        return _assemble(coords, basis, 2, 1e-12, f"cfg{k}", d, nocc)
    if k == 3:
        n = natom or 32
        side = 10.5 * (n / 32.0) ** (1.0 / 3.0)
        coords = _uniform_cube(g, n, side, 1.8)
        ks = b.integers(1, 4, size=11)
        shells = [(0, int(ks[0])), (0, int(ks[1])), (0, int(ks[2])), (0, int(ks[3])),
                  (1, int(ks[4])), (1, int(ks[5])), (1, int(ks[6])),
                  (2, int(ks[7])), (2, int(ks[8])), (3, int(ks[9])), (4, int(ks[10]))]
        basis = _atom_basis(b, shells, 0.1, 50.0)
        nocc = 120 if natom is None else max(1, int(round(3.75 * n)))
        return _assemble(coords, basis, 2, 1e-12, "cfg3", d, nocc)
    raise ValueError(f"unknown config {k}")


def make_batch(nmol: int = 64, amin: int = 10, amax: int = 120) -> list[Molecule]:
    """The batched workload: nmol molecules with round(linspace(amin, amax, nmol)) atoms
    (shuffled), clustered geometry, 3s2p1d1f shells, each with its own density."""
    g = np.random.default_rng(SEED_BASE + 50 + 0)
    b = np.random.default_rng(SEED_BASE + 50 + 1)
    d = np.random.default_rng(SEED_BASE + 50 + 2)
    counts = np.round(np.linspace(amin, amax, nmol)).astype(int)
    g.shuffle(counts)
    basis = _atom_basis(b, BASIS_3S2P1D1F, 0.15, 3000.0)
    mols = []
    for i, n in enumerate(counts):
        coords = _clusters(g, int(n))
        mols.append(_assemble(coords, basis, 2, 1e-12, f"cfg5_{i}", d, int(round(2.5 * n))))
    return mols


def custom(coords, shells, amin, amax, pure_from_l=2, thresh=0.0, nocc=None, seed=0):
    """Small ad-hoc molecule: ``shells`` is a list of (l, K) shared by every atom."""
    coords = np.asarray(coords, dtype=np.float64)
    b = np.random.default_rng(SEED_BASE + 1000 + seed)
    d = np.random.default_rng(SEED_BASE + 2000 + seed)
    basis = _atom_basis(b, shells, amin, amax)
    mol = _assemble(coords, basis, pure_from_l, thresh, "custom", d, 1)
    if nocc is None:
        nocc = max(1, mol.nbf // 4)
    mol.D = random_density(d, mol.nbf, nocc)
    return mol
