"""Seeded synthetic workloads for the SHG integral engine.

This module only draws random geometry and basis data and builds neighbour
lists. It contains none of the integral arithmetic, so both the HIP path and
the CPU oracle can take their inputs from here.

Basis shells follow the problem statement of the two-center integrals
(Sec. II, eq. contracted_phi): a shell is a center, an angular momentum l,
K exponents and K raw contraction coefficients (the library applies the
normalisation N_l itself).

Workloads (all seeded with ``1000 + k`` for workload k):

1. ``overlap200``    200 isolated atom pairs, l in {0,1,2}, K=3, overlap only.
2. ``five_ops500``   500 atoms in a 20 bohr cube, 4 shells/atom (l 0..4, K 1..7),
                     all ordered atom pairs within 12 bohr (self pairs included).
3. ``aab2000``       2000 atoms in a 40 bohr cube, orbital l=0..3 (K=5) and
                     uncontracted RI l=0..6 per atom, ordered pairs within 10 bohr.
4. ``molecules256``  256 molecules of 10..400 atoms (log-uniform), config-2 basis,
                     unordered intra-molecule shell pairs within 12 bohr.
5. ``screen5000``    5000 atoms in a 60 bohr cube, config-2 basis, ordered
                     shell pairs within 12 bohr.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import cKDTree


@dataclass
class Shells:
    """Structure-of-arrays shell table (host, numpy)."""
    center: np.ndarray      # (n, 3) float64, bohr
    l: np.ndarray           # (n,) int32
    nprim: np.ndarray       # (n,) int32
    prim_off: np.ndarray    # (n,) int64
    exps: np.ndarray        # (P,) float64, bohr^-2, sorted descending per shell
    coefs: np.ndarray       # (P,) float64, raw contraction coefficients
    atom: np.ndarray        # (n,) int32 atom index of each shell

    @property
    def n(self) -> int:
        return int(self.l.shape[0])

    def subset(self, idx) -> "Shells":
        """Shells `idx` repacked into a fresh table."""
        idx = np.asarray(idx, dtype=np.int64)
        nprim = self.nprim[idx].astype(np.int32)
        off = np.zeros(len(idx), dtype=np.int64)
        if len(idx):
            off[1:] = np.cumsum(nprim[:-1], dtype=np.int64)
        sel = np.concatenate([np.arange(self.prim_off[i], self.prim_off[i] + self.nprim[i])
                              for i in idx]) if len(idx) else np.zeros(0, np.int64)
        return Shells(self.center[idx].copy(), self.l[idx].astype(np.int32), nprim, off,
                      self.exps[sel].copy(), self.coefs[sel].copy(), self.atom[idx].astype(np.int32))


@dataclass
class Workload:
    name: str
    shells: Shells
    pairs: np.ndarray                      # (n, 2) int32 shell indices (a on A, b on B)
    ops: tuple = ("overlap",)
    omega: dict = field(default_factory=dict)
    deriv: bool = False
    aux: Shells | None = None              # RI shells for the (ab a~) workload
    triples: np.ndarray | None = None      # (n, 3) int32 (a on A, a~ on A, b on B)
    mol_of_pair: np.ndarray | None = None  # (n,) molecule id for batched serving
    n_atoms: int = 0

    def block_sizes(self) -> np.ndarray:
        if self.triples is not None:
            la = self.shells.l[self.triples[:, 0]].astype(np.int64)
            lt = self.aux.l[self.triples[:, 1]].astype(np.int64)
            lb = self.shells.l[self.triples[:, 2]].astype(np.int64)
            return (2 * la + 1) * (2 * lt + 1) * (2 * lb + 1)
        la = self.shells.l[self.pairs[:, 0]].astype(np.int64)
        lb = self.shells.l[self.pairs[:, 1]].astype(np.int64)
        return (2 * la + 1) * (2 * lb + 1)

    def out_offsets(self) -> tuple[np.ndarray, int]:
        """Exclusive prefix sum of the block sizes (element offsets) and the total."""
        sz = self.block_sizes()
        off = np.zeros(len(sz), dtype=np.int64)
        if len(sz):
            off[1:] = np.cumsum(sz[:-1])
        return off, int(sz.sum())


OMEGA = {"overlap": 0.0, "coulomb": 0.0, "erfc": 0.11, "erf": 0.33, "gauss": 1.0}
FIVE_OPS = ("overlap", "coulomb", "erfc", "erf", "gauss")


def _log_uniform(rng, lo, hi, size):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size))


def random_shells(rng, centers, l_list, k_list, exp_lo, exp_hi, atom_of):
    """Shells with log-uniform exponents (sorted descending) and U[0.1,1] coefficients."""
    n = len(l_list)
    nprim = np.asarray(k_list, dtype=np.int32)
    off = np.zeros(n, dtype=np.int64)
    if n:
        off[1:] = np.cumsum(nprim[:-1], dtype=np.int64)
    exps = np.empty(int(nprim.sum()))
    coefs = np.empty(int(nprim.sum()))
    for i in range(n):
        k = int(nprim[i])
        e = np.sort(_log_uniform(rng, exp_lo, exp_hi, k))[::-1]
        c = rng.uniform(0.1, 1.0, k)
        exps[off[i]:off[i] + k] = e
        coefs[off[i]:off[i] + k] = c
    return Shells(np.asarray(centers, dtype=np.float64).reshape(n, 3),
                  np.asarray(l_list, dtype=np.int32), nprim, off, exps, coefs,
                  np.asarray(atom_of, dtype=np.int32))


def _normalise_l2(sh: Shells) -> None:
    """Scale each shell's raw coefficients to unit 2-norm (reproducibility only:
    results do not depend on the scale of c, the library applies N_l)."""
    for i in range(sh.n):
        s = slice(sh.prim_off[i], sh.prim_off[i] + sh.nprim[i])
        sh.coefs[s] /= np.linalg.norm(sh.coefs[s])


def _atom_basis(rng, pos, shells_per_atom=4, lmax=4, kmax=7, exp_lo=0.05, exp_hi=50.0):
    na = len(pos)
    ls = rng.integers(0, lmax + 1, size=(na, shells_per_atom))
    ks = rng.integers(1, kmax + 1, size=(na, shells_per_atom))
    centers = np.repeat(pos, shells_per_atom, axis=0)
    atom_of = np.repeat(np.arange(na), shells_per_atom)
    return random_shells(rng, centers, ls.ravel(), ks.ravel(), exp_lo, exp_hi, atom_of)


def atom_pairs_within(pos, cutoff, ordered=True, include_self=True):
    """Atom pairs (i, j) with |R_i - R_j| <= cutoff, as an (m, 2) int64 array."""
    tree = cKDTree(pos)
    pr = tree.query_pairs(cutoff, output_type="ndarray").astype(np.int64)
    parts = [pr]
    if ordered:
        parts.append(pr[:, ::-1])
    if include_self:
        idx = np.arange(len(pos), dtype=np.int64)
        parts.append(np.stack([idx, idx], axis=1))
    ap = np.concatenate(parts, axis=0)
    order = np.lexsort((ap[:, 1], ap[:, 0]))
    return ap[order]


def expand_shell_pairs(atom_pairs, shells_per_atom):
    """All shell pairs of each atom pair (shells of atom i are i*s .. i*s+s-1)."""
    s = shells_per_atom
    a = atom_pairs[:, 0:1] * s + np.arange(s)[None, :]
    b = atom_pairs[:, 1:2] * s + np.arange(s)[None, :]
    sa = np.repeat(a, s, axis=1).reshape(-1)
    sb = np.tile(b, (1, s)).reshape(-1)
    return np.stack([sa, sb], axis=1).astype(np.int32)


def overlap200(seed: int = 1001, n: int = 200) -> Workload:
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.5, 5.0, n)
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    centers = np.zeros((2 * n, 3))
    centers[1::2] = d[:, None] * u
    ls = rng.integers(0, 3, size=2 * n)
    sh = random_shells(rng, centers, ls, np.full(2 * n, 3), 0.1, 10.0, np.arange(2 * n))
    _normalise_l2(sh)
    pairs = np.stack([np.arange(0, 2 * n, 2), np.arange(1, 2 * n, 2)], axis=1).astype(np.int32)
    return Workload("overlap200", sh, pairs, ("overlap",), dict(OMEGA), False, n_atoms=2 * n)


def five_ops500(seed: int = 1002, n_atoms: int = 500, box: float = 20.0,
                cutoff: float = 12.0) -> Workload:
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, box, size=(n_atoms, 3))
    sh = _atom_basis(rng, pos)
    ap = atom_pairs_within(pos, cutoff)
    pairs = expand_shell_pairs(ap, 4)
    return Workload("five_ops500", sh, pairs, FIVE_OPS, dict(OMEGA), True, n_atoms=n_atoms)


def aab2000(seed: int = 1003, n_atoms: int = 2000, box: float = 40.0,
            cutoff: float = 10.0) -> Workload:
    """Three-index overlap workload. Each atom carries orbital shells l=0..3 (K=5)
    and uncontracted RI shells l=0..6; a triple is (orbital on X, RI on X,
    orbital on Y) for every ordered atom pair (X, Y) within the cutoff."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, box, size=(n_atoms, 3))
    orb_l = np.tile(np.arange(4), n_atoms)
    orb = random_shells(rng, np.repeat(pos, 4, axis=0), orb_l, np.full(4 * n_atoms, 5),
                        0.05, 50.0, np.repeat(np.arange(n_atoms), 4))
    aux_l = np.tile(np.arange(7), n_atoms)
    aux = random_shells(rng, np.repeat(pos, 7, axis=0), aux_l, np.ones(7 * n_atoms, np.int32),
                        0.1, 20.0, np.repeat(np.arange(n_atoms), 7))
    ap = atom_pairs_within(pos, cutoff)
    triples = aab_triples(ap, 4, 7)
    return Workload("aab2000", orb, np.zeros((0, 2), np.int32), ("aab",), {}, True,
                    aux=aux, triples=triples, n_atoms=n_atoms)


def aab_triples(atom_pairs, orb_per_atom, aux_per_atom):
    """(orbital shell on X, RI shell on X, orbital shell on Y) for each atom pair (X, Y)."""
    no, nx = orb_per_atom, aux_per_atom
    X = atom_pairs[:, 0].astype(np.int64)
    Y = atom_pairs[:, 1].astype(np.int64)
    ia = np.arange(no)
    it = np.arange(nx)
    ib = np.arange(no)
    A, T, B = np.meshgrid(ia, it, ib, indexing="ij")
    A, T, B = A.ravel(), T.ravel(), B.ravel()
    sa = (X[:, None] * no + A[None, :]).ravel()
    st = (X[:, None] * nx + T[None, :]).ravel()
    sb = (Y[:, None] * no + B[None, :]).ravel()
    return np.stack([sa, st, sb], axis=1).astype(np.int32)


def molecules256(seed: int = 1004, n_mol: int = 256, cutoff: float = 12.0,
                 density: float = 0.0625, min_dist: float = 1.0) -> Workload:
    """Uneven molecules: n atoms log-uniform in [10, 400], uniform in a cube of
    the config-2 density with a minimum separation, config-2 basis, unordered
    intra-molecule shell pairs (self pairs included) within the cutoff."""
    rng = np.random.default_rng(seed)
    all_pos, mol_of_atom = [], []
    for m in range(n_mol):
        n = int(round(np.exp(rng.uniform(np.log(10), np.log(400)))))
        side = (n / density) ** (1.0 / 3.0)
        pts = np.empty((0, 3))
        while len(pts) < n:
            p = rng.uniform(0, side, 3)
            if len(pts) == 0 or np.min(np.linalg.norm(pts - p, axis=1)) >= min_dist:
                pts = np.vstack([pts, p])
        # molecules are placed far apart so no cross-molecule pair is in range
        all_pos.append(np.asarray(pts) + np.array([m * 1000.0, 0, 0]))
        mol_of_atom.append(np.full(n, m))
    pos = np.concatenate(all_pos)
    mol = np.concatenate(mol_of_atom)
    sh = _atom_basis(rng, pos)
    ap = atom_pairs_within(pos, cutoff, ordered=False, include_self=True)
    ap = ap[ap[:, 0] <= ap[:, 1]]
    pairs = expand_shell_pairs(ap, 4)
    same = ap[:, 0] == ap[:, 1]
    # for a self atom pair keep each unordered shell pair once
    keep = np.ones(len(pairs), dtype=bool)
    sp = np.repeat(same, 16)
    keep[sp] = pairs[sp, 0] <= pairs[sp, 1]
    pairs = pairs[keep]
    mol_of_pair = mol[sh.atom[pairs[:, 0]]]
    return Workload("molecules256", sh, pairs, FIVE_OPS, dict(OMEGA), True,
                    mol_of_pair=mol_of_pair.astype(np.int32), n_atoms=len(pos))


def screen5000(seed: int = 1005, n_atoms: int = 5000, box: float = 60.0,
               cutoff: float = 12.0) -> Workload:
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, box, size=(n_atoms, 3))
    sh = _atom_basis(rng, pos)
    ap = atom_pairs_within(pos, cutoff)
    pairs = expand_shell_pairs(ap, 4)
    return Workload("screen5000", sh, pairs, ("coulomb", "erfc"), dict(OMEGA), False,
                    n_atoms=n_atoms)


def small_pairs(seed: int, n: int, lmax: int = 4, kmax: int = 7, exp_lo=0.05, exp_hi=50.0,
                dmax: float = 6.0, same_center_frac: float = 0.1) -> Workload:
    """Small random pair list covering every (la, lb) class, for parity tests."""
    rng = np.random.default_rng(seed)
    la = rng.integers(0, lmax + 1, n)
    lb = rng.integers(0, lmax + 1, n)
    ka = rng.integers(1, kmax + 1, n)
    kb = rng.integers(1, kmax + 1, n)
    d = rng.uniform(0.0, dmax, n)
    d[rng.uniform(size=n) < same_center_frac] = 0.0
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    base = rng.uniform(-5, 5, size=(n, 3))
    centers = np.empty((2 * n, 3))
    centers[0::2] = base
    centers[1::2] = base + d[:, None] * u
    ls = np.empty(2 * n, dtype=np.int64)
    ls[0::2], ls[1::2] = la, lb
    ks = np.empty(2 * n, dtype=np.int64)
    ks[0::2], ks[1::2] = ka, kb
    sh = random_shells(rng, centers, ls, ks, exp_lo, exp_hi, np.arange(2 * n))
    pairs = np.stack([np.arange(0, 2 * n, 2), np.arange(1, 2 * n, 2)], axis=1).astype(np.int32)
    return Workload(f"small{n}", sh, pairs, FIVE_OPS, dict(OMEGA), True, n_atoms=2 * n)


def small_triples(seed: int, n: int, lmax: int = 3, ltmax: int = 6, kmax: int = 5,
                  dmax: float = 5.0) -> Workload:
    """Small random (a, a~, b) list: a and a~ share a center, b sits elsewhere."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.0, dmax, n)
    d[rng.uniform(size=n) < 0.1] = 0.0
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    A = rng.uniform(-5, 5, size=(n, 3))
    B = A + d[:, None] * u
    orb_c = np.empty((2 * n, 3))
    orb_c[0::2], orb_c[1::2] = A, B
    orb_l = rng.integers(0, lmax + 1, 2 * n)
    orb_k = rng.integers(1, kmax + 1, 2 * n)
    orb = random_shells(rng, orb_c, orb_l, orb_k, 0.05, 50.0, np.arange(2 * n))
    aux = random_shells(rng, A, rng.integers(0, ltmax + 1, n), np.ones(n, np.int32),
                        0.1, 20.0, np.arange(n))
    triples = np.stack([np.arange(0, 2 * n, 2), np.arange(n), np.arange(1, 2 * n, 2)],
                       axis=1).astype(np.int32)
    return Workload(f"smalltri{n}", orb, np.zeros((0, 2), np.int32), ("aab",), {}, True,
                    aux=aux, triples=triples, n_atoms=2 * n)


WORKLOADS = {1: overlap200, 2: five_ops500, 3: aab2000, 4: molecules256, 5: screen5000}
