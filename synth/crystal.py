"""Synthetic crystal structures, Gamma-centred q-grids and space-group operations.

This module only builds inputs (geometry and bookkeeping).  It contains none of the
scattering-rate arithmetic.

Conventions
-----------
* Lattice vectors are the ROWS of ``A`` (Angstrom).  A site is ``(s, R)`` with ``s`` the
  basis index and ``R`` an integer 3-vector of lattice coordinates; its Cartesian position
  is ``R @ A + tau[s]``.
* Reciprocal vectors are the rows of ``B = 2 pi inv(A).T`` so that ``A @ B.T = 2 pi I``.
* A Gamma-centred grid N1 x N2 x N3 has points ``q = sum_d (n_d / N_d) b_d`` with
  ``n_d in [0, N_d)`` and flat index ``iq = n1 + N1 * (n2 + N2 * n3)``.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Crystal:
    name: str
    A: np.ndarray            # (3,3) rows = lattice vectors, Angstrom
    tau: np.ndarray          # (nat,3) Cartesian basis positions, Angstrom
    mass: np.ndarray         # (nat,) amu
    # space-group operations as (T, t): r -> T r + t (Cartesian); always contains identity
    ops: list = field(default_factory=list)

    @property
    def natoms(self) -> int:
        return int(self.tau.shape[0])

    @property
    def nb(self) -> int:
        return 3 * self.natoms

    @property
    def B(self) -> np.ndarray:
        return 2.0 * np.pi * np.linalg.inv(self.A).T

    def position(self, s: int, R) -> np.ndarray:
        return np.asarray(R, dtype=float) @ self.A + self.tau[s]

    def locate(self, r: np.ndarray, tol: float = 1e-6):
        """Return (s, R) of the site at Cartesian position r (raises if none)."""
        Ainv = np.linalg.inv(self.A)
        for s in range(self.natoms):
            f = (r - self.tau[s]) @ Ainv
            Rf = np.rint(f)
            if np.max(np.abs(f - Rf)) < tol:
                return s, tuple(int(x) for x in Rf)
        raise ValueError(f"no site at {r}")


# ----------------------------------------------------------------------------- structures

def _td_rotations() -> list[np.ndarray]:
    """The 24 signed permutation matrices of point group Td (-43m): every coordinate
    permutation combined with an even number of sign flips."""
    mats = []
    for perm in itertools.permutations(range(3)):
        P = np.zeros((3, 3))
        for i, p in enumerate(perm):
            P[i, p] = 1.0
        for signs in itertools.product((1.0, -1.0), repeat=3):
            if np.prod(signs) > 0:
                mats.append(np.diag(signs) @ P)
    assert len(mats) == 24
    return mats


def diamond(a: float = 5.43, mass: float = 28.0) -> Crystal:
    """Two-atom diamond-structure cell (Fd-3m), FCC primitive vectors a/2 (0,1,1),
    (1,0,1), (1,1,0); basis at 0 and a/4 (1,1,1).

    The 48 space-group operations with the origin on atom 0 are the 24 Td operations
    (which fix atom 0) and those 24 composed with inversion through the bond centre
    a/8 (1,1,1), i.e. r -> -T r + a/4 (1,1,1)."""
    A = 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    tau = np.array([[0.0, 0.0, 0.0], [0.25 * a] * 3])
    ops = []
    shift = np.array([0.25 * a] * 3)
    for T in _td_rotations():
        ops.append((T, np.zeros(3)))
    for T in _td_rotations():
        ops.append((-T, shift.copy()))
    cr = Crystal("diamond", A, tau, np.array([mass, mass]), ops)
    check_ops(cr)
    return cr


def wurtzite_like(a: float = 3.25, c_over_a: float = 1.65, u: float = 0.375,
                  masses=(28.0, 14.0)) -> Crystal:
    """Four-atom hexagonal wurtzite-like cell.  Only the identity is used as a symmetry
    operation (the generator does not need the full P6_3mc group for this cell)."""
    c = c_over_a * a
    A = np.array([[a, 0.0, 0.0], [-0.5 * a, 0.5 * np.sqrt(3.0) * a, 0.0], [0.0, 0.0, c]])
    frac = np.array([[1 / 3, 2 / 3, 0.0], [2 / 3, 1 / 3, 0.5],
                     [1 / 3, 2 / 3, u], [2 / 3, 1 / 3, 0.5 + u]])
    tau = frac @ A
    m = np.array([masses[0], masses[0], masses[1], masses[1]])
    return Crystal("wurtzite_like", A, tau, m, [(np.eye(3), np.zeros(3))])


def layered_rhombohedral(a_h: float = 2.82, c_h: float = 14.05,
                         masses=(7.0, 56.0, 16.0, 16.0), z_o: float = 0.26) -> Crystal:
    """Four-atom layered rhombohedral cell (R-3m, LiCoO2-like, light/heavy mass 1:8).
    Rhombohedral primitive vectors from the hexagonal setting; Li at 0, Co at 1/2,
    O at +-z_o along the 3-fold axis.  Only the identity is used as a symmetry operation."""
    ah = np.array([a_h, 0.0, 0.0])
    bh = np.array([-0.5 * a_h, 0.5 * np.sqrt(3.0) * a_h, 0.0])
    ch = np.array([0.0, 0.0, c_h])
    a1 = (2 * ah + bh + ch) / 3.0
    a2 = (-ah + bh + ch) / 3.0
    a3 = (-ah - 2 * bh + ch) / 3.0
    A = np.array([a1, a2, a3])
    cvec = a1 + a2 + a3            # = ch (hexagonal c axis)
    tau = np.array([0.0 * cvec, 0.5 * cvec, z_o * cvec, -z_o * cvec])
    return Crystal("layered_rhombohedral", A, tau, np.array(masses, dtype=float),
                   [(np.eye(3), np.zeros(3))])


def layered_three_atom(a_h: float = 2.82, c_h: float = 14.05,
                       masses=(7.0, 56.0, 16.0), z_o: float = 0.26) -> Crystal:
    """Three-atom cell (9 branches): the layered rhombohedral cell without its second O.
    Only the identity is used as a symmetry operation."""
    full = layered_rhombohedral(a_h, c_h, tuple(masses) + (16.0,), z_o)
    return Crystal("layered_three_atom", full.A, full.tau[:3].copy(),
                   np.array(masses, dtype=float), [(np.eye(3), np.zeros(3))])


def fcc_one_atom(a: float = 3.6, mass: float = 63.5) -> Crystal:
    """One-atom FCC cell (3 branches), primitive vectors a/2 (0,1,1), (1,0,1), (1,1,0).
    Only the identity is used as a symmetry operation."""
    A = 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    return Crystal("fcc_one_atom", A, np.zeros((1, 3)), np.array([mass]),
                   [(np.eye(3), np.zeros(3))])


def ortho_one_atom(a=(3.0, 3.3, 3.6), mass: float = 40.0) -> Crystal:
    """One-atom simple orthorhombic cell (3 branches): orthogonal lattice vectors, so the
    first-Brillouin-zone image of a grid point splits axis by axis.  Only the identity is
    used as a symmetry operation."""
    return Crystal("ortho_one_atom", np.diag(np.asarray(a, dtype=float)), np.zeros((1, 3)),
                   np.array([mass]), [(np.eye(3), np.zeros(3))])


def check_ops(cr: Crystal, tol: float = 1e-8) -> None:
    """Assert every stored operation maps every site onto a site."""
    for T, t in cr.ops:
        for s in range(cr.natoms):
            for R in [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, -1, 0)]:
                cr.locate(T @ cr.position(s, R) + t, tol)


def apply_op(cr: Crystal, op, site):
    T, t = op
    s, R = site
    return cr.locate(T @ cr.position(s, R) + t)


# ----------------------------------------------------------------------------- neighbours

def sites_within(cr: Crystal, center, rc: float, nmax: int = 4):
    """All sites (s, R) within distance rc of the position `center` (Cartesian)."""
    out = []
    rng = range(-nmax, nmax + 1)
    for R in itertools.product(rng, rng, rng):
        for s in range(cr.natoms):
            d = np.linalg.norm(cr.position(s, R) - center)
            if d <= rc + 1e-9:
                out.append((s, tuple(R)))
    return out


def distance(cr: Crystal, a, b) -> float:
    return float(np.linalg.norm(cr.position(*a) - cr.position(*b)))


def shell_distances(cr: Crystal, nshell: int, tol: float = 1e-4, rmax: float = 12.0):
    """Sorted distinct interatomic distances (first nshell shells over all sites)."""
    ds = []
    for s in range(cr.natoms):
        for nb in sites_within(cr, cr.position(s, (0, 0, 0)), rmax):
            d = distance(cr, (s, (0, 0, 0)), nb)
            if d > 1e-6:
                ds.append(d)
    ds = np.sort(np.array(ds))
    shells = [ds[0]]
    for d in ds[1:]:
        if d - shells[-1] > tol:
            shells.append(d)
        if len(shells) >= nshell:
            break
    return shells


# ----------------------------------------------------------------------------- q-grids

def grid_points(grid) -> np.ndarray:
    """(N,3) integer index triples n in flat order iq = n1 + N1*(n2 + N2*n3)."""
    N1, N2, N3 = grid
    n3, n2, n1 = np.meshgrid(np.arange(N3), np.arange(N2), np.arange(N1), indexing="ij")
    return np.stack([n1.ravel(), n2.ravel(), n3.ravel()], axis=1).astype(np.int64)


def flat_index(n, grid) -> np.ndarray:
    n = np.asarray(n) % np.asarray(grid)
    return n[..., 0] + grid[0] * (n[..., 1] + grid[1] * n[..., 2])


def minus_index(grid) -> np.ndarray:
    """For each iq, the flat index of -q folded back into the grid."""
    return flat_index(-grid_points(grid), grid)


def q_cart(cr: Crystal, grid) -> np.ndarray:
    n = grid_points(grid).astype(float)
    return (n / np.asarray(grid, dtype=float)) @ cr.B


def bloch_phase(grid, n, R) -> np.ndarray:
    """exp(i q.R) for grid point n and integer cell R, from an integer reduction so that
    a reciprocal-lattice shift of q gives exactly the same value."""
    grid = np.asarray(grid)
    Ntot = int(np.prod(grid))
    k = np.zeros(np.broadcast(n[..., 0], R[..., 0]).shape, dtype=np.int64)
    for d in range(3):
        k = k + ((n[..., d] * R[..., d]) % grid[d]) * (Ntot // grid[d])
    k %= Ntot
    return np.exp(2j * np.pi * k / Ntot)
