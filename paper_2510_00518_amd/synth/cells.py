"""Crystal cells for the synthetic workloads: diamond structure, 2-atom FCC
primitive cell and 8-atom simple-cubic conventional cell.

The paper benchmarks on silicon (Results section); its DFT inputs are not
available, so these cells carry silicon's structure and mass with seeded
model force constants instead.
"""
from dataclasses import dataclass

import numpy as np

A_SI = 5.431  # cubic lattice constant, Angstrom (diamond silicon)
M_SI = 28.0   # amu


@dataclass
class Cell:
    """lattice: rows a1, a2, a3 (Angstrom); pos: Cartesian atom positions in the home cell."""
    lattice: np.ndarray   # (3, 3)
    pos: np.ndarray       # (n_at, 3)
    masses: np.ndarray    # (n_at,)

    @property
    def n_at(self):
        return len(self.masses)

    @property
    def nb(self):
        return 3 * self.n_at

    @property
    def volume(self):
        return abs(float(np.linalg.det(self.lattice)))

    @property
    def recip(self):
        """Rows b1, b2, b3 with b_i . a_j = 2 pi delta_ij (1/Angstrom)."""
        return 2.0 * np.pi * np.linalg.inv(self.lattice).T

    def site_xyz(self, atom, cell):
        return self.pos[atom] + np.asarray(cell, dtype=float) @ self.lattice


def diamond_primitive(a=A_SI, mass=M_SI):
    lat = 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    pos = np.array([[0.0, 0.0, 0.0], [0.25 * a, 0.25 * a, 0.25 * a]])
    return Cell(lat, pos, np.full(2, float(mass)))


def diamond_conventional(a=A_SI, mass=M_SI):
    lat = a * np.eye(3)
    fcc = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
    pos = a * np.concatenate([fcc, fcc + 0.25])
    return Cell(lat, pos, np.full(8, float(mass)))


def neighbour_shells(cell, n_shells=3, reach=3, tol=1e-6):
    """Return (distances, pairs) where pairs[s] lists (a, b, cell_vec) with atom a in
    the home cell and atom b in cell `cell_vec` at the s-th shell distance."""
    rng = range(-reach, reach + 1)
    found = []
    for a in range(cell.n_at):
        for b in range(cell.n_at):
            for i in rng:
                for j in rng:
                    for k in rng:
                        d = np.linalg.norm(cell.site_xyz(b, (i, j, k)) - cell.pos[a])
                        if d > tol:
                            found.append((d, a, b, (i, j, k)))
    dists = []
    for d, *_ in sorted(found):
        if not dists or d - dists[-1] > tol:
            dists.append(d)
        if len(dists) == n_shells:
            break
    pairs = [[] for _ in dists]
    for d, a, b, c in found:
        for s, ds in enumerate(dists):
            if abs(d - ds) < tol:
                pairs[s].append((a, b, c))
    for p in pairs:
        p.sort()
    return np.array(dists), pairs
