"""Irreducible q1 sets: stars of the cubic point group Oh (which contains inversion,
so time reversal is included) acting on a Gamma-centred mesh.  Representative =
smallest mesh index in the star, weight = star size (weights sum to N)."""
import itertools

import numpy as np

from .harmonic import mesh_coords, mesh_index


def cubic_ops():
    ops = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            S = np.zeros((3, 3))
            for i in range(3):
                S[i, perm[i]] = signs[i]
            ops.append(S)
    return ops


def irreducible_q(cell, mesh):
    """Return (q1 indices int32, weights float64) for the Oh stars of the mesh."""
    mesh = np.asarray(mesh)
    coords = mesh_coords(mesh)
    B = cell.recip
    A = cell.lattice
    qcart = (coords / mesh) @ B
    nq = len(coords)
    star_of = -np.ones(nq, dtype=np.int64)
    reps, weights = [], []
    for iq in range(nq):
        if star_of[iq] >= 0:
            continue
        members = set()
        for S in cubic_ops():
            qr = (S @ qcart[iq]) @ A.T / (2.0 * np.pi) * mesh
            n = np.rint(qr).astype(np.int64)
            if np.max(np.abs(qr - n)) > 1e-8:
                raise ValueError("mesh not invariant under the cubic group")
            members.add(int(mesh_index(n, mesh)))
        for m in members:
            star_of[m] = len(reps)
        reps.append(iq)
        weights.append(len(members))
    return np.array(reps, dtype=np.int32), np.array(weights, dtype=np.float64)
