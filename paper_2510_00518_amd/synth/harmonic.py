"""Harmonic inputs on a Gamma-centred q-mesh: omega, eigenvectors, group velocities.

Model: central springs, one constant per neighbour shell (nearest and next-nearest),
Phi(0a, Rb) = -k rhat rhat^T, on-site block fixed by the acoustic sum rule.

Conventions (the ones the scattering-rate inputs assume):
  * mesh point n = (n0, n1, n2), q = sum_d n_d b_d / N_d, index iq = (n0*N1 + n1)*N2 + n2
  * global mode index g = iq*nb + j, branch index j fastest
  * D(q)_{a alpha, b beta} = sum_R Phi_{alpha beta}(0a; Rb) exp(i q.R) / sqrt(M_a M_b),
    phases on lattice vectors only, so e(q + G) = e(q) and q.R = 2 pi sum_d n_d m_d / N_d
  * e(-q) is stored as conj(e(q)); at time-reversal-invariant q (2q = 0 mod G) D is real
    and a real eigenbasis is used
  * the three acoustic modes at Gamma get omega = 0 exactly and the exact rigid
    translations as eigenvectors
  * omega in rad/ps, velocities in Angstrom/ps, eigenvector components indexed 3*atom+alpha
"""
import numpy as np

from .cells import neighbour_shells

# eV expressed in amu * Angstrom^2 / ps^2 (CODATA 2018 SI values)
_EV = 1.602176634e-19 / (1.66053906660e-27 * 1e-20 * 1e24)


def mesh_coords(mesh):
    """Integer coordinates (nq, 3) in index order iq = (n0*N1 + n1)*N2 + n2."""
    n0, n1, n2 = np.meshgrid(np.arange(mesh[0]), np.arange(mesh[1]), np.arange(mesh[2]), indexing="ij")
    return np.stack([n0.ravel(), n1.ravel(), n2.ravel()], axis=1).astype(np.int64)


def mesh_index(coords, mesh):
    c = np.mod(np.asarray(coords, dtype=np.int64), np.asarray(mesh))
    return (c[..., 0] * mesh[1] + c[..., 1]) * mesh[2] + c[..., 2]


def spring_fc2(cell, k_shell):
    """Second-order force constants in eV/A^2 as a list of (a, b, cell_vec, 3x3 block)."""
    _, shells = neighbour_shells(cell, n_shells=len(k_shell))
    blocks = {}
    onsite = [np.zeros((3, 3)) for _ in range(cell.n_at)]
    for k, pairs in zip(k_shell, shells):
        for a, b, c in pairs:
            r = cell.site_xyz(b, c) - cell.pos[a]
            rr = np.outer(r, r) / np.dot(r, r)
            blocks[(a, b, c)] = blocks.get((a, b, c), 0.0) - k * rr
            onsite[a] += k * rr
    for a in range(cell.n_at):
        blocks[(a, a, (0, 0, 0))] = blocks.get((a, a, (0, 0, 0)), 0.0) + onsite[a]
    return [(a, b, np.array(c), blk) for (a, b, c), blk in sorted(blocks.items())]


def _roots(n, m, mesh):
    """exp(2 pi i sum_d n_d m_d / N_d) evaluated from the exactly reduced fraction."""
    ang = 0.0
    for d in range(3):
        ang = ang + np.mod(n[..., d] * m[d], mesh[d]) / mesh[d]
    ang = np.mod(ang, 1.0)
    return np.exp(2j * np.pi * ang)


def _dynmat(cell, fc2, n, mesh, with_grad=False):
    nb = cell.nb
    D = np.zeros((nb, nb), dtype=complex)
    dD = np.zeros((3, nb, nb), dtype=complex) if with_grad else None
    m = cell.masses
    for a, b, c, blk in fc2:
        ph = _roots(np.asarray(n), c, mesh)
        w = blk * _EV / np.sqrt(m[a] * m[b])
        D[3 * a:3 * a + 3, 3 * b:3 * b + 3] += w * ph
        if with_grad:
            R = c @ cell.lattice
            for x in range(3):
                dD[x, 3 * a:3 * a + 3, 3 * b:3 * b + 3] += 1j * R[x] * w * ph
    D = 0.5 * (D + D.conj().T)
    return D, dD


def phonons(cell, fc2, mesh):
    """Return omega (nq, nb), evec (nq, nb, nb) complex [q][j][3*atom+alpha], vel (nq, nb, 3)."""
    mesh = tuple(int(x) for x in mesh)
    coords = mesh_coords(mesh)
    nq, nb = len(coords), cell.nb
    omega = np.zeros((nq, nb))
    evec = np.zeros((nq, nb, nb), dtype=complex)
    vel = np.zeros((nq, nb, 3))
    minus = mesh_index(-coords, mesh)
    done = np.zeros(nq, dtype=bool)
    for iq in range(nq):
        if done[iq]:
            continue
        n = coords[iq]
        D, dD = _dynmat(cell, fc2, n, mesh, with_grad=True)
        if minus[iq] == iq:
            w2, e = np.linalg.eigh(D.real)
            e = e.astype(complex)
        else:
            w2, e = np.linalg.eigh(D)
        om = np.sqrt(np.clip(w2, 0.0, None))
        if iq == 0:
            om[:3] = 0.0
            tr = np.zeros((nb, 3))
            msum = cell.masses.sum()
            for a in range(cell.n_at):
                for x in range(3):
                    tr[3 * a + x, x] = np.sqrt(cell.masses[a] / msum)
            e[:, :3] = tr
        v = np.zeros((nb, 3))
        for j in range(nb):
            # v(-q) = -v(q), so v vanishes where -q = q
            if om[j] > 0.0 and minus[iq] != iq:
                for x in range(3):
                    v[j, x] = np.real(np.vdot(e[:, j], dD[x] @ e[:, j])) / (2.0 * om[j])
        omega[iq], evec[iq], vel[iq] = om, e.T, v
        done[iq] = True
        mq = minus[iq]
        if mq != iq:
            omega[mq], evec[mq], vel[mq] = om, e.T.conj(), -v
            done[mq] = True
    return omega, evec, vel
