"""Invariants of the seeded synthetic inputs (the generator feeds both the HIP
path and the oracle, so every pin downstream depends on these)."""
import itertools

import numpy as np
import pytest

from paper_2510_00518_amd.synth import (diamond_conventional, diamond_primitive, irreducible_q, make_config,
                                        mesh_coords, mesh_index, small_config)
from paper_2510_00518_amd.synth.configs import _cell, springs
from paper_2510_00518_amd.synth.harmonic import spring_fc2

EV = 1.602176634e-19 / (1.66053906660e-27 * 1e-20 * 1e24)


def _ifc_dict(ifc):
    d = {}
    for t in range(len(ifc["atoms"])):
        key = (tuple(int(x) for x in ifc["atoms"][t]), tuple(tuple(int(v) for v in c) for c in ifc["cells"][t]))
        d[key] = ifc["phi"][t]
    return d


@pytest.mark.parametrize("cell,order,n", [("prim", 3, 32), ("prim", 4, 96), ("prim", 3, 64), ("prim", 4, 160),
                                          ("conv", 4, 200)])
def test_ifc_acoustic_sum_rule(cell, order, n):
    from paper_2510_00518_amd.synth.configs import _ifc
    ifc = _ifc(cell, order, n)
    phi = ifc["phi"].reshape((-1,) + (3,) * order)
    scale = np.abs(phi).max()
    # sum over the last slot's (atom, cell) with everything else fixed
    groups = {}
    for t in range(len(phi)):
        key = (tuple(ifc["atoms"][t][:-1]), tuple(map(tuple, ifc["cells"][t][:-1])))
        groups[key] = groups.get(key, 0.0) + phi[t]
    worst = max(np.abs(v).max() for v in groups.values())
    assert worst < 1e-12 * scale


@pytest.mark.parametrize("cell,order,n", [("prim", 3, 32), ("prim", 4, 96), ("conv", 4, 200)])
def test_ifc_permutation_symmetry(cell, order, n):
    from paper_2510_00518_amd.synth.configs import _ifc
    ifc = _ifc(cell, order, n)
    d = _ifc_dict(ifc)
    for (atoms, cells), phi in d.items():
        sites = [(atoms[0], (0, 0, 0))] + [(atoms[r], cells[r - 1]) for r in range(1, order)]
        blk = phi.reshape((3,) * order)
        for perm in itertools.permutations(range(order)):
            ps = [sites[p] for p in perm]
            c0 = np.array(ps[0][1])
            key = (tuple(s[0] for s in ps), tuple(tuple(int(v) for v in np.array(s[1]) - c0) for s in ps[1:]))
            assert key in d
            np.testing.assert_allclose(d[key].reshape((3,) * order), np.transpose(blk, perm), rtol=0,
                                       atol=1e-13 * np.abs(blk).max())


@pytest.mark.parametrize("cell,order,n", [("prim", 3, 32), ("prim", 4, 96), ("conv", 4, 200)])
def test_ifc_blocks_not_cartesian_symmetric(cell, order, n):
    """Three-body clusters make blocks asymmetric in their Cartesian indices, so a
    transposed operand in any contraction changes the result."""
    from paper_2510_00518_amd.synth.configs import _ifc
    phi = _ifc(cell, order, n)["phi"].reshape((-1,) + (3,) * order)
    for a, b in itertools.combinations(range(order), 2):
        assert np.abs(phi - np.swapaxes(phi, a + 1, b + 1)).max() > 0.1 * np.abs(phi).max()


def test_ifc_counts_and_scale():
    c2, c3, c4 = make_config("fcc8_4ph"), make_config("fcc16_34ph"), make_config("sc10_4ph_uneven")
    # counts the greedy cluster pass reaches for targets 32, 96, 64, 160, 200
    assert c2["ifc3"]["n_terms"] == 32
    assert c2["ifc4"]["n_terms"] == 94
    assert c3["ifc3"]["n_terms"] == 62
    assert c3["ifc4"]["n_terms"] == 164
    assert c4["ifc4"]["n_terms"] == 198
    assert np.sqrt(np.mean(c2["ifc3"]["phi"] ** 2)) == pytest.approx(1.0, rel=1e-12)
    assert np.sqrt(np.mean(c2["ifc4"]["phi"] ** 2)) == pytest.approx(0.3, rel=1e-12)


def test_star_counts():
    """Oh stars of Gamma-centred meshes: 8/29/145 points for FCC 4^3/8^3/16^3, 56 for SC 10^3."""
    p, c = diamond_primitive(), diamond_conventional()
    for cell, n, expect in ((p, 4, 8), (p, 8, 29), (p, 16, 145), (c, 10, 56)):
        reps, w = irreducible_q(cell, (n, n, n))
        assert len(reps) == expect
        assert w.sum() == n ** 3


def _dyn_cartesian(cell, fc2, qcart):
    """Dynamical matrix from Cartesian phases exp(i q_cart . R_cart) (independent of mesh integers)."""
    nb = cell.nb
    D = np.zeros((nb, nb), dtype=complex)
    for a, b, c, blk in fc2:
        R = np.asarray(c) @ cell.lattice
        D[3 * a:3 * a + 3, 3 * b:3 * b + 3] += blk * EV * np.exp(1j * qcart @ R) / np.sqrt(
            cell.masses[a] * cell.masses[b])
    return D


@pytest.mark.parametrize("kind,mesh", [("prim", 4), ("prim", 8), ("conv", 3)])
def test_harmonic_eigenproblem(kind, mesh):
    cell = _cell(kind)
    if kind == "prim":
        cfg = small_config(mesh) if mesh != 8 else make_config("fcc8_4ph")
    else:
        cfg = small_config(mesh, n3=0, n4=0, cell="conv")
    fc2 = spring_fc2(cell, springs())
    om, ev, vel = cfg["omega"], cfg["evec"], cfg["vel"]
    coords = mesh_coords((mesh,) * 3)
    minus = mesh_index(-coords, (mesh,) * 3)
    for iq, n in enumerate(coords):
        qc = (n / mesh) @ cell.recip
        D = _dyn_cartesian(cell, fc2, qc)
        E = ev[iq].T  # columns are eigenvectors
        np.testing.assert_allclose(E.conj().T @ E, np.eye(cell.nb), atol=1e-12)
        resid = D @ E - E * (om[iq] ** 2)[None, :]
        assert np.abs(resid).max() < 1e-9 * np.abs(D).max()
        # e(-q) = conj e(q) exactly, real at time-reversal-invariant q
        np.testing.assert_array_equal(ev[minus[iq]], ev[iq].conj())
        np.testing.assert_array_equal(vel[minus[iq]], -vel[iq])
        if minus[iq] == iq:
            assert np.all(ev[iq].imag == 0.0)
        if iq == 0:
            assert np.all(om[0, :3] == 0.0)
        else:
            assert om[iq].min() > 1.0
    # group velocity against a central difference of omega along x (non-degenerate modes only)
    h = 1e-5
    for iq in (1, 2, 5):
        qc = (coords[iq] / mesh) @ cell.recip
        wp = np.sqrt(np.clip(np.linalg.eigvalsh(_dyn_cartesian(cell, fc2, qc + [h, 0, 0])), 0, None))
        wm = np.sqrt(np.clip(np.linalg.eigvalsh(_dyn_cartesian(cell, fc2, qc - [h, 0, 0])), 0, None))
        w0 = om[iq]
        for j in range(cell.nb):
            gaps = np.abs(w0 - w0[j])
            gaps[j] = np.inf
            if gaps.min() > 1e-2:
                assert vel[iq, j, 0] == pytest.approx((wp[j] - wm[j]) / (2 * h), rel=1e-5, abs=1e-6)
