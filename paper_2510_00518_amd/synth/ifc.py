"""Seeded anharmonic force constants with exact translational invariance and full
permutation symmetry.

The paper never shows the cubic/quartic IFC tables its matrix element consumes
(the arguments of the inlined Vp evaluation are elided in the appendix
algorithms), so the tables here are synthetic.  They are built as m-th
derivatives of a translation-invariant cluster energy

    U_m = sum_L sum_c P_c({u_{L+x} - u_{L+x0}} for x in c \\ x0),

each P_c a homogeneous degree-m polynomial with a seeded Gaussian coefficient
tensor.  Differentiating gives, with D_c[k, y] = delta(y, x_k) - delta(y, x_0),

    Phi^{a1..am}_{y1..ym} = m! sum_{k1..km} sym(T_c)[(k1 a1)..(km am)] prod_r D_c[k_r, y_r],

which sums to zero over any one site index (acoustic sum rule) and is symmetric
under any permutation of the (site, component) pairs.  Each ordered site tuple is
then translated so its first site lies in the home cell; contributions with the
same (atoms, cells) key are added.

Output format (one "term" per key):
    atoms (n, m) int32          atom index of each slot, slot 0 in the home cell
    cells (n, m-1, 3) int32     integer lattice coordinates of slots 1..m-1
    phi   (n, 3**m) float64     eV/Angstrom^m, row-major over [alpha0][alpha1]...
"""
import itertools
import math

import numpy as np

from .cells import neighbour_shells


def _canonical(sites):
    """Translation- and order-independent key of a cluster of (atom, cell) sites."""
    best = None
    for anchor in sites:
        c0 = np.array(anchor[1])
        key = tuple(sorted((a, tuple(int(v) for v in np.array(c) - c0)) for a, c in sites))
        if best is None or key < best:
            best = key
    return best


def candidate_clusters(cell, n_shells=3):
    """Candidate cluster groups, in the order they are offered: nearest-neighbour angle
    triples, then pair clusters by increasing shell.  Pair clusters alone would give
    blocks that are fully symmetric in their Cartesian indices (a pair energy depends
    on one relative displacement only); the three-body clusters break that, so the
    tables exercise every index of the contraction."""
    _, shells = neighbour_shells(cell, n_shells=n_shells)
    groups, seen = [], set()
    grp = []
    for a in range(cell.n_at):
        nn = [(b, tuple(c)) for aa, b, c in shells[0] if aa == a]
        for s1, s2 in itertools.combinations(nn, 2):
            key = _canonical(((a, (0, 0, 0)), s1, s2))
            if key not in seen:
                seen.add(key)
                grp.append(key)
    groups.append(grp)
    for pairs in shells:
        grp = []
        for a, b, c in pairs:
            sites = ((a, (0, 0, 0)), (b, tuple(c)))
            key = _canonical(sites)
            if key not in seen:
                seen.add(key)
                grp.append(key)
        groups.append(grp)
    return groups


def _sym(T):
    m = T.ndim
    out = np.zeros_like(T)
    for p in itertools.permutations(range(m)):
        out += np.transpose(T, p)
    return out / math.factorial(m)


def _cluster_blocks(sites, order, T):
    """Yield (site tuple, 3**order block) for one cluster with coefficient tensor T."""
    K = len(sites) - 1
    D = np.zeros((K, K + 1))
    for k in range(K):
        D[k, k + 1] += 1.0
        D[k, 0] -= 1.0
    Ts = _sym(T).reshape((K, 3) * order)
    # contract every (k, alpha) slot with D[k, y] -> (y, alpha)
    full = Ts
    for r in range(order):
        # axis 2r is k of slot r; bring result axis y into the same place
        full = np.moveaxis(np.tensordot(D, full, axes=([0], [2 * r])), 0, 2 * r)
    full = math.factorial(order) * full
    # full has axes (y0, a0, y1, a1, ...)
    for ys in itertools.product(range(K + 1), repeat=order):
        idx = []
        for y in ys:
            idx.extend([y, slice(None)])
        blk = full[tuple(idx)]
        if np.any(blk != 0.0):
            yield ys, blk.reshape(-1)


def _terms_from_clusters(clusters, order, tensors):
    acc = {}
    for sites, T in zip(clusters, tensors):
        for ys, blk in _cluster_blocks(sites, order, T):
            a0, c0 = sites[ys[0]]
            atoms = tuple(sites[y][0] for y in ys)
            cells = tuple(tuple(int(v) for v in np.array(sites[y][1]) - np.array(c0)) for y in ys[1:])
            key = (atoms, cells)
            acc[key] = acc.get(key, 0.0) + blk
    return acc


def build_ifc(cell, order, target_terms, rng, rms):
    """Return dict(atoms, cells, phi, n_terms, clusters) with about `target_terms` terms.

    One seeded three-body cluster is taken first; pair clusters are then offered
    shell by shell in a seeded order, and a cluster is kept if it
    brings the term count closer to the target or adds no new term (it then only
    enriches existing blocks), so the count ends at the nearest value this greedy
    pass reaches.  A final global rescale sets the RMS of all entries to `rms`
    (linear, so invariance and symmetry are kept).
    """
    groups = candidate_clusters(cell)
    chosen, tensors, count_keys = [], [], set()
    for gi, grp in enumerate(groups):
        order_idx = rng.permutation(len(grp))
        if gi == 0:
            order_idx = order_idx[:1]   # one three-body cluster, the rest pairs
        for i in order_idx:
            sites = grp[i]
            K = len(sites) - 1
            T = rng.standard_normal((3 * K,) * order)
            keys = set(_terms_from_clusters([sites], order, [T]).keys())
            n_new = len(count_keys | keys)
            if n_new == len(count_keys) or abs(n_new - target_terms) < abs(len(count_keys) - target_terms):
                chosen.append(sites)
                tensors.append(T)
                count_keys |= keys
    acc = _terms_from_clusters(chosen, order, tensors)
    keys = sorted(acc.keys())
    n = len(keys)
    atoms = np.array([k[0] for k in keys], dtype=np.int32).reshape(n, order)
    cells = np.array([k[1] for k in keys], dtype=np.int32).reshape(n, order - 1, 3)
    phi = np.array([acc[k] for k in keys], dtype=np.float64).reshape(n, 3 ** order)
    scale = rms / np.sqrt(np.mean(phi * phi))
    phi = phi * scale
    return dict(atoms=atoms, cells=cells, phi=phi, n_terms=n, clusters=chosen)


def to_supercell_dict(atoms, cells):
    """(term index) keyed by site tuple, for tests that need the full tensor."""
    out = {}
    for t in range(len(atoms)):
        out[(tuple(atoms[t]), tuple(map(tuple, cells[t])))] = t
    return out
