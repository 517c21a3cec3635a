"""Scalar-loop version of the same step, for brute-force checks on tiny grids.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Plain Python loops over nodes, species and directions, with matrix inverses by
Gauss-Jordan elimination written out here, so that it shares neither the
vectorised index bookkeeping of ``lbm`` nor numpy's linear algebra.  Same
problem definition (``lbm.Problem``) and the same readings of the paper.  Use
only on grids of a few dozen nodes.
"""
from __future__ import annotations

import numpy as np

from . import lattice as _lat
from . import lbm as _lbm
from . import ms as _ms


def _inverse(a):
    """Gauss-Jordan inverse with partial pivoting of a small list-of-lists matrix."""
    n = len(a)
    aug = [list(map(float, row)) + [1.0 if i == j else 0.0 for j in range(n)] for i, row in enumerate(a)]
    for col in range(n):
        piv = max(range(col, n), key=lambda r: abs(aug[r][col]))
        aug[col], aug[piv] = aug[piv], aug[col]
        p = aug[col][col]
        aug[col] = [v / p for v in aug[col]]
        for r in range(n):
            if r != col:
                fac = aug[r][col]
                aug[r] = [vr - fac * vc for vr, vc in zip(aug[r], aug[col])]
    return [row[n:] for row in aug]


def _node_matrices(prob, xi_all):
    """B (Eq. (2-10), or Eqs. (2-16), (2-17) in dilute mode), D~ = B^-1, Lambda_1
    (Eq. (3-26)), Lambda_2 (Eq. (3-16)) at one node."""
    n = prob.N
    m = n - 1
    D = prob.D
    x = list(prob.xi_ref) if prob.xi_ref is not None else xi_all
    B = [[0.0] * m for _ in range(m)]
    for i in range(m):
        for j in range(m):
            if i != j:
                B[i][j] = 0.0 if prob.dilute else x[i] * (1.0 / D[i][n - 1] - 1.0 / D[i][j])
            else:
                s = 0.0 if prob.dilute else x[i] / D[i][n - 1]
                for k in range(n):
                    if k != i:
                        s += x[k] / D[i][k]
                B[i][i] = s
    Dt = _inverse(B)
    cs2 = prob.lat.cs2
    A = [[Dt[i][j] / cs2 + (0.5 if i == j else 0.0) for j in range(m)] for i in range(m)]
    L1 = _inverse(A)
    L2 = [row[:] for row in L1]
    if prob.relax == _ms.RELAX_PAPER:
        for i in range(m):
            L2[i][i] = 8.0 * (L1[i][i] - 2.0) / (L1[i][i] - 8.0)
    elif prob.relax == _ms.RELAX_TRT:
        # (1/l1 - 1/2)(1/l2 - 1/2) = magic, solved for l2
        for i in range(m):
            L2[i][i] = 1.0 / (0.5 + prob.magic / (1.0 / L1[i][i] - 0.5))
    return B, Dt, L1, L2


def _neighbour(prob, node, k):
    """Source node x - c_k of direction k, or (None, face) if it lies beyond a wall."""
    c = prob.lat.c[k]
    src = []
    for a in range(prob.lat.d):
        s = node[a] - int(c[a])
        n = prob.shape[a]
        if s < 0 or s >= n:
            side = 0 if s < 0 else 1
            if prob.bc[a][side] == _lbm.PERIODIC:
                s %= n
            else:
                return None, (a, side)
        src.append(s)
    return tuple(src), None


def _nodes(prob):
    if prob.lat.d == 1:
        return [(x,) for x in range(prob.shape[0])]
    if prob.lat.d == 2:
        return [(x, y) for y in range(prob.shape[1]) for x in range(prob.shape[0])]
    return [(x, y, z) for z in range(prob.shape[2]) for y in range(prob.shape[1]) for x in range(prob.shape[0])]


def step(prob, f):
    """One collide-and-stream step on f given as a dict {node: [[f_k^i]]} (lists)."""
    lat = prob.lat
    q, m = lat.q, prob.m
    M0 = [list(r) for r in lat.M0]
    M0inv = _inverse(M0)
    order = lat.row_order
    fpost = {}
    for node, fn in f.items():
        xi = [sum(fn[i]) for i in range(m)]
        xi_all = xi + [1.0 - sum(xi)]
        _, _, L1, L2 = _node_matrices(prob, xi_all)
        L0 = L1 if prob.relax == _ms.RELAX_SRT else [[prob.lambda0] * m for _ in range(m)]
        fam = (L0, L1, L2)
        # Eq. (3-2): f+ = f - M0^-1 Lambda M0 (f - f^eq); the conserved moment of
        # f - f^eq is exactly zero (Eq. (3-15)).
        neq = [[fn[i][k] - lat.w[k] * xi[i] for k in range(q)] for i in range(m)]
        dm = [[0.0 if r == 0 else sum(M0[r][k] * neq[i][k] for k in range(q)) for r in range(q)] for i in range(m)]
        rel = [[sum(fam[_lat.relaxation_family(order[r])][i][j] * dm[j][r] for j in range(m)) for r in range(q)]
               for i in range(m)]
        fpost[node] = [[fn[i][k] - sum(M0inv[k][r] * rel[i][r] for r in range(q)) for k in range(q)]
                       for i in range(m)]
    opp = lat.opposite
    out = {}
    for node in f:
        fn = [[0.0] * q for _ in range(m)]
        for k in range(q):
            src, face = _neighbour(prob, node, k)
            for i in range(m):
                if src is not None:
                    fn[i][k] = fpost[src][i][k]
                else:
                    back = fpost[node][i][opp[k]]
                    kind = prob.bc[face[0]][face[1]]
                    if kind == _lbm.ZERO_FLUX:
                        fn[i][k] = back
                    else:
                        xb = prob.xi_wall[face][i]
                        fn[i][k] = -back + 2.0 * lat.w[opp[k]] * xb
        out[node] = fn
    return out


def from_array(prob, f):
    """Array layout (m, q, *nodes[z, y, x]) -> dict keyed by (x[, y[, z]])."""
    out = {}
    for node in _nodes(prob):
        idx = tuple(reversed(node))
        out[node] = [[float(f[(i, k) + idx]) for k in range(prob.lat.q)] for i in range(prob.m)]
    return out


def to_array(prob, fd):
    f = np.zeros((prob.m, prob.lat.q) + prob.nodes)
    for node, fn in fd.items():
        idx = tuple(reversed(node))
        for i in range(prob.m):
            for k in range(prob.lat.q):
                f[(i, k) + idx] = fn[i][k]
    return f


def init(prob, xi0):
    """f_k^i(x, 0) = w_k xi_i(x, 0) (initialisation rule of Sec. 4)."""
    xi0 = np.asarray(xi0, dtype=np.float64)
    out = {}
    for node in _nodes(prob):
        idx = tuple(reversed(node))
        out[node] = [[float(prob.lat.w[k] * xi0[(i,) + idx]) for k in range(prob.lat.q)]
                     for i in range(prob.m)]
    return out


def run(prob, xi0, nsteps):
    f = init(prob, xi0)
    for _ in range(nsteps):
        f = step(prob, f)
    return to_array(prob, f)
