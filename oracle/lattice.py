"""Lattice descriptors (velocity sets, weights, moment matrices).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Velocity sets and weights follow Sec. 3.1, Eqs. (3-4) (D1Q2), (3-5) (D1Q3),
(3-6) (D2Q4), (3-7) (D2Q5), (3-8) (D2Q9), (3-9) (D3Q6), (3-10) (D3Q7) and
(3-11) (D3Q15), in the paper's direction order.  Velocities are in lattice units
(c = dx/dt = 1; the scale invariance M0^-1 Lambda M0 = M^-1 Lambda M after
Eq. (3-14) makes the C_d factor irrelevant).

The moment matrix M0 is given by the paper only for D2Q5 (Eq. (3-14)).  For the
other lattices we use matrices built the same way: row 0 is the conserved
zeroth moment, then one row per first-order moment (the velocity components),
then second-order rows.  Every row is either even or odd under k -> opposite(k).
The lattices without a rest direction (D1Q2, D2Q4, D3Q6) have q = 2d: D1Q2 has
no second-order row, D2Q4 one (c_x^2 - c_y^2), D3Q6 two.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Lattice:
    name: str
    d: int                 # spatial dimension
    c: np.ndarray          # (q, 3) integer velocities (unused axes are 0)
    w: np.ndarray          # (q,) weights omega_k
    M0: np.ndarray         # (q, q) moment matrix
    row_order: tuple       # moment order of each row of M0: 0 .. 4

    @property
    def q(self) -> int:
        return len(self.w)

    @property
    def opposite(self) -> np.ndarray:
        """Index kbar with c_kbar = -c_k (used by the bounce-back rules, Sec. 4)."""
        opp = np.empty(self.q, dtype=np.int64)
        for k in range(self.q):
            hit = [j for j in range(self.q) if np.array_equal(self.c[j], -self.c[k])]
            assert len(hit) == 1
            opp[k] = hit[0]
        return opp

    @property
    def cs2(self) -> float:
        """Lattice sound speed squared, sum_k w_k c_kx^2.

        The Chapman-Enskog analysis of Sec. 3.2 is carried out on D2Q5, where the
        second moment of the weights is c^2/3 (Eqs. (3-22), (3-26), (3-27)).  On a
        general lattice the same derivation produces sum_k w_k c_kx^2 in that
        place: 1/3 on D1Q3, D2Q5 and D3Q6, 1/4 on D3Q7, 1/2 on D2Q4, 1 on D1Q2.
        """
        return float(np.sum(self.w * self.c[:, 0] ** 2))


def _vel(rows):
    c = np.zeros((len(rows), 3), dtype=np.int64)
    for k, r in enumerate(rows):
        c[k, : len(r)] = r
    return c


# Eq. (3-5): D1Q3, w = (2/3, 1/6, 1/6), c = (0, 1, -1).
D1Q3 = Lattice(
    name="D1Q3",
    d=1,
    c=_vel([(0,), (1,), (-1,)]),
    w=np.array([2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0]),
    M0=np.array(
        [
            [1.0, 1.0, 1.0],    # zeroth moment
            [0.0, 1.0, -1.0],   # c_x
            [-2.0, 1.0, 1.0],   # second order (even), orthogonal to row 0
        ]
    ),
    row_order=(0, 1, 2),
)

# Eq. (3-7): D2Q5, w = (1/3, 1/6 x4); directions (0,0), (1,0), (0,1), (-1,0), (0,-1).
# M0 is Eq. (3-14) with c = 1.
D2Q5 = Lattice(
    name="D2Q5",
    d=2,
    c=_vel([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1)]),
    w=np.array([1.0 / 3.0] + [1.0 / 6.0] * 4),
    M0=np.array(
        [
            [1.0, 1.0, 1.0, 1.0, 1.0],
            [0.0, 1.0, 0.0, -1.0, 0.0],
            [0.0, 0.0, 1.0, 0.0, -1.0],
            [0.0, 1.0, -1.0, 1.0, -1.0],
            [-4.0, 1.0, 1.0, 1.0, 1.0],
        ]
    ),
    row_order=(0, 1, 1, 2, 2),
)

# Eq. (3-10): D3Q7, w = (1/4, 1/8 x6); directions 0, +x, -x, +y, -y, +z, -z.
D3Q7 = Lattice(
    name="D3Q7",
    d=3,
    c=_vel([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]),
    w=np.array([1.0 / 4.0] + [1.0 / 8.0] * 6),
    M0=np.array(
        [
            [1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0],
            [0.0, 1.0, -1.0, 0.0, 0.0, 0.0, 0.0],
            [0.0, 0.0, 0.0, 1.0, -1.0, 0.0, 0.0],
            [0.0, 0.0, 0.0, 0.0, 0.0, 1.0, -1.0],
            [-6.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0],
            [0.0, 2.0, 2.0, -1.0, -1.0, -1.0, -1.0],
            [0.0, 0.0, 0.0, 1.0, 1.0, -1.0, -1.0],
        ]
    ),
    row_order=(0, 1, 1, 1, 2, 2, 2),
)

# Eq. (3-4): D1Q2, w = (1/2, 1/2), c = (1, -1).
D1Q2 = Lattice(
    name="D1Q2",
    d=1,
    c=_vel([(1,), (-1,)]),
    w=np.array([0.5, 0.5]),
    M0=np.array(
        [
            [1.0, 1.0],     # zeroth moment
            [1.0, -1.0],    # c_x
        ]
    ),
    row_order=(0, 1),
)

# Eq. (3-6): D2Q4, w = 1/4; directions (1,0), (0,1), (-1,0), (0,-1).
D2Q4 = Lattice(
    name="D2Q4",
    d=2,
    c=_vel([(1, 0), (0, 1), (-1, 0), (0, -1)]),
    w=np.array([0.25] * 4),
    M0=np.array(
        [
            [1.0, 1.0, 1.0, 1.0],
            [1.0, 0.0, -1.0, 0.0],
            [0.0, 1.0, 0.0, -1.0],
            [1.0, -1.0, 1.0, -1.0],    # c_x^2 - c_y^2
        ]
    ),
    row_order=(0, 1, 1, 2),
)

# Eq. (3-9): D3Q6, w = 1/6; directions +x, -x, +y, -y, +z, -z.
D3Q6 = Lattice(
    name="D3Q6",
    d=3,
    c=_vel([(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]),
    w=np.array([1.0 / 6.0] * 6),
    M0=np.array(
        [
            [1.0, 1.0, 1.0, 1.0, 1.0, 1.0],
            [1.0, -1.0, 0.0, 0.0, 0.0, 0.0],
            [0.0, 0.0, 1.0, -1.0, 0.0, 0.0],
            [0.0, 0.0, 0.0, 0.0, 1.0, -1.0],
            [2.0, 2.0, -1.0, -1.0, -1.0, -1.0],   # 2 c_x^2 - c_y^2 - c_z^2
            [0.0, 0.0, 1.0, 1.0, -1.0, -1.0],     # c_y^2 - c_z^2
        ]
    ),
    row_order=(0, 1, 1, 1, 2, 2),
)

def _poly_rows(c, polys):
    """Moment matrix rows from polynomials of the velocity components."""
    return np.array([[float(pfun(*ck)) for ck in c] for pfun in polys])


# Eq. (3-8): D2Q9, w = (4/9, 1/9 x4, 1/36 x4); directions (0,0), (1,0), (0,1),
# (-1,0), (0,-1), (1,1), (-1,1), (-1,-1), (1,-1).  The paper gives no moment
# matrix for it: rows are polynomials of definite parity (1; c_x, c_y;
# c^2, c_x^2 - c_y^2, c_x c_y; c^2 c_x, c^2 c_y; c^4).
_c2q9 = _vel([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)])
D2Q9 = Lattice(
    name="D2Q9",
    d=2,
    c=_c2q9,
    w=np.array([4.0 / 9.0] + [1.0 / 9.0] * 4 + [1.0 / 36.0] * 4),
    M0=_poly_rows(_c2q9[:, :2], [
        lambda x, y: 1,
        lambda x, y: x, lambda x, y: y,
        lambda x, y: x * x + y * y, lambda x, y: x * x - y * y, lambda x, y: x * y,
        lambda x, y: (x * x + y * y) * x, lambda x, y: (x * x + y * y) * y,
        lambda x, y: (x * x + y * y) ** 2,
    ]),
    row_order=(0, 1, 1, 2, 2, 2, 3, 3, 4),
)

# Eq. (3-11): D3Q15, w = (2/9, 1/9 x6, 1/72 x8), in the paper's direction order.
# Rows: 1; c_x, c_y, c_z; c^2, 3c_x^2 - c^2, c_y^2 - c_z^2, c_x c_y, c_y c_z,
# c_z c_x; c^2 c_x, c^2 c_y, c^2 c_z, c_x c_y c_z; c^4.
_c3q15 = _vel([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
               (1, 1, 1), (1, -1, -1), (1, -1, 1), (1, 1, -1), (-1, 1, 1), (-1, -1, -1), (-1, -1, 1), (-1, 1, -1)])
D3Q15 = Lattice(
    name="D3Q15",
    d=3,
    c=_c3q15,
    w=np.array([2.0 / 9.0] + [1.0 / 9.0] * 6 + [1.0 / 72.0] * 8),
    M0=_poly_rows(_c3q15, [
        lambda x, y, z: 1,
        lambda x, y, z: x, lambda x, y, z: y, lambda x, y, z: z,
        lambda x, y, z: x * x + y * y + z * z, lambda x, y, z: 2 * x * x - y * y - z * z,
        lambda x, y, z: y * y - z * z, lambda x, y, z: x * y, lambda x, y, z: y * z, lambda x, y, z: z * x,
        lambda x, y, z: (x * x + y * y + z * z) * x, lambda x, y, z: (x * x + y * y + z * z) * y,
        lambda x, y, z: (x * x + y * y + z * z) * z, lambda x, y, z: x * y * z,
        lambda x, y, z: (x * x + y * y + z * z) ** 2,
    ]),
    row_order=(0, 1, 1, 1, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 4),
)

LATTICES = {"D1Q2": D1Q2, "D1Q3": D1Q3, "D2Q4": D2Q4, "D2Q5": D2Q5, "D3Q6": D3Q6, "D3Q7": D3Q7,
            "D2Q9": D2Q9, "D3Q15": D3Q15}


def relaxation_family(order: int) -> int:
    """Which relaxation matrix a moment row of this order takes: 0 the conserved
    row (its m - m^eq is zero), 1 (Lambda_1) the odd orders, 2 (Lambda_2) the even
    ones.  Eq. (3-14) assigns Lambda_1 to the first-order and Lambda_2 to the
    second-order moments of D2Q5; for lattices with higher-order moments the odd
    ones relax with Lambda_1 and the even ones with Lambda_2, the two-relaxation-
    time grouping the paper names after Eq. (3-14)."""
    return 0 if order == 0 else (1 if order % 2 else 2)


def get(name: str) -> Lattice:
    return LATTICES[name]
