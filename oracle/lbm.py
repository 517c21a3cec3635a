"""The MRT lattice Boltzmann step for N-component Maxwell-Stefan diffusion.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Everything is FP64 numpy, vectorised over nodes, following the paper's order
of operations with no fusion: moments -> B -> D~ = B^-1 -> Lambda_1 (Eq. (3-26))
-> Lambda_2 (Eq. (3-16)) -> moment-space relaxation of the non-equilibrium part
and back-transform (Eq. (3-2)) -> propagation with the boundary rules of Sec. 4
(Eq. (3-13b)).

Array conventions
-----------------
* ``shape`` is (nx,), (nx, ny) or (nx, ny, nz); node arrays are stored with x
  fastest, i.e. numpy shape ``shape[::-1]`` (z, y, x).
* distributions ``f``: (m, q, *nodes) with m = N - 1 evolved species
  (Sec. 3.1: the evolution equation (3-2) is written for i <= n - 1; the last
  species follows from Eq. (2-3b)).
* mole fractions: (N, *nodes); gradients and fluxes: (m, d, *nodes) with the
  vector components ordered x, y, z.
* node j on an axis of n nodes sits at the cell centre (j + 1/2) dx; walls lie
  half-way between the boundary node and its missing neighbour (the half-way
  bounce-back rules of Sec. 4).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import lattice as _lat
from . import ms as _ms

PERIODIC = "periodic"
ZERO_FLUX = "zero_flux"     # half-way bounce-back (Sec. 4)
DIRICHLET = "dirichlet"     # half-way anti-bounce-back (Sec. 4)


@dataclass
class Problem:
    """One mixture on one lattice, in lattice units (dx = dt = 1).

    lattice : "D1Q2" | "D1Q3" | "D2Q4" | "D2Q5" | "D3Q6" | "D3Q7"
    D       : (N, N) symmetric Maxwell-Stefan diffusivities in lattice units
    shape   : (nx,), (nx, ny) or (nx, ny, nz)
    bc      : per axis a pair (low face, high face) of PERIODIC / ZERO_FLUX /
              DIRICHLET; default all periodic
    xi_wall : Dirichlet face values {(axis, 0|1): (N,) mole fractions}
    relax   : ms.RELAX_PAPER (Eq. (3-16)), ms.RELAX_SRT (Lambda_2 = Lambda_1) or
              ms.RELAX_TRT (Lambda_2 from the product rule with parameter `magic`)
    magic   : TRT parameter (1/lambda_1^ii - 1/2)(1/lambda_2^ii - 1/2) (> 0)
    lambda0 : value of every lambda_0^ij (Sec. 3.1 sets it to 1; it multiplies
              m_0 - m_0^eq, which is identically zero)
    c_t     : total molar concentration in the flux law (Eq. (2-12))
    xi_ref  : if given, B is evaluated at these fixed mole fractions instead of
              the local ones (the linearised theory with constant effective
              diffusivities, Sec. 1)
    dilute  : if true, B is the dilute-species approximation of Remark III
              (diagonal, Eqs. (2-16), (2-17)) instead of Eq. (2-10)
    """

    lattice: str
    D: np.ndarray
    shape: tuple
    bc: tuple = None
    xi_wall: dict = field(default_factory=dict)
    relax: str = _ms.RELAX_PAPER
    magic: float = _ms.MAGIC_PAPER
    lambda0: float = 1.0
    c_t: float = 1.0
    xi_ref: np.ndarray = None
    dilute: bool = False

    def __post_init__(self):
        self.D = np.asarray(self.D, dtype=np.float64)
        _ms.check_diffusivities(self.D)
        self.lat = _lat.get(self.lattice)
        self.shape = tuple(int(s) for s in self.shape)
        if len(self.shape) != self.lat.d:
            raise ValueError("shape must have one extent per lattice dimension")
        if self.bc is None:
            self.bc = tuple((PERIODIC, PERIODIC) for _ in range(self.lat.d))
        self.bc = tuple(tuple(b) for b in self.bc)
        for lo, hi in self.bc:
            if (lo == PERIODIC) != (hi == PERIODIC):
                raise ValueError("periodic faces must come in pairs")
        if self.xi_ref is not None:
            self.xi_ref = np.asarray(self.xi_ref, dtype=np.float64)

    @property
    def N(self) -> int:
        return self.D.shape[0]

    @property
    def m(self) -> int:
        return self.N - 1

    @property
    def nodes(self) -> tuple:
        return self.shape[::-1]


def _array_axis(prob: Problem, a: int) -> int:
    """numpy axis of node arrays (z, y, x order) that carries lattice axis a."""
    return prob.lat.d - 1 - a


# ----------------------------------------------------------------------------
# Initialisation and moments
# ----------------------------------------------------------------------------

def init(prob: Problem, xi0: np.ndarray) -> np.ndarray:
    """f_k^i(x, 0) = f_k^{i,eq} = w_k xi_i(x, 0) (initialisation rule of Sec. 4, Eq. (3-3)).

    xi0: (N, *nodes) or (m, *nodes); only the evolved species are used.
    """
    xi0 = np.asarray(xi0, dtype=np.float64)
    w = prob.lat.w
    f = w[(None, slice(None)) + (None,) * prob.lat.d] * xi0[: prob.m, None]
    return np.ascontiguousarray(f)


def mole_fractions(f: np.ndarray) -> np.ndarray:
    """xi_i = sum_k f_k^i for i < N (Eq. (3-15)); xi_N = 1 - sum_{i<N} xi_i (Eq. (2-3b))."""
    xi_e = f.sum(axis=1)
    xi_last = 1.0 - xi_e.sum(axis=0)
    return np.concatenate([xi_e, xi_last[None]], axis=0)


def first_moments(prob: Problem, f: np.ndarray) -> np.ndarray:
    """m1^i = sum_k c_k f_k^i, shape (m, d, *nodes) (the sums in Eq. (3-27))."""
    d = prob.lat.d
    c = prob.lat.c[:, :d].astype(np.float64)
    return np.einsum("ka,ik...->ia...", c, f)


def relaxation_matrices(prob: Problem, xi: np.ndarray):
    """B, D~, Lambda_1, Lambda_2 at every node from the mole fractions xi (N, *nodes).

    B by Eq. (2-10) (by Eqs. (2-16), (2-17) in dilute mode), D~ = B^-1 by
    Eq. (2-11), Lambda_1 by inverting Eq. (3-26), Lambda_2 by Eq. (3-16) (or =
    Lambda_1 in SRT mode).  All (*nodes, m, m).
    """
    if prob.xi_ref is not None:
        xi_b = np.broadcast_to(prob.xi_ref, prob.nodes + (prob.N,))
    else:
        xi_b = np.moveaxis(xi, 0, -1)
    B = (_ms.ms_B_dilute if prob.dilute else _ms.ms_B)(xi_b, prob.D)
    Dt = _ms.fick_matrix(B)
    L1 = _ms.lambda1_from_fick(Dt, prob.lat.cs2, 1.0)
    L2 = _ms.lambda2_from_lambda1(L1, prob.relax, prob.magic)
    return B, Dt, L1, L2


# ----------------------------------------------------------------------------
# Collision (Eq. (3-13a)) and propagation (Eq. (3-13b))
# ----------------------------------------------------------------------------

def collide(prob: Problem, f: np.ndarray) -> np.ndarray:
    """Post-collision distributions in the form of the evolution equation (3-2)/(3-1a):

        f^{i,+} = f^i - sum_j M0^-1 Lambda^{ij} M0 (f^j - f^{j,eq}),   f^{j,eq}_k = w_k xi_j (Eq. (3-3))

    with the diagonal relaxation Lambda^{ij} = diag(lambda_0^ij, lambda_1^ij, ..., lambda_2^ij, ...)
    of Eq. (3-14b): every first-order row of M0 uses Lambda_1, every second-order row
    Lambda_2 (higher orders by parity, lattice.relaxation_family).  The zeroth (conserved) moment of f - f^eq is zero exactly, since
    m_0 = sum_k f_k = xi (Eq. (3-15)) = m_0^eq (Eq. (m0A)); it is set to that exact value
    rather than to its floating-point residual, which would otherwise feed a systematic
    rounding drift of the species totals into every step.
    """
    lat = prob.lat
    xi = mole_fractions(f)
    xi_e = xi[: prob.m]
    _, _, L1, L2 = relaxation_matrices(prob, xi)
    if prob.relax == _ms.RELAX_SRT:
        L0 = L1
    else:
        L0 = np.full_like(L1, prob.lambda0)
    family = (L0, L1, L2)

    feq = lat.w[(None, slice(None)) + (None,) * lat.d] * xi_e[:, None]
    dm = np.einsum("rk,ik...->ir...", lat.M0, f - feq)       # m - m^eq (Eq. (3-11))
    dm[:, 0] = 0.0                                           # conserved moment
    relaxed = np.empty_like(dm)
    for r in range(lat.q):
        relaxed[:, r] = np.einsum("...ij,j...->i...", family[_lat.relaxation_family(lat.row_order[r])], dm[:, r])
    return f - np.einsum("kr,ir...->ik...", np.linalg.inv(lat.M0), relaxed)


def stream(prob: Problem, fpost: np.ndarray) -> np.ndarray:
    """Propagation f_k^i(x + c_k, t + 1) = f_k^{i,+}(x, t) (Eq. (3-13b)) with boundaries.

    Periodic faces wrap.  At a wall face the unknown incoming population of a
    boundary node x_f (the one whose source node lies outside) is, following
    Sec. 4:
      zero flux (half-way bounce-back):   f_k(x_f, t+1) =  f_kbar^+(x_f, t)
      Dirichlet (half-way anti-bounce-back):
                                          f_k(x_f, t+1) = -f_kbar^+(x_f, t) + 2 w_kbar xi_b
    """
    lat = prob.lat
    opp = lat.opposite
    out = np.empty_like(fpost)
    for k in range(lat.q):
        ck = lat.c[k]
        axes = [a for a in range(lat.d) if ck[a] != 0]
        moved = fpost[:, k]
        for a in axes:
            moved = np.roll(moved, shift=int(ck[a]), axis=1 + _array_axis(prob, a))
        out[:, k] = moved
        # Boundary nodes whose source x - c_k lies beyond a wall take the face
        # rule.  A diagonal direction can leave through two or three faces at an
        # edge or corner; there the face of the lowest axis decides (applied last).
        for a in reversed(axes):
            side = 0 if ck[a] > 0 else 1        # face whose boundary nodes miss their source
            kind = prob.bc[a][side]
            if kind == PERIODIC:
                continue
            ax = 1 + _array_axis(prob, a)       # axis in (m, *nodes) arrays
            idx = [slice(None)] * out[:, k].ndim
            idx[ax] = 0 if side == 0 else prob.shape[a] - 1
            idx = tuple(idx)
            back = fpost[:, opp[k]][idx]
            if kind == ZERO_FLUX:
                out[:, k][idx] = back
            elif kind == DIRICHLET:
                xi_b = np.asarray(prob.xi_wall[(a, side)], dtype=np.float64)[: prob.m]
                shape = (prob.m,) + (1,) * (back.ndim - 1)
                out[:, k][idx] = -back + 2.0 * lat.w[opp[k]] * xi_b.reshape(shape)
            else:
                raise ValueError(f"unknown boundary kind {kind!r}")
    return out


def step(prob: Problem, f: np.ndarray) -> np.ndarray:
    """One time step: collision followed by propagation (Eq. (3-13))."""
    return stream(prob, collide(prob, f))


def run(prob: Problem, xi0: np.ndarray, nsteps: int, f: np.ndarray = None) -> np.ndarray:
    """Initialise (unless f is given) and advance nsteps; returns pre-collision f at t = nsteps."""
    if f is None:
        f = init(prob, xi0)
    for _ in range(int(nsteps)):
        f = step(prob, f)
    return f


# ----------------------------------------------------------------------------
# Observables and diagnostics
# ----------------------------------------------------------------------------

def observables(prob: Problem, f: np.ndarray):
    """Mole fractions, gradients and diffusion fluxes at the current (pre-collision) state.

    grad xi_i = -(1/(cs2 dt)) sum_j lambda_1^ij sum_k c_k f_k^j   (Eq. (3-27), with the
                 D2Q5 factor c^2/3 read as the lattice's cs2)
    J = -c_t D~ grad xi                                        (Eq. (2-12))
    Returns (xi (N, *nodes), grad (m, d, *nodes), J (m, d, *nodes)).
    """
    xi = mole_fractions(f)
    _, Dt, L1, _ = relaxation_matrices(prob, xi)
    m1 = first_moments(prob, f)
    grad = np.zeros_like(m1)
    for i in range(prob.m):
        for j in range(prob.m):
            grad[i] -= L1[..., i, j][None, ...] * m1[j] / prob.lat.cs2
    J = _ms.fick_flux(Dt, grad, prob.c_t)
    return xi, grad, J


def diagnostics(prob: Problem, f: np.ndarray):
    """Per-species totals sum_x xi_i (conserved by Eq. (2-1) for closed domains),
    per-species min and max, and the number of non-finite values."""
    xi = mole_fractions(f)
    flat = xi.reshape(prob.N, -1)
    finite = np.isfinite(flat)
    return (
        flat.sum(axis=1),
        np.where(finite, flat, np.inf).min(axis=1),
        np.where(finite, flat, -np.inf).max(axis=1),
        int((~finite).sum()),
    )


def rel_l2_error(analytic: np.ndarray, numeric: np.ndarray) -> float:
    """Relative L2 error E(phi) of Sec. 4."""
    analytic = np.asarray(analytic, dtype=np.float64)
    numeric = np.asarray(numeric, dtype=np.float64)
    return float(np.sqrt(np.sum((analytic - numeric) ** 2) / np.sum(analytic ** 2)))


def cell_centres(n: int, lo: float, hi: float) -> np.ndarray:
    """Node positions (j + 1/2) dx on [lo, hi] with n nodes (half-way walls)."""
    dx = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * dx
