"""Maxwell-Stefan algebra: matrix B, generalised Fick matrix, relaxation matrices.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Species are indexed 0..N-1 here (the paper's 1..n); the last one is the species
whose flux and gradient equation are eliminated (Sec. 2, Eq. (2-8a)).  ``D`` is
the symmetric N x N matrix of Maxwell-Stefan diffusivities D_ij (Eq. (2-7));
its diagonal is never used.
"""
from __future__ import annotations

import numpy as np


def check_diffusivities(D: np.ndarray) -> None:
    """D_ij = 1/sigma_ij with sigma_ij = sigma_ji > 0 (Sec. 2, after Eq. (2-7))."""
    D = np.asarray(D, dtype=np.float64)
    n = D.shape[0]
    if D.shape != (n, n) or n < 2:
        raise ValueError("D must be a square matrix with N >= 2")
    off = ~np.eye(n, dtype=bool)
    if not np.all(D[off] > 0):
        raise ValueError("off-diagonal D_ij must be positive")
    if not np.allclose(D, D.T, rtol=0, atol=0):
        raise ValueError("D must be symmetric")


def ms_B(xi: np.ndarray, D: np.ndarray) -> np.ndarray:
    """Matrix B of Eq. (2-10) at every node.

    xi: (..., N) mole fractions of all N species.  Returns (..., N-1, N-1):

        B_ij = xi_i (1/D_iN - 1/D_ij)                       i != j
        B_ii = xi_i / D_iN + sum_{k != i, k = 1..N} xi_k / D_ik
    """
    xi = np.asarray(xi, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    n = D.shape[0]
    m = n - 1
    B = np.empty(xi.shape[:-1] + (m, m), dtype=np.float64)
    for i in range(m):
        for j in range(m):
            if i != j:
                B[..., i, j] = xi[..., i] * (1.0 / D[i, n - 1] - 1.0 / D[i, j])
            else:
                s = xi[..., i] / D[i, n - 1]
                for k in range(n):
                    if k != i:
                        s = s + xi[..., k] / D[i, k]
                B[..., i, i] = s
    return B


def ms_B_dilute(xi: np.ndarray, D: np.ndarray) -> np.ndarray:
    """The dilute-species approximation of B (Remark III, Eqs. (2-16), (2-17)),
    applied to every evolved species: B is diagonal with

        B_ii = 1 / D_eff,i = sum_{k != i, k = 1..N} xi_k / D_ik,

    so each species follows Fick's law with its own composition-dependent
    effective diffusivity.  xi: (..., N); returns (..., N-1, N-1).
    """
    xi = np.asarray(xi, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    n = D.shape[0]
    m = n - 1
    B = np.zeros(xi.shape[:-1] + (m, m), dtype=np.float64)
    for i in range(m):
        s = np.zeros(xi.shape[:-1])
        for k in range(n):
            if k != i:
                s = s + xi[..., k] / D[i, k]
        B[..., i, i] = s
    return B


def fick_matrix(B: np.ndarray) -> np.ndarray:
    """Generalised Fick diffusivity D~ = B^-1 (Eq. (2-11)); B is invertible (Sec. 2)."""
    return np.linalg.inv(B)


def fick_flux(Dt: np.ndarray, grad_xi: np.ndarray, c_t: float = 1.0) -> np.ndarray:
    """Generalised Fick law J_i = -c_t sum_j D~_ij grad xi_j (Eq. (2-12)).

    Dt: (*nodes, m, m); grad_xi: (m, d, *nodes).  Returns (m, d, *nodes).
    """
    m = grad_xi.shape[0]
    out = np.zeros_like(grad_xi)
    for i in range(m):
        for j in range(m):
            out[i] -= c_t * Dt[..., i, j][None, ...] * grad_xi[j]
    return out


def lambda1_from_fick(Dt: np.ndarray, cs2: float, dt: float = 1.0) -> np.ndarray:
    """Relaxation matrix Lambda_1 that realises a given D~ (Eq. (3-26) solved for Lambda_1).

    Eq. (3-26): D~ = cs2 dt (Lambda_1^-1 - I/2)  =>  Lambda_1 = (D~/(cs2 dt) + I/2)^-1.
    """
    m = Dt.shape[-1]
    eye = np.eye(m)
    return np.linalg.inv(Dt / (cs2 * dt) + 0.5 * eye)


def fick_from_lambda1(L1: np.ndarray, cs2: float, dt: float = 1.0) -> np.ndarray:
    """Eq. (3-26) as printed: D~ = cs2 dt (Lambda_1^-1 - I/2)."""
    m = L1.shape[-1]
    return cs2 * dt * (np.linalg.inv(L1) - 0.5 * np.eye(m))


RELAX_PAPER = "paper"   # Eq. (3-16)
RELAX_SRT = "srt"       # all relaxation parameters equal (Sec. 3.1, after Eq. (3-14))
RELAX_TRT = "trt"       # odd and even moments with two parameters (Sec. 3.1, after Eq. (3-14))

MAGIC_PAPER = 3.0 / 16.0


def lambda2_from_lambda1(L1: np.ndarray, rule: str = RELAX_PAPER, magic: float = MAGIC_PAPER) -> np.ndarray:
    """Second-order relaxation matrix Lambda_2.

    Paper rule, Eq. (3-16): lambda_2^ij = lambda_1^ij for i != j and
    lambda_2^ii = 8 (lambda_1^ii - 2) / (lambda_1^ii - 8), applied entry by entry
    to the coupled matrix Lambda_1.  SRT: Lambda_2 = Lambda_1.

    TRT (the two-relaxation-time case named after Eq. (3-14): odd moments with
    lambda_o = lambda_1, even ones with lambda_e = lambda_2): the even parameter of
    each species is fixed by the product (1/lambda_1^ii - 1/2)(1/lambda_2^ii - 1/2)
    = magic, i.e. lambda_2^ii = 2 (2 - l) / (2 + (4 magic - 1) l) with l = lambda_1^ii;
    off-diagonal entries as in the paper rule.  Eq. (3-16) is this rule with
    magic = 3/16.
    """
    L2 = np.array(L1, dtype=np.float64, copy=True)
    if rule == RELAX_SRT:
        return L2
    if rule not in (RELAX_PAPER, RELAX_TRT):
        raise ValueError(f"unknown relaxation rule {rule!r}")
    if rule == RELAX_TRT and not (np.isfinite(magic) and magic > 0):
        raise ValueError("the TRT parameter must be positive")
    m = L1.shape[-1]
    for i in range(m):
        l1 = L1[..., i, i]
        if rule == RELAX_PAPER:
            L2[..., i, i] = 8.0 * (l1 - 2.0) / (l1 - 8.0)
        else:
            L2[..., i, i] = 2.0 * (2.0 - l1) / (2.0 + (4.0 * magic - 1.0) * l1)
    return L2
