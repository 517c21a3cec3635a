"""Torch-CPU FP64 twin of the oracle step, for reference gradients by autograd.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The same algorithm as ``lbm`` in the same order (moments, B of Eq. (2-10),
D~ = B^-1, Lambda_1 by inverting Eq. (3-26), Lambda_2 by Eq. (3-16), the
collision in the form of Eq. (3-2) with the conserved moment of f - f^eq zero,
propagation with the face rules of Sec. 4), written with differentiable torch
operations so that torch.autograd yields dL/dD_ij and dL/dxi(0).  Its forward
pass is pinned to ``lbm`` and its gradients to finite differences of ``lbm``.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lattice as _lat
from . import lbm as _lbm
from . import ms as _ms


def pairs_to_matrix(d_pairs: torch.Tensor, N: int) -> torch.Tensor:
    """Symmetric N x N matrix (unit diagonal) from its upper-triangle entries,
    listed row by row: D_01, D_02, ..., D_12, ..."""
    rows = []
    it = 0
    idx = {}
    for i in range(N):
        for j in range(i + 1, N):
            idx[(i, j)] = idx[(j, i)] = it
            it += 1
    one = torch.ones((), dtype=d_pairs.dtype)
    for i in range(N):
        rows.append(torch.stack([one if i == j else d_pairs[idx[(i, j)]] for j in range(N)]))
    return torch.stack(rows)


def matrix_to_pairs(D: np.ndarray) -> np.ndarray:
    N = D.shape[0]
    return np.array([D[i, j] for i in range(N) for j in range(i + 1, N)])


class Twin:
    """One problem (same fields as lbm.Problem) evolved with torch operations."""

    def __init__(self, prob: _lbm.Problem):
        self.prob = prob
        self.lat = _lat.get(prob.lattice)
        self.w = torch.tensor(self.lat.w, dtype=torch.float64)
        self.M0 = torch.tensor(self.lat.M0, dtype=torch.float64)
        self.M0inv = torch.linalg.inv(self.M0)

    def _B(self, xi_b: torch.Tensor, D: torch.Tensor) -> torch.Tensor:
        """Eq. (2-10), or in dilute mode the diagonal B of Eqs. (2-16), (2-17);
        xi_b: (*nodes, N)."""
        N = D.shape[0]
        m = N - 1
        dilute = self.prob.dilute
        rows = []
        for i in range(m):
            cols = []
            for j in range(m):
                if i != j:
                    if dilute:
                        cols.append(torch.zeros_like(xi_b[..., i]))
                    else:
                        cols.append(xi_b[..., i] * (1.0 / D[i, N - 1] - 1.0 / D[i, j]))
                else:
                    s = torch.zeros_like(xi_b[..., i]) if dilute else xi_b[..., i] / D[i, N - 1]
                    for k in range(N):
                        if k != i:
                            s = s + xi_b[..., k] / D[i, k]
                    cols.append(s)
            rows.append(torch.stack(cols, dim=-1))
        return torch.stack(rows, dim=-2)

    def collide(self, f: torch.Tensor, D: torch.Tensor) -> torch.Tensor:
        p = self.prob
        d = self.lat.d
        m = f.shape[0]
        xi_e = f.sum(dim=1)
        xi_all = torch.cat([xi_e, (1.0 - xi_e.sum(dim=0))[None]], dim=0)
        if p.xi_ref is not None:
            xi_b = torch.tensor(p.xi_ref, dtype=torch.float64).expand(*xi_e.shape[1:], m + 1)
        else:
            xi_b = torch.movedim(xi_all, 0, -1)
        B = self._B(xi_b, D)
        Dt = torch.linalg.inv(B)
        eye = torch.eye(m, dtype=torch.float64)
        L1 = torch.linalg.inv(Dt / self.lat.cs2 + 0.5 * eye)
        if p.relax == _ms.RELAX_SRT:
            L2 = L1
            L0 = L1
        else:
            diag = torch.diagonal(L1, dim1=-2, dim2=-1)
            if p.relax == _ms.RELAX_TRT:
                l2 = 2.0 * (2.0 - diag) / (2.0 + (4.0 * p.magic - 1.0) * diag)
            else:
                l2 = 8.0 * (diag - 2.0) / (diag - 8.0)
            L2 = L1 - torch.diag_embed(diag) + torch.diag_embed(l2)
            L0 = torch.full_like(L1, p.lambda0)
        fam = (L0, L1, L2)
        feq = self.w.reshape((1, -1) + (1,) * d) * xi_e[:, None]
        dm = torch.einsum("rk,ik...->ir...", self.M0, f - feq)
        mask = torch.ones(self.lat.q, dtype=torch.float64)
        mask[0] = 0.0
        dm = dm * mask.reshape((1, -1) + (1,) * d)                 # conserved moment exactly zero
        rel = torch.stack([torch.einsum("...ij,j...->i...", fam[_lat.relaxation_family(self.lat.row_order[r])], dm[:, r])
                           for r in range(self.lat.q)], dim=1)
        return f - torch.einsum("kr,ir...->ik...", self.M0inv, rel)

    def stream(self, fpost: torch.Tensor) -> torch.Tensor:
        p = self.prob
        lat = self.lat
        opp = lat.opposite
        outs = []
        for k in range(lat.q):
            ck = lat.c[k]
            axes = [a for a in range(lat.d) if ck[a] != 0]
            if not axes:
                outs.append(fpost[:, k])
                continue
            out = fpost[:, k]
            for a in axes:
                out = torch.roll(out, shifts=int(ck[a]), dims=1 + (lat.d - 1 - a))
            # face rules, the lowest axis last (it decides at edges and corners)
            for a in reversed(axes):
                ax = 1 + (lat.d - 1 - a)
                side = 0 if ck[a] > 0 else 1
                kind = p.bc[a][side]
                if kind == _lbm.PERIODIC:
                    continue
                n = p.shape[a]
                pos = 0 if side == 0 else n - 1
                sel = torch.zeros(n, dtype=torch.float64)
                sel[pos] = 1.0
                sel = sel.reshape((1,) + tuple(n if i == ax else 1 for i in range(1, out.ndim)))
                back = fpost[:, opp[k]]
                if kind == _lbm.ZERO_FLUX:
                    face = back
                else:
                    xb = torch.tensor(np.asarray(p.xi_wall[(a, side)], dtype=np.float64)[: p.m])
                    face = -back + 2.0 * lat.w[opp[k]] * xb.reshape((-1,) + (1,) * (out.ndim - 1))
                out = out * (1.0 - sel) + face * sel
            outs.append(out)
        return torch.stack(outs, dim=1)

    def run(self, xi0: torch.Tensor, D: torch.Tensor, steps: int) -> torch.Tensor:
        """Pre-collision f at t = steps from xi0 (N or N-1 planes), differentiable."""
        d = self.lat.d
        f = self.w.reshape((1, -1) + (1,) * d) * xi0[: self.prob.m, None]
        for _ in range(int(steps)):
            f = self.stream(self.collide(f, D))
        return f

    @staticmethod
    def mole_fractions(f: torch.Tensor) -> torch.Tensor:
        xi_e = f.sum(dim=1)
        return torch.cat([xi_e, (1.0 - xi_e.sum(dim=0))[None]], dim=0)


def misfit_gradients(prob: _lbm.Problem, xi0: np.ndarray, target: np.ndarray, steps: int):
    """L = sum_x sum_i (xi_i(T) - target_i)^2 and its gradients with respect to the
    pair diffusivities (returned as a symmetric N x N matrix of pair derivatives,
    zero diagonal) and the evolved species' initial fields (N-1 planes)."""
    N = prob.N
    tw = Twin(prob)
    d_pairs = torch.tensor(matrix_to_pairs(prob.D), dtype=torch.float64, requires_grad=True)
    x0 = torch.tensor(xi0, dtype=torch.float64, requires_grad=True)
    D = pairs_to_matrix(d_pairs, N)
    f = tw.run(x0, D, steps)
    xi = tw.mole_fractions(f)
    L = ((xi - torch.tensor(target, dtype=torch.float64)) ** 2).sum()
    L.backward()
    gD = np.zeros((N, N))
    if d_pairs.grad is not None:            # None when L does not depend on D (no step)
        it = 0
        for i in range(N):
            for j in range(i + 1, N):
                gD[i, j] = gD[j, i] = d_pairs.grad[it].item()
                it += 1
    return float(L.item()), gD, x0.grad.numpy()[: N - 1].copy()
