"""Dense reference of the differentiable FV solve -- TEST INFRASTRUCTURE.

For L(kappa, B) = sum_r ||x_r - t_r||^2 with A(kappa) X = B:
  Lambda = A^{-T} dL/dX,  dL/dB = Lambda,
  dL/dkappa_c = - sum_r lambda_r^T (dA/dkappa_c) x_r,
  dL/dA_ij = - sum_r lambda_{i,r} x_{j,r}  (on the pattern).
dA/dkappa_c is written out from the discretisation of Eq. (pde) (cell-centred
finite volumes): an interior face between cells c and m carries
T = 2 k_c k_m / ((k_c + k_m) h^2) on A_cc, A_mm and -T on A_cm, A_mc, so
dT/dk_c = 2 k_m^2 / ((k_c + k_m)^2 h^2); a Dirichlet face of c (y = 0 or 1)
adds 2 k_c / h^2 to A_cc (derivative 2 / h^2).  Convection does not depend on
kappa.  Dense numpy solves; only for small grids.
"""
from __future__ import annotations

import numpy as np


def dA_dkappa_dense(n: int, dim: int, kappa: np.ndarray, c: int) -> np.ndarray:
    """Dense N x N derivative of A with respect to kappa_c."""
    N = n ** dim
    h2 = (1.0 / n) ** 2
    D = np.zeros((N, N))
    idx = [c % n, (c // n) % n] + ([c // (n * n)] if dim == 3 else [])
    stride = [1, n, n * n]
    kc = kappa[c]
    for d in range(dim):
        for side in (-1, 1):
            j = idx[d] + side
            if 0 <= j < n:
                m = c + side * stride[d]
                km = kappa[m]
                dT = 2.0 * km * km / ((kc + km) ** 2 * h2)
                D[c, c] += dT
                D[m, m] += dT
                D[c, m] -= dT
                D[m, c] -= dT
            elif d == 1:
                D[c, c] += 2.0 / h2
    return D


def dense_loss_and_grads(A: np.ndarray, B: np.ndarray, Xt: np.ndarray, n: int, dim: int,
                         kappa: np.ndarray):
    """Loss, X, Lambda, dL/dB, dL/dkappa for the dense matrix A = A(kappa)."""
    X = np.linalg.solve(A, B)
    G = 2.0 * (X - Xt)
    Lam = np.linalg.solve(A.T, G)
    loss = float(np.sum((X - Xt) ** 2))
    gk = np.zeros(n ** dim)
    for c in range(n ** dim):
        D = dA_dkappa_dense(n, dim, kappa, c)
        gk[c] = -np.sum(Lam * (D @ X))
    return loss, X, Lam, Lam.copy(), gk


def pattern_grad_dense(rowptr, col, Lam, X):
    """dL/dA values on the CSR pattern."""
    g = np.empty(len(col))
    for i in range(len(rowptr) - 1):
        for p in range(rowptr[i], rowptr[i + 1]):
            g[p] = -np.dot(Lam[i], X[col[p]])
    return g
