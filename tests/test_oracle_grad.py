"""Pins of the dense gradient reference (oracle/grad.py) against central
finite differences of the generator's assembly and of the loss."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import grad as OG


def _A(n, dim, kap, vel):
    rp, ci, va = W.fv_matrix(n, dim, kap, vel)
    return sp.csr_matrix((va, ci, rp), shape=(n ** dim, n ** dim)).toarray()


@pytest.mark.parametrize("n,dim,vel", [(8, 2, W.velocity_const((1.0, 0.5))), (6, 2, W.velocity_rotating(10.0)),
                                       (4, 3, W.velocity_const((1.0, 1.0, 1.0)))])
def test_dA_dkappa_matches_fd_of_assembly(n, dim, vel):
    rng = np.random.default_rng(0)
    kap = 10.0 ** rng.uniform(-2, 2, n ** dim)
    for c in rng.choice(n ** dim, 6, replace=False):
        d = 1e-6 * kap[c]
        kp, km = kap.copy(), kap.copy()
        kp[c] += d
        km[c] -= d
        fd = (_A(n, dim, kp, vel) - _A(n, dim, km, vel)) / (2 * d)
        ex = OG.dA_dkappa_dense(n, dim, kap, c)
        assert np.abs(fd - ex).max() <= 1e-6 * np.abs(ex).max()


def test_adjoint_gradient_matches_fd_of_loss():
    n, dim = 8, 2
    vel = W.velocity_const((1.0, 0.5))
    rng = np.random.default_rng(1)
    kap = 10.0 ** rng.uniform(-1, 1, n * n)
    B = rng.uniform(-1, 1, (n * n, 3))
    Xt = rng.uniform(-1, 1, (n * n, 3))
    A = _A(n, dim, kap, vel)
    loss, X, Lam, gB, gk = OG.dense_loss_and_grads(A, B, Xt, n, dim, kap)

    def L(kp, Bp):
        Xp = np.linalg.solve(_A(n, dim, kp, vel), Bp)
        return np.sum((Xp - Xt) ** 2)
    for c in (0, 9, 27, 63):
        d = 1e-5 * kap[c]
        kp, km = kap.copy(), kap.copy()
        kp[c] += d
        km[c] -= d
        fd = (L(kp, B) - L(km, B)) / (2 * d)
        assert abs(fd - gk[c]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gk).max())
    for (i, r) in ((5, 0), (40, 2)):
        Bp, Bm = B.copy(), B.copy()
        Bp[i, r] += 1e-6
        Bm[i, r] -= 1e-6
        fd = (L(kap, Bp) - L(kap, Bm)) / 2e-6
        assert abs(fd - gB[i, r]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gB).max())
    # pattern gradient: directional derivative along a random pattern perturbation
    S = sp.csr_matrix(A)
    S.sort_indices()
    g = OG.pattern_grad_dense(S.indptr, S.indices, Lam, X)
    dv = rng.standard_normal(len(S.data))
    eps = 1e-7

    def Lv(v):
        Av = sp.csr_matrix((v, S.indices, S.indptr), shape=A.shape).toarray()
        return np.sum((np.linalg.solve(Av, B) - Xt) ** 2)
    fd = (Lv(S.data + eps * dv) - Lv(S.data - eps * dv)) / (2 * eps)
    assert abs(fd - g @ dv) <= 1e-5 * abs(fd)
