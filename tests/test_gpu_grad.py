"""Differentiable solve on the GPU: FV assembly, adjoint gradients against the
dense oracle (32x32, 16 right-hand sides) and central finite differences on
the 512x512 workload (32 cells)."""
import sys
import time

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import grad as OG  # noqa: E402
from paper_1105_3468_amd import autograd as AG  # noqa: E402
from paper_1105_3468_amd import gmg as G  # noqa: E402


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n,dim,vel", [(64, 2, W.velocity_const((1.0, 0.5))), (96, 2, W.velocity_rotating(10.0)),
                                       (20, 3, W.velocity_const((1.0, 1.0, 1.0))), (1, 2, None),
                                       (37, 2, W.velocity_rotating(3.0))])
def test_fv_assembly_bit_exact(n, dim, vel):
    _say(f"[case] assemble n={n} dim={dim}")
    rng = np.random.default_rng(3)
    kap = 10.0 ** rng.uniform(-4, 4, n ** dim)
    rp, ci, va = W.fv_matrix(n, dim, kap, vel)
    vt = AG.face_velocities(n, dim, vel)
    grp, gci, gva = G.fv_assemble(n, dim, torch.as_tensor(kap, device="cuda"), vt)
    assert np.array_equal(grp.cpu().numpy(), rp) and np.array_equal(gci.cpu().numpy(), ci)
    assert np.array_equal(gva.cpu().numpy().view(np.uint64), va.view(np.uint64))


def test_gradients_match_dense_oracle_32():
    """32x32 with 16 right-hand sides: dL/dkappa, dL/dB and the loss against
    dense solves with the exact dA/dkappa (relative 1e-6)."""
    _say("[case] dense 32x32")
    p = W.make("fv2d_32_grad")
    n, dim = 32, 2
    vt = AG.face_velocities(n, dim, p.velocity)
    kap = torch.as_tensor(p.kappa, device="cuda").requires_grad_(True)
    B = torch.as_tensor(p.b, device="cuda").requires_grad_(True)
    Xt = torch.as_tensor(p.x_target, device="cuda")
    X = AG.fv_solve(kap, B, n, dim, vt, tol=1e-12)
    loss = ((X - Xt) ** 2).sum()
    loss.backward()
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n_rows, p.n_rows)).toarray()
    lo, Xo, Lam, gB, gk = OG.dense_loss_and_grads(A, p.b, p.x_target, n, dim, p.kappa)
    assert abs(loss.item() - lo) <= 1e-9 * lo
    g = kap.grad.cpu().numpy()
    assert np.abs(g - gk).max() <= 1e-6 * np.abs(gk).max()
    assert np.abs(B.grad.cpu().numpy() - gB).max() <= 1e-6 * np.abs(gB).max()


def test_pattern_gradient_matches_dense():
    _say("[case] pattern grad")
    p = W.scaled("fv2d", 24, nrhs=4)
    rng = np.random.default_rng(5)
    Xt = rng.uniform(-1, 1, p.b.shape)
    val = torch.as_tensor(p.val, device="cuda").requires_grad_(True)
    B = torch.as_tensor(p.b, device="cuda")
    X = AG.sparse_solve(torch.as_tensor(p.rowptr, device="cuda"), torch.as_tensor(p.col, device="cuda"), val, B,
                        tol=1e-12)
    loss = ((X - torch.as_tensor(Xt, device="cuda")) ** 2).sum()
    loss.backward()
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n_rows, p.n_rows)).toarray()
    Xd = np.linalg.solve(A, p.b)
    Lam = np.linalg.solve(A.T, 2 * (Xd - Xt))
    ref = OG.pattern_grad_dense(p.rowptr, p.col, Lam, Xd)
    assert np.abs(val.grad.cpu().numpy() - ref).max() <= 1e-6 * np.abs(ref).max()


@pytest.fixture(scope="module")
def fd512():
    """Central-difference reference on the 512x512 workload with 16 RHS, the
    perturbed systems solved directly (sparse LU on the host), contracted
    with the exact dL/dX = 2 (X - X_t) at the base point; Richardson
    extrapolation of steps d and 2d (d = 1e-3 kappa_c) removes the O(d^2)
    term while keeping the rounding noise of the two solves small against the
    difference.  32 seeded cells, and one seeded direction u for the
    directional derivative d/dh L(kappa * (1 + h u)) at h = 0 (a JVP of the
    whole solve, contracted with dL/dX)."""
    import scipy.sparse.linalg as spla
    p = W.make("fv2d_512_grad")
    n, dim = 512, 2

    def direct(Am):
        return spla.splu(sp.csc_matrix(Am)).solve(p.b)

    def solve_at(kp):
        rp, ci, va = W.fv_matrix(n, dim, kp, p.velocity)
        return direct(sp.csr_matrix((va, ci, rp), shape=(n * n, n * n)))

    X0 = solve_at(p.kappa)
    dLdX = 2.0 * (X0 - p.x_target)

    def central(c, d):
        Xs = []
        for sgn in (1, -1):
            kp = p.kappa.copy()
            kp[c] += sgn * d
            Xs.append(solve_at(kp))
        return np.sum(dLdX * (Xs[0] - Xs[1])) / (2 * d)

    cells = np.random.default_rng(7).choice(n * n, 32, replace=False)
    fd = np.empty(32)
    t0 = time.time()
    for i, c in enumerate(cells):
        d = 1e-3 * p.kappa[c]
        fd[i] = (4.0 * central(c, d) - central(c, 2 * d)) / 3.0
        if i % 8 == 7:
            _say(f"  fd {i + 1}/32 ({time.time() - t0:.0f}s)")
    u = np.random.default_rng(8).uniform(-1.0, 1.0, n * n)

    def along(h):
        return np.sum(dLdX * (solve_at(p.kappa * (1 + h * u)) - solve_at(p.kappa * (1 - h * u)))) / (2 * h)

    h = 1e-3
    dirfd = (4.0 * along(h) - along(2 * h)) / 3.0
    _say(f"  fd reference done ({time.time() - t0:.0f}s)")
    return p, cells, fd, u, dirfd


def _grad512(p, **opts):
    n, dim = 512, 2
    vt = AG.face_velocities(n, dim, p.velocity)
    kap = torch.as_tensor(p.kappa, device="cuda").requires_grad_(True)
    B = torch.as_tensor(p.b, device="cuda")
    Xt = torch.as_tensor(p.x_target, device="cuda")
    t0 = time.time()
    X = AG.fv_solve(kap, B, n, dim, vt, tol=1e-11, ilut_tau=1e-6, maxit=600, **opts)
    loss = ((X - Xt) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    _say(f"  gpu forward+backward {time.time() - t0:.2f}s ({opts})")
    return kap.grad.cpu().numpy()


def _check_cells(g, cells, fd):
    ref = np.maximum(np.abs(fd), 1e-3 * np.abs(fd).max())
    err = np.abs(g[cells] - fd) / ref
    _say(f"  max relative error on 32 cells {err.max():.2e}")
    assert err.max() <= 1e-6, err.max()


def test_gradients_match_central_fd_512(fd512):
    """The 512x512 workload with 16 RHS solved one column after another
    (unrestarted FGMRES): dL/dkappa on 32 seeded cells against the
    central-difference reference."""
    _say("[case] fd 512x512, column loop")
    p, cells, fd, u, dirfd = fd512
    _check_cells(_grad512(p, restart=300), cells, fd)


def test_gradients_batched_fgmres30_512(fd512):
    """The differentiable configuration as specified: 16 RHS batched through
    FGMRES(30) forward and adjoint (the batched path), dL/dkappa on the 32
    cells and the directional derivative along a random direction (every
    cell at once) against central differences, both within 1e-6."""
    _say("[case] fd 512x512, batched FGMRES(30)")
    p, cells, fd, u, dirfd = fd512
    g = _grad512(p, restart=30)
    _check_cells(g, cells, fd)
    dirg = float(np.sum(g * p.kappa * u))
    _say(f"  directional derivative {dirg:.10e} vs fd {dirfd:.10e}")
    assert abs(dirg - dirfd) <= 1e-6 * abs(dirfd), (dirg, dirfd)

