"""Newton solve of the discrete equilibrium of the improved scheme (oracle; test
infrastructure only).

At a state with u = 0 and a chemical potential that is uniform on the lattice,
the improved scheme's force vanishes (Eq. 24), the correction vanishes (Eq. 29,
u = 0) and the moving equilibrium populations depend on p_m = (1 + mu)/3 alone
(Eq. 27), so streaming reproduces the same populations: such a state is an exact
fixed point of the time step.  Its density solves, for an unknown constant mu0,

    mu_EOS(rho) - kappa lap_d(rho) = mu0,      sum_x rho = mass,

with lap_d the lattice Laplacian.  This module solves that system by Newton's
method with a sparse direct solver, with the Laplacian assembled here as a
sparse matrix from the stencil weights (not through the oracle's roll-based
operators).  It serves as an independent check of the time stepper; its own
pins are Table II (flat interfaces) and the Young-Laplace law (Eq. 32).
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def laplacian_matrix(shape, lat):
    """Sparse periodic lattice Laplacian, (2 / c_s^2) sum_a w_a [phi(x + e_a) - phi(x)].
    `shape` is (ny, nx) or (nz, ny, nx); flattening is C order (x fastest)."""
    D = len(shape)
    N = int(np.prod(shape))
    idx = np.arange(N).reshape(shape)
    rows, cols, vals = [], [], []
    w = lat.w.numpy()
    e = lat.e.numpy()
    for a in range(lat.Q):
        if not e[a].any():
            continue
        # neighbour x + e_a; axis k of the array holds component D-1-k
        nb = idx
        for k in range(D):
            nb = np.roll(nb, -int(e[a, D - 1 - k]), axis=k)
        rows.append(idx.ravel())
        cols.append(nb.ravel())
        vals.append(np.full(N, 6.0 * w[a]))
        rows.append(idx.ravel())
        cols.append(idx.ravel())
        vals.append(np.full(N, -6.0 * w[a]))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def solve(rho_init, eos, T, kappa, lat, tol=1e-13, maxiter=60):
    """Newton iteration from rho_init (numpy array).  Returns (rho, mu0, residual)."""
    shape = rho_init.shape
    L = laplacian_matrix(shape, lat)
    rho = np.array(rho_init, dtype=np.float64).ravel()
    mass = rho.sum()
    N = rho.size
    mu0 = float(np.mean(eos.mu(rho, T) - kappa * (L @ rho)))
    ones = np.ones((N, 1))
    res = np.inf
    for _ in range(maxiter):
        r = np.concatenate([eos.mu(rho, T) - kappa * (L @ rho) - mu0, [rho.sum() - mass]])
        res = np.abs(r).max()
        if res < tol:
            break
        dmu = eos.dp(rho, T) / rho          # d mu_EOS / d rho by Gibbs-Duhem
        J = sp.bmat([[sp.diags(dmu) - kappa * L, -ones], [ones.T, None]], format="csc")
        dx = spla.spsolve(J, -r)
        rho = rho + dx[:N]
        mu0 = mu0 + dx[N]
    return rho.reshape(shape), mu0, res
