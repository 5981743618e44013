"""Scalar per-node reference of one time step, for tiny lattices only.

Written independently of the vectorised oracle: explicit neighbour index
arithmetic with modulo wrap, velocity tables typed out here, and the equilibrium
and correction terms in their closed population-space forms (for D2Q9 these are
M^-1 of Eq. 27 and of Eq. 29's C; for D3Q19 the same construction rules).  Used
to pin the oracle on 3x3 .. 5x5 (x5) lattices.
"""

E2 = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
W2 = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
E3 = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
      (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
      (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
W3 = [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12

# Lallemand-Luo moment matrix typed out as integers (rows rho, e, eps, j_x, q_x,
# j_y, q_y, p_xx, p_xy; columns in the E2 velocity order).
MLL = [
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [-4, -1, -1, -1, -1, 2, 2, 2, 2],
    [4, -2, -2, -2, -2, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, -2, 0, 2, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [0, 0, -2, 0, 2, 1, 1, -1, -1],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 1, -1, 1, -1],
]


def step(f, dims, mu_eos, p_eos, kappa, tau, scheme, force_form="chempot", mrt=None, walls=None, c0=1.0):
    """f: dict {(a, node): value}; dims = (nx, ny) or (nx, ny, nz); node = (x, y[, z]).
    mrt (D2Q9 only): dict(s_e, s_eps, s_q, nu) -> collision in the moment basis MLL
    with rates (1, s_e, s_eps, 1, s_q, 1, s_q, s_v, s_v); s_v = 1/tau if nu is None,
    else 1/tau_v from nu = eta/rho with eta = rho/3 (tau_v - 1/2) (standard) or
    p_m (tau_v - 1/2) (improved).
    walls (D2Q9 only): (U_bottom, U_top); plates halfway outside rows 0 and ny-1.
    A stencil reaching past a plate reads the mirror node (row -1 -> 0, -2 -> 1,
    ny -> ny-1, ...), negated for the y component of phi u; a population
    leaving through a plate is pushed back into its own node reversed, plus the
    difference of the node's closed-form equilibrium (its rho and p_m) at the plate
    velocity between the reversed direction and the leaving one.
    Returns (f_next, fields)."""
    D = len(dims)
    E, W = (E2, W2) if D == 2 else (E3, W3)
    Q = len(E)
    nodes = [(x, y) for y in range(dims[1]) for x in range(dims[0])] if D == 2 else \
        [(x, y, z) for z in range(dims[2]) for y in range(dims[1]) for x in range(dims[0])]

    def nb(n, e, s=1):
        return tuple((n[d] + s * e[d]) % dims[d] for d in range(D))

    def val(field, n, e, odd=False):
        m = [n[d] + e[d] for d in range(D)]
        sign = 1.0
        if walls is not None and not 0 <= m[1] < dims[1]:
            m[1] = -1 - m[1] if m[1] < 0 else 2 * dims[1] - 1 - m[1]
            sign = -1.0 if odd else 1.0
        return sign * field[tuple(m[d] % dims[d] for d in range(D))]

    def grad(field, n, odd=False):
        return [3.0 * sum(W[a] * val(field, n, E[a], odd) * E[a][d] for a in range(Q)) for d in range(D)]

    def lap(field, n):
        return 6.0 * sum(W[a] * (val(field, n, E[a]) - field[n]) for a in range(1, Q))

    rho = {n: sum(f[(a, n)] for a in range(Q)) for n in nodes}
    j = {n: [sum(E[a][d] * f[(a, n)] for a in range(Q)) for d in range(D)] for n in nodes}
    lrho = {n: lap(rho, n) for n in nodes}
    mu = {n: mu_eos(rho[n]) - kappa * lrho[n] for n in nodes}
    F = {}
    for n in nodes:
        gmu = grad(mu, n)
        if scheme == "improved":
            F[n] = [(1 / 3 - rho[n]) * gmu[d] for d in range(D)]
        elif force_form == "chempot":
            grho = grad(rho, n)
            F[n] = [grho[d] / 3 - rho[n] * gmu[d] for d in range(D)]
    if scheme == "standard" and force_form == "ptensor":
        grho = {n: grad(rho, n) for n in nodes}
        P = {}
        for n in nodes:
            g2 = sum(x * x for x in grho[n])
            p = p_eos(rho[n]) - kappa * rho[n] * lrho[n] - 0.5 * kappa * g2
            P[n] = [[(p if i == k else 0.0) + kappa * grho[n][i] * grho[n][k] for k in range(D)] for i in range(D)]
        for n in nodes:
            grh = grho[n]
            div = []
            for k in range(D):
                s = 0.0
                for a in range(Q):
                    m = nb(n, E[a])
                    for i in range(D):
                        s += 3.0 * W[a] * E[a][i] * P[m][i][k]
                div.append(s)
            F[n] = [grh[k] / 3 - div[k] for k in range(D)]
    u = {n: [(j[n][d] + 0.5 * F[n][d]) / rho[n] for d in range(D)] for n in nodes}
    pm = {n: ((c0 + mu[n]) / 3 if scheme == "improved" else rho[n] / 3) for n in nodes}
    dcorr = {}
    if scheme == "improved":
        psi = [{n: (rho[n] / 3 - pm[n]) * u[n][d] for n in nodes} for d in range(D)]
        for n in nodes:
            dcorr[n] = [3.0 * sum(W[a] * val(psi[d], n, E[a], d == 1) * E[a][d] for a in range(Q)) for d in range(D)]

    out = {}
    for n in nodes:
        r, uu, FF = rho[n], u[n], F[n]
        usq = sum(x * x for x in uu)
        php = pm[n] - r / 3
        if scheme == "improved":
            Cii = [3.0 * x for x in dcorr[n]]
        def feq_of(a, vel):
            e = E[a]
            c2 = sum(x * x for x in e)
            eu = sum(e[d] * vel[d] for d in range(D))
            vsq = sum(x * x for x in vel)
            val = W[a] * r * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * vsq)
            if scheme == "improved":
                rest = 1.0 if a == 0 else 0.0
                if D == 2:
                    val += 3 * php * (W[a] - rest) + 4.5 * php * W[a] * eu * (3 * c2 - 4)
                else:
                    val += 3 * php * (W[a] - rest) + 9.0 * php * W[a] * eu * (3 * c2 - 5)
            return val

        feqs, srcs = [], []
        for a in range(Q):
            e = E[a]
            c2 = sum(x * x for x in e)
            eu = sum(e[d] * uu[d] for d in range(D))
            feq = feq_of(a, uu)
            G = W[a] * sum((3 * (e[d] - uu[d]) + 9 * eu * e[d]) * FF[d] for d in range(D))
            C = 0.0
            if scheme == "improved":
                if D == 2:
                    cx, cy = Cii
                    if a == 0:
                        C = -(cx + cy) / 3
                    elif c2 == 1:
                        C = (cx - 2 * cy) / 6 if e[0] != 0 else (cy - 2 * cx) / 6
                    else:
                        C = (cx + cy) / 6
                else:
                    if a == 0:
                        C = -5 * sum(Cii) / 21
                    elif c2 == 1:
                        i = [d for d in range(3) if e[d] != 0][0]
                        C = (Cii[i] - 6 * (sum(Cii) - Cii[i])) / 42
                    else:
                        ii = [d for d in range(3) if e[d] != 0]
                        k = [d for d in range(3) if e[d] == 0][0]
                        C = (5 * (Cii[ii[0]] + Cii[ii[1]]) - 2 * Cii[k]) / 42
            feqs.append(feq)
            srcs.append(G + C)
        if mrt is None:
            post = [f[(a, n)] - (f[(a, n)] - feqs[a]) / tau + (1 - 0.5 / tau) * srcs[a] for a in range(Q)]
        else:
            if mrt.get("nu") is None:
                tv = tau
            elif scheme == "improved":
                tv = mrt["nu"] * r / pm[n] + 0.5
            else:
                tv = 3.0 * mrt["nu"] + 0.5
            rates = [1.0, mrt["s_e"], mrt["s_eps"], 1.0, mrt["s_q"], 1.0, mrt["s_q"], 1.0 / tv, 1.0 / tv]
            mstar = []
            for k in range(9):
                mk = sum(MLL[k][a] * f[(a, n)] for a in range(9))
                mek = sum(MLL[k][a] * feqs[a] for a in range(9))
                sk = sum(MLL[k][a] * srcs[a] for a in range(9))
                mstar.append(mk - rates[k] * (mk - mek) + (1 - 0.5 * rates[k]) * sk)
            norms = [sum(MLL[k][a] ** 2 for a in range(9)) for k in range(9)]
            post = [sum(MLL[k][a] * mstar[k] / norms[k] for k in range(9)) for a in range(9)]
        for a in range(Q):
            ty = n[1] + E[a][1] if D == 2 else None
            if walls is not None and not 0 <= ty < dims[1]:
                b = E.index(tuple(-x for x in E[a]))
                U = walls[0] if ty < 0 else walls[1]
                out[(b, n)] = post[a] + feq_of(b, (U, 0.0)) - feq_of(a, (U, 0.0))
            else:
                out[(a, nb(n, E[a]))] = post[a]          # streaming, Eq. 10
    return out, {"rho": rho, "u": u, "mu": mu, "F": F}
