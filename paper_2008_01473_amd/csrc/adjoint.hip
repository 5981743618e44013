// Hand-written adjoint (vector-Jacobian product) of one D2Q9 time step, of the
// initialisation, and of the map f -> (rho, u), for the standard scheme with
// the chemical-potential force and for the improved scheme.
//
// Forward step at a node (all derivatives below are of these formulas):
//   rho = sum f, j = sum e f (Eq. 12);  mu = mu_EOS(rho) - kappa L rho (Eq. 2)
//   g = grad_d mu (Eq. 17);  F = (1/3 - rho) g (Eq. 24)  or  grad_d(rho)/3 - rho g (Eq. 13)
//   u = (j + F/2) / rho (Eq. 12);  p_m = (c0 + mu)/3 (improved; the paper: c0 = 1) or rho/3
//   phi = rho/3 - p_m, psi_i = phi u_i, d_i = d_i psi_i, C_ii = 3 d_i (Eq. 29)
//   f*_a = (1 - w) f_a + w feq_a(rho, u, p_m) + (1 - w/2) (G_a(u, F) + C_a(C_xx, C_yy))
//   f_a(x + e_a, t + 1) = f*_a(x) (Eq. 10)
// Adjoint of one step, given lam = dL/df(t+1) (post-streaming layout):
//   a_a(x)   = lam_a(x + e_a)                         (transpose of streaming)
//   from f*: direct (1 - w) a; feq_bar = w a; G_bar = C_bar = (1 - w/2) a
//   local partials of feq, G, C give rho_bar, u_bar, pm_bar, F_bar, d_bar
//   psi_bar_i = -d_i(d_bar_i)  (the transpose of the Eq. 17 stencil is its negative)
//   phi_bar = psi_bar . u; u_bar += phi psi_bar; rho_bar += phi_bar/3; pm_bar -= phi_bar
//   mu_bar = pm_bar/3 (improved; standard: rho_bar += pm_bar/3)
//   j_bar = u_bar/rho; F_bar += u_bar/(2 rho); rho_bar -= u_bar . u / rho
//   rho_bar -= F_bar . g; g_bar = (1/3 - rho) F_bar (improved) or -rho F_bar, and for the
//     standard force rho_bar -= div_d(F_bar)/3
//   mu_bar -= div_d(g_bar)
//   rho_bar += mu_EOS'(rho) mu_bar - kappa L mu_bar   (L is symmetric)
//   kappa_bar -= sum mu_bar L rho;  (T/Tc)_bar += sum mu_bar d mu_EOS / d(T/Tc)
//   dL/df_a(t) = (1 - w) a_a + rho_bar + e_a . j_bar
// All adjoint arithmetic is float64; the forward fields are recomputed in
// float64 from the stored state (float64 or float32 deviations).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "lbm_device.hpp"
#include "lbm_shared.hpp"

namespace lbm {
namespace adj {

__device__ constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr double W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                    1.0 / 36};

// Field indices in the adjoint workspace (each nnodes doubles).
enum Field {
    RHO, JX, JY, MU, LR, MUR, MUT, GX, GY, FX, FY, UX, UY,
    RB, UXB, UYB, PB, FXB, FYB, DXB, DYB, JXB, JYB, GXB, GYB, MUB,
    NFIELDS
};

struct AdjArgs {
    const void* state;      // forward state at time t (library storage, pull layout)
    const double* lam_in;   // dL/df(t+1), [9][N]
    double* lam_out;        // dL/df(t), [9][N]
    const double* rho_bar;  // cotangent of rho (fields mode) or null
    const double* u_bar;    // cotangent of u, [2][N] (fields mode) or null
    const double* rho0;     // initial density (init mode)
    double* grad_rho0;      // output of the init mode
    double* ws;             // NFIELDS * N doubles
    double* partial;        // 2 doubles per block
    double* grad;           // [kappa_bar, (T/Tc)_bar], incremented
    int pending;            // partials of the previous adjoint step wait in `partial` (blocks)
    LatticeRec rec;
    double dRT;             // d(R T) / d(T/Tc) = R T_c
    int N, nx, ny, improved, precision;
};

__device__ __forceinline__ double* F(const AdjArgs& a, int k) { return a.ws + (size_t)k * a.N; }

struct Nbr {
    int xm, xp, ym, yp, x, y;
};
// Neighbours of node (x, y), 0 <= x < nx, 0 <= y < ny (periodic).
__device__ __forceinline__ Nbr nbr_xy(int x, int y, int nx, int ny) {
    Nbr n;
    n.x = x;
    n.y = y;
    n.xm = x == 0 ? nx - 1 : x - 1;
    n.xp = x == nx - 1 ? 0 : x + 1;
    n.ym = y == 0 ? ny - 1 : y - 1;
    n.yp = y == ny - 1 ? 0 : y + 1;
    return n;
}
__device__ __forceinline__ Nbr nbr(int i, int nx, int ny) {
    Nbr n;
    n.x = i % nx;
    n.y = i / nx;
    n.xm = n.x == 0 ? nx - 1 : n.x - 1;
    n.xp = n.x == nx - 1 ? 0 : n.x + 1;
    n.ym = n.y == 0 ? ny - 1 : n.y - 1;
    n.yp = n.y == ny - 1 ? 0 : n.y + 1;
    return n;
}
__device__ __forceinline__ int at(const Nbr& n, int dx, int dy, int nx) {
    const int x = dx < 0 ? n.xm : (dx > 0 ? n.xp : n.x);
    const int y = dy < 0 ? n.ym : (dy > 0 ? n.yp : n.y);
    return y * nx + x;
}
// Eq. 17 gradient components and the isotropic Laplacian of a global field.
__device__ __forceinline__ double ddx(const double* p, const Nbr& n, int nx) {
    return (4.0 * (p[at(n, 1, 0, nx)] - p[at(n, -1, 0, nx)]) + (p[at(n, 1, 1, nx)] - p[at(n, -1, 1, nx)]) +
            (p[at(n, 1, -1, nx)] - p[at(n, -1, -1, nx)])) * (1.0 / 12.0);
}
__device__ __forceinline__ double ddy(const double* p, const Nbr& n, int nx) {
    return (4.0 * (p[at(n, 0, 1, nx)] - p[at(n, 0, -1, nx)]) + (p[at(n, 1, 1, nx)] + p[at(n, -1, 1, nx)]) -
            (p[at(n, -1, -1, nx)] + p[at(n, 1, -1, nx)])) * (1.0 / 12.0);
}
__device__ __forceinline__ double lap(const double* p, const Nbr& n, int nx) {
    const int c = n.y * nx + n.x;
    return (4.0 * (p[at(n, 1, 0, nx)] + p[at(n, -1, 0, nx)] + p[at(n, 0, 1, nx)] + p[at(n, 0, -1, nx)]) +
            (p[at(n, 1, 1, nx)] + p[at(n, -1, 1, nx)] + p[at(n, -1, -1, nx)] + p[at(n, 1, -1, nx)]) - 20.0 * p[c]) *
           (1.0 / 6.0);
}

// mu_EOS, d mu_EOS / d rho and d mu_EOS / d(T/Tc) for the two free energies.
// dRT = d(R T)/d(T/Tc) = R T_c, so d mu_EOS / d(T/Tc) = dRT * (mu_EOS + 2 a rho) / (R T).
__device__ __forceinline__ void eos_terms(const LatticeRec& R, double dRT, double rho, double& mu,
                                          double& dmu_drho, double& dmu_dt) {
    const double RT = R.RT, a = R.a, b = R.b;
    // one reciprocal of (1 - b rho) or (1 - h) and one of rho (rcp_nr); the
    // kernels' float64 logarithm (log_pos)
    const double ir = rcp_nr(rho);
    if (R.eos == 0) {
        const double ibr = rcp_nr(1.0 - b * rho);
        const double s = log_pos(rho * ibr) + ibr;
        mu = RT * s - 2.0 * a * rho;
        dmu_drho = RT * ir * (ibr * ibr) - 2.0 * a;
        dmu_dt = dRT * s;
    } else {
        const double h = 0.25 * b * rho, iom = rcp_nr(1.0 - h);
        const double iom3 = iom * iom * iom;
        const double s = log_pos(rho) + 1.0 + h * (8.0 - 9.0 * h + 3.0 * h * h) * iom3;
        mu = RT * s - 2.0 * a * rho;
        const double num = 1.0 + 4.0 * h + 4.0 * h * h - 4.0 * h * h * h + h * h * h * h;
        dmu_drho = RT * num * ir * (iom3 * iom) - 2.0 * a;
        dmu_dt = dRT * s;
    }
}

template <typename S>
__device__ __forceinline__ double state_f(const AdjArgs& a, int q, int x, int y) {
    // post-streaming f_q(x, y) = stored f*_q(x - e_q) + fbar_q
    const int nx = a.nx, ny = a.ny;
    int sx = x - EX[q], sy = y - EY[q];
    sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
    sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
    const S* st = reinterpret_cast<const S*>(a.state) + a.rec.state_offset * 9;
    return (double)st[(size_t)q * a.N + sy * nx + sx] + a.rec.fbar[q];
}

// ---- forward fields -----------------------------------------------------------
// mu and the EOS derivatives of the initial density (init mode).
__global__ void fwd_mu(AdjArgs a, int from_rho0) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const double* rho = from_rho0 ? a.rho0 : F(a, RHO);
    const Nbr n = nbr(i, a.nx, a.ny);
    double mu, dr, dt;
    eos_terms(a.rec, a.dRT, rho[i], mu, dr, dt);
    const double L = lap(rho, n, a.nx);
    F(a, MU)[i] = mu - a.rec.kappa * L;
    F(a, LR)[i] = L;
    F(a, MUR)[i] = dr;
    F(a, MUT)[i] = dt;
}

// ---- adjoint ---------------------------------------------------------------------
// A1: local adjoint of the collision at node i; lam[q] = lam_in(x + e_q).
__device__ __forceinline__ void collision_vjp(const AdjArgs& a, int i, const double (&lam)[9], double r, double ux,
                                              double uy, double Fx, double Fy, double mu) {
    // Every partial below is linear in lam with coefficients polynomial in e_q, so
    // it is assembled from a few moments of lam (q != 0 unless stated):
    //   W0 = sum w_q lam_q, W1 = sum w_q lam_q e_q, W2 = sum w_q lam_q e_q e_q^T,
    //   K1 = sum k_q lam_q e_q (k_q: coefficient of php (e.u) in the equilibrium,
    //   -1/2 on the axes, 1/4 on the diagonals), Cs = sum c_q lam_q (c_q: coefficient
    //   of p_m, 1/3 and 1/12), V0 = W0 + w_0 lam_0 (Guo forcing covers q = 0 too), and
    //   CX, CY = sum over all q of lam_q times the C_xx, C_yy coefficients of C_q.
    // Equilibrium (closed form of M^-1 Eq. 27): rest rho - 5 p_m/3 - (2/3) rho u^2;
    //   others c_q p_m + rho w_q (3 e.u + 4.5 (e.u)^2 - 1.5 u^2) + k_q php e.u.
    // Guo forcing (Eq. 14): w_q [3 (e - u).F + 9 (e.u)(e.F)].
    const double w = a.rec.omega, w2 = 1.0 - 0.5 * w;
    const double pm = a.improved ? (a.rec.c0 + mu) * (1.0 / 3.0) : r * (1.0 / 3.0);
    const double php = pm - r * (1.0 / 3.0);
    const double usq = ux * ux + uy * uy;
    const double ax = lam[1] + lam[3], ay = lam[2] + lam[4];            // axis pairs
    const double dxa = lam[1] - lam[3], dya = lam[2] - lam[4];
    const double dg = (lam[5] + lam[7]) + (lam[6] + lam[8]);            // diagonals
    const double dgx = (lam[5] - lam[7]) + (lam[8] - lam[6]);           // sum e_x lam over diagonals
    const double dgy = (lam[5] - lam[7]) + (lam[6] - lam[8]);           // sum e_y lam over diagonals
    const double dgxy = (lam[5] + lam[7]) - (lam[6] + lam[8]);          // sum e_x e_y lam
    const double W0 = (ax + ay) * (1.0 / 9.0) + dg * (1.0 / 36.0);
    const double W1x = dxa * (1.0 / 9.0) + dgx * (1.0 / 36.0), W1y = dya * (1.0 / 9.0) + dgy * (1.0 / 36.0);
    const double Wxx = ax * (1.0 / 9.0) + dg * (1.0 / 36.0), Wyy = ay * (1.0 / 9.0) + dg * (1.0 / 36.0);
    const double Wxy = dgxy * (1.0 / 36.0);
    const double K1x = -0.5 * dxa + 0.25 * dgx, K1y = -0.5 * dya + 0.25 * dgy;
    const double Cs = (ax + ay) * (1.0 / 3.0) + dg * (1.0 / 12.0);
    const double V0 = W0 + (4.0 / 9.0) * lam[0];
    const double l0 = lam[0];
    const double uK = ux * K1x + uy * K1y;
    const double W2ux = Wxx * ux + Wxy * uy, W2uy = Wxy * ux + Wyy * uy;      // W2 u
    const double W2Fx = Wxx * Fx + Wxy * Fy, W2Fy = Wxy * Fx + Wyy * Fy;      // W2 F
    const double rb = w * (l0 * (1.0 - (2.0 / 3.0) * usq) + 3.0 * (ux * W1x + uy * W1y) +
                           4.5 * (ux * W2ux + uy * W2uy) - 1.5 * usq * W0 - uK * (1.0 / 3.0));
    const double pb = w * (-(5.0 / 3.0) * l0 + Cs + uK);
    const double uxb = w * (-(4.0 / 3.0) * r * ux * l0 + r * (3.0 * W1x + 9.0 * W2ux - 3.0 * ux * W0) + php * K1x) +
                       w2 * (-3.0 * Fx * V0 + 9.0 * W2Fx);
    const double uyb = w * (-(4.0 / 3.0) * r * uy * l0 + r * (3.0 * W1y + 9.0 * W2uy - 3.0 * uy * W0) + php * K1y) +
                       w2 * (-3.0 * Fy * V0 + 9.0 * W2Fy);
    const double fxb = w2 * (3.0 * W1x - 3.0 * ux * V0 + 9.0 * W2ux);
    const double fyb = w2 * (3.0 * W1y - 3.0 * uy * V0 + 9.0 * W2uy);
    double cxxb = 0.0, cyyb = 0.0;
    if (a.improved) {
        // C_q coefficients (C_xx, C_yy): rest (-1/3, -1/3); +-x (1/6, -1/3); +-y (-1/3, 1/6); diagonals (1/6, 1/6)
        cxxb = w2 * (-(1.0 / 3.0) * l0 + (1.0 / 6.0) * ax - (1.0 / 3.0) * ay + (1.0 / 6.0) * dg);
        cyyb = w2 * (-(1.0 / 3.0) * l0 - (1.0 / 3.0) * ax + (1.0 / 6.0) * ay + (1.0 / 6.0) * dg);
    }
    F(a, RB)[i] = rb;
    F(a, UXB)[i] = uxb;
    F(a, UYB)[i] = uyb;
    F(a, PB)[i] = pb;
    F(a, FXB)[i] = fxb;
    F(a, FYB)[i] = fyb;
    F(a, DXB)[i] = 3.0 * cxxb;
    F(a, DYB)[i] = 3.0 * cyyb;
}

// A0 + A1 fused on a tile of TX x TY nodes: rho, j on the tile + 2 rings and mu on
// the tile + 1 ring in LDS, then at each node of the tile g = grad mu, F, u and the
// local adjoint of the collision (the same formulas, in the same order, as
// fwd_moments, fwd_mu, fwd_force and adj_local, which it replaces in the step and
// fields modes).
constexpr int TX = 32, TY = 8;
// Threads per work group: twice the tile, so that the ring stages (tile + 2: 432
// nodes, tile + 1: 340) take one pass each; the tile's own nodes use the first half.
constexpr int NTH = 2 * TX * TY;
constexpr int RW = TX + 4, RH = TY + 4;      // rho, j: tile + 2
constexpr int MW = TX + 2, MH = TY + 2;      // mu: tile + 1

__device__ __forceinline__ int wrapn(int v, int n) {
    // one period off in either direction needs no division; lattices narrower than
    // the tile's halo take the remainder
    v += v < 0 ? n : 0;
    v -= v >= n ? n : 0;
    if ((unsigned)v < (unsigned)n) return v;
    const int r = v % n;
    return r < 0 ? r + n : r;
}
template <int W>
__device__ __forceinline__ double lds_ddx(const double* p, int c) {
    return (4.0 * (p[c + 1] - p[c - 1]) + (p[c + W + 1] - p[c + W - 1]) + (p[c - W + 1] - p[c - W - 1])) *
           (1.0 / 12.0);
}
template <int W>
__device__ __forceinline__ double lds_ddy(const double* p, int c) {
    return (4.0 * (p[c + W] - p[c - W]) + (p[c + W + 1] + p[c + W - 1]) - (p[c - W - 1] + p[c - W + 1])) *
           (1.0 / 12.0);
}
template <int W>
__device__ __forceinline__ double lds_lap(const double* p, int c) {
    return (4.0 * (p[c + 1] + p[c - 1] + p[c + W] + p[c - W]) + (p[c + W + 1] + p[c + W - 1] + p[c - W - 1] +
                                                                   p[c - W + 1]) -
            20.0 * p[c]) *
           (1.0 / 6.0);
}

template <typename S>
__global__ __launch_bounds__(NTH) void adj_front(AdjArgs a, int fields_mode) {
    __shared__ double s_rho[RH * RW], s_jx[RH * RW], s_jy[RH * RW];
    __shared__ double s_mu[MH * MW];
    const int nx = a.nx, ny = a.ny;
    const int ntx = (nx + TX - 1) / TX;
    const int x0 = (blockIdx.x % ntx) * TX, y0 = (blockIdx.x / ntx) * TY;
    const int tid = threadIdx.x;
    // Within a segment the previous adjoint step's parameter partials are added
    // here (the sum adj_reduce would take, in the same order) before adj_back
    // overwrites them, which saves a launch per step.
    if (a.pending && blockIdx.x == 0 && tid < 64) {
        double k = 0, t = 0;
        for (int b = tid; b < a.pending; b += 64) {
            k += a.partial[2 * b];
            t += a.partial[2 * b + 1];
        }
        k = wave_sum(k);
        t = wave_sum(t);
        if (tid == 0) {
            a.grad[0] += k;
            a.grad[1] += t;
        }
    }
    const int lx = tid % TX, ly = tid / TX;
    const int gx = x0 + lx, gy = y0 + ly;
    const bool own = tid < TX * TY && gx < nx && gy < ny;
    const int i = own ? gy * nx + gx : 0;
    const Nbr n = own ? nbr_xy(gx, gy, nx, ny) : nbr_xy(0, 0, nx, ny);
    // the cotangents gathered by the collision adjoint, lam(x + e_q), are loaded
    // first so that their latency overlaps the stages below
    double lam[9];
    if (own && !fields_mode) {
#pragma unroll
        for (int q = 0; q < 9; ++q) lam[q] = a.lam_in[(size_t)q * a.N + at(n, EX[q], EY[q], nx)];
    }
    // rho and j on the tile + 2 rings (periodic): both of a thread's nodes' pulls
    // are issued before either is summed
    constexpr int NT = NTH, NR = (RH * RW + NT - 1) / NT;
    double fr[NR][9];
#pragma unroll
    for (int h = 0; h < NR; ++h) {
        const int k = tid + h * NT;
        if (k < RH * RW) {
            const int x = wrapn(x0 - 2 + k % RW, nx), y = wrapn(y0 - 2 + k / RW, ny);
#pragma unroll
            for (int q = 0; q < 9; ++q) fr[h][q] = state_f<S>(a, q, x, y);
        }
    }
#pragma unroll
    for (int h = 0; h < NR; ++h) {
        const int k = tid + h * NT;
        if (k < RH * RW) {
            double r = 0, jx = 0, jy = 0;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                r += fr[h][q];
                jx += EX[q] * fr[h][q];
                jy += EY[q] * fr[h][q];
            }
            s_rho[k] = r;
            s_jx[k] = jx;
            s_jy[k] = jy;
        }
    }
    __syncthreads();
    // mu on the tile + 1 ring; L, dmu/drho and dmu/d(T/Tc) of the tile's nodes
    for (int k = tid; k < MH * MW; k += NTH) {
        const int mx = k % MW, my = k / MW;
        const int c = (my + 1) * RW + mx + 1;
        double mu, dr, dt;
        eos_terms(a.rec, a.dRT, s_rho[c], mu, dr, dt);
        const double L = lds_lap<RW>(s_rho, c);
        s_mu[k] = mu - a.rec.kappa * L;
        const int hx = x0 - 1 + mx, hy = y0 - 1 + my;
        if (mx >= 1 && mx <= TX && my >= 1 && my <= TY && hx < nx && hy < ny) {
            const int ih = hy * nx + hx;
            F(a, LR)[ih] = L;
            F(a, MUR)[ih] = dr;
            F(a, MUT)[ih] = dt;
        }
    }
    __syncthreads();
    if (!own) return;
    const int cr = (ly + 2) * RW + lx + 2, cm = (ly + 1) * MW + lx + 1;
    const double r = s_rho[cr];
    const double gxv = lds_ddx<MW>(s_mu, cm), gyv = lds_ddy<MW>(s_mu, cm);
    double Fx, Fy;
    if (a.improved) {
        Fx = (1.0 / 3.0 - r) * gxv;
        Fy = (1.0 / 3.0 - r) * gyv;
    } else {
        Fx = lds_ddx<RW>(s_rho, cr) * (1.0 / 3.0) - r * gxv;
        Fy = lds_ddy<RW>(s_rho, cr) * (1.0 / 3.0) - r * gyv;
    }
    const double ir = rcp_nr(r);
    const double ux = (s_jx[cr] + 0.5 * Fx) * ir;
    const double uy = (s_jy[cr] + 0.5 * Fy) * ir;
    const double muv = s_mu[cm];
    F(a, RHO)[i] = r;
    F(a, MU)[i] = muv;
    F(a, GX)[i] = gxv;
    F(a, GY)[i] = gyv;
    F(a, UX)[i] = ux;
    F(a, UY)[i] = uy;
    if (fields_mode) {
        F(a, RB)[i] = a.rho_bar ? a.rho_bar[i] : 0.0;
        F(a, UXB)[i] = a.u_bar ? a.u_bar[i] : 0.0;
        F(a, UYB)[i] = a.u_bar ? a.u_bar[a.N + i] : 0.0;
        F(a, PB)[i] = 0.0;
        F(a, FXB)[i] = 0.0;
        F(a, FYB)[i] = 0.0;
        F(a, DXB)[i] = 0.0;
        F(a, DYB)[i] = 0.0;
        return;
    }
    collision_vjp(a, i, lam, r, ux, uy, Fx, Fy, muv);
}

// A2 - A4 fused on a tile (step and fields modes): on the tile + 2 rings the
// psi, phi, p_m, u and F adjoints (psi_bar = -d(d_bar)), on the tile + 1 ring
// mu_bar -= div(g_bar) (standard force: rho_bar -= div(F_bar)/3), and on the tile
// rho_bar through mu, the parameter partials and dL/df(t).  The same formulas,
// in the same order, as the per-node kernels they replaced.
__global__ __launch_bounds__(NTH) void adj_back(AdjArgs a, int mode) {
    constexpr int NT = NTH, VN = RH * RW, MN = MH * MW;
    __shared__ double s_gxb[VN], s_gyb[VN], s_fxb[VN], s_fyb[VN], s_rb[VN], s_mub[VN], s_jxb[VN], s_jyb[VN];
    __shared__ double s_mub2[MN], s_rb2[MN];
    __shared__ double sk[NT], st[NT];
    const int nx = a.nx, ny = a.ny;
    const int ntx = (nx + TX - 1) / TX;
    const int x0 = (blockIdx.x % ntx) * TX, y0 = (blockIdx.x / ntx) * TY;
    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    const int gx = x0 + lx, gy = y0 + ly;
    const bool own = tid < TX * TY && gx < nx && gy < ny;
    const int i = own ? gy * nx + gx : 0;
    const Nbr n = own ? nbr_xy(gx, gy, nx, ny) : nbr_xy(0, 0, nx, ny);
    double lam[9];
    if (own && mode == 0) {
#pragma unroll
        for (int q = 0; q < 9; ++q) lam[q] = a.lam_in[(size_t)q * a.N + at(n, EX[q], EY[q], nx)];
    }
    // psi, phi, p_m, u and F adjoints on the tile + 2 rings
    for (int k = tid; k < VN; k += NT) {
        const int x = wrapn(x0 - 2 + k % RW, nx), y = wrapn(y0 - 2 + k / RW, ny);
        const int j = y * nx + x;
        const Nbr m = nbr_xy(x, y, nx, ny);
        const double r = F(a, RHO)[j], ux = F(a, UX)[j], uy = F(a, UY)[j];
        double rb = F(a, RB)[j], uxb = F(a, UXB)[j], uyb = F(a, UYB)[j], pb = F(a, PB)[j];
        double fxb = F(a, FXB)[j], fyb = F(a, FYB)[j];
        double mub = 0.0;
        if (a.improved) {
            const double psixb = -ddx(F(a, DXB), m, nx);
            const double psiyb = -ddy(F(a, DYB), m, nx);
            const double pm = (a.rec.c0 + F(a, MU)[j]) * (1.0 / 3.0);
            const double phi = r * (1.0 / 3.0) - pm;
            const double phib = psixb * ux + psiyb * uy;
            uxb += phi * psixb;
            uyb += phi * psiyb;
            rb += phib * (1.0 / 3.0);
            pb -= phib;
            mub = pb * (1.0 / 3.0);
        } else {
            rb += pb * (1.0 / 3.0);
        }
        const double ir = rcp_nr(r);
        s_jxb[k] = uxb * ir;
        s_jyb[k] = uyb * ir;
        fxb += 0.5 * uxb * ir;
        fyb += 0.5 * uyb * ir;
        rb -= (uxb * ux + uyb * uy) * ir;
        rb -= fxb * F(a, GX)[j] + fyb * F(a, GY)[j];
        const double gfac = a.improved ? (1.0 / 3.0 - r) : -r;
        s_gxb[k] = gfac * fxb;
        s_gyb[k] = gfac * fyb;
        s_fxb[k] = fxb;
        s_fyb[k] = fyb;
        s_rb[k] = rb;
        s_mub[k] = mub;
    }
    __syncthreads();
    // mu_bar -= div(g_bar) on the tile + 1 ring
    for (int k = tid; k < MN; k += NT) {
        const int c = (k / MW + 1) * RW + k % MW + 1;
        s_mub2[k] = s_mub[c] - (lds_ddx<RW>(s_gxb, c) + lds_ddy<RW>(s_gyb, c));
        double rb = s_rb[c];
        if (!a.improved) rb -= (lds_ddx<RW>(s_fxb, c) + lds_ddy<RW>(s_fyb, c)) * (1.0 / 3.0);
        s_rb2[k] = rb;
    }
    __syncthreads();
    // rho_bar through mu, parameter partials, dL/df(t)
    double kb = 0.0, tb = 0.0;
    if (own) {
        const int cm = (ly + 1) * MW + lx + 1, cr = (ly + 2) * RW + lx + 2;
        const double mub = s_mub2[cm];
        double rb = s_rb2[cm];
        rb += F(a, MUR)[i] * mub - a.rec.kappa * lds_lap<MW>(s_mub2, cm);
        kb = -mub * F(a, LR)[i];
        tb = mub * F(a, MUT)[i];
        const double jxb = s_jxb[cr], jyb = s_jyb[cr];
        const double w1 = 1.0 - a.rec.omega;
        for (int q = 0; q < 9; ++q) {
            double v = rb + EX[q] * jxb + EY[q] * jyb;
            if (mode == 0) v += w1 * lam[q];
            a.lam_out[(size_t)q * a.N + i] = v;
        }
    }
    // tile partial sums of the parameter gradients, in a fixed order
    sk[tid] = kb;
    st[tid] = tb;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (tid < w) {
            sk[tid] += sk[tid + w];
            st[tid] += st[tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        a.partial[2 * blockIdx.x] = sk[0];
        a.partial[2 * blockIdx.x + 1] = st[0];
    }
}

// Init mode, after adj_init_local: rho_bar through mu (PB = mu_bar, RB = rho_bar),
// the parameter partials and dL/drho0 (mode 2; modes 0 and 1 are adj_back's).
__global__ __launch_bounds__(256) void adj_final(AdjArgs a, int mode) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double kb = 0.0, tb = 0.0;
    if (i < a.N) {
        const Nbr n = nbr(i, a.nx, a.ny);
        const double mub = F(a, PB)[i];
        double rb = (mode == 2) ? F(a, RB)[i] : F(a, DXB)[i];
        rb += F(a, MUR)[i] * mub - a.rec.kappa * lap(F(a, PB), n, a.nx);
        kb = -mub * F(a, LR)[i];
        tb = mub * F(a, MUT)[i];
        if (mode == 2) {
            a.grad_rho0[i] = rb;
        } else {
            const double jxb = F(a, JXB)[i], jyb = F(a, JYB)[i];
            const double w1 = 1.0 - a.rec.omega;
            for (int q = 0; q < 9; ++q) {
                double v = rb + EX[q] * jxb + EY[q] * jyb;
                if (mode == 0) v += w1 * a.lam_in[(size_t)q * a.N + at(n, EX[q], EY[q], a.nx)];
                a.lam_out[(size_t)q * a.N + i] = v;
            }
        }
    }
    // block partial sums of the parameter gradients, in a fixed order
    __shared__ double sk[256], st[256];
    sk[threadIdx.x] = kb;
    st[threadIdx.x] = tb;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sk[threadIdx.x] += sk[threadIdx.x + w];
            st[threadIdx.x] += st[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.partial[2 * blockIdx.x] = sk[0];
        a.partial[2 * blockIdx.x + 1] = st[0];
    }
}

// Init VJP, local part: f0 = feq(rho0, 0, p_m(mu(rho0))).
__global__ void adj_init_local(AdjArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    double rb = 0, pb = 0;
    for (int q = 0; q < 9; ++q) {
        const double l = a.lam_in[(size_t)q * a.N + i];
        if (q == 0) { rb += l; pb += -5.0 / 3.0 * l; }
        else pb += (q < 5 ? 1.0 / 3.0 : 1.0 / 12.0) * l;
    }
    if (a.improved) {
        F(a, PB)[i] = pb * (1.0 / 3.0);   // mu_bar
        F(a, RB)[i] = rb;
    } else {
        F(a, PB)[i] = 0.0;
        F(a, RB)[i] = rb + pb * (1.0 / 3.0);
    }
}

// Sum the block partials and add them to the two accumulators: one wave, lane l
// summing blocks l, l + 64, ... in order, then a fixed butterfly across the lanes,
// so that every run adds in the same order.  (A last-block-done reduction inside
// adj_final was measured slower: the device-scope fence of every block costs more
// than this launch.)
__global__ void adj_reduce(const double* partial, int nblocks, double* grad) {
    const int lane = threadIdx.x;
    double k = 0, t = 0;
    for (int b = lane; b < nblocks; b += 64) {
        k += partial[2 * b];
        t += partial[2 * b + 1];
    }
    k = wave_sum(k);
    t = wave_sum(t);
    if (lane == 0) {
        grad[0] += k;
        grad[1] += t;
    }
}

}  // namespace adj

// Fields and two partial sums per block: 256-node blocks (init mode) or tiles.
size_t adjoint_workspace_doubles(int nx, int ny) {
    const long long N = (long long)nx * ny;
    const long long tiles = (long long)((nx + adj::TX - 1) / adj::TX) * ((ny + adj::TY - 1) / adj::TY);
    const long long blocks = std::max<long long>((N + 255) / 256, tiles);
    return (size_t)adj::NFIELDS * (size_t)N + 2 * (size_t)blocks;
}

// Device workspace of the allocation-free adjoint step (lbm_adjoint_step_noalloc):
// a fixed array in each GPU's global memory, held until the process ends.  In host
// code `scratch` only names the symbol; its device address comes from
// hipGetSymbolAddress, once per device with that device current, and is kept here.
constexpr size_t kStaticScratchBytes = size_t(24) << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

size_t static_scratch_bytes() { return kStaticScratchBytes; }

// Device address of the current device's scratch array (resolved on the first
// call per device; later calls return the kept address).
hipError_t static_scratch(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// kind: 0 step, 1 fields (rho_bar/u_bar given), 2 init.  chain (steps of a
// segment): kAdjPending = the previous step's partials are still to be added,
// kAdjDeferReduce = leave this step's partials to the next step.
hipError_t adjoint_launch(int kind, const LatticeRec& rec, double dRT, int precision, int improved, const void* state,
                          const double* lam_in, double* lam_out, const double* rho_bar, const double* u_bar,
                          const double* rho0, double* grad_rho0, double* ws, double* grad, hipStream_t s,
                          int chain) {
    adj::AdjArgs a;
    a.state = state;
    a.lam_in = lam_in;
    a.lam_out = lam_out;
    a.rho_bar = rho_bar;
    a.u_bar = u_bar;
    a.rho0 = rho0;
    a.grad_rho0 = grad_rho0;
    a.rec = rec;
    a.dRT = dRT;
    a.nx = rec.nx;
    a.ny = rec.ny;
    a.N = (int)rec.nnodes;
    a.ws = ws;
    a.partial = ws + (size_t)adj::NFIELDS * a.N;
    a.improved = improved;
    a.precision = precision;
    a.grad = grad;
    a.pending = 0;
    const int B = 256, G = (a.N + B - 1) / B;
    if (kind == 2) {
        hipLaunchKernelGGL(adj::fwd_mu, dim3(G), dim3(B), 0, s, a, 1);
        hipLaunchKernelGGL(adj::adj_init_local, dim3(G), dim3(B), 0, s, a);
        hipLaunchKernelGGL(adj::adj_final, dim3(G), dim3(B), 0, s, a, 2);
        hipLaunchKernelGGL(adj::adj_reduce, dim3(1), dim3(64), 0, s, a.partial, G, grad);
        return hipGetLastError();
    }
    const int tiles = ((a.nx + adj::TX - 1) / adj::TX) * ((a.ny + adj::TY - 1) / adj::TY);
    a.pending = (chain & kAdjPending) ? tiles : 0;
    if (precision == 0)
        hipLaunchKernelGGL(adj::adj_front<double>, dim3(tiles), dim3(adj::NTH), 0, s, a, kind == 1 ? 1 : 0);
    else
        hipLaunchKernelGGL(adj::adj_front<float>, dim3(tiles), dim3(adj::NTH), 0, s, a, kind == 1 ? 1 : 0);
    hipLaunchKernelGGL(adj::adj_back, dim3(tiles), dim3(adj::NTH), 0, s, a, kind == 1 ? 1 : 0);
    if (!(chain & kAdjDeferReduce))
        hipLaunchKernelGGL(adj::adj_reduce, dim3(1), dim3(64), 0, s, a.partial, tiles, grad);
    return hipGetLastError();
}

}  // namespace lbm
