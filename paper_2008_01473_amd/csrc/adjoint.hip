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
    LatticeRec rec;
    double dRT;             // d(R T) / d(T/Tc) = R T_c
    int N, nx, ny, improved, precision;
};

__device__ __forceinline__ double* F(const AdjArgs& a, int k) { return a.ws + (size_t)k * a.N; }

struct Nbr {
    int xm, xp, ym, yp, x, y;
};
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
            (p[at(n, 1, -1, nx)] - p[at(n, -1, -1, nx)])) / 12.0;
}
__device__ __forceinline__ double ddy(const double* p, const Nbr& n, int nx) {
    return (4.0 * (p[at(n, 0, 1, nx)] - p[at(n, 0, -1, nx)]) + (p[at(n, 1, 1, nx)] + p[at(n, -1, 1, nx)]) -
            (p[at(n, -1, -1, nx)] + p[at(n, 1, -1, nx)])) / 12.0;
}
__device__ __forceinline__ double lap(const double* p, const Nbr& n, int nx) {
    const int c = n.y * nx + n.x;
    return (4.0 * (p[at(n, 1, 0, nx)] + p[at(n, -1, 0, nx)] + p[at(n, 0, 1, nx)] + p[at(n, 0, -1, nx)]) +
            (p[at(n, 1, 1, nx)] + p[at(n, -1, 1, nx)] + p[at(n, -1, -1, nx)] + p[at(n, 1, -1, nx)]) - 20.0 * p[c]) /
           6.0;
}

// mu_EOS, d mu_EOS / d rho and d mu_EOS / d(T/Tc) for the two free energies.
// dRT = d(R T)/d(T/Tc) = R T_c, so d mu_EOS / d(T/Tc) = dRT * (mu_EOS + 2 a rho) / (R T).
__device__ __forceinline__ void eos_terms(const LatticeRec& R, double dRT, double rho, double& mu,
                                          double& dmu_drho, double& dmu_dt) {
    const double RT = R.RT, a = R.a, b = R.b;
    if (R.eos == 0) {
        const double br = 1.0 - b * rho;
        const double s = log(rho / br) + 1.0 / br;
        mu = RT * s - 2.0 * a * rho;
        dmu_drho = RT / (rho * br * br) - 2.0 * a;
        dmu_dt = dRT * s;
    } else {
        const double h = 0.25 * b * rho, om = 1.0 - h;
        const double s = log(rho) + 1.0 + h * (8.0 - 9.0 * h + 3.0 * h * h) / (om * om * om);
        mu = RT * s - 2.0 * a * rho;
        const double num = 1.0 + 4.0 * h + 4.0 * h * h - 4.0 * h * h * h + h * h * h * h;
        dmu_drho = RT * num / (rho * om * om * om * om) - 2.0 * a;
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
template <typename S>
__global__ void fwd_moments(AdjArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const int x = i % a.nx, y = i / a.nx;
    double r = 0, jx = 0, jy = 0;
    for (int q = 0; q < 9; ++q) {
        const double f = state_f<S>(a, q, x, y);
        r += f;
        jx += EX[q] * f;
        jy += EY[q] * f;
    }
    F(a, RHO)[i] = r;
    F(a, JX)[i] = jx;
    F(a, JY)[i] = jy;
}

// mu and the EOS derivatives; the density comes from RHO (steps) or rho0 (init).
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

__global__ void fwd_force(AdjArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const Nbr n = nbr(i, a.nx, a.ny);
    const double r = F(a, RHO)[i];
    const double gx = ddx(F(a, MU), n, a.nx), gy = ddy(F(a, MU), n, a.nx);
    double Fx, Fy;
    if (a.improved) {
        Fx = (1.0 / 3.0 - r) * gx;
        Fy = (1.0 / 3.0 - r) * gy;
    } else {
        Fx = ddx(F(a, RHO), n, a.nx) / 3.0 - r * gx;
        Fy = ddy(F(a, RHO), n, a.nx) / 3.0 - r * gy;
    }
    F(a, GX)[i] = gx;
    F(a, GY)[i] = gy;
    F(a, FX)[i] = Fx;
    F(a, FY)[i] = Fy;
    F(a, UX)[i] = (F(a, JX)[i] + 0.5 * Fx) / r;
    F(a, UY)[i] = (F(a, JY)[i] + 0.5 * Fy) / r;
}

// ---- adjoint ---------------------------------------------------------------------
// A1: local adjoint of the collision (or the given field cotangents).
__global__ void adj_local(AdjArgs a, int fields_mode) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
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
    const Nbr n = nbr(i, a.nx, a.ny);
    const double w = a.rec.omega, w2 = 1.0 - 0.5 * w;
    const double r = F(a, RHO)[i], ux = F(a, UX)[i], uy = F(a, UY)[i];
    const double Fx = F(a, FX)[i], Fy = F(a, FY)[i];
    const double pm = a.improved ? (a.rec.c0 + F(a, MU)[i]) / 3.0 : r / 3.0;
    const double php = pm - r / 3.0;
    const double usq = ux * ux + uy * uy;
    double rb = 0, uxb = 0, uyb = 0, pb = 0, fxb = 0, fyb = 0, cxxb = 0, cyyb = 0;
    for (int q = 0; q < 9; ++q) {
        const double ab = a.lam_in[(size_t)q * a.N + at(n, EX[q], EY[q], a.nx)];   // lam(x + e_q)
        const double ex = EX[q], ey = EY[q];
        const double eu = ex * ux + ey * uy, eF = ex * Fx + ey * Fy;
        const double fe = w * ab, gb = w2 * ab;
        // equilibrium partials (closed form of M^-1 Eq. 27)
        if (q == 0) {
            rb += fe * (1.0 - (2.0 / 3.0) * usq);
            pb += fe * (-5.0 / 3.0);
            uxb += fe * (-(4.0 / 3.0) * r * ux);
            uyb += fe * (-(4.0 / 3.0) * r * uy);
        } else {
            const double wq = W[q];
            const double k = (q < 5) ? -0.5 : 0.25;             // coefficient of php * eu
            rb += fe * (wq * (3.0 * eu + 4.5 * eu * eu - 1.5 * usq) - k * eu / 3.0);
            pb += fe * ((q < 5 ? 1.0 / 3.0 : 1.0 / 12.0) + k * eu);
            uxb += fe * (r * wq * (3.0 * ex + 9.0 * eu * ex - 3.0 * ux) + k * php * ex);
            uyb += fe * (r * wq * (3.0 * ey + 9.0 * eu * ey - 3.0 * uy) + k * php * ey);
        }
        // Guo forcing G = w [3 (e - u).F + 9 (e.u)(e.F)]
        uxb += gb * W[q] * (-3.0 * Fx + 9.0 * ex * eF);
        uyb += gb * W[q] * (-3.0 * Fy + 9.0 * ey * eF);
        fxb += gb * W[q] * (3.0 * (ex - ux) + 9.0 * eu * ex);
        fyb += gb * W[q] * (3.0 * (ey - uy) + 9.0 * eu * ey);
        // correction C (linear in C_xx, C_yy)
        if (a.improved) {
            double cx, cy;
            if (q == 0) { cx = -1.0 / 3.0; cy = -1.0 / 3.0; }
            else if (q == 1 || q == 3) { cx = 1.0 / 6.0; cy = -1.0 / 3.0; }
            else if (q == 2 || q == 4) { cx = -1.0 / 3.0; cy = 1.0 / 6.0; }
            else { cx = 1.0 / 6.0; cy = 1.0 / 6.0; }
            cxxb += gb * cx;
            cyyb += gb * cy;
        }
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

// A2: psi_bar = -d(d_bar); phi, p_m, u and F adjoints at the node.
__global__ void adj_velocity(AdjArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const Nbr n = nbr(i, a.nx, a.ny);
    const double r = F(a, RHO)[i], ux = F(a, UX)[i], uy = F(a, UY)[i];
    double rb = F(a, RB)[i], uxb = F(a, UXB)[i], uyb = F(a, UYB)[i], pb = F(a, PB)[i];
    double fxb = F(a, FXB)[i], fyb = F(a, FYB)[i];
    double mub = 0.0;
    if (a.improved) {
        const double psixb = -ddx(F(a, DXB), n, a.nx);
        const double psiyb = -ddy(F(a, DYB), n, a.nx);
        const double pm = (a.rec.c0 + F(a, MU)[i]) / 3.0;
        const double phi = r / 3.0 - pm;
        const double phib = psixb * ux + psiyb * uy;
        uxb += phi * psixb;
        uyb += phi * psiyb;
        rb += phib / 3.0;
        pb -= phib;
        mub = pb / 3.0;
    } else {
        rb += pb / 3.0;
    }
    const double ir = 1.0 / r;
    F(a, JXB)[i] = uxb * ir;
    F(a, JYB)[i] = uyb * ir;
    fxb += 0.5 * uxb * ir;
    fyb += 0.5 * uyb * ir;
    rb -= (uxb * ux + uyb * uy) * ir;
    rb -= fxb * F(a, GX)[i] + fyb * F(a, GY)[i];
    const double gfac = a.improved ? (1.0 / 3.0 - r) : -r;
    F(a, GXB)[i] = gfac * fxb;
    F(a, GYB)[i] = gfac * fyb;
    F(a, FXB)[i] = fxb;
    F(a, FYB)[i] = fyb;
    F(a, RB)[i] = rb;
    F(a, MUB)[i] = mub;
}

// A3: mu_bar -= div(g_bar); standard force: rho_bar -= div(F_bar)/3.
__global__ void adj_mu(AdjArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const Nbr n = nbr(i, a.nx, a.ny);
    // written to separate slots: PB holds mu_bar, DXB the updated rho_bar
    const double mub = F(a, MUB)[i] - (ddx(F(a, GXB), n, a.nx) + ddy(F(a, GYB), n, a.nx));
    double rb = F(a, RB)[i];
    if (!a.improved) rb -= (ddx(F(a, FXB), n, a.nx) + ddy(F(a, FYB), n, a.nx)) / 3.0;
    F(a, PB)[i] = mub;
    F(a, DXB)[i] = rb;
}

// A4: rho_bar through mu; parameter gradients; dL/df(t) (or dL/drho0 in init mode).
// mode 0: step, 1: fields, 2: init (reads PB = mu_bar, RB = rho_bar from adj_init_local).
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
        F(a, PB)[i] = pb / 3.0;   // mu_bar
        F(a, RB)[i] = rb;
    } else {
        F(a, PB)[i] = 0.0;
        F(a, RB)[i] = rb + pb / 3.0;
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

size_t adjoint_workspace_doubles(long long N) {
    const long long blocks = (N + 255) / 256;
    return (size_t)adj::NFIELDS * (size_t)N + 2 * (size_t)blocks;
}

// kind: 0 step, 1 fields (rho_bar/u_bar given), 2 init
hipError_t adjoint_launch(int kind, const LatticeRec& rec, double dRT, int precision, int improved, const void* state,
                          const double* lam_in, double* lam_out, const double* rho_bar, const double* u_bar,
                          const double* rho0, double* grad_rho0, double* ws, double* grad, hipStream_t s) {
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
    const int B = 256, G = (a.N + B - 1) / B;
    if (kind == 2) {
        hipLaunchKernelGGL(adj::fwd_mu, dim3(G), dim3(B), 0, s, a, 1);
        hipLaunchKernelGGL(adj::adj_init_local, dim3(G), dim3(B), 0, s, a);
        hipLaunchKernelGGL(adj::adj_final, dim3(G), dim3(B), 0, s, a, 2);
        hipLaunchKernelGGL(adj::adj_reduce, dim3(1), dim3(64), 0, s, a.partial, G, grad);
        return hipGetLastError();
    }
    if (precision == 0)
        hipLaunchKernelGGL(adj::fwd_moments<double>, dim3(G), dim3(B), 0, s, a);
    else
        hipLaunchKernelGGL(adj::fwd_moments<float>, dim3(G), dim3(B), 0, s, a);
    hipLaunchKernelGGL(adj::fwd_mu, dim3(G), dim3(B), 0, s, a, 0);
    hipLaunchKernelGGL(adj::fwd_force, dim3(G), dim3(B), 0, s, a);
    hipLaunchKernelGGL(adj::adj_local, dim3(G), dim3(B), 0, s, a, kind == 1 ? 1 : 0);
    hipLaunchKernelGGL(adj::adj_velocity, dim3(G), dim3(B), 0, s, a);
    hipLaunchKernelGGL(adj::adj_mu, dim3(G), dim3(B), 0, s, a);
    hipLaunchKernelGGL(adj::adj_final, dim3(G), dim3(B), 0, s, a, kind == 1 ? 1 : 0);
    hipLaunchKernelGGL(adj::adj_reduce, dim3(1), dim3(64), 0, s, a.partial, G, grad);
    return hipGetLastError();
}

}  // namespace lbm
