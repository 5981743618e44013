// D2Q9 kernels: the fused time step (one work group per output tile, halos
// recomputed in LDS), the initialisation from (rho0, u0), and conversion of
// the stored state to and from post-streaming populations.
//
// Velocity order: 0 rest; 1 E (1,0); 2 N (0,1); 3 W (-1,0); 4 S (0,-1);
//                 5 NE (1,1); 6 NW (-1,1); 7 SW (-1,-1); 8 SE (1,-1).
// State layout: one buffer per time level holding, for population a at node x,
// the post-collision value f*_a(x) of the previous step (before streaming);
// population a of lattice L lives at state_offset(L)*9 + a*nnodes(L) + y*nx + x.
// A step pulls f_a(x) = f*_a(x - e_a) (Eq. 10) and writes f*_a(x) of the new
// time level at x itself.  In FP32 deviation mode the stored value is
// f - fbar with fbar the reference rest equilibrium of the lattice.

#include <hip/hip_runtime.h>

#include "lbm_device.hpp"
#include "lbm_shared.hpp"

namespace lbm {
namespace d2q9 {

// Pull the nine populations arriving at (xc, yc): f_a(x) = f*_a(x - e_a).
// p[a] is the (wave-uniform) base of population a, so each load is a scalar
// base plus a 32-bit lane offset.
template <typename S, typename T>
__device__ __forceinline__ void pull(const S* const (&p)[9], int nx, int xm, int xc, int xp, int ym, int yc,
                                     int yp, T f[9]) {
    const unsigned rc = (unsigned)(yc * nx), rm = (unsigned)(ym * nx), rp = (unsigned)(yp * nx);
    f[0] = (T)ld_off(p[0], rc + xc);
    f[1] = (T)ld_off(p[1], rc + xm);
    f[2] = (T)ld_off(p[2], rm + xc);
    f[3] = (T)ld_off(p[3], rc + xp);
    f[4] = (T)ld_off(p[4], rp + xc);
    f[5] = (T)ld_off(p[5], rm + xm);
    f[6] = (T)ld_off(p[6], rm + xp);
    f[7] = (T)ld_off(p[7], rp + xp);
    f[8] = (T)ld_off(p[8], rp + xm);
}

// Plates (lattices bounded in y, halfway between rows -1 / 0 and ny-1 / ny): the
// node whose fields stand at row y is its mirror image beyond a plate (clamped:
// rows further out than the stencils reach are never used).
__device__ __forceinline__ int plate_row(int y, int ny, bool& mirrored) {
    mirrored = y < 0 || y >= ny;
    y = y < 0 ? -1 - y : (y >= ny ? 2 * ny - 1 - y : y);
    return min(max(y, 0), ny - 1);
}

// Pull of a fluid node in row yc of a lattice with plates: populations that would
// come from beyond a plate are read from the node's own slot of the reversed
// direction, which the previous step stored already reflected (bounce-back).
// Loads for rows past a plate are clamped in bounds and then replaced.
template <typename S, typename T>
__device__ __forceinline__ void pull_plates(const S* const (&p)[9], int nx, int ny, int xm, int xc, int xp,
                                            int yc, T f[9]) {
    const int ym = yc > 0 ? yc - 1 : yc, yp = yc < ny - 1 ? yc + 1 : yc;
    pull<S, T>(p, nx, xm, xc, xp, ym, yc, yp, f);
    const unsigned own = (unsigned)(yc * nx + xc);
    if (yc == 0) {                     // N, NE, NW come back from the bottom plate
        f[2] = (T)ld_off(p[4], own);
        f[5] = (T)ld_off(p[7], own);
        f[6] = (T)ld_off(p[8], own);
    } else if (yc == ny - 1) {         // S, SW, SE come back from the top plate
        f[4] = (T)ld_off(p[2], own);
        f[7] = (T)ld_off(p[5], own);
        f[8] = (T)ld_off(p[6], own);
    }
}

// Sum of the moving populations, then the density deviation: the rest
// population (the large deviation in float32 storage) is added last, so that the
// sum is rounded once at its magnitude.
template <typename T>
__device__ __forceinline__ T moving9(const T f[9]) {
    return ((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8]));
}
template <typename T>
__device__ __forceinline__ T sum9(const T f[9]) { return f[0] + moving9(f); }
template <typename T>
__device__ __forceinline__ T jx9(const T f[9]) { return (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]); }
template <typename T>
__device__ __forceinline__ T jy9(const T f[9]) { return (f[2] - f[4]) + (f[5] - f[8]) + (f[6] - f[7]); }

// Isotropic stencils on an LDS plane of row width W (y + 1 is +W).
//   lap  = [4 (E + W + N + S) + (NE + NW + SW + SE) - 20 c] / 6
//   d/dx = [4 (E - W) + (NE - NW - SW + SE)] / 12          (Eq. 17)
//   d/dy = [4 (N - S) + (NE + NW - SW - SE)] / 12
template <int W, typename T>
__device__ __forceinline__ T lap(const T* s, int c) {
    const T ax = (s[c + 1] + s[c - 1]) + (s[c + W] + s[c - W]);
    const T dg = (s[c + W + 1] + s[c + W - 1]) + (s[c - W - 1] + s[c - W + 1]);
    return (T(4) * ax + dg - T(20) * s[c]) * T(1.0 / 6.0);
}
template <int W, typename T>
__device__ __forceinline__ T ddx(const T* s, int c) {
    return (T(4) * (s[c + 1] - s[c - 1]) + ((s[c + W + 1] - s[c + W - 1]) + (s[c - W + 1] - s[c - W - 1]))) *
           T(1.0 / 12.0);
}
template <int W, typename T>
__device__ __forceinline__ T ddy(const T* s, int c) {
    return (T(4) * (s[c + W] - s[c - W]) + ((s[c + W + 1] + s[c + W - 1]) - (s[c - W - 1] + s[c - W + 1]))) *
           T(1.0 / 12.0);
}

// BGK collision with Guo forcing (Eq. 14) and, for the improved scheme, the
// correction term C of Eqs. 28-29 in population form; f holds the incoming
// populations minus fbar and receives f* minus fbar.
//   drho = rho - rho_ref, Sm = the moving populations' sum (drho - f[0]),
//   dpm = p_m - pm_ref (standard: drho / 3),
//   php = p_m - rho/3 (zero in the standard scheme), Cxx = 3 d_x, Cyy = 3 d_y.
// Equilibrium minus reference (M^-1 of Eq. 27 / Eq. 11):
//   rest: drho - 5 dpm / 3 - (2/3) rho u^2
//   axis: dpm / 3  + rho/9  (3 eu + 4.5 eu^2 - 1.5 u^2) - php eu / 2
//   diag: dpm / 12 + rho/36 (3 eu + 4.5 eu^2 - 1.5 u^2) + php eu / 4
template <typename T>
__device__ __forceinline__ void collide(T f[9], T rho, T Sm, T ux, T uy, T Fx, T Fy, T dpm, T php, T Cxx,
                                        T Cyy, T omega) {
    const T usq = ux * ux + uy * uy;
    const T uF = ux * Fx + uy * Fy;
    const T om1 = T(1) - omega, om2 = T(1) - T(0.5) * omega;
    const T r9 = rho * T(1.0 / 9.0), r36 = rho * T(1.0 / 36.0);
    const T Ca = (Cxx - T(2) * Cyy) * T(1.0 / 6.0);   // +-x
    const T Cb = (Cyy - T(2) * Cxx) * T(1.0 / 6.0);   // +-y
    const T Cd = (Cxx + Cyy) * T(1.0 / 6.0);          // diagonals
    {
        // f0* = f0 + omega (feq0 - f0) + om2 (G0 + C0), feq0 - f0 = Sm - 5 dpm / 3 - (2/3) rho u^2
        const T dfeq = Sm - T(5.0 / 3.0) * dpm - T(2.0 / 3.0) * rho * usq;
        const T G = T(4.0 / 9.0) * (T(-3) * uF);
        f[0] += (omega * dfeq + om2 * (G - T(2) * Cd));
    }
    // axis pairs: w = 1/9, php coefficient -1/2;  diagonal pairs: w = 1/36, +1/4
    const T Ua = dpm * T(1.0 / 3.0) - T(1.5) * r9 * usq;
    const T Ud = dpm * T(1.0 / 12.0) - T(1.5) * r36 * usq;
    const T ea = omega * Ua - om2 * T(3.0 / 9.0) * uF, ed = omega * Ud - om2 * T(3.0 / 36.0) * uF;
    const T e1a = omega * T(4.5) * r9, e1d = omega * T(4.5) * r36;
    const T e2a = om2 * T(1.0), e2d = om2 * T(0.25);
    const T o1a = omega * (T(3) * r9 - T(0.5) * php), o1d = omega * (T(3) * r36 + T(0.25) * php);
    const T o2a = om2 * T(1.0 / 3.0), o2d = om2 * T(1.0 / 12.0);
    pair_update<T>(f[1], f[3], ux, Fx, ea + om2 * Ca, e1a, e2a, o1a, o2a, om1);
    pair_update<T>(f[2], f[4], uy, Fy, ea + om2 * Cb, e1a, e2a, o1a, o2a, om1);
    const T ed2 = ed + om2 * Cd;
    pair_update<T>(f[5], f[7], ux + uy, Fx + Fy, ed2, e1d, e2d, o1d, o2d, om1);
    pair_update<T>(f[6], f[8], uy - ux, Fy - Fx, ed2, e1d, e2d, o1d, o2d, om1);
}

// Multiple-relaxation-time collision (Eq. 9 / Eq. 28 with the relaxation matrix
// of Eq. 8) in the moment basis (rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy)
// with rows  e: -4 + 3|e|^2,  eps: 4 - 21|e|^2/2 + 9|e|^4/2,  q_i: (-5 + 3|e|^2) e_i,
// p_xx: e_x^2 - e_y^2,  p_xy: e_x e_y.  f holds populations minus fbar; the
// non-equilibrium moments are formed from drho = rho - rho_ref and
// dpm = p_m - pm_ref so that fbar's moments cancel; with ax, dg the sums of the
// axis and diagonal populations, e(f) + 4 drho = 3 ax + 6 dg and
// eps(f) - 4 drho = -6 ax - 3 dg, so the rest population drops out exactly:
//   e - e_eq     = e(f) + 4 drho - 6 dpm - 3 rho u^2       (e_eq = -4 rho + 3 rho u^2 + 6 p_m)
//   eps - eps_eq = eps(f) - 4 drho + 9 dpm + 3 rho u^2     (eps_eq = 4 rho - 3 rho u^2 - 9 p_m)
//   q_i - q_i,eq = q_i(f) - (3 php - rho) u_i              (q_eq = (3 p_m - 2 rho) u, Eq. 27)
//   p_xx - ..    = p_xx(f) - rho (u_x^2 - u_y^2),  p_xy - .. = p_xy(f) - rho u_x u_y
// Sources: S = M G (Eq. 14) = (0, 6 u.F, -6 u.F, F_x, -F_x, F_y, -F_y, 2(u_x F_x - u_y F_y),
// u_x F_y + u_y F_x) and C of Eq. 29 = (0, 3(Cxx + Cyy), 0, 0, 0, 0, 0, Cxx - Cyy, 0).
// With D_k = -s_k (m_k - m_k,eq) + (1 - s_k/2)(S_k + C_k) (D_rho = 0, D_j = F for any
// tau_c), f* = f + M^-1 D, M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4).
template <typename T>
__device__ __forceinline__ void collide_mrt(T f[9], T rho, T ux, T uy, T Fx, T Fy, T dpm, T php, T Cxx,
                                            T Cyy, T s_e, T s_eps, T s_q, T s_v) {
    const T ax = (f[1] + f[2]) + (f[3] + f[4]);
    const T dg = (f[5] + f[6]) + (f[7] + f[8]);
    const T m_e4 = T(3) * ax + T(6) * dg;           // e(f) + 4 drho
    const T m_eps4 = -(T(6) * ax + T(3) * dg);      // eps(f) - 4 drho
    const T m_qx = T(2) * (f[3] - f[1]) + ((f[5] - f[6]) + (f[8] - f[7]));
    const T m_qy = T(2) * (f[4] - f[2]) + ((f[5] + f[6]) - (f[7] + f[8]));
    const T m_pxx = (f[1] + f[3]) - (f[2] + f[4]);
    const T m_pxy = (f[5] + f[7]) - (f[6] + f[8]);
    const T ru2 = rho * (ux * ux + uy * uy);
    const T uF = ux * Fx + uy * Fy;
    const T g = T(3) * php - rho;
    const T d_e = -s_e * (m_e4 - T(6) * dpm - T(3) * ru2) + (T(1) - T(0.5) * s_e) * (T(6) * uF + T(3) * (Cxx + Cyy));
    const T d_eps = -s_eps * (m_eps4 + T(9) * dpm + T(3) * ru2) + (T(1) - T(0.5) * s_eps) * (T(-6) * uF);
    const T hq = T(1) - T(0.5) * s_q;
    const T d_qx = -s_q * (m_qx - g * ux) - hq * Fx;
    const T d_qy = -s_q * (m_qy - g * uy) - hq * Fy;
    const T hv = T(1) - T(0.5) * s_v;
    const T d_pxx = -s_v * (m_pxx - rho * (ux * ux - uy * uy)) + hv * (T(2) * (ux * Fx - uy * Fy) + (Cxx - Cyy));
    const T d_pxy = -s_v * (m_pxy - rho * ux * uy) + hv * (ux * Fy + uy * Fx);
    f[0] += (d_eps - d_e) * T(1.0 / 9.0);
    const T A = -(d_e + T(2) * d_eps) * T(1.0 / 36.0);
    const T B = (T(2) * d_e + d_eps) * T(1.0 / 36.0);
    const T Ax = Fx * T(1.0 / 6.0) - d_qx * T(1.0 / 6.0), Ay = Fy * T(1.0 / 6.0) - d_qy * T(1.0 / 6.0);
    const T P4 = d_pxx * T(0.25), X4 = d_pxy * T(0.25);
    f[1] += A + Ax + P4;
    f[3] += A - Ax + P4;
    f[2] += A + Ay - P4;
    f[4] += A - Ay - P4;
    const T X = Fx * T(1.0 / 6.0) + d_qx * T(1.0 / 12.0), Y = Fy * T(1.0 / 6.0) + d_qy * T(1.0 / 12.0);
    f[5] += B + X + Y + X4;
    f[6] += B - X + Y - X4;
    f[7] += B - X - Y + X4;
    f[8] += B + X - Y - X4;
}

// Equilibrium minus reference for initialisation (same closed forms, no force).
template <typename T>
__device__ __forceinline__ void equilibrium(T feq[9], T rho, T drho, T ux, T uy, T dpm, T php) {
    const T usq = ux * ux + uy * uy;
    const T r9 = rho * T(1.0 / 9.0), r36 = rho * T(1.0 / 36.0);
    feq[0] = drho - T(5.0 / 3.0) * dpm - T(2.0 / 3.0) * rho * usq;
    const T ua = dpm * T(1.0 / 3.0) - T(1.5) * r9 * usq;
    const T ud = dpm * T(1.0 / 12.0) - T(1.5) * r36 * usq;
    const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        const T eu = T(ex[a]) * ux + T(ey[a]) * uy;
        if (a < 5)
            feq[a] = ua + r9 * (T(3) * eu + T(4.5) * eu * eu) - T(0.5) * php * eu;
        else
            feq[a] = ud + r36 * (T(3) * eu + T(4.5) * eu * eu) + T(0.25) * php * eu;
    }
}

// ---------------------------------------------------------------------------
// Fused step.  Stages on one tile of BX x BY output nodes:
//   A  rho (and j) on the tile + 3 halo rings, from pulled populations
//   B  mu = mu_EOS(rho) - kappa lap(rho) on tile + 2 (Eq. 2); P on tile + 2 (P-tensor form)
//   C  F (Eq. 13 / Eq. 24), u = (j + F/2)/rho (Eq. 12), psi = phi u (Eq. 29) on tile + 1
//   D  collision (Eq. 9 / Eq. 28 with Lambda = I/tau) and store, or field output
// MODE (lbm::Mode) selects collide-and-store, or the read-out of rho, u, mu and
// the per-tile diagnostics of the input time level (no store).
// FEAT bit 1: lattices of the launch may use the MRT collision; bit 2: they may
// have plates (the lattice record decides); launches without them carry no such code.
// XT: work-group threads per own thread.  With XT = 2 the second half of the work
// group owns no node: it takes the halo pulls of stage A, and every thread takes a
// share of stages B and C, so that each stage is one pass over the tile's rings.
template <typename S, typename T, int V, int BX, int BY, int MODE, int FEAT, int NPT, int XT = 1>
__global__ __launch_bounds__(BX* BY* XT) void step_kernel(StepArgs args) {
    constexpr int NT = BX * BY;                    // threads that own nodes
    constexpr int TPB = NT * XT;                   // threads of the work group
    constexpr int TH = BY * NPT, NN = BX * TH;     // tile: BX x TH nodes, NPT per thread (rows BY apart)
    constexpr bool MRT = (FEAT & 1) != 0;
    constexpr bool PLATES = (FEAT & 2) != 0;
    constexpr int W3 = BX + 6, H3 = TH + 6, W2 = BX + 4, H2 = TH + 4, W1 = BX + 2, H1 = TH + 2;
    constexpr bool IMP = (V == kImproved);
    constexpr bool PT = (V == kStdPtensor);
    __shared__ T s_rho[H3 * W3];
    __shared__ T s_mu[H2 * W2];
    __shared__ T s_a[H1 * W1];            // j_x, then psi_x = phi u_x
    __shared__ T s_b[H1 * W1];            // j_y, then psi_y
    __shared__ T s_F[2 * NN], s_u[2 * NN];
    __shared__ T s_P[PT ? 3 * H2 * W2 : 1];
    __shared__ double s_red[7 * (TPB / 64)];
    __shared__ unsigned s_ured[TPB / 64 + 1];     // per-wave status bits, then the arrival count

    const int t_idx = tile_of_block(blockIdx.x, args.tiles_per_xcd);
    if (t_idx >= args.ntiles) return;
    // With one lattice the tile and the addressing come from the arguments, so
    // the population loads do not wait for the tile and lattice records.
    int lat, x0, y0, nx, ny, sx, sy;
    long long soff;
    if (args.single) {
        int tx, ty;
        band_order(t_idx, args.ntx, args.nty, args.band, tx, ty);
        lat = 0;
        x0 = tx * BX;
        y0 = ty * TH;
        nx = args.nx0;
        ny = args.ny0;
        sx = args.slow_x0;
        sy = args.slow_y0;
        soff = 0;
    } else {
        const Tile tile = args.tiles[t_idx];
        lat = tile.lat;
        x0 = tile.x0;
        y0 = tile.y0;
        nx = tile.nx;
        ny = tile.ny;
        sx = tile.slow & 1;
        sy = tile.slow >> 1;
        soff = tile.soff;
    }
    const LatticeRec& R = args.recs[lat];
    const int N = nx * ny;
    const S* __restrict__ src = reinterpret_cast<const S*>(args.src) + soff * 9;
    S* __restrict__ dst = reinterpret_cast<S*>(args.dst) + soff * 9;
    const S* pp[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) pp[a] = src + (size_t)a * N;
    const Eos<T> eos{R.eos, (T)R.a, (T)R.b, (T)R.RT};
    const T kappa = (T)R.kappa, omega = (T)R.omega;
    // LDS holds the density as x = rho - rho_ref and the chemical potential minus
    // muref.mu_off (float32: deviations from the reference state; float64: rho_ref
    // = 0, offset 0)
    constexpr bool F32 = sizeof(S) == 4;
    const T rho_ref = (T)R.rho_ref, pm_ref = (T)R.pm_ref, mu_ref = (T)R.mu_ref, c0 = (T)R.c0;
    const T phi0 = rho_ref * T(1.0 / 3.0) - pm_ref;      // float32: phi = phi0 + (x - (mu - mu_ref)) / 3
    const MuRef muref(R, F32);
    // Record fields used in stage D are read here, with the others: a load issued
    // in stage D would put a memory round trip at the end of every work group.
    const double rho_max = R.rho_max;
    const int mrt = MRT ? R.mrt : 0;
    const T mrt_nu = MRT ? (T)R.nu : T(0);
    const T mrt_se = MRT ? (T)R.s_e : T(0), mrt_seps = MRT ? (T)R.s_eps : T(0), mrt_sq = MRT ? (T)R.s_q : T(0);
    const T wall_u0 = PLATES ? (T)R.wall_u0 : T(0), wall_u1 = PLATES ? (T)R.wall_u1 : T(0);
    const long long field_offset = R.field_offset;
    const int tid = threadIdx.x;
    const int lx0 = tid % BX, ly0 = tid / BX;
    const bool owner = XT == 1 || tid < NT;
    // halo slot of this thread: helper threads first, then the owners
    const int hslot = XT == 1 ? tid : (tid >= NT ? tid - NT : tid + (TPB - NT));
    const int hwave = XT == 1 ? (tid & ~63) : ((tid & ~63) >= NT ? (tid & ~63) - NT : (tid & ~63) + (TPB - NT));

    // ---- stage A: the interior node owned by this thread (kept in registers for
    // stage D) and up to HP nodes of the three halo rings; every load is issued
    // before any is used.
    constexpr int HALO = H3 * W3 - NN;
    constexpr int HP = (HALO + TPB - 1) / TPB;
    T fown[NPT][9];
    T fh[HP][9];
    int hpos[HP];
    const bool plates = PLATES && R.walls;
    // A tile whose pulls (tile + 4 rings) stay inside the lattice needs no periodic
    // wrap: block-uniform, so the wrap arithmetic is skipped for most tiles.
    const bool inner = x0 >= 4 && x0 + BX + 4 <= nx && y0 >= 4 && y0 + TH + 4 <= ny;
    auto wx = [&](int v) { return inner ? v : wrap(v, nx, sx); };
    auto wy = [&](int v) { return inner ? v : wrap(v, ny, sy); };
    bool own_mirror[NPT];
    bool h_mirror[HP];
#pragma unroll
    for (int p = 0; p < NPT; ++p) {
        own_mirror[p] = false;
        if (!owner) continue;
        const int gx = x0 + lx0, gy = y0 + ly0 + p * BY;
        const int xc = wx(gx), xm = wx(gx - 1), xp = wx(gx + 1);
        if (plates) {
            pull_plates<S, T>(pp, nx, ny, xm, xc, xp, plate_row(gy, ny, own_mirror[p]), fown[p]);
        } else {
            const int yc = wy(gy), ym = wy(gy - 1), yp = wy(gy + 1);
            pull<S, T>(pp, nx, xm, xc, xp, ym, yc, yp, fown[p]);
        }
    }
#pragma unroll
    for (int q = 0; q < HP; ++q) {
        int k = hslot + q * TPB;
        k = k < HALO ? k : HALO - 1;          // idle lanes repeat the last halo node
        int lx, ly;
        if (k < 3 * W3) {
            ly = k / W3; lx = k % W3;
        } else if (k < 6 * W3) {
            const int k2 = k - 3 * W3;
            ly = H3 - 3 + k2 / W3; lx = k2 % W3;
        } else {
            const int k3 = k - 6 * W3;
            ly = 3 + k3 / 6;
            const int c = k3 % 6;
            lx = c < 3 ? c : W3 - 6 + c;
        }
        hpos[q] = ly * W3 + lx;
        const int gx = x0 - 3 + lx, gy = y0 - 3 + ly;
        const int xc = wx(gx), xm = wx(gx - 1), xp = wx(gx + 1);
        h_mirror[q] = false;
        if (hwave + q * TPB < HALO) {                 // waves with no halo node left skip the pulls
            if (plates) {
                pull_plates<S, T>(pp, nx, ny, xm, xc, xp, plate_row(gy, ny, h_mirror[q]), fh[q]);
            } else {
                const int yc = wy(gy), ym = wy(gy - 1), yp = wy(gy + 1);
                pull<S, T>(pp, nx, xm, xc, xp, ym, yc, yp, fh[q]);
            }
        }
    }
    // Blown-up lattices are frozen: steps skip them.  The flag can be raised by
    // other blocks while this one runs, so one thread reads it and the whole block
    // follows.  (The runtime leaves the tiles of lattices it has reported blown up
    // out of its plan, so this mostly catches lattices that blew up since.)  A
    // read-out, which stores no populations, covers every tile.
    __shared__ unsigned s_skip;
    if (tid == 0) {
        s_skip = __atomic_load_n(args.status + lat, __ATOMIC_RELAXED);
        s_ured[TPB / 64] = 0u;
    }
    // a mirror image beyond a plate carries the reflected momentum (j_y negated)
#pragma unroll
    for (int p = 0; p < NPT; ++p) {
        if (!owner) continue;
        const int ly = ly0 + p * BY;
        s_rho[(ly + 3) * W3 + lx0 + 3] = sum9(fown[p]);
        s_a[(ly + 1) * W1 + lx0 + 1] = jx9(fown[p]);
        s_b[(ly + 1) * W1 + lx0 + 1] = own_mirror[p] ? -jy9(fown[p]) : jy9(fown[p]);
    }
#pragma unroll
    for (int q = 0; q < HP; ++q) {
        if (hslot + q * TPB < HALO) {
            const int pos = hpos[q];
            const int ly = pos / W3, lx = pos - ly * W3;
            s_rho[pos] = sum9(fh[q]);
            if (lx >= 2 && lx < W3 - 2 && ly >= 2 && ly < H3 - 2) {
                s_a[(ly - 2) * W1 + lx - 2] = jx9(fh[q]);
                s_b[(ly - 2) * W1 + lx - 2] = h_mirror[q] ? -jy9(fh[q]) : jy9(fh[q]);
            }
        }
    }
    __syncthreads();
    if (MODE == kStep && s_skip != 0u) return;

    // ---- stage B: chemical potential (and pressure tensor) on tile + 2 ----
    for (int k = tid; k < H2 * W2; k += TPB) {
        const int lx = k % W2, ly = k / W2;
        const int c = (ly + 1) * W3 + lx + 1;
        const T x = s_rho[c];
        const T L = lap<W3>(s_rho, c);
        s_mu[k] = muref.dmu(eos, x) - kappa * L;
        if constexpr (PT) {
            const T r = rho_ref + x;
            const T gx = ddx<W3>(s_rho, c), gy = ddy<W3>(s_rho, c);
            const T p = eos.p(r) - kappa * r * L - T(0.5) * kappa * (gx * gx + gy * gy);   // Eq. 4
            s_P[k] = p + kappa * gx * gx;                                                 // Eq. 5
            s_P[H2 * W2 + k] = kappa * gx * gy;
            s_P[2 * H2 * W2 + k] = p + kappa * gy * gy;
        }
    }
    __syncthreads();

    // ---- stage C: force, velocity, psi on tile + 1 ----
    for (int k = tid; k < H1 * W1; k += TPB) {
        const int lx = k % W1, ly = k / W1;
        const int c2 = (ly + 1) * W2 + lx + 1;
        const int c3 = (ly + 2) * W3 + lx + 2;
        const T x = s_rho[c3];
        const T r = rho_ref + x;
        T Fx, Fy;
        if constexpr (IMP) {
            const T g = T(1.0 / 3.0) - r;                                                 // Eq. 24
            Fx = g * ddx<W2>(s_mu, c2);
            Fy = g * ddy<W2>(s_mu, c2);
        } else if constexpr (PT) {
            const T* Pxx = s_P;
            const T* Pxy = s_P + H2 * W2;
            const T* Pyy = s_P + 2 * H2 * W2;
            Fx = ddx<W3>(s_rho, c3) * T(1.0 / 3.0) - (ddx<W2>(Pxx, c2) + ddy<W2>(Pxy, c2));
            Fy = ddy<W3>(s_rho, c3) * T(1.0 / 3.0) - (ddx<W2>(Pxy, c2) + ddy<W2>(Pyy, c2));
        } else {
            Fx = ddx<W3>(s_rho, c3) * T(1.0 / 3.0) - r * ddx<W2>(s_mu, c2);
            Fy = ddy<W3>(s_rho, c3) * T(1.0 / 3.0) - r * ddy<W2>(s_mu, c2);
        }
        const T ir = dev_rcp(r);
        const T ux = (s_a[k] + T(0.5) * Fx) * ir;
        const T uy = (s_b[k] + T(0.5) * Fy) * ir;
        if constexpr (IMP) {
            // Eq. 29: phi = rho/3 - p_m
            const T phi = F32 ? phi0 + (x - s_mu[c2]) * T(1.0 / 3.0)
                              : r * T(1.0 / 3.0) - (c0 + s_mu[c2]) * T(1.0 / 3.0);
            s_a[k] = phi * ux;
            s_b[k] = phi * uy;
        }
        if (lx >= 1 && lx <= BX && ly >= 1 && ly <= TH) {
            const int i0 = (ly - 1) * BX + lx - 1;
            s_F[i0] = Fx; s_F[NN + i0] = Fy;
            s_u[i0] = ux; s_u[NN + i0] = uy;
        }
    }
    __syncthreads();

    // ---- stage D: collide and store (or write fields) ----
    DiagAcc acc;
#pragma unroll
    for (int p = 0; p < NPT; ++p) {
    T (&fo)[9] = fown[p];
    const int ly = ly0 + p * BY, io = tid + p * NT;
    const int gx = x0 + lx0, gy = y0 + ly;
    if (owner && gx < nx && gy < ny) {
        const int c3 = (ly + 3) * W3 + lx0 + 3, c2 = (ly + 2) * W2 + lx0 + 2, c1 = (ly + 1) * W1 + lx0 + 1;
        const T x = s_rho[c3];
        const T r = rho_ref + x;
        const T dmu = s_mu[c2];                                 // mu - mu_off
        const double mu = muref.mu_off + (double)dmu;
        const T Fx = s_F[io], Fy = s_F[NN + io], ux = s_u[io], uy = s_u[NN + io];
        const T Sm = moving9(fo);
        const T drho = fo[0] + Sm;
        const double m_in = F32 ? mass_in<9, T>(fo) : 0.0;      // exact node mass (float32 storage)
        const int node = gy * nx + gx;
        if constexpr (MODE == kFields) {
            const long long o = field_offset + node;
            if (args.rho_out) args.rho_out[o] = muref.rho_ref + (double)x;
            if (args.mu_out) args.mu_out[o] = mu;
            if (args.u_out) {
                args.u_out[o] = (double)ux;
                args.u_out[args.field_total + o] = (double)uy;
            }
        } else {
            T dpm, php, Cxx = T(0), Cyy = T(0);
            if constexpr (IMP) {
                if constexpr (F32) {
                    dpm = dmu * T(1.0 / 3.0);
                    php = -(phi0 + (x - dmu) * T(1.0 / 3.0));
                } else {
                    dpm = (dmu - mu_ref) * T(1.0 / 3.0);
                    php = (c0 + dmu) * T(1.0 / 3.0) - r * T(1.0 / 3.0);
                }
                Cxx = T(3) * ddx<W1>(s_a, c1);
                Cyy = T(3) * ddy<W1>(s_b, c1);
            } else {
                dpm = drho * T(1.0 / 3.0);
                php = T(0);
            }
            if (MRT && mrt) {
                // shear rate: 1/tau, or from the constant kinematic viscosity nu = eta / rho with
                // eta = p_m (tau_v - 1/2) (improved, Sec. III) or rho/3 (tau_v - 1/2) (standard)
                T s_v = omega;
                if (mrt_nu > T(0)) {
                    const T nu = mrt_nu;
                    s_v = IMP ? dev_rcp(nu * r * dev_rcp(pm_ref + dpm) + T(0.5)) : dev_rcp(T(3) * nu + T(0.5));
                }
                collide_mrt<T>(fo, r, ux, uy, Fx, Fy, dpm, php, Cxx, Cyy, mrt_se, mrt_seps, mrt_sq, s_v);
            } else {
                collide<T>(fo, r, Sm, ux, uy, Fx, Fy, dpm, php, Cxx, Cyy, omega);
            }
            if constexpr (F32) keep_mass_on_axes<9, 4, T>(fo, m_in);
            if (plates && (gy == 0 || gy == ny - 1)) {
                // Populations heading into a plate are stored reflected for the next pull:
                // f*_a + feq_-a - feq_a at the plate velocity U (along x).  The odd part of
                // both equilibria on the diagonals is (p_m / 2)(e . U) per pair (Eq. 11:
                // 6 w rho = rho / 6 = p_m / 2; Eq. 27 adds php / 2), and zero on N, S.
                const T pm = IMP ? pm_ref + dpm : r * T(1.0 / 3.0);
                if (gy == 0) {
                    const T w = T(0.5) * pm * wall_u0;
                    fo[7] += w;              // SW returns as NE
                    fo[8] -= w;              // SE returns as NW
                }
                if (gy == ny - 1) {
                    const T w = T(0.5) * pm * wall_u1;
                    fo[5] -= w;              // NE returns as SW
                    fo[6] += w;              // NW returns as SE
                }
            }
            if (args.write_through) {
#pragma unroll
                for (int a = 0; a < 9; ++a) st_dev(dst + (size_t)a * N, (unsigned)node, (S)fo[a]);
            } else {
#pragma unroll
                for (int a = 0; a < 9; ++a) st_off(dst + (size_t)a * N, (unsigned)node, (S)fo[a]);
            }
        }
        acc.mass += F32 ? m_in : (double)drho;
        acc.mx += (double)(r * ux);
        acc.my += (double)(r * uy);
        acc.umax2 = fmax(acc.umax2, (double)(ux * ux + uy * uy));
        acc.mumin = fmin(acc.mumin, mu);
        acc.mumax = fmax(acc.mumax, mu);
        acc.status |= blowup_bits<T>(r, ux, uy, T(0), rho_max);
    }
    }
    if constexpr (MODE == kStep) {
        if (acc.status) atomicOr(args.status + lat, acc.status);
    } else {
        const unsigned st = block_reduce_store<TPB>(acc, args.partial + t_idx, s_red, s_ured);
        if (st != 0u) atomicOr(args.status + lat, st);
    }
}

// Where the pull of population a at node (x, y) reads: slot a of node x - e_a
// (periodic), or, for a population coming back from a plate, the node's own slot
// of the reversed direction.  Index within the lattice's state block.
__device__ __forceinline__ long long slot_of(int a, int x, int y, const LatticeRec& R) {
    const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    const int nx = R.nx, ny = R.ny;
    const long long N = (long long)nx * ny;
    const int sy = y - ey[a];
    if (R.walls && (sy < 0 || sy >= ny)) return opp[a] * N + (long long)y * nx + x;
    const int sx = ((x - ex[a]) % nx + nx) % nx, syw = (sy % ny + ny) % ny;
    return a * N + (long long)syw * nx + sx;
}

// Initialisation: f(x, 0) = f_eq(rho0, u0) (minus fbar), written where a pull
// finds it (slot_of).  One thread per node of all lattices.
template <typename S, typename T, int V>
__global__ void init_kernel(S* state, const LatticeRec* recs, int nlat, const double* rho0, const double* u0,
                            long long field_total) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int L = 0;
    while (L + 1 < nlat && gid >= recs[L + 1].field_offset) ++L;
    const LatticeRec& R = recs[L];
    const long long local = gid - R.field_offset;
    if (local < 0 || local >= R.nnodes) return;
    const int nx = R.nx, ny = R.ny, N = nx * ny;
    const int x = (int)(local % nx), y = (int)(local / nx);
    const double* r0 = rho0 + R.field_offset;
    auto at = [&](int dx, int dy) {
        const int xx = ((x + dx) % nx + nx) % nx;
        bool m;
        const int yy = R.walls ? plate_row(y + dy, ny, m) : ((y + dy) % ny + ny) % ny;
        return (T)r0[yy * nx + xx];
    };
    const T r = at(0, 0);
    T ux = T(0), uy = T(0);
    if (u0) {
        ux = (T)u0[R.field_offset + local];
        uy = (T)u0[field_total + R.field_offset + local];
    }
    T dpm, php;
    if (V == kImproved) {
        const T ax = (at(1, 0) + at(-1, 0)) + (at(0, 1) + at(0, -1));
        const T dg = (at(1, 1) + at(-1, 1)) + (at(-1, -1) + at(1, -1));
        const T L2 = (T(4) * ax + dg - T(20) * r) * T(1.0 / 6.0);
        const Eos<T> eos{R.eos, (T)R.a, (T)R.b, (T)R.RT};
        const T mu = eos.mu(r) - (T)R.kappa * L2;
        dpm = (mu - (T)R.mu_ref) * T(1.0 / 3.0);
        php = ((T)R.c0 + mu) * T(1.0 / 3.0) - r * T(1.0 / 3.0);
    } else {
        dpm = (r - (T)R.rho_ref) * T(1.0 / 3.0);
        php = T(0);
    }
    T feq[9];
    equilibrium<T>(feq, r, r - (T)R.rho_ref, ux, uy, dpm, php);
    S* st = state + R.state_offset * 9;
#pragma unroll
    for (int a = 0; a < 9; ++a) st[slot_of(a, x, y, R)] = (S)feq[a];
}

// Post-streaming populations f_a(x, t) as float64 (fbar added back), or the reverse.
template <typename S, bool GET>
__global__ void convert_kernel(S* state, const LatticeRec* recs, int nlat, double* f, long long field_total) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int L = 0;
    while (L + 1 < nlat && gid >= recs[L + 1].field_offset) ++L;
    const LatticeRec& R = recs[L];
    const long long local = gid - R.field_offset;
    if (local < 0 || local >= R.nnodes) return;
    const int nx = R.nx, ny = R.ny, N = nx * ny;
    const int x = (int)(local % nx), y = (int)(local / nx);
    S* st = state + R.state_offset * 9;
    for (int a = 0; a < 9; ++a) {
        const long long fo = (long long)a * field_total + R.field_offset + local;
        const long long so = slot_of(a, x, y, R);
        if (GET)
            f[fo] = (double)st[so] + R.fbar[a];
        else
            st[so] = (S)(f[fo] - R.fbar[a]);
    }
}

}  // namespace d2q9

// ---------------------------------------------------------------------------
// Host-side launchers (called by the runtime).

namespace {
template <typename S, typename T, int V, int BX, int BY, int MODE, int NPT, int XT>
void launch_feat(const StepArgs& a, int feat, dim3 g, dim3 b, hipStream_t s) {
    switch (feat) {
        case 1: hipLaunchKernelGGL((d2q9::step_kernel<S, T, V, BX, BY, MODE, 1, NPT, XT>), g, b, 0, s, a); return;
        case 2:
            if constexpr (V != kStdPtensor)      // plates are not offered with the pressure-tensor force
                hipLaunchKernelGGL((d2q9::step_kernel<S, T, V, BX, BY, MODE, 2, NPT, XT>), g, b, 0, s, a);
            return;
        case 3:
            if constexpr (V != kStdPtensor)
                hipLaunchKernelGGL((d2q9::step_kernel<S, T, V, BX, BY, MODE, 3, NPT, XT>), g, b, 0, s, a);
            return;
        default: hipLaunchKernelGGL((d2q9::step_kernel<S, T, V, BX, BY, MODE, 0, NPT, XT>), g, b, 0, s, a); return;
    }
}

template <typename S, typename T, int V, int BX, int BY, int NPT = 1, int XT = 1>
hipError_t launch_step_t(const StepArgs& a, int grid, hipStream_t s, int mode) {
    const dim3 g(grid), b(BX * BY * XT);
    const int feat = (a.any_mrt ? 1 : 0) | (a.any_plates ? 2 : 0);
    if (mode == kFields) {
        if constexpr (V != kStdPtensor) {
            if (a.any_plates) {
                hipLaunchKernelGGL((d2q9::step_kernel<S, T, V, BX, BY, kFields, 2, NPT, XT>), g, b, 0, s, a);
                return hipGetLastError();
            }
        }
        hipLaunchKernelGGL((d2q9::step_kernel<S, T, V, BX, BY, kFields, 0, NPT, XT>), g, b, 0, s, a);
    } else {
        launch_feat<S, T, V, BX, BY, kStep, NPT, XT>(a, feat, g, b, s);
    }
    return hipGetLastError();
}

template <typename S, typename T, int V>
hipError_t launch_shape(const StepArgs& a, int grid, hipStream_t s, int fields, int shape) {
    switch (shape) {
        case 0: return launch_step_t<S, T, V, 32, 16>(a, grid, s, fields);
        case 1: return launch_step_t<S, T, V, 64, 8>(a, grid, s, fields);
        case 2: return launch_step_t<S, T, V, 32, 8>(a, grid, s, fields);
        case 3: return launch_step_t<S, T, V, 16, 16>(a, grid, s, fields);
        case 4: return launch_step_t<S, T, V, 64, 16>(a, grid, s, fields);
        case 5: return launch_step_t<S, T, V, 128, 8>(a, grid, s, fields);
        case 6:    // 128 x 16 nodes, two per thread: float32 only (float64 exceeds the LDS)
            if constexpr (sizeof(S) == 4) return launch_step_t<S, T, V, 128, 8, 2>(a, grid, s, fields);
            return hipErrorInvalidValue;
        case 7: return launch_step_t<S, T, V, 64, 8, 2>(a, grid, s, fields);     // 64 x 16 nodes, two per thread
        case 8: return launch_step_t<S, T, V, 32, 16, 1, 2>(a, grid, s, fields);   // 32 x 16 nodes, 1024 threads
        case 9: return launch_step_t<S, T, V, 32, 8, 1, 2>(a, grid, s, fields);    // 32 x 8 nodes, 512 threads
        case 10: return launch_step_t<S, T, V, 64, 8, 1, 2>(a, grid, s, fields);   // 64 x 8 nodes, 1024 threads
        case 11: return launch_step_t<S, T, V, 16, 16, 1, 2>(a, grid, s, fields);  // 16 x 16 nodes, 512 threads
        default: return hipErrorInvalidValue;
    }
}
}  // namespace

extern const int kD2Q9Shapes[][2];
const int kD2Q9Shapes[][2] = {{32, 16}, {64, 8}, {32, 8}, {16, 16}, {64, 16}, {128, 8}, {128, 16}, {64, 16},
                              {32, 16}, {32, 8}, {64, 8}, {16, 16}};
extern const int kNumD2Q9Shapes;
const int kNumD2Q9Shapes = 12;
// Nodes each thread owns (rows by / nodes-per-thread apart), or -2: work groups of
// two threads per node, half of them owning none (the XT = 2 kernels).
extern const int kD2Q9NodesPerThread[];
const int kD2Q9NodesPerThread[] = {1, 1, 1, 1, 1, 1, 2, 2, -2, -2, -2, -2};

hipError_t d2q9_launch_step(const StepArgs& a, int grid, hipStream_t s, int precision, int variant, int shape,
                            int fields) {
    if (precision == 0) {
        switch (variant) {
            case kStdChempot: return launch_shape<double, double, kStdChempot>(a, grid, s, fields, shape);
            case kStdPtensor: return launch_shape<double, double, kStdPtensor>(a, grid, s, fields, shape);
            case kImproved: return launch_shape<double, double, kImproved>(a, grid, s, fields, shape);
        }
    } else {
        switch (variant) {
            case kStdChempot: return launch_shape<float, float, kStdChempot>(a, grid, s, fields, shape);
            case kStdPtensor: return launch_shape<float, float, kStdPtensor>(a, grid, s, fields, shape);
            case kImproved: return launch_shape<float, float, kImproved>(a, grid, s, fields, shape);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t d2q9_launch_init(void* state, const LatticeRec* recs, int nlat, const double* rho0, const double* u0,
                            long long total, hipStream_t s, int precision, int variant) {
    const int B = 256;
    const int grid = (int)((total + B - 1) / B);
    if (grid == 0) return hipSuccess;
    const bool imp = variant == kImproved;
    if (precision == 0) {
        if (imp)
            hipLaunchKernelGGL((d2q9::init_kernel<double, double, kImproved>), dim3(grid), dim3(B), 0, s,
                               (double*)state, recs, nlat, rho0, u0, total);
        else
            hipLaunchKernelGGL((d2q9::init_kernel<double, double, kStdChempot>), dim3(grid), dim3(B), 0, s,
                               (double*)state, recs, nlat, rho0, u0, total);
    } else {
        if (imp)
            hipLaunchKernelGGL((d2q9::init_kernel<float, float, kImproved>), dim3(grid), dim3(B), 0, s,
                               (float*)state, recs, nlat, rho0, u0, total);
        else
            hipLaunchKernelGGL((d2q9::init_kernel<float, float, kStdChempot>), dim3(grid), dim3(B), 0, s,
                               (float*)state, recs, nlat, rho0, u0, total);
    }
    return hipGetLastError();
}

hipError_t d2q9_launch_convert(void* state, const LatticeRec* recs, int nlat, double* f, long long total,
                               hipStream_t s, int precision, bool get) {
    const int B = 256;
    const int grid = (int)((total + B - 1) / B);
    if (grid == 0) return hipSuccess;
    if (precision == 0) {
        if (get)
            hipLaunchKernelGGL((d2q9::convert_kernel<double, true>), dim3(grid), dim3(B), 0, s, (double*)state,
                               recs, nlat, f, total);
        else
            hipLaunchKernelGGL((d2q9::convert_kernel<double, false>), dim3(grid), dim3(B), 0, s, (double*)state,
                               recs, nlat, f, total);
    } else {
        if (get)
            hipLaunchKernelGGL((d2q9::convert_kernel<float, true>), dim3(grid), dim3(B), 0, s, (float*)state,
                               recs, nlat, f, total);
        else
            hipLaunchKernelGGL((d2q9::convert_kernel<float, false>), dim3(grid), dim3(B), 0, s, (float*)state,
                               recs, nlat, f, total);
    }
    return hipGetLastError();
}

}  // namespace lbm
