// D3Q19 kernels: the fused time step as a 2.5D sweep (one work group per
// BX x BY column of output nodes and a chunk of z-slices, rings of slices in
// LDS), the initialisation from (rho0, u0), and conversion of the stored state
// to and from post-streaming populations.
//
// Velocity order: 0 rest; 1 +x; 2 -x; 3 +y; 4 -y; 5 +z; 6 -z;
//   7 (1,1,0) 8 (-1,-1,0) 9 (1,-1,0) 10 (-1,1,0) 11 (1,0,1) 12 (-1,0,-1)
//   13 (1,0,-1) 14 (-1,0,1) 15 (0,1,1) 16 (0,-1,-1) 17 (0,1,-1) 18 (0,-1,1).
// State layout and pull convention as in the D2Q9 kernels: population a of a
// lattice at state_offset*19 + a*nnodes + (z*ny + y)*nx + x holds f*_a(x) of the
// previous step; a step reads f_a(x) = f*_a(x - e_a) (Eq. 10).
//
// The D3Q19 forms of the improved equilibrium and of the correction term are
// the paper's D2Q9 constructions carried to 19 velocities by the same rules:
// second moments p_m I + rho u u (Eq. 25), third moments of Eq. 26, fourth
// moments shifted by (p_m - rho/3)/3 as Eq. 27 does on D2Q9; C with zero mass
// and momentum, second moments diag(3 d_i) and no higher orthogonal moments.

#include <hip/hip_runtime.h>

#include <type_traits>

#include "lbm_device.hpp"
#include "lbm_shared.hpp"

namespace lbm {
namespace d3q19 {

__device__ constexpr int EX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__device__ constexpr int EY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__device__ constexpr int EZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

// Pull the 19 populations arriving at a node (Eq. 10: population a comes from
// x - e_a).  xy[k] is the byte offset of the in-plane neighbour (dx, dy) =
// (k % 3 - 1, k / 3 - 1) within a plane, fixed over a sweep; zb[k] the byte offset
// of plane z - 1 + k (wave-uniform), so each load costs one vector add.  Offsets are
// unsigned 32-bit: one population array may span up to 4 GB.
template <typename S, typename T>
__device__ __forceinline__ void pull(const S* const (&p)[19], const int (&xy)[9], const unsigned (&zb)[3], T f[19]) {
#pragma unroll
    for (int a = 0; a < 19; ++a)
        f[a] = (T)*reinterpret_cast<const S*>(reinterpret_cast<const char*>(p[a]) +
                                             ((unsigned)xy[(1 - EY[a]) * 3 + (1 - EX[a])] + zb[1 - EZ[a]]));
}

// Sum of the moving populations, then the density deviation with the rest
// population (the large deviation in float32 storage) added last: one rounding
// at its magnitude.
template <typename T>
__device__ __forceinline__ T moving19(const T f[19]) {
    const T s0 = ((f[1] + f[2]) + (f[3] + f[4])) + (f[5] + f[6]);
    const T s1 = (f[7] + f[8]) + (f[9] + f[10]) + (f[11] + f[12]);
    const T s2 = (f[13] + f[14]) + (f[15] + f[16]) + (f[17] + f[18]);
    return s0 + (s1 + s2);
}
template <typename T>
__device__ __forceinline__ T sum19(const T f[19]) { return f[0] + moving19(f); }
template <typename T>
__device__ __forceinline__ void mom19(const T f[19], T& jx, T& jy, T& jz) {
    jx = (f[1] - f[2]) + (f[7] - f[8]) + (f[9] - f[10]) + (f[11] - f[12]) + (f[13] - f[14]);
    jy = (f[3] - f[4]) + (f[7] - f[8]) + (f[10] - f[9]) + (f[15] - f[16]) + (f[17] - f[18]);
    jz = (f[5] - f[6]) + (f[11] - f[12]) + (f[14] - f[13]) + (f[15] - f[16]) + (f[18] - f[17]);
}

// Isotropic stencils on three consecutive LDS slices (Dn = z-1, P = z, U = z+1)
// of row width W:  grad = 3 sum_a w_a phi(x + e_a) e_a  (Eq. 17),
// lap = 6 sum_a w_a [phi(x + e_a) - phi(x)] = (1/3) sum_axis + (1/6) sum_edge - 4 phi.
template <int W, typename T>
__device__ __forceinline__ T gx(const T* Dn, const T* P, const T* U, int c) {
    return T(1.0 / 6.0) * (P[c + 1] - P[c - 1]) +
           T(1.0 / 12.0) * ((P[c + W + 1] - P[c - W - 1]) + (P[c - W + 1] - P[c + W - 1]) +
                            (U[c + 1] - Dn[c - 1]) + (Dn[c + 1] - U[c - 1]));
}
template <int W, typename T>
__device__ __forceinline__ T gy(const T* Dn, const T* P, const T* U, int c) {
    return T(1.0 / 6.0) * (P[c + W] - P[c - W]) +
           T(1.0 / 12.0) * ((P[c + W + 1] - P[c - W - 1]) + (P[c + W - 1] - P[c - W + 1]) +
                            (U[c + W] - Dn[c - W]) + (Dn[c + W] - U[c - W]));
}
template <int W, typename T>
__device__ __forceinline__ T gz(const T* Dn, const T* P, const T* U, int c) {
    return T(1.0 / 6.0) * (U[c] - Dn[c]) +
           T(1.0 / 12.0) * ((U[c + 1] - Dn[c - 1]) + (U[c - 1] - Dn[c + 1]) + (U[c + W] - Dn[c - W]) +
                            (U[c - W] - Dn[c + W]));
}
template <int W, typename T>
__device__ __forceinline__ T lap(const T* Dn, const T* P, const T* U, int c) {
    const T ax = (P[c + 1] + P[c - 1]) + (P[c + W] + P[c - W]) + (U[c] + Dn[c]);
    const T ed = (P[c + W + 1] + P[c + W - 1]) + (P[c - W + 1] + P[c - W - 1]) + (U[c + 1] + U[c - 1]) +
                 (U[c + W] + U[c - W]) + (Dn[c + 1] + Dn[c - 1]) + (Dn[c + W] + Dn[c - W]);
    return T(1.0 / 3.0) * ax + T(1.0 / 6.0) * ed - T(4) * P[c];
}

// The same gradient with an accessor v(dx, dy, dz) giving the field at x + (dx, dy, dz).
template <typename T, class F>
__device__ __forceinline__ T agx(F v) {
    return T(1.0 / 6.0) * (v(1, 0, 0) - v(-1, 0, 0)) +
           T(1.0 / 12.0) * ((v(1, 1, 0) - v(-1, -1, 0)) + (v(1, -1, 0) - v(-1, 1, 0)) + (v(1, 0, 1) - v(-1, 0, -1)) +
                            (v(1, 0, -1) - v(-1, 0, 1)));
}
template <typename T, class F>
__device__ __forceinline__ T agy(F v) {
    return T(1.0 / 6.0) * (v(0, 1, 0) - v(0, -1, 0)) +
           T(1.0 / 12.0) * ((v(1, 1, 0) - v(-1, -1, 0)) + (v(-1, 1, 0) - v(1, -1, 0)) + (v(0, 1, 1) - v(0, -1, -1)) +
                            (v(0, 1, -1) - v(0, -1, 1)));
}
template <typename T, class F>
__device__ __forceinline__ T agz(F v) {
    return T(1.0 / 6.0) * (v(0, 0, 1) - v(0, 0, -1)) +
           T(1.0 / 12.0) * ((v(1, 0, 1) - v(-1, 0, -1)) + (v(-1, 0, 1) - v(1, 0, -1)) + (v(0, 1, 1) - v(0, -1, -1)) +
                            (v(0, -1, 1) - v(0, 1, -1)));
}

// BGK collision with Guo forcing and the correction term (improved scheme);
// f holds populations minus fbar on entry and f* minus fbar on exit; Sm is the
// moving populations' sum.
// Equilibrium minus reference:
//   rest: drho - 2 dpm - rho u^2 / 2
//   axis: dpm / 6  + rho/18 (3 eu + 4.5 eu^2 - 1.5 u^2) - php eu
//   edge: dpm / 12 + rho/36 (3 eu + 4.5 eu^2 - 1.5 u^2) + php eu / 4
// Correction (C_ii = 3 d_i, S = C_xx + C_yy + C_zz):
//   rest -5S/21; +-i (C_ii - 6 (S - C_ii))/42; ij-edges (5 C_ii + 5 C_jj - 2 C_kk)/42.
template <typename T>
__device__ __forceinline__ void collide(T f[19], T rho, T Sm, T ux, T uy, T uz, T Fx, T Fy, T Fz, T dpm,
                                        T php, T Cxx, T Cyy, T Czz, T omega) {
    const T usq = ux * ux + uy * uy + uz * uz;
    const T uF = ux * Fx + uy * Fy + uz * Fz;
    const T om1 = T(1) - omega, om2 = T(1) - T(0.5) * omega;
    const T r18 = rho * T(1.0 / 18.0), r36 = rho * T(1.0 / 36.0);
    const T S = Cxx + Cyy + Czz;
    const T k42 = T(1.0 / 42.0);
    const T Cx = (T(7) * Cxx - T(6) * S) * k42, Cy = (T(7) * Cyy - T(6) * S) * k42, Cz = (T(7) * Czz - T(6) * S) * k42;
    const T Cxy = (T(7) * (Cxx + Cyy) - T(2) * S) * k42;
    const T Cxz = (T(7) * (Cxx + Czz) - T(2) * S) * k42;
    const T Cyz = (T(7) * (Cyy + Czz) - T(2) * S) * k42;
    {
        // f0* = f0 + omega (feq0 - f0) + om2 (G0 + C0), feq0 - f0 = Sm - 2 dpm - rho u^2 / 2
        const T dfeq = Sm - T(2) * dpm - T(0.5) * rho * usq;
        const T G = T(1.0 / 3.0) * (T(-3) * uF);
        f[0] += (omega * dfeq + om2 * (G + T(-5.0 / 21.0) * S));
    }
    // axis pairs: w = 1/18, php coefficient -1;  edge pairs: w = 1/36, +1/4
    const T Ua = dpm * T(1.0 / 6.0) - T(1.5) * r18 * usq;
    const T Ue = dpm * T(1.0 / 12.0) - T(1.5) * r36 * usq;
    const T ea = omega * Ua - om2 * T(3.0 / 18.0) * uF, ee = omega * Ue - om2 * T(3.0 / 36.0) * uF;
    const T e1a = omega * T(4.5) * r18, e1e = omega * T(4.5) * r36;
    const T e2a = om2 * T(0.5), e2e = om2 * T(0.25);
    const T o1a = omega * (T(3) * r18 - php), o1e = omega * (T(3) * r36 + T(0.25) * php);
    const T o2a = om2 * T(1.0 / 6.0), o2e = om2 * T(1.0 / 12.0);
    pair_update<T>(f[1], f[2], ux, Fx, ea + om2 * Cx, e1a, e2a, o1a, o2a, om1);
    pair_update<T>(f[3], f[4], uy, Fy, ea + om2 * Cy, e1a, e2a, o1a, o2a, om1);
    pair_update<T>(f[5], f[6], uz, Fz, ea + om2 * Cz, e1a, e2a, o1a, o2a, om1);
    const T exy = ee + om2 * Cxy, exz = ee + om2 * Cxz, eyz = ee + om2 * Cyz;
    pair_update<T>(f[7], f[8], ux + uy, Fx + Fy, exy, e1e, e2e, o1e, o2e, om1);
    pair_update<T>(f[9], f[10], ux - uy, Fx - Fy, exy, e1e, e2e, o1e, o2e, om1);
    pair_update<T>(f[11], f[12], ux + uz, Fx + Fz, exz, e1e, e2e, o1e, o2e, om1);
    pair_update<T>(f[13], f[14], ux - uz, Fx - Fz, exz, e1e, e2e, o1e, o2e, om1);
    pair_update<T>(f[15], f[16], uy + uz, Fy + Fz, eyz, e1e, e2e, o1e, o2e, om1);
    pair_update<T>(f[17], f[18], uy - uz, Fy - Fz, eyz, e1e, e2e, o1e, o2e, om1);
}

template <typename T>
__device__ __forceinline__ void equilibrium(T feq[19], T rho, T drho, T ux, T uy, T uz, T dpm, T php) {
    const T usq = ux * ux + uy * uy + uz * uz;
    const T r18 = rho * T(1.0 / 18.0), r36 = rho * T(1.0 / 36.0);
    feq[0] = drho - T(2) * dpm - T(0.5) * rho * usq;
    const T ua = dpm * T(1.0 / 6.0) - T(1.5) * r18 * usq;
    const T ue = dpm * T(1.0 / 12.0) - T(1.5) * r36 * usq;
#pragma unroll
    for (int a = 1; a < 19; ++a) {
        const T eu = T(EX[a]) * ux + T(EY[a]) * uy + T(EZ[a]) * uz;
        feq[a] = (a < 7) ? ua + r18 * (T(3) * eu + T(4.5) * eu * eu) - php * eu
                         : ue + r36 * (T(3) * eu + T(4.5) * eu * eu) + T(0.25) * php * eu;
    }
}

// ---------------------------------------------------------------------------
// Fused step as a sweep over z.  Iteration `it` handles slice za = z0 - 3 + it:
//   A  pull populations of slice za, rho on tile + 3 rings, j on tile + 1
//   B  mu (and P) of slice za - 1 on tile + 2
//   C  F and u (and psi = phi u, improved) of slice za - 2
//   D  collide and store slice za - 3 (the thread's own populations, pulled
//      three iterations earlier, wait in a register FIFO when FIFO is set)
// rho is kept for 4 slices (slot (z - z0 + 8) & 3); mu, j, psi and P for 3
// (slot (z - z0 + 9) % 3); F and u of the tile for 2.
// WT: store the populations at device scope (LBM_STORES_DEVICE) instead of
// non-temporally; a template parameter so that each kernel holds one store loop.
template <typename S, typename T, int V, int BX, int BY, int MODE, bool WT>
__global__ __launch_bounds__(BX* BY) void step_kernel(StepArgs args) {
    constexpr int NT = BX * BY;
    constexpr int W3 = BX + 6, H3 = BY + 6, A3 = W3 * H3;
    constexpr int W2 = BX + 4, H2 = BY + 4, A2 = W2 * H2;
    constexpr int W1 = BX + 2, H1 = BY + 2, A1 = W1 * H1;
    constexpr bool IMP = (V == kImproved);
    constexpr bool PT = (V == kStdPtensor);
    constexpr bool FIFO = sizeof(T) == 4;       // float64 re-reads its populations in stage D instead
    __shared__ T s_rho[4 * A3];
    __shared__ T s_mu[3 * A2];
    __shared__ T s_j[3 * 3 * A1];               // component stride 3 * A1
    __shared__ T s_psi[IMP ? 3 * 3 * A1 : 1];
    __shared__ T s_P[PT ? 4 * 3 * A2 : 1];      // p, d_x rho, d_y rho, d_z rho; ring of 3 slices
    __shared__ T s_fu[6 * 2 * NT];              // Fx Fy Fz ux uy uz of the tile, 2 slices
    __shared__ double s_red[7 * (NT / 64)];
    __shared__ unsigned s_ured[NT / 64 + 1];      // per-wave status bits, then the arrival count

    const int t_idx = tile_of_block(blockIdx.x, args.tiles_per_xcd);
    if (t_idx >= args.ntiles) return;
    const Tile tile = args.tiles[t_idx];
    const LatticeRec& R = args.recs[tile.lat];
    // Blown-up lattices are frozen: steps skip them.  The flag can be raised by
    // other blocks while this one starts, so one thread reads it and the whole
    // block follows.  A read-out, which stores no populations, covers every tile.
    __shared__ unsigned s_skip;
    if (threadIdx.x == 0) {
        s_skip = __atomic_load_n(args.status + tile.lat, __ATOMIC_RELAXED);
        s_ured[NT / 64] = 0u;
    }
    __syncthreads();
    if (MODE == kStep && s_skip != 0u) return;

    const int nx = R.nx, ny = R.ny, nz = R.nz;
    const int N = nx * ny * nz, NXY = nx * ny;
    const int sx = R.slow_x, sy = R.slow_y, sz = R.slow_z;
    const S* __restrict__ src = reinterpret_cast<const S*>(args.src) + R.state_offset * 19;
    S* __restrict__ dst = reinterpret_cast<S*>(args.dst) + R.state_offset * 19;
    const S* pp[19];
#pragma unroll
    for (int a = 0; a < 19; ++a) pp[a] = src + (size_t)a * N;
    const Eos<T> eos{R.eos, (T)R.a, (T)R.b, (T)R.RT};
    const T kappa = (T)R.kappa, omega = (T)R.omega;
    // LDS holds the density as x = rho - rho_ref and the chemical potential minus
    // muref.mu_off (float32: deviations from the reference state; float64: rho_ref
    // = 0, offset 0)
    constexpr bool F32 = sizeof(S) == 4;
    const T rho_ref = (T)R.rho_ref, pm_ref = (T)R.pm_ref, mu_ref = (T)R.mu_ref, c0 = (T)R.c0;
    const T phi0 = rho_ref * T(1.0 / 3.0) - pm_ref;      // float32: phi = phi0 + (x - (mu - mu_ref)) / 3
    const MuRef muref(R, F32);
    // Record fields used in stage D are read here with the others: a load issued in
    // stage D waits (in issue order) behind every pull before it and puts a memory
    // round trip into each slice
    const double rho_max = R.rho_max;
    const long long field_offset = R.field_offset;
    const int x0 = tile.x0, y0 = tile.y0, z0 = tile.z0, zn = tile.zn;
    const int tid = threadIdx.x;
    const int lx0 = tid % BX, ly0 = tid / BX;
    const int gx0 = x0 + lx0, gy0 = y0 + ly0;
    const bool own_valid = gx0 < nx && gy0 < ny;

    // byte offsets of the owned column's in-plane neighbourhood (fixed over the sweep)
    constexpr int WS = (int)sizeof(S);
    int oxy[9];
    {
        int X[3], Y[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            X[k] = wrap(gx0 - 1 + k, nx, sx);
            Y[k] = wrap(gy0 - 1 + k, ny, sy) * nx;
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) oxy[k] = (Y[k / 3] + X[k % 3]) * WS;
    }
    const unsigned plane_bytes = (unsigned)NXY * (unsigned)WS;
    auto zbytes = [&](int z, unsigned (&zb)[3]) {
#pragma unroll
        for (int k = 0; k < 3; ++k) zb[k] = (unsigned)wrap(z - 1 + k, nz, sz) * plane_bytes;
    };

    T fifo[FIFO ? 4 : 1][19];
    DiagAcc acc;

    // Halo nodes of stage A handled by this thread: their in-slice position and
    // wrapped x / y neighbour offsets do not change along the sweep, so they are
    // decoded once here (idle lanes repeat the last halo node and store nothing).
    constexpr int HALO = A3 - NT;
    constexpr int HP = (HALO + NT - 1) / NT;
    int hxy[HP][9], hpos[HP], hpos1[HP];
#pragma unroll
    for (int q = 0; q < HP; ++q) {
        int k = tid + q * NT;
        k = k < HALO ? k : HALO - 1;
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
        const int hx = x0 - 3 + lx, hy = y0 - 3 + ly;
        int X[3], Y[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            X[d] = wrap(hx - 1 + d, nx, sx);
            Y[d] = wrap(hy - 1 + d, ny, sy) * nx;
        }
#pragma unroll
        for (int d = 0; d < 9; ++d) hxy[q][d] = (Y[d / 3] + X[d % 3]) * WS;
        hpos[q] = (tid + q * NT < HALO) ? ly * W3 + lx : -1;
        hpos1[q] = (lx >= 2 && lx < W3 - 2 && ly >= 2 && ly < H3 - 2) ? (ly - 2) * W1 + lx - 2 : -1;
    }

    // The sweep is unrolled by four so that the FIFO slot written by stage A
    // (it mod 4) and the one read by stage D (three iterations later) are
    // compile-time register names.  Iterations past NIT only pass the barriers.
    const int NIT = zn + 6;
    auto iteration = [&](const int it, auto slot) {
        constexpr int KW = decltype(slot)::value;
        constexpr int KR = (KW + 1) & 3;
        const int za = z0 - 3 + it;
        const int slA = (za - z0 + 8) & 3;
        const int slA3 = (za - z0 + 9) % 3;

        // ---- A: interior column of this thread, then its halo nodes; all loads
        // are issued before any is used ----
        if (it < NIT) {
            T f[19];
            T fh[HP][19];
            unsigned zb[3];
            zbytes(za, zb);
            pull<S, T>(pp, oxy, zb, f);
#pragma unroll
            for (int q = 0; q < HP; ++q)
                if ((tid & ~63) + q * NT < HALO)          // waves with no halo node left skip the pulls
                    pull<S, T>(pp, hxy[q], zb, fh[q]);
            s_rho[slA * A3 + (ly0 + 3) * W3 + lx0 + 3] = sum19(f);
            T jx, jy, jz;
            mom19(f, jx, jy, jz);
            const int c1 = slA3 * A1 + (ly0 + 1) * W1 + lx0 + 1;
            s_j[c1] = jx; s_j[3 * A1 + c1] = jy; s_j[6 * A1 + c1] = jz;
            if constexpr (FIFO) {
#pragma unroll
                for (int a = 0; a < 19; ++a) fifo[KW][a] = f[a];
            }
#pragma unroll
            for (int q = 0; q < HP; ++q) {
                if (hpos[q] >= 0) {
                    s_rho[slA * A3 + hpos[q]] = sum19(fh[q]);
                    if (hpos1[q] >= 0) {
                        T hx_, hy_, hz_;
                        mom19(fh[q], hx_, hy_, hz_);
                        const int h1 = slA3 * A1 + hpos1[q];
                        s_j[h1] = hx_; s_j[3 * A1 + h1] = hy_; s_j[6 * A1 + h1] = hz_;
                    }
                }
            }
        }
        __syncthreads();

        // ---- B: mu (and P) of slice za - 1 on tile + 2 ----
        if (it >= 2 && it < NIT) {
            const int zb = za - 1;
            const T* Rd = s_rho + ((zb - 1 - z0 + 8) & 3) * A3;
            const T* Rp = s_rho + ((zb - z0 + 8) & 3) * A3;
            const T* Ru = s_rho + ((zb + 1 - z0 + 8) & 3) * A3;
            const int slB = (zb - z0 + 9) % 3;
            for (int k = tid; k < A2; k += NT) {
                const int lx = k % W2, ly = k / W2;
                const int c = (ly + 1) * W3 + lx + 1;
                const T x = Rp[c];
                const T L = lap<W3>(Rd, Rp, Ru, c);
                s_mu[slB * A2 + k] = muref.dmu(eos, x) - kappa * L;
                if constexpr (PT) {
                    const T r = rho_ref + x;
                    const T g0 = gx<W3>(Rd, Rp, Ru, c), g1 = gy<W3>(Rd, Rp, Ru, c), g2 = gz<W3>(Rd, Rp, Ru, c);
                    // Eq. 4; the tensor of Eq. 5 is rebuilt from (p, grad rho) where it is differentiated
                    const T p = eos.p(r) - kappa * r * L - T(0.5) * kappa * (g0 * g0 + g1 * g1 + g2 * g2);
                    T* P = s_P + ((zb - z0 + 9) % 3) * A2 + k;
                    P[0] = p;
                    P[3 * A2] = g0;
                    P[6 * A2] = g1;
                    P[9 * A2] = g2;
                }
            }
        }
        __syncthreads();

        // ---- C: F, u (and psi) of slice za - 2 ----
        if (it >= 4 && it < NIT) {
            const int zc = za - 2;
            const int sd = (zc - 1 - z0 + 8) & 3, sp = (zc - z0 + 8) & 3, su = (zc + 1 - z0 + 8) & 3;
            const int md = (zc - 1 - z0 + 9) % 3, mp = (zc - z0 + 9) % 3, mu3 = (zc + 1 - z0 + 9) % 3;
            const int sfu = (zc - z0 + 8) & 1;
            constexpr int NC = IMP ? A1 : NT;          // improved needs psi on tile + 1
            for (int k = tid; k < NC; k += NT) {
                int lx, ly;     // tile + 1 coordinates
                if (IMP) { lx = k % W1; ly = k / W1; } else { lx = k % BX + 1; ly = k / BX + 1; }
                const int c2 = (ly + 1) * W2 + lx + 1;
                const int c3 = (ly + 2) * W3 + lx + 2;
                const T x = s_rho[sp * A3 + c3];
                const T r = rho_ref + x;
                T Fx, Fy, Fz;
                const T* Md = s_mu + md * A2;
                const T* Mp = s_mu + mp * A2;
                const T* Mu = s_mu + mu3 * A2;
                if constexpr (IMP) {
                    const T g = T(1.0 / 3.0) - r;                                       // Eq. 24
                    Fx = g * gx<W2>(Md, Mp, Mu, c2);
                    Fy = g * gy<W2>(Md, Mp, Mu, c2);
                    Fz = g * gz<W2>(Md, Mp, Mu, c2);
                } else {
                    const T* Rd = s_rho + sd * A3;
                    const T* Rp = s_rho + sp * A3;
                    const T* Ru = s_rho + su * A3;
                    const T ax = gx<W3>(Rd, Rp, Ru, c3) * T(1.0 / 3.0);
                    const T ay = gy<W3>(Rd, Rp, Ru, c3) * T(1.0 / 3.0);
                    const T az = gz<W3>(Rd, Rp, Ru, c3) * T(1.0 / 3.0);
                    if constexpr (PT) {
                        // P_ij = p delta_ij + kappa d_i rho d_j rho (Eq. 5); (div P)_j = sum_i d_i P_ij (Eq. 17)
                        auto at = [&](int q, int dx, int dy, int dz) {
                            return s_P[q * 3 * A2 + ((zc + dz - z0 + 9) % 3) * A2 + c2 + dy * W2 + dx];
                        };
                        auto Pf = [&](int i, int j) {
                            return [&, i, j](int dx, int dy, int dz) {
                                const T v = kappa * at(1 + i, dx, dy, dz) * at(1 + j, dx, dy, dz);
                                return i == j ? v + at(0, dx, dy, dz) : v;
                            };
                        };
                        const T dPx = agx<T>(Pf(0, 0)) + agy<T>(Pf(1, 0)) + agz<T>(Pf(2, 0));
                        const T dPy = agx<T>(Pf(0, 1)) + agy<T>(Pf(1, 1)) + agz<T>(Pf(2, 1));
                        const T dPz = agx<T>(Pf(0, 2)) + agy<T>(Pf(1, 2)) + agz<T>(Pf(2, 2));
                        Fx = ax - dPx; Fy = ay - dPy; Fz = az - dPz;
                    } else {
                        Fx = ax - r * gx<W2>(Md, Mp, Mu, c2);
                        Fy = ay - r * gy<W2>(Md, Mp, Mu, c2);
                        Fz = az - r * gz<W2>(Md, Mp, Mu, c2);
                    }
                }
                const int c1 = mp * A1 + ly * W1 + lx;
                const T ir = dev_rcp(r);
                const T ux = (s_j[c1] + T(0.5) * Fx) * ir;
                const T uy = (s_j[3 * A1 + c1] + T(0.5) * Fy) * ir;
                const T uz = (s_j[6 * A1 + c1] + T(0.5) * Fz) * ir;
                if constexpr (IMP) {
                    // Eq. 29: phi = rho/3 - p_m
                    const T phi = F32 ? phi0 + (x - Mp[c2]) * T(1.0 / 3.0)
                                      : r * T(1.0 / 3.0) - (c0 + Mp[c2]) * T(1.0 / 3.0);
                    s_psi[c1] = phi * ux;
                    s_psi[3 * A1 + c1] = phi * uy;
                    s_psi[6 * A1 + c1] = phi * uz;
                }
                if (lx >= 1 && lx <= BX && ly >= 1 && ly <= BY) {
                    T* fu = s_fu + sfu * 6 * NT + (ly - 1) * BX + lx - 1;
                    fu[0] = Fx; fu[NT] = Fy; fu[2 * NT] = Fz;
                    fu[3 * NT] = ux; fu[4 * NT] = uy; fu[5 * NT] = uz;
                }
            }
        }
        __syncthreads();

        // ---- D: collide and store slice za - 3 ----
        if (it >= 6 && it < NIT && own_valid) {
            const int zd = za - 3;
            const int sp = (zd - z0 + 8) & 3;
            const int md = (zd - 1 - z0 + 9) % 3, mp = (zd - z0 + 9) % 3, mu3 = (zd + 1 - z0 + 9) % 3;
            const int sfu = (zd - z0 + 8) & 1;
            const T x = s_rho[sp * A3 + (ly0 + 3) * W3 + lx0 + 3];
            const T r = rho_ref + x;
            const T dmu = s_mu[mp * A2 + (ly0 + 2) * W2 + lx0 + 2];    // mu - mu_off
            const double mu = muref.mu_off + (double)dmu;
            const T* fu = s_fu + sfu * 6 * NT + tid;
            const T Fx = fu[0], Fy = fu[NT], Fz = fu[2 * NT], ux = fu[3 * NT], uy = fu[4 * NT], uz = fu[5 * NT];
            T f[19];
            if constexpr (FIFO) {
#pragma unroll
                for (int a = 0; a < 19; ++a) f[a] = fifo[KR][a];
            } else {
                unsigned zb[3];
                zbytes(zd, zb);
                pull<S, T>(pp, oxy, zb, f);
            }
            const T Sm = moving19(f);
            const T drho = f[0] + Sm;
            const double m_in = F32 ? mass_in<19, T>(f) : 0.0;    // exact node mass (float32 storage)
            const int node = zd * NXY + gy0 * nx + gx0;
            if constexpr (MODE == kFields) {
                const long long o = field_offset + node;
                if (args.rho_out) args.rho_out[o] = muref.rho_ref + (double)x;
                if (args.mu_out) args.mu_out[o] = mu;
                if (args.u_out) {
                    args.u_out[o] = (double)ux;
                    args.u_out[args.field_total + o] = (double)uy;
                    args.u_out[2 * args.field_total + o] = (double)uz;
                }
            } else {
                T dpm, php, Cxx = T(0), Cyy = T(0), Czz = T(0);
                if constexpr (IMP) {
                    const int c1 = (ly0 + 1) * W1 + lx0 + 1;
                    const T* Xd = s_psi + md * A1; const T* Xp = s_psi + mp * A1; const T* Xu = s_psi + mu3 * A1;
                    const T* Yd = Xd + 3 * A1; const T* Yp = Xp + 3 * A1; const T* Yu = Xu + 3 * A1;
                    const T* Zdd = Xd + 6 * A1; const T* Zp = Xp + 6 * A1; const T* Zu = Xu + 6 * A1;
                    Cxx = T(3) * gx<W1>(Xd, Xp, Xu, c1);
                    Cyy = T(3) * gy<W1>(Yd, Yp, Yu, c1);
                    Czz = T(3) * gz<W1>(Zdd, Zp, Zu, c1);
                    if constexpr (F32) {
                        dpm = dmu * T(1.0 / 3.0);
                        php = -(phi0 + (x - dmu) * T(1.0 / 3.0));
                    } else {
                        dpm = (dmu - mu_ref) * T(1.0 / 3.0);
                        php = (c0 + dmu) * T(1.0 / 3.0) - r * T(1.0 / 3.0);
                    }
                } else {
                    dpm = drho * T(1.0 / 3.0);
                    php = T(0);
                }
                collide<T>(f, r, Sm, ux, uy, uz, Fx, Fy, Fz, dpm, php, Cxx, Cyy, Czz, omega);
                if constexpr (F32) keep_mass_on_axes<19, 6, T>(f, m_in);
                if constexpr (WT) {
#pragma unroll
                    for (int a = 0; a < 19; ++a) st_dev(dst + (size_t)a * N, (unsigned)node, (S)f[a]);
                } else {
#pragma unroll
                    for (int a = 0; a < 19; ++a) st_off(dst + (size_t)a * N, (unsigned)node, (S)f[a]);
                }
            }
            acc.mass += F32 ? m_in : (double)drho;
            acc.mx += (double)(r * ux);
            acc.my += (double)(r * uy);
            acc.mz += (double)(r * uz);
            acc.umax2 = fmax(acc.umax2, (double)(ux * ux + uy * uy + uz * uz));
            acc.mumin = fmin(acc.mumin, mu);
            acc.mumax = fmax(acc.mumax, mu);
            acc.status |= blowup_bits<T>(r, ux, uy, uz, rho_max);
        }
        __syncthreads();
    };
    for (int it0 = 0; it0 < NIT; it0 += 4) {
        iteration(it0, std::integral_constant<int, 0>{});
        iteration(it0 + 1, std::integral_constant<int, 1>{});
        iteration(it0 + 2, std::integral_constant<int, 2>{});
        iteration(it0 + 3, std::integral_constant<int, 3>{});
    }
    if constexpr (MODE == kStep) {
        if (acc.status) atomicOr(args.status + tile.lat, acc.status);
    } else {
        const unsigned st = block_reduce_store<NT>(acc, args.partial + t_idx, s_red, s_ured);
        if (st != 0u) atomicOr(args.status + tile.lat, st);
    }
}

template <typename S, typename T, int V>
__global__ void init_kernel(S* state, const LatticeRec* recs, int nlat, const double* rho0, const double* u0,
                            long long field_total) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int L = 0;
    while (L + 1 < nlat && gid >= recs[L + 1].field_offset) ++L;
    const LatticeRec& R = recs[L];
    const long long local = gid - R.field_offset;
    if (local < 0 || local >= R.nnodes) return;
    const int nx = R.nx, ny = R.ny, nz = R.nz, NXY = nx * ny, N = NXY * nz;
    const int x = (int)(local % nx), y = (int)((local / nx) % ny), z = (int)(local / NXY);
    const double* r0 = rho0 + R.field_offset;
    auto at = [&](int dx, int dy, int dz) {
        const int xx = ((x + dx) % nx + nx) % nx, yy = ((y + dy) % ny + ny) % ny, zz = ((z + dz) % nz + nz) % nz;
        return (T)r0[(zz * ny + yy) * nx + xx];
    };
    const T r = at(0, 0, 0);
    T ux = T(0), uy = T(0), uz = T(0);
    if (u0) {
        ux = (T)u0[R.field_offset + local];
        uy = (T)u0[field_total + R.field_offset + local];
        uz = (T)u0[2 * field_total + R.field_offset + local];
    }
    T dpm, php;
    if (V == kImproved) {
        T ax = T(0), ed = T(0);
#pragma unroll
        for (int a = 1; a < 19; ++a) {
            const T v = at(EX[a], EY[a], EZ[a]);
            if (a < 7) ax += v; else ed += v;
        }
        const T L2 = T(1.0 / 3.0) * ax + T(1.0 / 6.0) * ed - T(4) * r;
        const Eos<T> eos{R.eos, (T)R.a, (T)R.b, (T)R.RT};
        const T mu = eos.mu(r) - (T)R.kappa * L2;
        dpm = (mu - (T)R.mu_ref) * T(1.0 / 3.0);
        php = ((T)R.c0 + mu) * T(1.0 / 3.0) - r * T(1.0 / 3.0);
    } else {
        dpm = (r - (T)R.rho_ref) * T(1.0 / 3.0);
        php = T(0);
    }
    T feq[19];
    equilibrium<T>(feq, r, r - (T)R.rho_ref, ux, uy, uz, dpm, php);
    S* st = state + R.state_offset * 19;
#pragma unroll
    for (int a = 0; a < 19; ++a) {
        const int sx = ((x - EX[a]) % nx + nx) % nx, sy = ((y - EY[a]) % ny + ny) % ny,
                  sz = ((z - EZ[a]) % nz + nz) % nz;
        st[(size_t)a * N + (sz * ny + sy) * nx + sx] = (S)feq[a];
    }
}

template <typename S, bool GET>
__global__ void convert_kernel(S* state, const LatticeRec* recs, int nlat, double* f, long long field_total) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int L = 0;
    while (L + 1 < nlat && gid >= recs[L + 1].field_offset) ++L;
    const LatticeRec& R = recs[L];
    const long long local = gid - R.field_offset;
    if (local < 0 || local >= R.nnodes) return;
    const int nx = R.nx, ny = R.ny, nz = R.nz, NXY = nx * ny, N = NXY * nz;
    const int x = (int)(local % nx), y = (int)((local / nx) % ny), z = (int)(local / NXY);
    S* st = state + R.state_offset * 19;
    for (int a = 0; a < 19; ++a) {
        const int sx = ((x - EX[a]) % nx + nx) % nx, sy = ((y - EY[a]) % ny + ny) % ny,
                  sz = ((z - EZ[a]) % nz + nz) % nz;
        const long long fo = (long long)a * field_total + R.field_offset + local;
        const long long so = (long long)a * N + (sz * ny + sy) * nx + sx;
        if (GET)
            f[fo] = (double)st[so] + R.fbar[a];
        else
            st[so] = (S)(f[fo] - R.fbar[a]);
    }
}

}  // namespace d3q19

namespace {
template <typename S, typename T, int V, int BX, int BY>
hipError_t launch3_t(const StepArgs& a, int grid, hipStream_t s, int mode) {
    if constexpr (sizeof(T) == 8 && BX * BY > 256) {
        return hipErrorInvalidValue;      // float64 rings of this tile exceed the 160 KB of LDS
    } else {
    const dim3 g(grid), b(BX * BY);
    if (mode == kFields)
        hipLaunchKernelGGL((d3q19::step_kernel<S, T, V, BX, BY, kFields, false>), g, b, 0, s, a);
    else if (a.write_through)
        hipLaunchKernelGGL((d3q19::step_kernel<S, T, V, BX, BY, kStep, true>), g, b, 0, s, a);
    else
        hipLaunchKernelGGL((d3q19::step_kernel<S, T, V, BX, BY, kStep, false>), g, b, 0, s, a);
    return hipGetLastError();
    }
}
template <typename S, typename T, int V>
hipError_t launch3_shape(const StepArgs& a, int grid, hipStream_t s, int fields, int shape) {
    switch (shape) {
        case 0: return launch3_t<S, T, V, 32, 8>(a, grid, s, fields);
        case 1: return launch3_t<S, T, V, 32, 16>(a, grid, s, fields);
        case 2: return launch3_t<S, T, V, 16, 16>(a, grid, s, fields);
        case 3: return launch3_t<S, T, V, 64, 4>(a, grid, s, fields);
        default: return hipErrorInvalidValue;
    }
}
}  // namespace

extern const int kD3Q19Shapes[][2];
const int kD3Q19Shapes[][2] = {{32, 8}, {32, 16}, {16, 16}, {64, 4}};
extern const int kNumD3Q19Shapes;
const int kNumD3Q19Shapes = 4;

hipError_t d3q19_launch_step(const StepArgs& a, int grid, hipStream_t s, int precision, int variant, int shape,
                             int fields) {
    if (precision == 0) {
        switch (variant) {
            case kStdChempot: return launch3_shape<double, double, kStdChempot>(a, grid, s, fields, shape);
            case kStdPtensor: return launch3_shape<double, double, kStdPtensor>(a, grid, s, fields, shape);
            case kImproved: return launch3_shape<double, double, kImproved>(a, grid, s, fields, shape);
        }
    } else {
        switch (variant) {
            case kStdChempot: return launch3_shape<float, float, kStdChempot>(a, grid, s, fields, shape);
            case kStdPtensor: return launch3_shape<float, float, kStdPtensor>(a, grid, s, fields, shape);
            case kImproved: return launch3_shape<float, float, kImproved>(a, grid, s, fields, shape);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t d3q19_launch_init(void* state, const LatticeRec* recs, int nlat, const double* rho0, const double* u0,
                             long long total, hipStream_t s, int precision, int variant) {
    const int B = 256;
    const int grid = (int)((total + B - 1) / B);
    if (grid == 0) return hipSuccess;
    const bool imp = variant == kImproved;
    if (precision == 0) {
        if (imp)
            hipLaunchKernelGGL((d3q19::init_kernel<double, double, kImproved>), dim3(grid), dim3(B), 0, s,
                               (double*)state, recs, nlat, rho0, u0, total);
        else
            hipLaunchKernelGGL((d3q19::init_kernel<double, double, kStdChempot>), dim3(grid), dim3(B), 0, s,
                               (double*)state, recs, nlat, rho0, u0, total);
    } else {
        if (imp)
            hipLaunchKernelGGL((d3q19::init_kernel<float, float, kImproved>), dim3(grid), dim3(B), 0, s,
                               (float*)state, recs, nlat, rho0, u0, total);
        else
            hipLaunchKernelGGL((d3q19::init_kernel<float, float, kStdChempot>), dim3(grid), dim3(B), 0, s,
                               (float*)state, recs, nlat, rho0, u0, total);
    }
    return hipGetLastError();
}

hipError_t d3q19_launch_convert(void* state, const LatticeRec* recs, int nlat, double* f, long long total,
                                hipStream_t s, int precision, bool get) {
    const int B = 256;
    const int grid = (int)((total + B - 1) / B);
    if (grid == 0) return hipSuccess;
    if (precision == 0) {
        if (get)
            hipLaunchKernelGGL((d3q19::convert_kernel<double, true>), dim3(grid), dim3(B), 0, s, (double*)state,
                               recs, nlat, f, total);
        else
            hipLaunchKernelGGL((d3q19::convert_kernel<double, false>), dim3(grid), dim3(B), 0, s, (double*)state,
                               recs, nlat, f, total);
    } else {
        if (get)
            hipLaunchKernelGGL((d3q19::convert_kernel<float, true>), dim3(grid), dim3(B), 0, s, (float*)state,
                               recs, nlat, f, total);
        else
            hipLaunchKernelGGL((d3q19::convert_kernel<float, false>), dim3(grid), dim3(B), 0, s, (float*)state,
                               recs, nlat, f, total);
    }
    return hipGetLastError();
}

}  // namespace lbm
