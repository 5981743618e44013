// Plain data records shared by the host runtime and the kernels.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace lbm {

constexpr int kMaxQ = 19;

// Scheme variants compiled into the kernels.
enum Variant : int {
    kStdChempot = 0,   // Eq. 13 right: F = grad(rho/3) - rho grad(mu)
    kStdPtensor = 1,   // Eq. 13 left:  F = grad(rho/3) - div P, P from Eqs. 4-5
    kImproved = 2      // Eq. 24, Eq. 27, Eqs. 28-29
};

// What a step-kernel launch does at its output nodes.
enum Mode : int {
    kStep = 0,         // collide and store; only the blow-up flags are checked
    kFields = 1        // write rho, u, mu (any may be absent) and the per-tile diagnostics
};

// Per-lattice record, uploaded once at bind time.
struct LatticeRec {
    int nx, ny, nz, eos;
    int slow_x, slow_y, slow_z, q;      // slow_*: extent too small for single-step wrap
    long long state_offset;             // first node of this lattice in the state buffers
    long long field_offset;             // first node of this lattice in field arrays
    long long nnodes;
    double a, b, RT, kappa, omega, rho_max;
    double rho_ref, pm_ref, mu_ref;     // FP32 deviation reference (zero for FP64)
    double fbar[kMaxQ];                 // reference populations f_eq(rho_ref, 0, pm_ref)
    int tile_begin, tile_end;           // range of this lattice's tiles in the tile list
    // D2Q9 MRT (Eq. 8): mrt != 0 selects it; rates of e, eps, q; shear rate
    // omega (nu <= 0) or from the constant kinematic viscosity nu.
    int mrt, pad_mrt;
    double s_e, s_eps, s_q, nu;
    // D2Q9 plates bounding y (walls != 0): x-velocities of the bottom and top plate.
    int walls, pad_walls;
    double wall_u0, wall_u1;
    double c0;                          // improved scheme: p_m = (c0 + mu)/3 (the paper: 1)
    // Float32 chemical potential in deviation form (see MuRef): q0 = 1/(1 - b rho_ref)
    // (vdW) or 1/(1 - b rho_ref / 4) (CS), and the constant part k0 of
    // mu_EOS(rho_ref + x) - mu_ref that does not depend on x.
    double dev_q0, dev_k0;
};

// Chaining flags of consecutive adjoint steps (adjoint_launch).
enum AdjChain : int { kAdjPending = 1, kAdjDeferReduce = 2 };

// One unit of work: an output tile (2D) or an output column chunk (3D).  It also
// carries its lattice's extents, wrap flags and state offset, so that a batch's
// tile can issue its pulls as soon as this record has arrived.
struct Tile {
    int lat, x0, y0, z0, zn;
    int nx, ny;
    int slow;                 // bit 0: slow wrap in x, bit 1: in y (lattice narrower than a tile + 8)
    long long soff;           // the lattice's state offset in nodes
};

// Order of the D2Q9 tiles of one lattice: bands of `band` tile columns, taken
// left to right, each band row-major.  Work groups are dealt to the XCDs in
// contiguous runs of this order, so the tiles resident on one XCD at a time
// form a compact block whose halo rows are still in that XCD's L2 when the next
// rows of the band read them.
__host__ __device__ inline void band_order(int t, int ntx, int nty, int band, int& tx, int& ty) {
    const int per_band = band * nty;
    const int b = t / per_band;
    const int r = t - b * per_band;
    const int left = ntx - b * band;
    const int wb = left < band ? left : band;
    ty = r / wb;
    tx = b * band + (r - ty * wb);
}

// Per-tile partial diagnostics, reduced per lattice in a fixed order.
struct DiagPartial {
    double mass, momx, momy, momz, umax2, mumin, mumax;
    unsigned int status, pad;
};

// Per-lattice reduced diagnostics (device side image of lbm_diag's sums).
struct DiagOut {
    double mass, momx, momy, momz, umax, mumin, mumax;
    unsigned int status, pad;
};

struct StepArgs {
    const void* src;          // state at time t (post-collision at t-1, unstreamed)
    void* dst;                // state at time t+1
    const LatticeRec* recs;
    const Tile* tiles;
    int ntiles;
    int tiles_per_xcd;        // XCD-aware block -> tile mapping
    DiagPartial* partial;     // one per tile
    unsigned int* status;     // one per lattice (sticky blow-up flags)
    double* rho_out;          // fields mode outputs (may be null)
    double* u_out;
    double* mu_out;
    long long field_total;    // total nodes of all lattices (vector-field stride)
    // One lattice only (single != 0): the kernels derive their tile from the
    // block index with band_order and take the extents below from the
    // arguments instead of loading the tile and lattice records first.
    int single, ntx, nty, band;
    int nx0, ny0, slow_x0, slow_y0;
    int any_mrt;              // some lattice of the launch uses the MRT collision (D2Q9)
    int any_plates;           // some lattice of the launch has plates (D2Q9)
    int write_through;        // store the populations at device scope (st_dev), not non-temporally
};

}  // namespace lbm
