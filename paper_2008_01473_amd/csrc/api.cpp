// Host runtime behind the C ABI of include/lbm.h: parameter checks, tiling
// plans, workspace layout, kernel launches, HIP graph replay of many steps,
// diagnostics read-back and the tile-shape autotuner.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/lbm.h"
#include "host_thermo.hpp"
#include "lbm_shared.hpp"

namespace lbm {
hipError_t d2q9_launch_step(const StepArgs& a, int grid, hipStream_t s, int precision, int variant, int shape,
                            int mode);
hipError_t d2q9_launch_init(void* state, const LatticeRec* recs, int nlat, const double* rho0, const double* u0,
                            long long total, hipStream_t s, int precision, int variant);
hipError_t d2q9_launch_convert(void* state, const LatticeRec* recs, int nlat, double* f, long long total,
                               hipStream_t s, int precision, bool get);
hipError_t d3q19_launch_step(const StepArgs& a, int grid, hipStream_t s, int precision, int variant, int shape,
                             int mode);
hipError_t d3q19_launch_init(void* state, const LatticeRec* recs, int nlat, const double* rho0, const double* u0,
                             long long total, hipStream_t s, int precision, int variant);
hipError_t d3q19_launch_convert(void* state, const LatticeRec* recs, int nlat, double* f, long long total,
                                hipStream_t s, int precision, bool get);
hipError_t launch_finalize(const DiagPartial* partial, const LatticeRec* recs, const unsigned* status,
                           DiagOut* out, int nlat, hipStream_t s);
hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
size_t adjoint_workspace_doubles(int nx, int ny);
size_t static_scratch_bytes();
hipError_t static_scratch(void** out);
hipError_t adjoint_launch(int kind, const LatticeRec& rec, double dRT, int precision, int improved, const void* state,
                          const double* lam_in, double* lam_out, const double* rho_bar, const double* u_bar,
                          const double* rho0, double* grad_rho0, double* ws, double* grad, hipStream_t s,
                          int chain);
extern const int kD2Q9Shapes[][2];
extern const int kNumD2Q9Shapes;
extern const int kD2Q9NodesPerThread[];
extern const int kD3Q19Shapes[][2];
extern const int kNumD3Q19Shapes;
}  // namespace lbm

using namespace lbm;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

#define HIP_TRY(call)                                                                             \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(LBM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));          \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int kGraphChunk = 256;   // even, so replaying a chunk keeps the buffer parity

// Work-group counts the D3Q19 z-chunking may aim at (256 CUs): fewer, longer
// chunks re-read fewer warm-up slices; more chunks fill the CUs better.
constexpr int kNumZTargets = 3;
constexpr long long kZTargets[kNumZTargets] = {512, 1024, 256};
constexpr int kMinZChunk = 16;     // shortest z-chunk lbm_set_zchunk accepts (below: mostly warm-up)

}  // namespace

struct lbm_ctx {
    std::vector<lbm_params> params;
    int lattice = 0, Q = 9, D = 2, variant = 0, precision = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    std::vector<LatticeRec> recs;
    std::vector<Tile> tiles;
    int shape = 0;
    int zchunk_fixed = 0;     // D3Q19: z-chunk length set by lbm_set_zchunk (0: from the tuning index)
    int store_mode = LBM_STORES_STREAMING;   // how the step kernels store f* (lbm_set_store_mode)
    long long field_total = 0, state_nodes = 0;
    size_t state_bytes = 0, ws_bytes = 0;
    size_t off_recs = 0, off_tiles = 0, off_partial = 0, off_status = 0, off_diag = 0;
    int max_tiles = 0;
    char* ws = nullptr;
    void* buf[2] = {nullptr, nullptr};
    int cur = 0;
    long long t = 0, t_diag = -1;
    bool bound = false, inited = false;
    bool use_graphs = true;
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;
    // Lattices reported blown up by lbm_diagnostics: left out of the plan (frozen)
    // until the next reset of the status flags.  Their last diagnostics stay
    // readable from a host copy until the next step produces new ones.
    std::vector<char> dropped;
    std::vector<DiagOut> frozen_diag;       // a dropped lattice's diagnostics when it was reported
    std::vector<long long> frozen_step;
    std::vector<DiagOut> diag_cache;
    bool diag_cache_valid = false;
    // lbm_step leaves the reduction of its last input's diagnostics to
    // lbm_diagnostics, which reads that time level from the other buffer
    bool diag_pending = false;

    // A tuning index names a kernel tile shape and, for D3Q19, also how many
    // work groups the z-chunking aims at (kZTargets): index = shape * 3 + target.
    int num_shapes() const { return lattice == LBM_D2Q9 ? kNumD2Q9Shapes : kNumD3Q19Shapes * kNumZTargets; }
    int kernel_shape(int s) const { return lattice == LBM_D2Q9 ? s : s / kNumZTargets; }
    void shape_dims(int s, int& bx, int& by) const {
        if (lattice == LBM_D2Q9) {
            bx = kD2Q9Shapes[s][0];
            by = kD2Q9Shapes[s][1];
        } else {
            bx = kD3Q19Shapes[kernel_shape(s)][0];
            by = kD3Q19Shapes[kernel_shape(s)][1];
        }
    }
    LatticeRec* d_recs() const { return reinterpret_cast<LatticeRec*>(ws + off_recs); }
    Tile* d_tiles() const { return reinterpret_cast<Tile*>(ws + off_tiles); }
    DiagPartial* d_partial() const { return reinterpret_cast<DiagPartial*>(ws + off_partial); }
    unsigned* d_status() const { return reinterpret_cast<unsigned*>(ws + off_status); }
    DiagOut* d_diag() const { return reinterpret_cast<DiagOut*>(ws + off_diag); }
    int zchunk_for(int s) const;
    std::vector<Tile> plan(int s, std::vector<LatticeRec>& rr) const;
    // Adjoint segments (lbm_adjoint_segment) replayed from graphs, keyed by the
    // segment length, the buffer parity and the caller's buffers.
    using SegKey = std::tuple<int, int, const void*, const void*, const void*, const void*, const void*>;
    std::map<SegKey, hipGraphExec_t> seg_graphs;
    // lbm_adjoint_sweep: recompute (kind 0) and adjoint-step (kind 1) graphs keyed by
    // (kind, segment length, arena, lam, lam2, ws, grad); a second stream for the
    // recomputation and the events that order the two streams.
    std::map<SegKey, hipGraphExec_t> sweep_graphs;
    hipStream_t side_stream = nullptr;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    void drop_graphs() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);   // teardown: nothing to report
        graphs.clear();
        for (auto& kv : seg_graphs) (void)hipGraphExecDestroy(kv.second);
        seg_graphs.clear();
        for (auto& kv : sweep_graphs) (void)hipGraphExecDestroy(kv.second);
        sweep_graphs.clear();
    }
};

// Width (in tiles) of the D2Q9 tile bands: about 512 nodes, so that the tiles
// resident on one XCD cover a block a few bands tall rather than whole rows.
static int band_width(int ntx, int bx) { return std::max(1, std::min(ntx, 512 / bx)); }

int lbm_ctx::zchunk_for(int s) const {
    if (lattice == LBM_D2Q9) return 1;
    if (zchunk_fixed > 0) return zchunk_fixed;
    int bx, by;
    shape_dims(s, bx, by);
    long long cols = 0;
    int nzmax = 1;
    for (const auto& p : params) {
        cols += (long long)((p.nx + bx - 1) / bx) * ((p.ny + by - 1) / by);
        nzmax = std::max(nzmax, p.nz);
    }
    // aim for the index's work-group count, chunks of >= 16 slices
    const long long want = kZTargets[s % kNumZTargets];
    int chunks = (int)std::max<long long>(1, (want + cols - 1) / cols);
    int zc = (nzmax + chunks - 1) / chunks;
    zc = std::max(zc, std::min(16, nzmax));
    return zc;
}

static Tile tile_of(const LatticeRec& R, int L) {
    Tile t{};
    t.lat = L;
    t.nx = R.nx;
    t.ny = R.ny;
    t.slow = (R.slow_x ? 1 : 0) | (R.slow_y ? 2 : 0);
    t.soff = R.state_offset;
    return t;
}

std::vector<Tile> lbm_ctx::plan(int s, std::vector<LatticeRec>& rr) const {
    int bx, by;
    shape_dims(s, bx, by);
    const int zc = zchunk_for(s);
    std::vector<Tile> out;
    for (size_t L = 0; L < rr.size(); ++L) {
        LatticeRec& R = rr[L];
        R.slow_x = R.nx < bx + 8;
        R.slow_y = R.ny < by + 8;
        R.slow_z = R.nz < 8;
        R.tile_begin = (int)out.size();
        if (dropped[L]) {             // reported blown up: frozen, no work
            R.tile_end = R.tile_begin;
            continue;
        }
        const int ntx = (R.nx + bx - 1) / bx, nty = (R.ny + by - 1) / by;
        if (lattice == LBM_D2Q9) {
            const int band = band_width(ntx, bx);
            for (int k = 0; k < ntx * nty; ++k) {
                int tx, ty;
                band_order(k, ntx, nty, band, tx, ty);
                Tile t = tile_of(R, (int)L);
                t.x0 = tx * bx;
                t.y0 = ty * by;
                t.z0 = 0;
                t.zn = 1;
                out.push_back(t);
            }
        } else {
            const int nzc = (R.nz + zc - 1) / zc;
            for (int kz = 0; kz < nzc; ++kz)
                for (int ty = 0; ty < nty; ++ty)
                    for (int tx = 0; tx < ntx; ++tx) {
                        Tile t = tile_of(R, (int)L);
                        t.x0 = tx * bx;
                        t.y0 = ty * by;
                        t.z0 = kz * zc;
                        t.zn = std::min(zc, R.nz - kz * zc);
                        out.push_back(t);
                    }
        }
        R.tile_end = (int)out.size();
    }
    return out;
}

namespace {

int check_params(const lbm_params& p) {
    if (p.lattice != LBM_D2Q9 && p.lattice != LBM_D3Q19) return fail(LBM_ERR_ARG, "lattice must be D2Q9 or D3Q19");
    if (p.nx < 1 || p.ny < 1 || p.nz < 1) return fail(LBM_ERR_ARG, "lattice extents must be >= 1");
    if (p.lattice == LBM_D2Q9 && p.nz != 1) return fail(LBM_ERR_ARG, "D2Q9 requires nz == 1");
    const long long n = (long long)p.nx * p.ny * p.nz;
    // the kernels address one population array with unsigned 32-bit byte offsets
    if (n * (p.precision == LBM_FP32_DEV ? 4 : 8) > (1LL << 32))
        return fail(LBM_ERR_UNSUPPORTED,
                    "one population array of a lattice may span at most 4 GB (2^30 nodes in float32, 2^29 in float64)");
    if (p.eos != LBM_EOS_VDW && p.eos != LBM_EOS_CS) return fail(LBM_ERR_ARG, "eos must be VDW or CS");
    if (!(p.a >= 0) || !(p.b > 0) || !(p.R > 0)) return fail(LBM_ERR_ARG, "EOS constants need a >= 0, b > 0, R > 0");
    if (!(p.T_over_Tc > 0)) return fail(LBM_ERR_ARG, "T_over_Tc must be > 0");
    if (!(p.kappa >= 0)) return fail(LBM_ERR_ARG, "kappa must be >= 0");
    if (!(p.tau > 0.5)) return fail(LBM_ERR_ARG, "tau must be > 0.5");
    if (p.scheme != LBM_STANDARD && p.scheme != LBM_IMPROVED) return fail(LBM_ERR_ARG, "bad scheme");
    if (p.force_form != LBM_FORCE_CHEMPOT && p.force_form != LBM_FORCE_PTENSOR) return fail(LBM_ERR_ARG, "bad force form");
    if (p.force_form == LBM_FORCE_PTENSOR && p.scheme != LBM_STANDARD)
        return fail(LBM_ERR_ARG, "the pressure-tensor force is defined for the standard scheme only");
    if (p.precision != LBM_FP64 && p.precision != LBM_FP32_DEV) return fail(LBM_ERR_ARG, "bad precision");
    if (p.a == 0) return fail(LBM_ERR_ARG, "a must be > 0 (T_c is proportional to a)");
    if (p.collision != LBM_BGK && p.collision != LBM_MRT) return fail(LBM_ERR_ARG, "bad collision");
    if (p.collision == LBM_MRT) {
        if (p.lattice != LBM_D2Q9) return fail(LBM_ERR_UNSUPPORTED, "the MRT collision is implemented for D2Q9");
        if (!(p.tau_e > 0.5) || !(p.tau_s > 0.5) || !(p.tau_q > 0.5))
            return fail(LBM_ERR_ARG, "MRT relaxation times tau_e, tau_s, tau_q must be > 0.5");
        if (!(p.nu == p.nu)) return fail(LBM_ERR_ARG, "nu must be a number");
    }
    if (!(p.c0 >= 0) || !std::isfinite(p.c0)) return fail(LBM_ERR_ARG, "c0 must be >= 0 (0 selects 1)");
    if (p.walls != 0) {
        if (p.walls != 1) return fail(LBM_ERR_ARG, "walls must be 0 or 1");
        if (p.lattice != LBM_D2Q9) return fail(LBM_ERR_UNSUPPORTED, "plates are implemented for D2Q9");
        if (p.force_form != LBM_FORCE_CHEMPOT)
            return fail(LBM_ERR_UNSUPPORTED, "plates are implemented with the chemical-potential force");
        if (p.ny < 4) return fail(LBM_ERR_ARG, "a lattice with plates needs ny >= 4");
        if (!std::isfinite(p.wall_u_bottom) || !std::isfinite(p.wall_u_top))
            return fail(LBM_ERR_ARG, "plate velocities must be finite");
    }
    return LBM_OK;
}

// Constants of the float32 chemical potential in deviation form (MuRef in the
// kernels): mu_EOS(rho_ref + x) - mu_ref = k0 + RT [ln(rho q) + b x q q0] - 2 a x
// (vdW, q = 1/(1 - b rho)) or k0 + RT [ln rho + g(h) - g(h0)] - 2 a x (CS).
void set_dev_constants(LatticeRec& R, double Rgas) {
    if (!(R.rho_ref > 0)) {
        R.dev_q0 = R.dev_k0 = 0.0;
        return;
    }
    const double T = R.RT / Rgas;
    const double mu0 = host::mu_eos(R.eos, R.a, R.b, Rgas, T, R.rho_ref) - R.mu_ref;
    if (R.eos == LBM_EOS_VDW) {
        R.dev_q0 = 1.0 / (1.0 - R.b * R.rho_ref);
        R.dev_k0 = mu0 - R.RT * std::log(R.rho_ref * R.dev_q0);
    } else {
        R.dev_q0 = 1.0 / (1.0 - 0.25 * R.b * R.rho_ref);
        R.dev_k0 = mu0 - R.RT * std::log(R.rho_ref);
    }
}

LatticeRec make_rec(const lbm_params& p, int variant, int Q) {
    LatticeRec R;
    std::memset(&R, 0, sizeof(R));
    R.nx = p.nx;
    R.ny = p.ny;
    R.nz = p.nz;
    R.eos = p.eos;
    R.q = Q;
    R.nnodes = (long long)p.nx * p.ny * p.nz;
    R.a = p.a;
    R.b = p.b;
    R.RT = p.R * p.T_over_Tc * host::critical_temperature(p.eos, p.a, p.b, p.R);
    R.kappa = p.kappa;
    R.omega = 1.0 / p.tau;
    R.rho_max = host::rho_limit(p.eos, p.b);
    R.c0 = p.c0 > 0 ? p.c0 : 1.0;
    if (p.walls) {
        R.walls = 1;
        R.wall_u0 = p.wall_u_bottom;
        R.wall_u1 = p.wall_u_top;
    }
    if (p.collision == LBM_MRT) {
        R.mrt = 1;
        R.s_e = 1.0 / p.tau_e;
        R.s_eps = 1.0 / p.tau_s;
        R.s_q = 1.0 / p.tau_q;
        R.nu = p.nu > 0 ? p.nu : 0.0;
    }
    if (p.precision == LBM_FP64) {
        R.rho_ref = 0.0;
        R.pm_ref = 0.0;
        R.mu_ref = -R.c0;    // so that p_m - pm_ref = (mu - mu_ref)/3 = p_m
        return R;
    }
    double rho_ref = p.rho_ref, pm_ref = p.pm_ref;
    if (!(rho_ref > 0) || !(pm_ref > 0)) {
        double rg, rl, mu, ps;
        double T = R.RT / p.R;
        double rr, mm;
        if (host::maxwell(p.eos, p.a, p.b, p.R, p.T_over_Tc, &rg, &rl, &mu, &ps) == 0) {
            rr = 0.5 * (rg + rl);
            mm = mu;
        } else {   // no coexistence: single-phase reference at the critical density
            rr = p.eos == LBM_EOS_VDW ? 1.0 / (3.0 * p.b) : 0.5217755367698157 / p.b;
            mm = host::mu_eos(p.eos, p.a, p.b, p.R, T, rr);
        }
        if (!(rho_ref > 0)) rho_ref = rr;
        if (!(pm_ref > 0)) pm_ref = (variant == kImproved) ? (R.c0 + mm) / 3.0 : rho_ref / 3.0;
    }
    R.rho_ref = rho_ref;
    R.pm_ref = pm_ref;
    R.mu_ref = 3.0 * pm_ref - R.c0;
    if (variant != kImproved) R.pm_ref = rho_ref / 3.0;
    set_dev_constants(R, p.R);
    const double pmr = R.pm_ref;
    if (Q == 9) {
        R.fbar[0] = rho_ref - 5.0 * pmr / 3.0;
        for (int a = 1; a < 5; ++a) R.fbar[a] = pmr / 3.0;
        for (int a = 5; a < 9; ++a) R.fbar[a] = pmr / 12.0;
    } else {
        R.fbar[0] = rho_ref - 2.0 * pmr;
        for (int a = 1; a < 7; ++a) R.fbar[a] = pmr / 6.0;
        for (int a = 7; a < 19; ++a) R.fbar[a] = pmr / 12.0;
    }
    return R;
}

hipError_t launch_step(lbm_ctx* h, const StepArgs& a, int mode, hipStream_t s) {
    const int ntiles = (int)h->tiles.size();
    const int per = (ntiles + 7) / 8;
    StepArgs b = a;
    b.ntiles = ntiles;
    b.tiles_per_xcd = per;
    const int grid = 8 * per;
    if (grid == 0) return hipSuccess;
    for (const auto& R : h->recs) {
        b.any_mrt |= R.mrt;
        b.any_plates |= R.walls;
    }
    b.write_through = h->store_mode == LBM_STORES_DEVICE;
    if (h->lattice == LBM_D2Q9 && h->params.size() == 1) {
        int bx, by;
        h->shape_dims(h->shape, bx, by);
        const lbm_params& p = h->params[0];
        b.single = 1;
        b.ntx = (p.nx + bx - 1) / bx;
        b.nty = (p.ny + by - 1) / by;
        b.band = band_width(b.ntx, bx);
        b.nx0 = p.nx;
        b.ny0 = p.ny;
        b.slow_x0 = p.nx < bx + 8;
        b.slow_y0 = p.ny < by + 8;
    }
    if (h->lattice == LBM_D2Q9) return d2q9_launch_step(b, grid, s, h->precision, h->variant, h->shape, mode);
    return d3q19_launch_step(b, grid, s, h->precision, h->variant, h->kernel_shape(h->shape), mode);
}

StepArgs base_args(lbm_ctx* h) {
    StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.recs = h->d_recs();
    a.tiles = h->d_tiles();
    a.partial = h->d_partial();
    a.status = h->d_status();
    a.field_total = h->field_total;
    return a;
}

int upload_tables(lbm_ctx* h) {
    HIP_TRY(hipMemcpyAsync(h->d_recs(), h->recs.data(), h->recs.size() * sizeof(LatticeRec), hipMemcpyHostToDevice,
                           h->stream));
    HIP_TRY(hipMemcpyAsync(h->d_tiles(), h->tiles.data(), h->tiles.size() * sizeof(Tile), hipMemcpyHostToDevice,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

// Rebuild the tile list for the current shape and the current set of frozen
// lattices; graphs captured with the old list are dropped.
int replan(lbm_ctx* h) {
    h->tiles = h->plan(h->shape, h->recs);
    h->drop_graphs();
    return upload_tables(h);
}

// Clear every lattice's blow-up flags and bring frozen lattices back into the plan.
int reset_status(lbm_ctx* h) {
    HIP_TRY(launch_zero_u32(h->d_status(), (int)h->recs.size(), h->stream));
    h->diag_cache_valid = false;
    bool any = false;
    for (char& d : h->dropped) {
        any |= d != 0;
        d = 0;
    }
    return any ? replan(h) : LBM_OK;
}

int enqueue_steps(lbm_ctx* h, int n, hipStream_t s, int mode = kStep) {
    for (int i = 0; i < n; ++i) {
        StepArgs a = base_args(h);
        a.src = h->buf[h->cur];
        a.dst = h->buf[h->cur ^ 1];
        HIP_TRY(launch_step(h, a, mode, s));
        h->cur ^= 1;
    }
    return LBM_OK;
}

int graph_for(lbm_ctx* h, int n, hipGraphExec_t* out) {
    auto key = std::make_pair(n, h->cur);
    auto it = h->graphs.find(key);
    if (it != h->graphs.end()) {
        *out = it->second;
        return LBM_OK;
    }
    if (!h->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    const int saved = h->cur;
    HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_steps(h, n, h->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
    h->cur = saved;
    if (rc != LBM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    h->graphs[key] = ex;
    // the executable graph goes to the device now, so that its first replay does
    // not pay for the upload
    e = hipGraphUpload(ex, h->stream);
    if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("hipGraphUpload: ") + hipGetErrorString(e));
    *out = ex;
    return LBM_OK;
}

}  // namespace

namespace {
// Launches of one kind captured once per key and replayed.
template <class Enqueue>
int cached_graph(lbm_ctx* h, std::map<lbm_ctx::SegKey, hipGraphExec_t>& cache, const lbm_ctx::SegKey& key,
                 Enqueue&& enqueue, hipGraphExec_t* out) {
    auto it = cache.find(key);
    if (it != cache.end()) {
        *out = it->second;
        return LBM_OK;
    }
    if (cache.size() >= 16) {                  // callers with fresh buffers every time: keep a few
        for (auto& kv : cache) (void)hipGraphExecDestroy(kv.second);
        cache.clear();
    }
    if (!h->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue(h->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
    if (rc != LBM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    cache[key] = ex;
    *out = ex;
    return LBM_OK;
}
}  // namespace

extern "C" {

const char* lbm_error_string(int code) {
    switch (code) {
        case LBM_OK: return "ok";
        case LBM_ERR_ARG: return "invalid argument";
        case LBM_ERR_UNSUPPORTED: return "unsupported";
        case LBM_ERR_HIP: return "HIP runtime error";
        case LBM_ERR_BLOWUP: return "lattice blew up (NaN/Inf or density out of range)";
        case LBM_ERR_DOMAIN: return "no liquid-gas coexistence at this temperature";
        case LBM_ERR_STATE: return "call out of order";
        default: return "unknown error";
    }
}

const char* lbm_last_error(void) { return g_last_error.c_str(); }

int lbm_create_batch(const lbm_params* p, int count, void* hip_stream, lbm_ctx** out) {
    if (!p || !out || count < 1) return fail(LBM_ERR_ARG, "null argument or count < 1");
    *out = nullptr;
    for (int i = 0; i < count; ++i) {
        int rc = check_params(p[i]);
        if (rc != LBM_OK) return rc;
        if (p[i].lattice != p[0].lattice || p[i].scheme != p[0].scheme || p[i].force_form != p[0].force_form ||
            p[i].precision != p[0].precision)
            return fail(LBM_ERR_ARG, "lattices of one batch must share lattice, scheme, force form and precision");
    }
    lbm_ctx* h = new (std::nothrow) lbm_ctx();
    if (!h) return fail(LBM_ERR_ARG, "out of host memory");
    h->params.assign(p, p + count);
    h->lattice = p[0].lattice;
    h->Q = h->lattice == LBM_D2Q9 ? 9 : 19;
    h->D = h->lattice == LBM_D2Q9 ? 2 : 3;
    h->variant = p[0].scheme == LBM_IMPROVED ? kImproved : (p[0].force_form == LBM_FORCE_PTENSOR ? kStdPtensor
                                                                                                : kStdChempot);
    h->precision = p[0].precision;
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    long long foff = 0, soff = 0;
    for (int i = 0; i < count; ++i) {
        LatticeRec R = make_rec(p[i], h->variant, h->Q);
        R.field_offset = foff;
        R.state_offset = soff;
        foff += R.nnodes;
        soff += (R.nnodes + 63) / 64 * 64;
        h->recs.push_back(R);
    }
    h->dropped.assign(count, 0);
    h->frozen_diag.assign(count, DiagOut{});
    h->frozen_step.assign(count, -1);
    h->field_total = foff;
    h->state_nodes = soff;
    const size_t word = h->precision == LBM_FP64 ? 8 : 4;
    h->state_bytes = align256((size_t)soff * h->Q * word);
    // the largest tile list over all shapes, so that re-tiling fits the workspace;
    // for D3Q19 also with the shortest z-chunk lbm_set_zchunk accepts
    for (int s = 0; s < h->num_shapes(); ++s) {
        std::vector<LatticeRec> rr = h->recs;
        h->max_tiles = std::max<int>(h->max_tiles, (int)h->plan(s, rr).size());
        if (h->lattice == LBM_D3Q19) {
            h->zchunk_fixed = kMinZChunk;
            rr = h->recs;
            h->max_tiles = std::max<int>(h->max_tiles, (int)h->plan(s, rr).size());
            h->zchunk_fixed = 0;
        }
    }
    h->shape = 0;
    h->tiles = h->plan(h->shape, h->recs);
    size_t o = 0;
    h->off_recs = o;
    o = align256(o + count * sizeof(LatticeRec));
    h->off_tiles = o;
    o = align256(o + (size_t)h->max_tiles * sizeof(Tile));
    h->off_partial = o;
    o = align256(o + (size_t)h->max_tiles * sizeof(DiagPartial));
    h->off_status = o;
    o = align256(o + count * sizeof(unsigned));
    h->off_diag = o;
    o = align256(o + count * sizeof(DiagOut));
    h->ws_bytes = o;
    *out = h;
    return LBM_OK;
}

int lbm_create(const lbm_params* p, void* hip_stream, lbm_ctx** out) { return lbm_create_batch(p, 1, hip_stream, out); }

size_t lbm_state_bytes(const lbm_ctx* h) { return h ? h->state_bytes : 0; }
size_t lbm_workspace_bytes(const lbm_ctx* h) { return h ? h->ws_bytes : 0; }
long long lbm_num_nodes(const lbm_ctx* h) { return h ? h->field_total : 0; }
int lbm_count(const lbm_ctx* h) { return h ? (int)h->recs.size() : 0; }
long long lbm_node_offset(const lbm_ctx* h, int i) {
    if (!h || i < 0 || i >= (int)h->recs.size()) return -1;
    return h->recs[i].field_offset;
}
long long lbm_time(const lbm_ctx* h) { return h ? h->t : -1; }

int lbm_bind(lbm_ctx* h, void* f_a, void* f_b, void* workspace) {
    if (!h || !f_a || !f_b || !workspace) return fail(LBM_ERR_ARG, "null argument");
    if (((uintptr_t)f_a | (uintptr_t)f_b | (uintptr_t)workspace) & 255)
        return fail(LBM_ERR_ARG, "buffers must be 256-byte aligned");
    h->drop_graphs();
    h->buf[0] = f_a;
    h->buf[1] = f_b;
    h->ws = reinterpret_cast<char*>(workspace);
    h->cur = 0;
    int rc = upload_tables(h);
    if (rc != LBM_OK) return rc;
    if (int rc0 = reset_status(h); rc0 != LBM_OK) return rc0;
    h->bound = true;
    h->inited = false;
    return LBM_OK;
}

int lbm_init(lbm_ctx* h, const double* rho0, const double* u0) {
    if (!h || !rho0) return fail(LBM_ERR_ARG, "null argument");
    if (!h->bound) return fail(LBM_ERR_STATE, "lbm_bind first");
    h->cur = 0;
    if (h->lattice == LBM_D2Q9)
        HIP_TRY(d2q9_launch_init(h->buf[0], h->d_recs(), (int)h->recs.size(), rho0, u0, h->field_total, h->stream,
                                 h->precision, h->variant));
    else
        HIP_TRY(d3q19_launch_init(h->buf[0], h->d_recs(), (int)h->recs.size(), rho0, u0, h->field_total, h->stream,
                                  h->precision, h->variant));
    if (int rc0 = reset_status(h); rc0 != LBM_OK) return rc0;
    h->t = 0;
    h->t_diag = -1;
    h->diag_pending = false;
    h->inited = true;
    return LBM_OK;
}

int lbm_step(lbm_ctx* h, int n) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (n < 0) return fail(LBM_ERR_ARG, "n must be >= 0");
    if (!h->inited) return fail(LBM_ERR_STATE, "lbm_init or lbm_set_f first");
    if (n == 0) return LBM_OK;
    const long long t0 = h->t;
    // graph replays of even length (the current buffer is unchanged by an even
    // number of steps), then single launches
    int left = n;
    if (h->use_graphs) {
        while (left >= 2) {
            const int len = left >= kGraphChunk ? kGraphChunk : (left & ~1);
            hipGraphExec_t ex;
            int rc = graph_for(h, len, &ex);
            if (rc != LBM_OK) return rc;
            HIP_TRY(hipGraphLaunch(ex, h->stream));
            left -= len;
        }
    }
    int rc = enqueue_steps(h, left, h->stream, kStep);
    if (rc != LBM_OK) return rc;
    h->t = t0 + n;
    // The diagnostics refer to the last step's input, which the other buffer
    // holds until the next step; lbm_diagnostics reduces them when asked.
    h->t_diag = h->t - 1;
    h->diag_pending = true;
    h->diag_cache_valid = false;
    return LBM_OK;
}

int lbm_prepare_steps(lbm_ctx* h, int n) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (n < 0) return fail(LBM_ERR_ARG, "n must be >= 0");
    if (!h->bound) return fail(LBM_ERR_STATE, "lbm_bind first");
    if (!h->use_graphs) return LBM_OK;
    int left = n;
    while (left >= 2) {
        const int len = left >= kGraphChunk ? kGraphChunk : (left & ~1);
        hipGraphExec_t ex;
        int rc = graph_for(h, len, &ex);
        if (rc != LBM_OK) return rc;
        left -= len;
    }
    return LBM_OK;
}

int lbm_moments(lbm_ctx* h, double* rho, double* u, double* mu) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (!h->inited) return fail(LBM_ERR_STATE, "lbm_init or lbm_set_f first");
    StepArgs a = base_args(h);
    a.src = h->buf[h->cur];
    a.dst = nullptr;
    a.rho_out = rho;
    a.u_out = u;
    a.mu_out = mu;
    HIP_TRY(launch_step(h, a, kFields, h->stream));
    h->t_diag = h->t;
    h->diag_pending = false;
    h->diag_cache_valid = false;
    return LBM_OK;
}

// The read-out of the last step's input (the other buffer) into the per-tile
// partials, if lbm_step left it to be done; enqueued with the lattice records the
// steps used.
static int reduce_pending_diag(lbm_ctx* h) {
    if (!h->diag_pending) return LBM_OK;
    StepArgs a = base_args(h);
    a.src = h->buf[h->cur ^ 1];
    HIP_TRY(launch_step(h, a, kFields, h->stream));
    h->diag_pending = false;
    return LBM_OK;
}

int lbm_diagnostics(lbm_ctx* h, lbm_diag* out) {
    if (!h || !out) return fail(LBM_ERR_ARG, "null argument");
    if (!h->inited || h->t_diag < 0) return fail(LBM_ERR_STATE, "no diagnostics yet (step or moments first)");
    const int n = (int)h->recs.size();
    std::vector<DiagOut> tmp(n);
    if (h->diag_cache_valid) {
        tmp = h->diag_cache;
    } else {
        if (int rc0 = reduce_pending_diag(h); rc0 != LBM_OK) return rc0;
        HIP_TRY(launch_finalize(h->d_partial(), h->d_recs(), h->d_status(), h->d_diag(), n, h->stream));
        HIP_TRY(hipMemcpyAsync(tmp.data(), h->d_diag(), n * sizeof(DiagOut), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        // Lattices newly reported blown up leave the plan.  Their state is copied
        // into the other buffer so that it stays as it is (the ping-pong buffers
        // would otherwise alternate between two time levels), and the sums are
        // kept on the host: a new plan renumbers the per-tile partials.
        bool fresh = false;
        const size_t word = h->precision == LBM_FP64 ? 8 : 4;
        for (int i = 0; i < n; ++i) {
            if (!tmp[i].status || h->dropped[i]) continue;
            h->dropped[i] = fresh = true;
            h->frozen_diag[i] = tmp[i];
            h->frozen_step[i] = h->t_diag;
            const LatticeRec& R = h->recs[i];
            const size_t off = (size_t)R.state_offset * h->Q * word;
            const size_t len = (size_t)((R.nnodes + 63) / 64 * 64) * h->Q * word;
            HIP_TRY(hipMemcpyAsync(static_cast<char*>(h->buf[h->cur ^ 1]) + off,
                                   static_cast<const char*>(h->buf[h->cur]) + off, len, hipMemcpyDeviceToDevice,
                                   h->stream));
        }
        if (fresh) {
            h->diag_cache = tmp;
            h->diag_cache_valid = true;
            if (int rc0 = replan(h); rc0 != LBM_OK) return rc0;
        }
    }
    int rc = LBM_OK;
    for (int i = 0; i < n; ++i) {
        // a lattice out of the plan has no tiles: it reports what it had when it left
        const DiagOut& d = h->dropped[i] ? h->frozen_diag[i] : tmp[i];
        out[i].mass = d.mass;
        out[i].mom[0] = d.momx;
        out[i].mom[1] = d.momy;
        out[i].mom[2] = d.momz;
        out[i].max_u = d.umax;
        out[i].mu_min = d.mumin;
        out[i].mu_max = d.mumax;
        out[i].step = h->dropped[i] ? h->frozen_step[i] : h->t_diag;
        out[i].status = (int)(d.status | tmp[i].status);
        out[i].reserved = 0;
        if (out[i].status) rc = LBM_ERR_BLOWUP;
    }
    if (rc != LBM_OK) fail(rc, "at least one lattice has its blow-up flags set");
    return rc;
}

int lbm_get_f(lbm_ctx* h, double* f) {
    if (!h || !f) return fail(LBM_ERR_ARG, "null argument");
    if (!h->inited) return fail(LBM_ERR_STATE, "no state");
    if (h->lattice == LBM_D2Q9)
        HIP_TRY(d2q9_launch_convert(h->buf[h->cur], h->d_recs(), (int)h->recs.size(), f, h->field_total, h->stream,
                                    h->precision, true));
    else
        HIP_TRY(d3q19_launch_convert(h->buf[h->cur], h->d_recs(), (int)h->recs.size(), f, h->field_total, h->stream,
                                     h->precision, true));
    return LBM_OK;
}

int lbm_set_f(lbm_ctx* h, const double* f) {
    if (!h || !f) return fail(LBM_ERR_ARG, "null argument");
    if (!h->bound) return fail(LBM_ERR_STATE, "lbm_bind first");
    if (h->lattice == LBM_D2Q9)
        HIP_TRY(d2q9_launch_convert(h->buf[h->cur], h->d_recs(), (int)h->recs.size(), const_cast<double*>(f),
                                    h->field_total, h->stream, h->precision, false));
    else
        HIP_TRY(d3q19_launch_convert(h->buf[h->cur], h->d_recs(), (int)h->recs.size(), const_cast<double*>(f),
                                     h->field_total, h->stream, h->precision, false));
    if (int rc0 = reset_status(h); rc0 != LBM_OK) return rc0;
    h->inited = true;
    h->t_diag = -1;
    h->diag_pending = false;
    return LBM_OK;
}

int lbm_get_state(lbm_ctx* h, void* dst, long long* step) {
    if (!h || !dst) return fail(LBM_ERR_ARG, "null argument");
    if (!h->inited) return fail(LBM_ERR_STATE, "no state");
    HIP_TRY(hipMemcpyAsync(dst, h->buf[h->cur], h->state_bytes, hipMemcpyDeviceToDevice, h->stream));
    if (step) *step = h->t;
    return LBM_OK;
}

int lbm_set_state(lbm_ctx* h, const void* src, long long step) {
    if (!h || !src) return fail(LBM_ERR_ARG, "null argument");
    if (!h->bound) return fail(LBM_ERR_STATE, "lbm_bind first");
    HIP_TRY(hipMemcpyAsync(h->buf[h->cur], src, h->state_bytes, hipMemcpyDeviceToDevice, h->stream));
    if (int rc0 = reset_status(h); rc0 != LBM_OK) return rc0;
    h->t = step;
    h->t_diag = -1;
    h->diag_pending = false;
    h->inited = true;
    return LBM_OK;
}

int lbm_maxwell(int eos, double a, double b, double R, double T_over_Tc, double* rho_g, double* rho_l,
                double* mu_sat, double* p_sat) {
    if (eos != LBM_EOS_VDW && eos != LBM_EOS_CS) return fail(LBM_ERR_ARG, "bad eos");
    const int rc = host::maxwell(eos, a, b, R, T_over_Tc, rho_g, rho_l, mu_sat, p_sat);
    if (rc == -1) return fail(LBM_ERR_ARG, "EOS constants and T_over_Tc must be positive");
    if (rc != 0) return fail(LBM_ERR_DOMAIN, "no liquid-gas coexistence at this temperature");
    return LBM_OK;
}

double lbm_critical_temperature(int eos, double a, double b, double R) {
    return host::critical_temperature(eos, a, b, R);
}

int lbm_num_tile_shapes(const lbm_ctx* h) { return h ? h->num_shapes() : 0; }
int lbm_get_tile_shape(const lbm_ctx* h) { return h ? h->shape : -1; }

int lbm_describe_tile_shape(const lbm_ctx* h, int s, int* bx, int* by, int* bz) {
    if (!h || s < 0 || s >= h->num_shapes()) return fail(LBM_ERR_ARG, "bad shape index");
    int x, y;
    h->shape_dims(s, x, y);
    if (bx) *bx = x;
    if (by) *by = y;
    if (bz) *bz = h->lattice == LBM_D2Q9 ? kD2Q9NodesPerThread[s] : h->zchunk_for(s);
    return LBM_OK;
}

int lbm_set_tile_shape(lbm_ctx* h, int s) {
    if (!h || s < 0 || s >= h->num_shapes()) return fail(LBM_ERR_ARG, "bad shape index");
    {
        int bx, by;
        h->shape_dims(s, bx, by);
        if (h->lattice == LBM_D3Q19 && h->precision == LBM_FP64 && bx * by > 256)
            return fail(LBM_ERR_UNSUPPORTED, "this D3Q19 tile shape needs more LDS than float64 allows");
        if (h->lattice == LBM_D2Q9 && h->precision == LBM_FP64 && bx * by > 1024)
            return fail(LBM_ERR_UNSUPPORTED, "this D2Q9 tile shape (two nodes per thread) is float32 only");
    }
    std::vector<LatticeRec> rr = h->recs;
    std::vector<Tile> tt = h->plan(s, rr);
    if ((int)tt.size() > h->max_tiles) return fail(LBM_ERR_UNSUPPORTED, "tile list does not fit the workspace");
    if (h->bound) HIP_TRY(hipStreamSynchronize(h->stream));
    h->recs = rr;
    h->tiles = tt;
    h->shape = s;
    h->drop_graphs();
    if (h->bound) return upload_tables(h);
    return LBM_OK;
}

int lbm_set_zchunk(lbm_ctx* h, int bz) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (h->lattice != LBM_D3Q19) return bz == 0 ? LBM_OK : fail(LBM_ERR_UNSUPPORTED, "z-chunks are D3Q19 only");
    if (bz != 0 && bz < kMinZChunk) return fail(LBM_ERR_ARG, "a fixed z-chunk must be 0 (automatic) or >= 16");
    const int old = h->zchunk_fixed;
    h->zchunk_fixed = bz;
    const int rc = lbm_set_tile_shape(h, h->shape);      // re-plan with the new chunk length
    if (rc != LBM_OK) h->zchunk_fixed = old;
    return rc;
}

int lbm_get_zchunk(const lbm_ctx* h) { return h ? h->zchunk_fixed : -1; }

int lbm_set_store_mode(lbm_ctx* h, int mode) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (mode != LBM_STORES_STREAMING && mode != LBM_STORES_DEVICE) return fail(LBM_ERR_ARG, "bad store mode");
    if (mode != h->store_mode) {
        h->store_mode = mode;
        h->drop_graphs();             // the captured launches carry the old mode
    }
    return LBM_OK;
}

int lbm_get_store_mode(const lbm_ctx* h) { return h ? h->store_mode : -1; }

int lbm_set_use_graphs(lbm_ctx* h, int on) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    h->use_graphs = on != 0;
    return LBM_OK;
}

int lbm_autotune(lbm_ctx* h, int steps, void* scratch) {
    if (!h || !scratch || steps < 1) return fail(LBM_ERR_ARG, "bad argument");
    if (!h->inited) return fail(LBM_ERR_STATE, "lbm_init first");
    long long t0;
    int rc = lbm_get_state(h, scratch, &t0);
    if (rc != LBM_OK) return rc;
    const int cur0 = h->cur;
    // the trial steps may flag lattices: the flags are restored with the state
    std::vector<unsigned> st0(h->recs.size());
    HIP_TRY(hipMemcpyAsync(st0.data(), h->d_status(), st0.size() * sizeof(unsigned), hipMemcpyDeviceToHost,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    int best = h->shape, best_mode = h->store_mode;
    float best_ms = 1e30f;
    const int modes[2] = {LBM_STORES_STREAMING, LBM_STORES_DEVICE};
    for (int s = 0; s < h->num_shapes() && rc == LBM_OK; ++s) {
        rc = lbm_set_tile_shape(h, s);
        if (rc == LBM_ERR_UNSUPPORTED) {       // a shape this lattice or precision does not offer
            rc = LBM_OK;
            continue;
        }
        for (const int m : modes) {
            if (rc != LBM_OK) break;
            rc = lbm_set_store_mode(h, m);
            if (rc != LBM_OK) break;
            float ms_min = 1e30f;
            for (int rep = 0; rep < 2 && rc == LBM_OK; ++rep) {     // best of two: short trials are noisy
                rc = lbm_step(h, 2);                 // warm-up and graph capture
                if (rc != LBM_OK) break;
                HIP_TRY(hipEventRecord(e0, h->stream));
                rc = lbm_step(h, steps);
                if (rc != LBM_OK) break;
                HIP_TRY(hipEventRecord(e1, h->stream));
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                ms_min = std::min(ms_min, ms);
                h->cur = cur0;
                HIP_TRY(hipMemcpyAsync(h->buf[h->cur], scratch, h->state_bytes, hipMemcpyDeviceToDevice,
                                       h->stream));
                // every trial starts from the same flags, so a lattice flagged in
                // one trial is not skipped (less work) in the next
                HIP_TRY(hipMemcpyAsync(h->d_status(), st0.data(), st0.size() * sizeof(unsigned),
                                       hipMemcpyHostToDevice, h->stream));
                HIP_TRY(hipStreamSynchronize(h->stream));
                h->t = t0;
            }
            if (rc == LBM_OK && ms_min < best_ms) {
                best_ms = ms_min;
                best = s;
                best_mode = m;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != LBM_OK) return rc;
    rc = lbm_set_tile_shape(h, best);
    if (rc != LBM_OK) return rc;
    rc = lbm_set_store_mode(h, best_mode);
    if (rc != LBM_OK) return rc;
    HIP_TRY(hipMemcpyAsync(h->d_status(), st0.data(), st0.size() * sizeof(unsigned), hipMemcpyHostToDevice,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->t_diag = -1;
    h->diag_pending = false;
    h->diag_cache_valid = false;
    return best;
}

int lbm_set_physics(lbm_ctx* h, int i, double kappa, double T_over_Tc) {
    if (!h || i < 0 || i >= (int)h->recs.size()) return fail(LBM_ERR_ARG, "bad handle or lattice index");
    if (!(kappa >= 0) || !(T_over_Tc > 0)) return fail(LBM_ERR_ARG, "kappa >= 0 and T_over_Tc > 0 required");
    // diagnostics still owed for the last step are reduced with the physics it used
    if (h->bound) {
        if (int rc0 = reduce_pending_diag(h); rc0 != LBM_OK) return rc0;
    }
    lbm_params& p = h->params[i];
    p.kappa = kappa;
    p.T_over_Tc = T_over_Tc;
    LatticeRec& R = h->recs[i];
    R.kappa = kappa;
    R.RT = p.R * T_over_Tc * host::critical_temperature(p.eos, p.a, p.b, p.R);
    set_dev_constants(R, p.R);
    // The adjoint kernels take the lattice record by value, so captured segment
    // graphs hold the old kappa and RT: drop every captured graph.
    h->drop_graphs();
    if (h->bound) {
        HIP_TRY(hipStreamSynchronize(h->stream));
        return upload_tables(h);
    }
    return LBM_OK;
}

namespace {
int adjoint_check(lbm_ctx* h) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (h->lattice != LBM_D2Q9 || h->recs.size() != 1 || h->variant == kStdPtensor || h->recs[0].mrt ||
        h->recs[0].walls)
        return fail(LBM_ERR_UNSUPPORTED,
                    "the adjoint is implemented for one D2Q9 BGK lattice, improved or chemical-potential standard "
                    "scheme");
    if (!h->bound) return fail(LBM_ERR_STATE, "lbm_bind first");
    return LBM_OK;
}
double adjoint_dRT(const lbm_ctx* h) {
    const lbm_params& p = h->params[0];
    return p.R * host::critical_temperature(p.eos, p.a, p.b, p.R);
}
}  // namespace

size_t lbm_adjoint_workspace_bytes(const lbm_ctx* h) {
    if (!h || h->lattice != LBM_D2Q9 || h->recs.size() != 1 || h->recs[0].mrt || h->recs[0].walls) return 0;
    return align256(adjoint_workspace_doubles(h->recs[0].nx, h->recs[0].ny) * sizeof(double));
}

int lbm_adjoint_step(lbm_ctx* h, const void* state_t, const double* lam_next, double* lam_out, void* ws,
                     double* grad) {
    int rc = adjoint_check(h);
    if (rc != LBM_OK) return rc;
    if (!state_t || !lam_next || !lam_out || !ws || !grad) return fail(LBM_ERR_ARG, "null argument");
    if (lam_next == lam_out) return fail(LBM_ERR_ARG, "lam_next and lam_out must not alias");
    HIP_TRY(adjoint_launch(0, h->recs[0], adjoint_dRT(h), h->precision, h->variant == kImproved, state_t, lam_next,
                           lam_out, nullptr, nullptr, nullptr, nullptr, reinterpret_cast<double*>(ws), grad,
                           h->stream, 0));
    return LBM_OK;
}

int lbm_adjoint_step_noalloc(lbm_ctx* h, const void* state_t, const double* lam_next, double* lam_out,
                             double* grad) {
    int rc = adjoint_check(h);
    if (rc != LBM_OK) return rc;
    if (!state_t || !lam_next || !lam_out || !grad) return fail(LBM_ERR_ARG, "null argument");
    if (lam_next == lam_out) return fail(LBM_ERR_ARG, "lam_next and lam_out must not alias");
    const size_t need = adjoint_workspace_doubles(h->recs[0].nx, h->recs[0].ny) * sizeof(double);
    if (need > static_scratch_bytes())
        return fail(LBM_ERR_UNSUPPORTED, "this lattice's adjoint workspace (" + std::to_string(need) +
                                             " bytes) exceeds the static scratch of " +
                                             std::to_string(static_scratch_bytes()) + " bytes");
    void* ws = nullptr;
    HIP_TRY(static_scratch(&ws));
    HIP_TRY(adjoint_launch(0, h->recs[0], adjoint_dRT(h), h->precision, h->variant == kImproved, state_t, lam_next,
                           lam_out, nullptr, nullptr, nullptr, nullptr, reinterpret_cast<double*>(ws), grad,
                           h->stream, 0));
    return LBM_OK;
}

size_t lbm_adjoint_noalloc_max_bytes(void) { return static_scratch_bytes(); }

namespace {

// The work of one adjoint segment after its checkpoint has been restored: the
// recompute of states t0 .. t0 + m - 1 (each kept in `states`) and the adjoint
// steps back through them.  Leaves h->cur as the recompute leaves it.
// The adjoint steps of a segment over its states (slots m-1 down to 0 of `states`):
// on entry lam holds dL/df(t0+m), on exit dL/df(t0).
int enqueue_adjoint_steps(lbm_ctx* h, int m, void* states, double* lam, double* lam2, void* ws, double* grad,
                          hipStream_t s) {
    char* st = reinterpret_cast<char*>(states);
    double* in = lam;
    double* out = lam2;
    for (int k = m - 1; k >= 0; --k) {
        HIP_TRY(adjoint_launch(0, h->recs[0], adjoint_dRT(h), h->precision, h->variant == kImproved,
                               st + (size_t)k * h->state_bytes, in, out, nullptr, nullptr, nullptr, nullptr,
                               reinterpret_cast<double*>(ws), grad, s,
                               (k < m - 1 ? kAdjPending : 0) | (k > 0 ? kAdjDeferReduce : 0)));
        std::swap(in, out);
    }
    if (in != lam) HIP_TRY(launch_copy(lam, in, (size_t)9 * h->recs[0].nnodes * sizeof(double), s));
    return LBM_OK;
}

int enqueue_segment(lbm_ctx* h, int m, void* states, double* lam, double* lam2, void* ws, double* grad,
                    hipStream_t s) {
    // slot 0 holds the checkpoint; each recompute step writes the next slot, the
    // last one the handle's current buffer (the handle ends at t0 + m)
    char* st = reinterpret_cast<char*>(states);
    for (int k = 0; k < m; ++k) {
        StepArgs a = base_args(h);
        a.src = st + (size_t)k * h->state_bytes;
        a.dst = k + 1 < m ? static_cast<void*>(st + (size_t)(k + 1) * h->state_bytes) : h->buf[h->cur];
        HIP_TRY(launch_step(h, a, kStep, s));
    }
    return enqueue_adjoint_steps(h, m, states, lam, lam2, ws, grad, s);
}

// The states a segment's adjoint steps need: slot 0 holds the checkpoint (time
// level t0), slots 1 .. m-1 receive t0+1 .. t0+m-1.
int enqueue_recompute(lbm_ctx* h, int m, void* states, hipStream_t s) {
    char* st = reinterpret_cast<char*>(states);
    for (int k = 0; k + 1 < m; ++k) {
        StepArgs a = base_args(h);
        a.src = st + (size_t)k * h->state_bytes;
        a.dst = st + (size_t)(k + 1) * h->state_bytes;
        HIP_TRY(launch_step(h, a, kStep, s));
    }
    return LBM_OK;
}


// A segment's launches captured once and replayed (keyed by the buffers, so a
// caller that keeps its buffers replays one graph per segment).
int segment_graph(lbm_ctx* h, int m, void* states, double* lam, double* lam2, void* ws, double* grad,
                  hipGraphExec_t* out) {
    const lbm_ctx::SegKey key{m, h->cur, states, lam, lam2, ws, grad};
    auto it = h->seg_graphs.find(key);
    if (it != h->seg_graphs.end()) {
        *out = it->second;
        return LBM_OK;
    }
    if (h->seg_graphs.size() >= 8) {           // callers with fresh buffers every time: keep a few
        for (auto& kv : h->seg_graphs) (void)hipGraphExecDestroy(kv.second);
        h->seg_graphs.clear();
    }
    if (!h->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    const int saved = h->cur;
    HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_segment(h, m, states, lam, lam2, ws, grad, h->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
    h->cur = saved;
    if (rc != LBM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(LBM_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    h->seg_graphs[key] = ex;
    *out = ex;
    return LBM_OK;
}

}  // namespace

int lbm_adjoint_segment(lbm_ctx* h, const void* checkpoint, long long t0, int m, void* states, double* lam,
                        double* lam2, void* ws, double* grad) {
    int rc = adjoint_check(h);
    if (rc != LBM_OK) return rc;
    if (!checkpoint || !states || !lam || !lam2 || !ws || !grad) return fail(LBM_ERR_ARG, "null argument");
    if (m < 1) return fail(LBM_ERR_ARG, "m must be >= 1");
    if (lam == lam2) return fail(LBM_ERR_ARG, "lam and lam2 must not alias");
    if (((uintptr_t)states | (uintptr_t)lam | (uintptr_t)lam2 | (uintptr_t)checkpoint) & 15)
        return fail(LBM_ERR_ARG, "checkpoint, states, lam and lam2 must be 16-byte aligned");
    rc = reset_status(h);
    if (rc != LBM_OK) return rc;
    HIP_TRY(launch_copy(states, checkpoint, h->state_bytes, h->stream));
    if (h->use_graphs) {
        hipGraphExec_t ex = nullptr;
        rc = segment_graph(h, m, states, lam, lam2, ws, grad, &ex);
        if (rc != LBM_OK) return rc;
        HIP_TRY(hipGraphLaunch(ex, h->stream));
    } else {
        rc = enqueue_segment(h, m, states, lam, lam2, ws, grad, h->stream);
        if (rc != LBM_OK) return rc;
    }
    h->t = t0 + m;
    h->t_diag = -1;
    h->diag_pending = false;
    h->inited = true;
    return LBM_OK;
}

int lbm_adjoint_sweep(lbm_ctx* h, const void* const* checkpoints, const long long* t0, const int* m, int nseg,
                      void* states, double* lam, double* lam2, void* ws, double* grad) {
    int rc = adjoint_check(h);
    if (rc != LBM_OK) return rc;
    if (!checkpoints || !t0 || !m || !states || !lam || !lam2 || !ws || !grad) return fail(LBM_ERR_ARG, "null argument");
    if (nseg < 1) return fail(LBM_ERR_ARG, "nseg must be >= 1");
    if (lam == lam2) return fail(LBM_ERR_ARG, "lam and lam2 must not alias");
    if (((uintptr_t)states | (uintptr_t)lam | (uintptr_t)lam2) & 15)
        return fail(LBM_ERR_ARG, "states, lam and lam2 must be 16-byte aligned");
    int kmax = 0;
    for (int i = 0; i < nseg; ++i) {
        if (!checkpoints[i] || ((uintptr_t)checkpoints[i] & 15))
            return fail(LBM_ERR_ARG, "every checkpoint must be a 16-byte aligned device pointer");
        if (m[i] < 1) return fail(LBM_ERR_ARG, "every segment needs m >= 1");
        if (i > 0 && t0[i] != t0[i - 1] + m[i - 1]) return fail(LBM_ERR_ARG, "segments must be consecutive");
        kmax = std::max(kmax, m[i]);
    }
    rc = reset_status(h);
    if (rc != LBM_OK) return rc;
    if (!h->side_stream) HIP_TRY(hipStreamCreateWithFlags(&h->side_stream, hipStreamNonBlocking));
    for (hipEvent_t& e : h->ev)
        if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    hipStream_t A = h->stream, B = h->side_stream;
    hipEvent_t entry = h->ev[0], rdone[2] = {h->ev[1], h->ev[2]}, adone[2] = {h->ev[3], h->ev[4]};
    char* arena[2] = {reinterpret_cast<char*>(states), reinterpret_cast<char*>(states) + (size_t)kmax * h->state_bytes};
    // segment i recomputes into arena i % 2 on B; its adjoint steps run on A
    auto recompute = [&](int i) -> int {
        char* st = arena[i % 2];
        HIP_TRY(launch_copy(st, checkpoints[i], h->state_bytes, B));
        if (m[i] < 2) return LBM_OK;
        if (h->use_graphs) {
            hipGraphExec_t ex = nullptr;
            const lbm_ctx::SegKey key{0, m[i], st, nullptr, nullptr, nullptr, nullptr};
            int r = cached_graph(h, h->sweep_graphs, key,
                                 [&](hipStream_t s) { return enqueue_recompute(h, m[i], st, s); }, &ex);
            if (r != LBM_OK) return r;
            HIP_TRY(hipGraphLaunch(ex, B));
            return LBM_OK;
        }
        return enqueue_recompute(h, m[i], st, B);
    };
    auto backward = [&](int i) -> int {
        char* st = arena[i % 2];
        if (h->use_graphs) {
            hipGraphExec_t ex = nullptr;
            const lbm_ctx::SegKey key{1, m[i], st, lam, lam2, ws, grad};
            int r = cached_graph(
                h, h->sweep_graphs, key,
                [&](hipStream_t s) { return enqueue_adjoint_steps(h, m[i], st, lam, lam2, ws, grad, s); }, &ex);
            if (r != LBM_OK) return r;
            HIP_TRY(hipGraphLaunch(ex, A));
            return LBM_OK;
        }
        return enqueue_adjoint_steps(h, m[i], st, lam, lam2, ws, grad, A);
    };
    // B starts after everything already queued on A (the checkpoints, lam)
    HIP_TRY(hipEventRecord(entry, A));
    HIP_TRY(hipStreamWaitEvent(B, entry, 0));
    rc = recompute(nseg - 1);
    if (rc != LBM_OK) return rc;
    HIP_TRY(hipEventRecord(rdone[(nseg - 1) % 2], B));
    for (int i = nseg - 1; i >= 0; --i) {
        HIP_TRY(hipStreamWaitEvent(A, rdone[i % 2], 0));
        if (i > 0) {
            // segment i-1 reuses the arena of segment i+1, whose adjoint steps must be done
            if (i + 1 < nseg) HIP_TRY(hipStreamWaitEvent(B, adone[(i + 1) % 2], 0));
            rc = recompute(i - 1);
            if (rc != LBM_OK) return rc;
            HIP_TRY(hipEventRecord(rdone[(i - 1) % 2], B));
        }
        rc = backward(i);
        if (rc != LBM_OK) return rc;
        HIP_TRY(hipEventRecord(adone[i % 2], A));
    }
    h->diag_cache_valid = false;
    h->t_diag = -1;
    h->diag_pending = false;
    return LBM_OK;
}

int lbm_adjoint_fields(lbm_ctx* h, const void* state_t, const double* rho_bar, const double* u_bar, double* lam_out,
                       void* ws, double* grad) {
    int rc = adjoint_check(h);
    if (rc != LBM_OK) return rc;
    if (!state_t || !lam_out || !ws || !grad) return fail(LBM_ERR_ARG, "null argument");
    HIP_TRY(adjoint_launch(1, h->recs[0], adjoint_dRT(h), h->precision, h->variant == kImproved, state_t, nullptr,
                           lam_out, rho_bar, u_bar, nullptr, nullptr, reinterpret_cast<double*>(ws), grad,
                           h->stream, 0));
    return LBM_OK;
}

int lbm_adjoint_init(lbm_ctx* h, const double* rho0, const double* lam0, double* grad_rho0, void* ws,
                     double* grad) {
    int rc = adjoint_check(h);
    if (rc != LBM_OK) return rc;
    if (!rho0 || !lam0 || !grad_rho0 || !ws || !grad) return fail(LBM_ERR_ARG, "null argument");
    HIP_TRY(adjoint_launch(2, h->recs[0], adjoint_dRT(h), h->precision, h->variant == kImproved, nullptr, lam0,
                           nullptr, nullptr, nullptr, rho0, grad_rho0, reinterpret_cast<double*>(ws), grad,
                           h->stream, 0));
    return LBM_OK;
}

int lbm_copy_kernel(void* dst, const void* src, size_t bytes, void* hip_stream) {
    if (!dst || !src) return fail(LBM_ERR_ARG, "null argument");
    if (((uintptr_t)dst | (uintptr_t)src) & 15) return fail(LBM_ERR_ARG, "buffers must be 16-byte aligned");
    HIP_TRY(launch_copy(dst, src, bytes, reinterpret_cast<hipStream_t>(hip_stream)));
    return LBM_OK;
}

void lbm_destroy(lbm_ctx* h) {
    if (!h) return;
    h->drop_graphs();
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->side_stream) (void)hipStreamDestroy(h->side_stream);
    for (hipEvent_t e : h->ev)
        if (e) (void)hipEventDestroy(e);
    delete h;
}

}  // extern "C"
