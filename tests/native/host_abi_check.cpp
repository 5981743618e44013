// Host-side checks of the C ABI for a sanitizer build (AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code): parameter checking, planning,
// size queries, tile and chunk selection, store modes, the Maxwell construction
// and every error path that needs no GPU.  Exits non-zero on the first mismatch.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/lbm.h"

static int failures = 0;
#define CHECK(cond)                                                                  \
    do {                                                                             \
        if (!(cond)) {                                                               \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                              \
        }                                                                            \
    } while (0)

static lbm_params base(int lattice, int nx, int ny, int nz) {
    lbm_params p;
    std::memset(&p, 0, sizeof(p));
    p.lattice = lattice;
    p.nx = nx;
    p.ny = ny;
    p.nz = nz;
    p.eos = LBM_EOS_VDW;
    p.a = 9.0 / 392.0;
    p.b = 2.0 / 21.0;
    p.R = 1.0;
    p.T_over_Tc = 0.8;
    p.kappa = 0.02;
    p.tau = 1.0;
    p.scheme = LBM_IMPROVED;
    return p;
}

int main() {
    // Maxwell construction: Table II's analytical column (vdW, T/Tc = 0.8) and the domain check
    double rg, rl, mu, ps;
    CHECK(lbm_maxwell(LBM_EOS_VDW, 9.0 / 392.0, 2.0 / 21.0, 1.0, 0.8, &rg, &rl, &mu, &ps) == LBM_OK);
    CHECK(std::fabs(rg - 0.83883) < 1e-5 && std::fabs(rl - 6.76447) < 1e-5 && std::fabs(mu - 0.018302) < 1e-6);
    CHECK(lbm_maxwell(LBM_EOS_VDW, 9.0 / 392.0, 2.0 / 21.0, 1.0, 1.2, &rg, &rl, &mu, &ps) == LBM_ERR_DOMAIN);
    CHECK(lbm_maxwell(LBM_EOS_VDW, -1.0, 2.0 / 21.0, 1.0, 0.8, &rg, &rl, &mu, &ps) == LBM_ERR_ARG);
    CHECK(lbm_maxwell(7, 1.0, 1.0, 1.0, 0.8, &rg, &rl, &mu, &ps) == LBM_ERR_ARG);
    for (double t = 0.5; t < 0.99; t += 0.05) {
        CHECK(lbm_maxwell(LBM_EOS_CS, 0.0282217394824, 0.149078724791, 1.0, t, &rg, &rl, &mu, &ps) == LBM_OK);
        CHECK(rg > 0 && rl > rg);
    }
    CHECK(std::fabs(lbm_critical_temperature(LBM_EOS_VDW, 9.0 / 392.0, 2.0 / 21.0, 1.0) - 1.0 / 14.0) < 1e-15);

    // parameter checks
    lbm_ctx* h = nullptr;
    lbm_params p = base(LBM_D2Q9, 32, 24, 1);
    CHECK(lbm_create(&p, nullptr, &h) == LBM_OK && h);
    CHECK(lbm_state_bytes(h) % 256 == 0 && lbm_state_bytes(h) >= 9 * 8 * 32 * 24);
    CHECK(lbm_workspace_bytes(h) > 0);
    CHECK(lbm_num_nodes(h) == 32 * 24 && lbm_count(h) == 1 && lbm_node_offset(h, 0) == 0);
    CHECK(lbm_node_offset(h, 1) == -1);
    for (int s = 0; s < lbm_num_tile_shapes(h); ++s) {
        int bx = 0, by = 0, bz = 0;
        // D2Q9: bz > 0 nodes per thread, or -2 for two threads per node
        CHECK(lbm_describe_tile_shape(h, s, &bx, &by, &bz) == LBM_OK && bx > 0 && by > 0 && (bz > 0 || bz == -2));
        const int rc = lbm_set_tile_shape(h, s);       // unbound: plans only
        CHECK(rc == LBM_OK || rc == LBM_ERR_UNSUPPORTED);
    }
    CHECK(lbm_set_tile_shape(h, -1) == LBM_ERR_ARG);
    CHECK(lbm_set_zchunk(h, 0) == LBM_OK && lbm_set_zchunk(h, 32) == LBM_ERR_UNSUPPORTED);
    CHECK(lbm_set_store_mode(h, LBM_STORES_DEVICE) == LBM_OK && lbm_get_store_mode(h) == LBM_STORES_DEVICE);
    CHECK(lbm_set_store_mode(h, 9) == LBM_ERR_ARG);
    CHECK(lbm_step(h, 1) == LBM_ERR_STATE);              // not bound, not initialised
    CHECK(lbm_step(h, -1) == LBM_ERR_ARG);
    CHECK(lbm_init(h, nullptr, nullptr) == LBM_ERR_ARG);
    lbm_diag d;
    CHECK(lbm_diagnostics(h, &d) == LBM_ERR_STATE);
    CHECK(lbm_set_physics(h, 0, 0.03, 0.85) == LBM_OK);
    CHECK(lbm_set_physics(h, 1, 0.03, 0.85) == LBM_ERR_ARG);
    CHECK(lbm_adjoint_workspace_bytes(h) > 0);
    CHECK(lbm_adjoint_noalloc_max_bytes() == (size_t(24) << 20));
    CHECK(std::strlen(lbm_error_string(LBM_ERR_BLOWUP)) > 0 && std::strlen(lbm_error_string(-99)) > 0);
    lbm_destroy(h);

    // every invalid field is refused, with a message
    struct Bad { const char* what; void (*edit)(lbm_params&); int code; };
    const Bad bad[] = {
        {"lattice", [](lbm_params& q) { q.lattice = 5; }, LBM_ERR_ARG},
        {"nx", [](lbm_params& q) { q.nx = 0; }, LBM_ERR_ARG},
        {"nz in 2D", [](lbm_params& q) { q.nz = 2; }, LBM_ERR_ARG},
        {"eos", [](lbm_params& q) { q.eos = 3; }, LBM_ERR_ARG},
        {"b", [](lbm_params& q) { q.b = 0; }, LBM_ERR_ARG},
        {"a", [](lbm_params& q) { q.a = 0; }, LBM_ERR_ARG},
        {"T", [](lbm_params& q) { q.T_over_Tc = -1; }, LBM_ERR_ARG},
        {"kappa", [](lbm_params& q) { q.kappa = -1; }, LBM_ERR_ARG},
        {"tau", [](lbm_params& q) { q.tau = 0.5; }, LBM_ERR_ARG},
        {"scheme", [](lbm_params& q) { q.scheme = 4; }, LBM_ERR_ARG},
        {"ptensor improved", [](lbm_params& q) { q.force_form = LBM_FORCE_PTENSOR; }, LBM_ERR_ARG},
        {"precision", [](lbm_params& q) { q.precision = 9; }, LBM_ERR_ARG},
        {"mrt rates", [](lbm_params& q) { q.collision = LBM_MRT; q.tau_e = 0.4; q.tau_s = 1; q.tau_q = 1; }, LBM_ERR_ARG},
        {"c0", [](lbm_params& q) { q.c0 = -1; }, LBM_ERR_ARG},
        {"walls", [](lbm_params& q) { q.walls = 2; }, LBM_ERR_ARG},
        {"population array beyond 4 GB", [](lbm_params& q) { q.nx = 1 << 15; q.ny = (1 << 14) + 1; },
         LBM_ERR_UNSUPPORTED},
    };
    for (const Bad& b : bad) {
        lbm_params q = base(LBM_D2Q9, 32, 24, 1);
        b.edit(q);
        lbm_ctx* hb = nullptr;
        const int rc = lbm_create(&q, nullptr, &hb);
        if (rc != b.code) std::fprintf(stderr, "%s: got %d\n", b.what, rc);
        CHECK(rc == b.code && hb == nullptr && std::strlen(lbm_last_error()) > 0);
    }

    // D3Q19 batch of unequal lattices: offsets, fixed z-chunks, refusals
    std::vector<lbm_params> batch = {base(LBM_D3Q19, 20, 18, 40), base(LBM_D3Q19, 70, 12, 260),
                                     base(LBM_D3Q19, 9, 9, 9)};
    batch[1].precision = LBM_FP32_DEV;
    CHECK(lbm_create_batch(batch.data(), 3, nullptr, &h) == LBM_ERR_ARG);     // mixed precision
    batch[1].precision = LBM_FP64;
    CHECK(lbm_create_batch(batch.data(), 3, nullptr, &h) == LBM_OK);
    CHECK(lbm_node_offset(h, 1) == 20 * 18 * 40 && lbm_node_offset(h, 2) == 20 * 18 * 40 + 70 * 12 * 260);
    for (int bz : {16, 32, 128, 0}) CHECK(lbm_set_zchunk(h, bz) == LBM_OK);
    CHECK(lbm_set_zchunk(h, 8) == LBM_ERR_ARG);
    for (int s = 0; s < lbm_num_tile_shapes(h); ++s) {
        const int rc = lbm_set_tile_shape(h, s);
        CHECK(rc == LBM_OK || rc == LBM_ERR_UNSUPPORTED);
    }
    CHECK(lbm_adjoint_workspace_bytes(h) == 0);
    lbm_destroy(h);
    lbm_destroy(nullptr);

    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("host ABI checks passed\n");
    return 0;
}
