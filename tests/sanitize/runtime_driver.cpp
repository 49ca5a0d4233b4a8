// Host-side paths of the C ABI under the host sanitizers (AddressSanitizer,
// UndefinedBehaviorSanitizer): parameter validation, workspace layout,
// context creation and destruction, launch-shape and mode checks, and the
// argument checks of every entry point.  Nothing here reaches a HIP call
// (each call is either host-only or rejected before its first HIP call), so
// the program needs no GPU.  Exit status 0 when every expectation holds.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>

#include "../../include/mrt_lbm.h"

static int g_fail = 0;
#define EXPECT(cond)                                                         \
    do {                                                                     \
        if (!(cond)) {                                                       \
            std::printf("FAILED line %d: %s (%s)\n", __LINE__, #cond, lbm_last_error()); \
            ++g_fail;                                                        \
        }                                                                    \
    } while (0)

static lbm_params base() {
    lbm_params p;
    lbm_params_default(&p);
    return p;
}

int main() {
    size_t b = 0;
    lbm_params p = base();
    EXPECT(lbm_workspace_bytes(&p, &b) == LBM_OK && b > 0);
    EXPECT(lbm_workspace_bytes(nullptr, &b) == LBM_ERR_INVALID_ARG);
    EXPECT(lbm_workspace_bytes(&p, nullptr) == LBM_ERR_INVALID_ARG);

    // Invalid parameters, one field at a time.
    const double nan = std::numeric_limits<double>::quiet_NaN();
    struct Bad {
        const char *name;
        void (*set)(lbm_params &);
        lbm_status want;
    } bad[] = {
        {"nx=0", [](lbm_params &q) { q.nx = 0; }, LBM_ERR_INVALID_ARG},
        {"ny<0", [](lbm_params &q) { q.ny = -3; }, LBM_ERR_INVALID_ARG},
        {"huge", [](lbm_params &q) { q.nx = q.ny = q.nz = 1 << 20; }, LBM_ERR_INVALID_ARG},
        {"wall_z=2", [](lbm_params &q) { q.wall_z = 2; }, LBM_ERR_INVALID_ARG},
        {"walls nz=1", [](lbm_params &q) { q.wall_z = 1; q.nz = 1; }, LBM_ERR_INVALID_ARG},
        {"op", [](lbm_params &q) { q.op = 7; }, LBM_ERR_INVALID_ARG},
        {"storage", [](lbm_params &q) { q.storage = 9; }, LBM_ERR_INVALID_ARG},
        {"psi_form", [](lbm_params &q) { q.psi_form = 5; }, LBM_ERR_INVALID_ARG},
        {"f16_exp", [](lbm_params &q) { q.f16_exp = 30; }, LBM_ERR_INVALID_ARG},
        {"s_nu=2", [](lbm_params &q) { q.s_nu = 2.0; }, LBM_ERR_INVALID_ARG},
        {"s_e nan", [](lbm_params &q) { q.s_e = std::numeric_limits<double>::quiet_NaN(); }, LBM_ERR_INVALID_ARG},
        {"G>0", [](lbm_params &q) { q.G = 0.5; }, LBM_ERR_INVALID_ARG},
        {"T<0", [](lbm_params &q) { q.T_over_Tc = -1.0; }, LBM_ERR_INVALID_ARG},
        {"theta=180", [](lbm_params &q) { q.theta_wall_deg = 180.0; }, LBM_ERR_INVALID_ARG},
        {"nu_ratio<0", [](lbm_params &q) { q.nu_ratio = -1.0; }, LBM_ERR_INVALID_ARG},
        {"visc range", [](lbm_params &q) { q.nu_ratio = 5.0; q.visc_rho_L = 0.1; q.visc_rho_V = 0.4; },
         LBM_ERR_INVALID_ARG},
        {"gravity inf", [](lbm_params &q) { q.gravity[2] = std::numeric_limits<double>::infinity(); },
         LBM_ERR_INVALID_ARG},
        {"diag_every<0", [](lbm_params &q) { q.diag_every = -1; }, LBM_ERR_INVALID_ARG},
        {"orth_meq=2", [](lbm_params &q) { q.orth_meq = 2; }, LBM_ERR_INVALID_ARG},
        {"orth_sigma<0", [](lbm_params &q) { q.orth_sigma = -1; }, LBM_ERR_INVALID_ARG},
        {"lid without wall", [](lbm_params &q) { q.lid_u[0] = 0.1; }, LBM_ERR_INVALID_ARG},
        {"x walls multiphase", [](lbm_params &q) { q.wall_x = 1; }, LBM_ERR_UNSUPPORTED},
        {"five planes > 4 GiB", [](lbm_params &q) { q.nx = q.ny = 1024; q.nz = 512; q.storage = LBM_STORE_F64; },
         LBM_ERR_UNSUPPORTED},
    };
    (void)nan;
    for (const Bad &x : bad) {
        lbm_params q = base();
        x.set(q);
        const lbm_status s = lbm_workspace_bytes(&q, &b);
        if (s != x.want) std::printf("case %s: got %d\n", x.name, s);
        EXPECT(s == x.want);
        EXPECT(std::strlen(lbm_last_error()) > 0);
    }

    // Contexts over a fake (never touched) aligned workspace, every storage,
    // operator and wall combination; mode and tile checks.
    alignas(256) static unsigned char fake[512];
    for (int st = 0; st < 3; ++st)
        for (int op = 0; op < 2; ++op)
            for (int w = 0; w < 2; ++w) {
                lbm_params q = base();
                q.storage = st;
                q.op = op;
                q.wall_z = w;
                q.nx = 68;
                q.ny = 37;
                q.nz = 21;
                q.rho_ref = 0.01;
                q.f16_exp = 10;
                size_t need = 0;
                EXPECT(lbm_workspace_bytes(&q, &need) == LBM_OK);
                lbm_ctx *c = nullptr;
                EXPECT(lbm_create(&q, fake, 16, nullptr, &c) == LBM_ERR_BUFFER_TOO_SMALL && c == nullptr);
                EXPECT(lbm_create(&q, fake + 8, need, nullptr, &c) == LBM_ERR_INVALID_ARG);
                EXPECT(lbm_create(&q, fake, need, nullptr, &c) == LBM_OK && c != nullptr);
                int32_t mode = -1, slab = -1;
                EXPECT(lbm_get_step_mode(c, &mode, &slab) == LBM_OK);
                EXPECT(mode == (st == LBM_STORE_F64 ? LBM_STEP_FUSED : LBM_STEP_SPLIT));
                for (int m = 0; m <= 4; ++m) {
                    const lbm_status s = lbm_set_step_mode(c, m, 8);
                    EXPECT(s == LBM_OK || s == LBM_ERR_UNSUPPORTED);
                    lbm_tile t{};
                    EXPECT(lbm_get_tile(c, &t) == LBM_OK);
                    EXPECT(lbm_set_tile(c, &t) == LBM_OK);  // the current tile is always valid
                }
                EXPECT(lbm_set_step_mode(c, 9, 8) == LBM_ERR_INVALID_ARG);
                EXPECT(lbm_set_step_mode(c, LBM_STEP_FUSED, 0) == LBM_ERR_INVALID_ARG);
                lbm_tile t{0, 4, 8, 0};
                EXPECT(lbm_set_tile(c, &t) == LBM_ERR_INVALID_ARG);
                t = {2048, 1, 8, 0};
                EXPECT(lbm_set_tile(c, &t) == LBM_ERR_INVALID_ARG);
                t = {64, 64, 8, 0};
                EXPECT(lbm_set_tile(c, &t) == LBM_ERR_INVALID_ARG);
                EXPECT(lbm_set_store_policy(c, 7) == LBM_ERR_INVALID_ARG);
                EXPECT(lbm_set_store_policy(c, LBM_STORE_STREAM) == LBM_OK);
                EXPECT(lbm_set_write_check(c, 1) == LBM_OK);
                EXPECT(lbm_set_graph_steps(c, -1) == LBM_ERR_INVALID_ARG);
                EXPECT(lbm_set_graph_steps(c, 4) == LBM_OK);
                EXPECT(lbm_set_timing(c, 0) == LBM_OK);
                EXPECT(lbm_step(c, -1) == LBM_ERR_INVALID_ARG);
                EXPECT(lbm_step(c, 0) == LBM_OK);
                EXPECT(lbm_step_count(c) == 0);
                size_t sb = 0;
                EXPECT(lbm_state_bytes(c, &sb) == LBM_OK && sb > 0);
                EXPECT(lbm_save_state(c, nullptr, sb) == LBM_ERR_INVALID_ARG);
                EXPECT(lbm_save_state(c, fake, 8) == LBM_ERR_BUFFER_TOO_SMALL);
                EXPECT(lbm_load_state(c, fake, 8) == LBM_ERR_BUFFER_TOO_SMALL);
                EXPECT(lbm_init_fields(c, nullptr, nullptr) == LBM_ERR_INVALID_ARG);
                lbm_droplet d{};
                EXPECT(lbm_init_droplets(c, &d, 0, 0.4, 0.01, 2.0) == LBM_ERR_INVALID_ARG);
                EXPECT(lbm_init_droplets(c, &d, 1, 0.4, 0.01, 0.0) == LBM_ERR_INVALID_ARG);
                EXPECT(lbm_read_populations(c, nullptr) == LBM_ERR_INVALID_ARG);
                EXPECT(lbm_write_populations(c, nullptr) == LBM_ERR_INVALID_ARG);
                EXPECT(lbm_diagnostics(c, nullptr, nullptr) == LBM_ERR_INVALID_ARG);
                lbm_diag_request rq{};
                rq.r_in = -1.0;
                lbm_diag out{};
                EXPECT(lbm_diagnostics(c, &rq, &out) == LBM_ERR_INVALID_ARG);
                EXPECT(lbm_autotune(c, 0, nullptr) == LBM_ERR_INVALID_ARG);
                EXPECT(lbm_destroy(c) == LBM_OK);
            }
    EXPECT(lbm_destroy(nullptr) == LBM_ERR_INVALID_ARG);
    EXPECT(lbm_step(nullptr, 1) == LBM_ERR_INVALID_ARG);
    EXPECT(lbm_step_count(nullptr) == -1);

    // The allocation-free step rejects its bad arguments before any HIP call.
    {
        lbm_params q = base();
        q.nx = q.ny = 2048;
        q.nz = 2;
        q.wall_z = 1;
        q.storage = LBM_STORE_F64;
        alignas(256) static unsigned char src[256], dst[256];
        EXPECT(lbm_step_noalloc(&q, src, dst, nullptr) == LBM_ERR_UNSUPPORTED);
        q = base();
        EXPECT(lbm_step_noalloc(&q, src, src, nullptr) == LBM_ERR_INVALID_ARG);
        EXPECT(lbm_step_noalloc(&q, nullptr, dst, nullptr) == LBM_ERR_INVALID_ARG);
        EXPECT(lbm_step_noalloc(&q, src + 4, dst, nullptr) == LBM_ERR_INVALID_ARG);
        EXPECT(lbm_step_noalloc(nullptr, src, dst, nullptr) == LBM_ERR_INVALID_ARG);
    }

    // Batches: sizes and argument checks.
    {
        lbm_params runs[3] = {base(), base(), base()};
        runs[1].nx = runs[1].ny = runs[1].nz = 48;
        runs[2].nx = 40;
        size_t bb = 0;
        EXPECT(lbm_batch_workspace_bytes(runs, 3, &bb) == LBM_OK && bb > 0);
        EXPECT(lbm_batch_workspace_bytes(runs, 0, &bb) == LBM_ERR_INVALID_ARG);
        EXPECT(lbm_batch_workspace_bytes(nullptr, 3, &bb) == LBM_ERR_INVALID_ARG);
        runs[2].wall_z = 1;
        EXPECT(lbm_batch_workspace_bytes(runs, 3, &bb) != LBM_OK);
        lbm_batch *bt = nullptr;
        EXPECT(lbm_batch_create(runs, 3, nullptr, 0, nullptr, &bt) != LBM_OK && bt == nullptr);
        EXPECT(lbm_batch_runs(nullptr) == 0);
        EXPECT(lbm_batch_nodes(nullptr) == -1);
        EXPECT(lbm_batch_destroy(nullptr) == LBM_ERR_INVALID_ARG);
    }
    for (int s = -6; s <= 1; ++s) EXPECT(lbm_status_string(s) != nullptr);

    std::printf("%s: %d failure(s)\n", g_fail ? "FAIL" : "OK", g_fail);
    return g_fail ? 1 : 0;
}
