// Host-side check of the runtime behind include/lbm.h: every entry point,
// every storage, temperature model and collision operator, the wall
// families, launch policies, graphs, state save/restore and batches, on
// small lattices, with the runtime's host code built under address and
// undefined-behaviour sanitizers (the kernels are not instrumented).  Exits
// 0 and prints "host check ok" when every call returned what it should.
#include "lbm.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <vector>

static int g_fail = 0;

#define EXPECT(cond)                                                            \
    do {                                                                        \
        if (!(cond)) {                                                          \
            fprintf(stderr, "host check: %s:%d: %s\n", __FILE__, __LINE__, #cond); \
            ++g_fail;                                                           \
        }                                                                       \
    } while (0)

static lbm_params cavity(int model, int coll, bool nee, bool px) {
    lbm_params p;
    lbm_params_default(&p);
    p.ra = 1e4;
    p.u_c = 0.1;
    p.collision = coll;
    if (model == LBM_MODEL_ISOTHERMAL) {
        p.ra = 0.0;
        p.s_nu = 1.3;
        p.zeta_alpha = 1.0;
        p.wall_u[LBM_TOP][0] = 0.05;
    }
    for (int side = 0; side < 4; ++side) {
        const bool periodic = px && side < 2;
        p.bc_flow[side] = periodic ? LBM_BC_PERIODIC : (nee ? LBM_BC_NEE : LBM_BC_WALL);
        if (periodic) p.bc_temp[side] = LBM_T_PERIODIC;
        else if (side < 2) p.bc_temp[side] = nee ? LBM_T_NEE_DIRICHLET : LBM_T_DIRICHLET;
        else p.bc_temp[side] = nee ? LBM_T_NEE_ADIABATIC : LBM_T_ADIABATIC;
    }
    if (px) {  // heated from below instead
        p.bc_temp[LBM_BOTTOM] = nee ? LBM_T_NEE_DIRICHLET : LBM_T_DIRICHLET;
        p.bc_temp[LBM_TOP] = nee ? LBM_T_NEE_DIRICHLET : LBM_T_DIRICHLET;
        p.wall_T[LBM_BOTTOM] = 1.0;
        p.wall_T[LBM_TOP] = 0.0;
    }
    return p;
}

static void one_solver(int nx, int ny, int storage, int model, int coll, bool nee, bool px) {
    lbm_solver* h = nullptr;
    if (lbm_create(&h, nx, ny, storage, model, nullptr) != LBM_OK) {
        fprintf(stderr, "host check: create %dx%d: %s\n", nx, ny, lbm_last_error(nullptr));
        ++g_fail;
        return;
    }
    lbm_params p = cavity(model, coll, nee, px);
    const int rc = lbm_set_params(h, &p);
    if (rc != LBM_OK) {  // a combination the library rejects must say why
        EXPECT(rc == LBM_ERR_ARG && strlen(lbm_last_error(h)) > 0);
        lbm_destroy(h);
        return;
    }
    const size_t n = (size_t)nx * ny;
    const int ng = model == LBM_MODEL_D2Q5 ? 5 : (model == LBM_MODEL_D2Q9T ? 9 : 0);
    std::vector<double> T(n), rho(n), ux(n), uy(n), t2(n), f(9 * n), g((ng ? ng : 1) * n);
    for (size_t c = 0; c < n; ++c) T[c] = 0.5 + 0.1 * sin(0.37 * (double)c);
    if (ng) EXPECT(lbm_init_temperature(h, T.data()) == LBM_OK);
    else EXPECT(lbm_init_temperature(h, T.data()) != LBM_OK);
    EXPECT(lbm_step(h, 5) == LBM_OK);
    EXPECT(lbm_moments(h, rho.data(), ux.data(), uy.data(), ng ? t2.data() : nullptr) == LBM_OK);
    for (size_t c = 0; c < n; ++c) EXPECT(isfinite(rho[c]) && fabs(rho[c] - 1.0) < 0.1);
    double r = 0.0;
    int64_t bad = -1;
    EXPECT(lbm_residual(h, &r, &bad) == LBM_OK && bad == 0);
    EXPECT(lbm_step(h, 3) == LBM_OK);
    EXPECT(lbm_residual(h, &r, &bad) == LBM_OK && bad == 0 && isfinite(r));
    if (ng) {
        const int side = px ? LBM_BOTTOM : LBM_LEFT;
        double mean = 0.0, mx = 0.0;
        int32_t imax = -1;
        const int depth = px ? ny : nx;
        const int want = depth >= 2 + (nee ? 1 : 0) ? LBM_OK : LBM_ERR_ARG;
        EXPECT(lbm_nusselt(h, side, &mean, &mx, &imax) == want);
        std::vector<double> loc(px ? nx : ny);
        EXPECT(lbm_nusselt_local(h, side, loc.data()) == want);
    }
    EXPECT(lbm_get_populations(h, f.data(), ng ? g.data() : nullptr) == LBM_OK);
    EXPECT(lbm_set_populations(h, f.data(), ng ? g.data() : nullptr) == LBM_OK);
    uint64_t sb = 0;
    EXPECT(lbm_state_bytes(h, &sb) == LBM_OK && sb > 0);
    std::vector<unsigned char> blob(sb);
    EXPECT(lbm_save_state(h, blob.data(), sb) == LBM_OK);
    EXPECT(lbm_save_state(h, blob.data(), sb - 1) != LBM_OK);
    for (int pol : {0, (int)(LBM_POLICY_XCD_BANDS | LBM_POLICY_KEEP_STORES), (int)LBM_POLICY_FUSE2,
                    (int)(LBM_POLICY_FUSEK | LBM_POLICY_FUSE2 | LBM_POLICY_XCD_BANDS), (int)LBM_POLICY_DEFAULT}) {
        EXPECT(lbm_set_launch(h, 0, 0, 0, pol) == LBM_OK);
        int32_t spl = 0;
        EXPECT(lbm_steps_per_launch(h, &spl) == LBM_OK && spl >= 1 && spl <= 4);
        EXPECT(lbm_step(h, 3) == LBM_OK);
        EXPECT(lbm_step(h, 5) == LBM_OK);
    }
    EXPECT(lbm_set_graph_steps(h, 4) == LBM_OK);
    EXPECT(lbm_step(h, 9) == LBM_OK);
    EXPECT(lbm_set_graph_steps(h, 3) == LBM_ERR_ARG);
    EXPECT(lbm_load_state(h, blob.data(), sb) == LBM_OK);
    int64_t t = -1;
    EXPECT(lbm_time(h, &t) == LBM_OK && t == 8);
    EXPECT(lbm_synchronize(h) == LBM_OK);
    lbm_destroy(h);
}

static void batches(int storage) {
    lbm_batch* b = nullptr;
    EXPECT(lbm_batch_create(&b, storage, nullptr) == LBM_OK);
    std::vector<lbm_solver*> members;
    const int sizes[][2] = {{64, 64}, {70, 33}, {20, 9}, {130, 41}};
    for (auto& sz : sizes) {
        lbm_solver* h = nullptr;
        EXPECT(lbm_create(&h, sz[0], sz[1], storage, LBM_MODEL_D2Q5, lbm_batch_stream(b)) == LBM_OK);
        lbm_params p = cavity(LBM_MODEL_D2Q5, LBM_COLLISION_MRT, false, false);
        EXPECT(lbm_set_params(h, &p) == LBM_OK);
        int32_t slot = -1;
        EXPECT(lbm_batch_add(b, h, &slot) == LBM_OK && slot >= 0);
        members.push_back(h);
    }
    for (int pol : {(int)LBM_POLICY_DEFAULT, 0, (int)LBM_POLICY_FUSE2, (int)(LBM_POLICY_FUSEK | LBM_POLICY_FUSE2),
                    (int)LBM_POLICY_FUSEK}) {
        EXPECT(lbm_batch_set_policy(b, pol) == LBM_OK);
        EXPECT(lbm_batch_step(b, 7) == LBM_OK);
    }
    EXPECT(lbm_batch_set_policy(b, 5) == LBM_ERR_ARG);
    EXPECT(lbm_batch_set_graph_steps(b, 6) == LBM_OK);
    EXPECT(lbm_batch_step(b, 13) == LBM_OK);
    std::vector<double> r(members.size());
    std::vector<int64_t> bad(members.size());
    EXPECT(lbm_batch_residual(b, r.data(), bad.data()) == LBM_OK);
    EXPECT(lbm_batch_remove(b, 1) == LBM_OK);
    EXPECT(lbm_batch_remove(b, 1) == LBM_ERR_ARG);
    EXPECT(lbm_batch_step(b, 4) == LBM_OK);
    int32_t active = 0, slots = 0;
    EXPECT(lbm_batch_size(b, &active, &slots) == LBM_OK && active == 3 && slots == 4);
    lbm_destroy(members[0]);  // a member destroyed while in the batch leaves it
    EXPECT(lbm_batch_step(b, 2) == LBM_OK);
    // the members launch on the batch's stream: destroy them before it
    for (size_t k = 1; k < members.size(); ++k) lbm_destroy(members[k]);
    lbm_batch_destroy(b);
}

int main() {
    EXPECT(lbm_abi_version() == LBM_ABI_VERSION);
    lbm_solver* h = nullptr;
    EXPECT(lbm_create(&h, 0, 5, LBM_F64, LBM_MODEL_D2Q5, nullptr) == LBM_ERR_ARG && h == nullptr);
    EXPECT(lbm_step(nullptr, 1) == LBM_ERR_ARG);
    lbm_destroy(nullptr);
    lbm_batch_destroy(nullptr);
    const int shapes[][2] = {{1, 1}, {3, 7}, {64, 4}, {70, 45}, {129, 9}};
    for (auto& s : shapes)
        for (int storage = LBM_F64; storage <= LBM_F16; ++storage)
            for (int model = LBM_MODEL_D2Q5; model <= LBM_MODEL_ISOTHERMAL; ++model)
                for (int coll = LBM_COLLISION_MRT; coll <= LBM_COLLISION_ORTHO_MRT; ++coll)
                    for (int nee = 0; nee < 2; ++nee)
                        for (int px = 0; px < 2; ++px) one_solver(s[0], s[1], storage, model, coll, nee, px);
    for (int storage = LBM_F64; storage <= LBM_F16; ++storage) batches(storage);
    if (g_fail) fprintf(stderr, "host check: %d failures\n", g_fail);
    else printf("host check ok\n");
    // Every object of ours is destroyed above.  End without running the
    // HIP runtime's global finalizers: under AddressSanitizer its teardown
    // frees runtime objects after the sanitizer's device allocator has
    // been told the device runtime is gone, which fails a sanitizer check.
    fflush(stdout);
    fflush(stderr);
    _exit(g_fail ? 1 : 0);
}
