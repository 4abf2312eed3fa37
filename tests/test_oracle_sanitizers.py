"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only; the oracle has no device code) and driven through
every entry point for every temperature model, collision operator and
wall family on lattices from 1 x 1 up, periodic or not on each axis: no
out-of-bounds access, leak, use of uninitialised memory the sanitizers
see, signed overflow or other undefined behaviour may occur."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

DRIVER = r"""
#include "orc_lbm.c"
#include <stdio.h>

static int run(int nx, int ny, int model, int coll, int nee, int px, int py) {
    orc_params p;
    memset(&p, 0, sizeof p);
    p.nx = nx;
    p.ny = ny;
    p.model = model;
    p.collision = coll;
    const double s[9] = {1, 1, 1, 1.6, 1.3, 1.3, 1.2, 1.2, 1.8};
    const double q[9] = {1, 1.1, 1.1, 1.9, 1.9, 1.7, 1.7, 1.4, 1.4};
    for (int k = 0; k < 9; ++k) { p.s[k] = s[k]; p.q[k] = q[k]; }
    p.varpi = 0.5; p.theta = 1.0; p.rho0 = 1.0; p.gbeta = 1e-3; p.T0 = 0.5; p.ax = 1e-5; p.ay = -2e-5;
    for (int side = 0; side < 4; ++side) {
        const int periodic = side < 2 ? px : py;
        p.bc_flow[side] = periodic ? FLOW_PERIODIC : (nee ? FLOW_NEE : FLOW_WALL);
        if (periodic) p.bc_temp[side] = TEMP_PERIODIC;
        else if (side < 2) p.bc_temp[side] = nee ? TEMP_NEE_DIRICHLET : TEMP_DIRICHLET;
        else p.bc_temp[side] = nee ? TEMP_NEE_ADIABATIC : TEMP_ADIABATIC;
    }
    p.wall_T[0] = 1.0;
    p.wall_u[3][0] = 0.05;
    p.wall_u[0][1] = 0.01;
    if (orc_check_params(&p) != 0) return 0;
    orc_lattice* L = orc_create(&p);
    if (!L) { fprintf(stderr, "create failed\n"); exit(2); }
    const size_t n = (size_t)nx * ny;
    const int ng = model == MODEL_D2Q5 ? 5 : (model == MODEL_D2Q9T ? 9 : 0);
    double* T = malloc(n * sizeof(double));
    double* f = malloc(9 * n * sizeof(double));
    double* g = malloc((ng ? ng : 1) * n * sizeof(double));
    double* m = malloc(4 * n * sizeof(double));
    double* loc = malloc((size_t)(nx > ny ? nx : ny) * sizeof(double));
    for (size_t c = 0; c < n; ++c) T[c] = 0.5 + 0.1 * sin(0.7 * (double)c);
    orc_init_equilibrium(L, T);
    orc_step(L, 3);
    orc_moments(L, m, m + n, m + 2 * n, m + 3 * n);
    double mean, mx;
    int32_t imax;
    if (ng && !px) (void)orc_nusselt(L, 0, (double)nx, 1.0, loc, &mean, &mx, &imax);
    orc_get_state(L, f, g);
    orc_set_state(L, f, g);
    orc_post_collision(L, f, g);
    double fo[9], go[9];
    orc_collide_node(&p, f, g, fo, go);
    orc_destroy(L);
    free(T); free(f); free(g); free(m); free(loc);
    return 1;
}

int main(void) {
    const int sizes[] = {1, 2, 3, 5, 16};
    int runs = 0;
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 5; ++b)
            for (int model = 0; model < 3; ++model)
                for (int coll = 0; coll < 3; ++coll)
                    for (int nee = 0; nee < 2; ++nee)
                        for (int px = 0; px < 2; ++px)
                            for (int py = 0; py < 2; ++py)
                                runs += run(sizes[a], sizes[b], model, coll, nee, px, py);
    printf("runs %d\n", runs);
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    src = tmp_path / "driver.c"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", ORACLE, "-o", str(exe), str(src), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    runs = int(r.stdout.split()[-1])
    assert runs > 1000, r.stdout
