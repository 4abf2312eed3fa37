/*
 * orc_lbm.c -- plain, slow, FP64 CPU oracle for the double-distribution
 * non-orthogonal MRT lattice Boltzmann method of Liu, He, Li & Li
 * (arXiv:1510.08224): a D2Q9 MRT equation for the incompressible flow
 * (Sec. 2.1) and an MRT equation for the temperature (Sec. 2.2), coupled
 * by the Boussinesq force (Eq. 4).  The temperature lattice is one of
 *   MODEL_D2Q5      the D2Q5 model (Eqs. 23-30), the paper's main one;
 *   MODEL_D2Q9T     the D2Q9 thermal model (Eqs. 31-32);
 *   MODEL_ISOTHERMAL no temperature field: the flow alone, driven by the
 *                   acceleration a and the walls (Secs. 3.1, 3.2).
 * The collision operator is the paper's non-orthogonal MRT, or one of the
 * two operators Sec. 3.2 compares it with:
 *   COLL_BGK        single relaxation time: fbar* = fbar - w (fbar - f^eq)
 *                   + (1 - w/2) S with w = s_nu and the Guo source S in
 *                   velocity space; g* = g - zeta (g - g^eq), zeta =
 *                   zeta_alpha;
 *   COLL_ORTHO      the classical MRT with an orthogonal basis: M_o is built
 *                   by Gram-Schmidt from the monomials 1, |e|^2, |e|^4, e_x,
 *                   e_x |e|^2, e_y, e_y |e|^2, e_x^2 - e_y^2, e_x e_y (the
 *                   paper does not print it), m^eq = M_o f^eq, source moments
 *                   M_o S, rates s_e, s_eps, s_q, s_nu on the energy, energy
 *                   square, heat-flux and stress moments; the temperature
 *                   keeps the model's own MRT.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the tests, the smoke check
 * and the CPU-baseline leg of the benchmark load this library.  It shares
 * no code, header or table with the GPU library.
 *
 * It is written to be checked by eye against the paper, not to be fast:
 *   - array-of-structures storage f[(y*nx+x)*9+i], g[(y*nx+x)*5+i];
 *   - the collision multiplies by the full dense matrices M (Eq. 13),
 *     M^-1 (App. A, Eq. A1), N (Eq. 26) and N^-1 (Eq. A2) exactly as
 *     printed in the paper;
 *   - the D2Q9 thermal equilibrium moments are the dense product M g^eq
 *     with g^eq of Eq. 31 (the definition n^eq = N g^eq);
 *   - the relaxation is the diagonal expression of Eq. 8 / Eq. 24;
 *   - streaming is a push (Eqs. 9 and 25) into a second array;
 *   - compiled with -O2 -ffp-contract=off (no fused multiply-add).
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *   R1 (Sec. 2.1, incompressible approximation after Eq. 19): the density
 *      rho enters m_0^eq, the 2rho/3 of m_3^eq and the rho/9 of m_8^eq;
 *      every velocity term of m^eq, every source moment and the momentum
 *      use the reference density rho0, i.e. j = rho0*u.
 *   R2 (Eq. 17): the printed S~_8 = (2/3) rho (ux Fy + uy Fx) is not M*S
 *      for the Guo source; the oracle uses (2/3) rho0 (ux Fx + uy Fy),
 *      which is.  A switch (s8_literal) keeps the printed form.
 *   R3 (Eqs. 4, 19, 27): at a node, T = sum g (pre-collision), then
 *      F = a + g*beta*(T - T0)*y_hat, then rho0*u = sum e_i fbar_i + rho0*F/2.
 *   R5 (Sec. 3, non-equilibrium extrapolation, the scheme of Guo, Zheng
 *      and Shi that the paper cites for its walls): with the NEE wall type
 *      the wall passes through the first/last node row or column.  After
 *      streaming, every population of a wall node x_b is rebuilt from its
 *      inward neighbour x_f:
 *        fbar_i(x_b) = f_i^eq(rho(x_f), u_w) + [fbar_i(x_f) - f_i^eq(rho(x_f), u(x_f))],
 *        g_i(x_b)    = g_i^eq(T_b, u_w)      + [g_i(x_f)    - g_i^eq(T(x_f), u(x_f))],
 *      with f^eq of Eq. 22 (reading R1), g^eq of Eq. 30, T_b = T_w for a
 *      Dirichlet wall and T(x_f) for an adiabatic one.  A corner node takes
 *      the diagonal inward neighbour, the velocity of its top/bottom wall,
 *      and a Dirichlet temperature if either of its walls has one (the
 *      top/bottom wall's first).
 *   R6 (Eqs. 31-32): the D2Q9 thermal model's N is the non-orthogonal
 *      D2Q9 matrix M of Eq. 13 (built from the same basis, Eq. 12), its
 *      relaxation diagonal is Eq. 32 and c_s^2 = 1/3; its Dirichlet
 *      anti-bounce-back adds twice the even part of Eq. 31 at the wall,
 *      2 w_i T_w [1 + theta (4.5 (e_i.u_w)^2 - 1.5 |u_w|^2)].
 *   R4 (Sec. 3 uses non-equilibrium extrapolation, not given in the
 *      text): the default walls are link-wise.  Flow: halfway bounce-back with the
 *      moving-wall term 6 w_i rho0 (e_i . u_w).  Temperature, Dirichlet:
 *      anti-bounce-back, -g*_opp + varpi*T_w/2.  Temperature, adiabatic:
 *      bounce-back.  A link that leaves through a top/bottom wall takes
 *      that wall's velocity, otherwise the left/right wall's.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- lattice (Eq. 5; weights after Eq. 22) -------------------------------- */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP9[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double W9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

/* ---- transformation matrices as printed --------------------------------- */
/* Eq. 13 */
static const double M9[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 1, 1, 1, 1, 2, 2, 2, 2},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 1, 1, -1, -1},
    {0, 0, 0, 0, 0, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 1, 1, 1, 1}};
/* Appendix A, Eq. A1 */
static const double MI9[9][9] = {
    {1, 0, 0, -1, 0, 0, 0, 0, 1},
    {0, 0.5, 0, 0.25, 0.25, 0, 0, -0.5, -0.5},
    {0, 0, 0.5, 0.25, -0.25, 0, -0.5, 0, -0.5},
    {0, -0.5, 0, 0.25, 0.25, 0, 0, 0.5, -0.5},
    {0, 0, -0.5, 0.25, -0.25, 0, 0.5, 0, -0.5},
    {0, 0, 0, 0, 0, 0.25, 0.25, 0.25, 0.25},
    {0, 0, 0, 0, 0, -0.25, 0.25, -0.25, 0.25},
    {0, 0, 0, 0, 0, 0.25, -0.25, -0.25, 0.25},
    {0, 0, 0, 0, 0, -0.25, -0.25, 0.25, 0.25}};
/* Eq. 26 */
static const double N5[5][5] = {
    {1, 1, 1, 1, 1},
    {0, 1, 0, -1, 0},
    {0, 0, 1, 0, -1},
    {0, 1, 1, 1, 1},
    {0, 1, -1, 1, -1}};
/* Appendix A, Eq. A2 */
static const double NI5[5][5] = {
    {1, 0, 0, -1, 0},
    {0, 0.5, 0, 0.25, 0.25},
    {0, 0, 0.5, 0.25, -0.25},
    {0, -0.5, 0, 0.25, 0.25},
    {0, 0, -0.5, 0.25, -0.25}};

enum { MODEL_D2Q5 = 0, MODEL_D2Q9T = 1, MODEL_ISOTHERMAL = 2 };
enum { COLL_MRT = 0, COLL_BGK = 1, COLL_ORTHO = 2 };
enum { SIDE_LEFT = 0, SIDE_RIGHT = 1, SIDE_BOTTOM = 2, SIDE_TOP = 3 };
enum { FLOW_PERIODIC = 0, FLOW_WALL = 1, FLOW_NEE = 2 };
enum { TEMP_PERIODIC = 0, TEMP_DIRICHLET = 1, TEMP_ADIABATIC = 2, TEMP_NEE_DIRICHLET = 3,
       TEMP_NEE_ADIABATIC = 4 };

typedef struct {
    int32_t nx, ny;
    int32_t model;     /* MODEL_* */
    double s[9];       /* Lambda = diag(s_0..s_8), Eq. 20 */
    double q[9];       /* Q = diag(zeta_0..), Eq. 29 (5 used) or Eq. 32 (9) */
    double varpi;      /* Eq. 28 (D2Q5) */
    double theta;      /* Eq. 31 (D2Q9 thermal), 0 or 1 */
    double rho0;       /* reference density */
    double gbeta;      /* g*beta of Eq. 4 */
    double T0;         /* reference temperature of Eq. 4 */
    double ax, ay;     /* external acceleration a of Eq. 4 */
    int32_t bc_flow[4];
    int32_t bc_temp[4];
    double wall_T[4];
    double wall_u[4][2];
    int32_t s8_literal;
    int32_t collision; /* COLL_* */
} orc_params;

typedef struct {
    orc_params p;
    int ng;              /* temperature populations per node: 5, 9 or 0 */
    double *f, *g;       /* pre-collision state at time t, AoS */
    double *fn, *gn;     /* streaming target */
    double *fp, *gp;     /* post-collision state (scratch) */
    int64_t t;
} orc_lattice;

/* ------------------------------------------------------------------------- */
/* Single-node collision: Eqs. 4, 8, 15-20 for f; Eqs. 24, 27-29 for g.      */
/* ------------------------------------------------------------------------- */
static int model_ng(const orc_params* p) {
    return p->model == MODEL_D2Q5 ? 5 : (p->model == MODEL_D2Q9T ? 9 : 0);
}

/* g_i^eq: Eq. 30 (D2Q5) or Eq. 31 (D2Q9 thermal, c_s^2 = 1/3). */
static double geq_i(const orc_params* p, int i, double T, double ux, double uy) {
    double eu = EX[i] * ux + EY[i] * uy;
    if (p->model == MODEL_D2Q9T) {
        double usq = ux * ux + uy * uy;
        return W9[i] * T * (1.0 + 3.0 * eu + p->theta * (4.5 * eu * eu - 1.5 * usq));
    }
    if (i == 0) return (1.0 - p->varpi) * T;
    return 0.25 * p->varpi * T + 0.5 * eu * T;
}

static void macroscopic(const orc_params* p, const double f[9], const double* g,
                        double* rho, double* ux, double* uy, double* T,
                        double* Fx, double* Fy) {
    /* Eq. 27: T = n_0 = sum g (no temperature field: T = T0, no buoyancy) */
    const int ng = model_ng(p);
    double t = ng ? 0.0 : p->T0;
    for (int i = 0; i < ng; ++i) t += g[i];
    /* Eq. 4: F = g beta (T - T0) j + a */
    double fx = p->ax;
    double fy = p->ay + p->gbeta * (t - p->T0);
    /* Eq. 18 */
    double r = 0.0;
    for (int i = 0; i < 9; ++i) r += f[i];
    /* Eq. 19 with j = rho0 u (reading R1) */
    double jx = 0.0, jy = 0.0;
    for (int i = 0; i < 9; ++i) {
        jx += EX[i] * f[i];
        jy += EY[i] * f[i];
    }
    jx += 0.5 * p->rho0 * fx;
    jy += 0.5 * p->rho0 * fy;
    *rho = r;
    *ux = jx / p->rho0;
    *uy = jy / p->rho0;
    *T = t;
    *Fx = fx;
    *Fy = fy;
}

/* f_i^eq of Eq. 22 under reading R1. */
static double feq_i(const orc_params* p, int i, double rho, double ux, double uy) {
    double eu = EX[i] * ux + EY[i] * uy;
    double usq = ux * ux + uy * uy;
    return W9[i] * (rho + p->rho0 * (3.0 * eu + 4.5 * eu * eu - 1.5 * usq));
}

/* The Guo forcing term in velocity space, whose moments Eq. 10 calls S~:
 * S_i = w_i rho0 [3 (e_i - u).F + 9 (e_i.u)(e_i.F)]. */
static double guo_i(const orc_params* p, int i, double ux, double uy, double Fx, double Fy) {
    double eu = EX[i] * ux + EY[i] * uy;
    double eF = EX[i] * Fx + EY[i] * Fy;
    double uF = ux * Fx + uy * Fy;
    return W9[i] * p->rho0 * (3.0 * (eF - uF) + 9.0 * eu * eF);
}

/* Orthogonal D2Q9 basis by Gram-Schmidt (plain dot product over the nine
 * velocities) of the monomials 1, |e|^2, |e|^4, e_x, e_x|e|^2, e_y,
 * e_y|e|^2, e_x^2 - e_y^2, e_x e_y; its inverse is M_o^T diag(1/|row|^2). */
static double MO9[9][9], MOI9[9][9];
static int mo9_ready = 0;

static void ortho_basis(void) {
    if (mo9_ready) return;
    double v[9][9];
    for (int i = 0; i < 9; ++i) {
        double x = EX[i], y = EY[i], r = x * x + y * y;
        v[0][i] = 1.0;
        v[1][i] = r;
        v[2][i] = r * r;
        v[3][i] = x;
        v[4][i] = x * r;
        v[5][i] = y;
        v[6][i] = y * r;
        v[7][i] = x * x - y * y;
        v[8][i] = x * y;
    }
    for (int k = 0; k < 9; ++k) {
        for (int j = 0; j < k; ++j) {
            double num = 0.0, den = 0.0;
            for (int i = 0; i < 9; ++i) {
                num += v[k][i] * MO9[j][i];
                den += MO9[j][i] * MO9[j][i];
            }
            for (int i = 0; i < 9; ++i) v[k][i] -= num / den * MO9[j][i];
        }
        for (int i = 0; i < 9; ++i) MO9[k][i] = v[k][i];
    }
    for (int k = 0; k < 9; ++k) {
        double n2 = 0.0;
        for (int i = 0; i < 9; ++i) n2 += MO9[k][i] * MO9[k][i];
        for (int i = 0; i < 9; ++i) MOI9[i][k] = MO9[k][i] / n2;
    }
    mo9_ready = 1;
}

static void collide_flow_bgk(const orc_params* p, const double f[9], double rho, double ux, double uy,
                             double Fx, double Fy, double fo[9]) {
    const double w = p->s[4];
    for (int i = 0; i < 9; ++i)
        fo[i] = f[i] - w * (f[i] - feq_i(p, i, rho, ux, uy)) + (1.0 - 0.5 * w) * guo_i(p, i, ux, uy, Fx, Fy);
}

static void collide_flow_ortho(const orc_params* p, const double f[9], double rho, double ux, double uy,
                               double Fx, double Fy, double fo[9]) {
    ortho_basis();
    /* rates along the basis: conserved moments 1, then e, eps, -, q_x, -,
     * q_y, p_xx, p_xy */
    const double s[9] = {1.0, p->s[3], p->s[8], 1.0, p->s[6], 1.0, p->s[6], p->s[4], p->s[4]};
    double feq[9], S[9], m[9], meq[9], ms[9], sm[9];
    for (int i = 0; i < 9; ++i) {
        feq[i] = feq_i(p, i, rho, ux, uy);
        S[i] = guo_i(p, i, ux, uy, Fx, Fy);
    }
    for (int k = 0; k < 9; ++k) {
        double a = 0.0, b = 0.0, c = 0.0;
        for (int i = 0; i < 9; ++i) {
            a += MO9[k][i] * f[i];
            b += MO9[k][i] * feq[i];
            c += MO9[k][i] * S[i];
        }
        m[k] = a;
        meq[k] = b;
        sm[k] = c;
    }
    for (int k = 0; k < 9; ++k) ms[k] = m[k] - s[k] * (m[k] - meq[k]) + (1.0 - 0.5 * s[k]) * sm[k];
    for (int i = 0; i < 9; ++i) {
        double acc = 0.0;
        for (int k = 0; k < 9; ++k) acc += MOI9[i][k] * ms[k];
        fo[i] = acc;
    }
}

/* The paper's flow collision: Eq. 8 in the moment space of M (Eq. 13). */
static void collide_flow_mrt(const orc_params* p, const double f[9], double rho, double ux, double uy,
                             double Fx, double Fy, double fo[9]) {
    const double r0 = p->rho0;
    /* m_bar = M fbar (Eq. 10, dense product) */
    double m[9];
    for (int k = 0; k < 9; ++k) {
        double acc = 0.0;
        for (int i = 0; i < 9; ++i) acc += M9[k][i] * f[i];
        m[k] = acc;
    }
    /* Eq. 16 under reading R1 */
    const double usq = ux * ux + uy * uy;
    double meq[9];
    meq[0] = rho;
    meq[1] = r0 * ux;
    meq[2] = r0 * uy;
    meq[3] = 2.0 / 3.0 * rho + r0 * usq;
    meq[4] = r0 * (ux * ux - uy * uy);
    meq[5] = r0 * ux * uy;
    meq[6] = 1.0 / 3.0 * r0 * uy;
    meq[7] = 1.0 / 3.0 * r0 * ux;
    meq[8] = 1.0 / 9.0 * rho + 1.0 / 3.0 * r0 * usq;
    /* Eq. 17 under readings R1, R2 */
    double S[9];
    S[0] = 0.0;
    S[1] = r0 * Fx;
    S[2] = r0 * Fy;
    S[3] = 2.0 * r0 * (ux * Fx + uy * Fy);
    S[4] = 2.0 * r0 * (ux * Fx - uy * Fy);
    S[5] = r0 * (ux * Fy + uy * Fx);
    S[6] = 1.0 / 3.0 * r0 * Fy;
    S[7] = 1.0 / 3.0 * r0 * Fx;
    S[8] = p->s8_literal ? 2.0 / 3.0 * r0 * (ux * Fy + uy * Fx)
                         : 2.0 / 3.0 * r0 * (ux * Fx + uy * Fy);
    /* Eq. 8 with diagonal Lambda (Eq. 20), delta_t = 1 */
    double ms[9];
    for (int k = 0; k < 9; ++k)
        ms[k] = m[k] - p->s[k] * (m[k] - meq[k]) + (1.0 - 0.5 * p->s[k]) * S[k];
    /* fbar* = M^-1 m_bar* (dense product with Eq. A1) */
    for (int i = 0; i < 9; ++i) {
        double acc = 0.0;
        for (int k = 0; k < 9; ++k) acc += MI9[i][k] * ms[k];
        fo[i] = acc;
    }
}

/* The temperature collision of the model: Eq. 24 in the moment space of N
 * (D2Q5) or of M (D2Q9, reading R6). */
static void collide_thermal_mrt(const orc_params* p, const double* g, double T, double ux, double uy,
                                double* go) {
    if (p->model == MODEL_ISOTHERMAL) return;
    if (p->model == MODEL_D2Q9T) {
        /* n = M g, n^eq = M g^eq (Eq. 31, reading R6), Q of Eq. 32 */
        double n9[9], ne9[9], geq[9], ns9[9];
        for (int i = 0; i < 9; ++i) geq[i] = geq_i(p, i, T, ux, uy);
        for (int k = 0; k < 9; ++k) {
            double acc = 0.0, acce = 0.0;
            for (int i = 0; i < 9; ++i) {
                acc += M9[k][i] * g[i];
                acce += M9[k][i] * geq[i];
            }
            n9[k] = acc;
            ne9[k] = acce;
        }
        for (int k = 0; k < 9; ++k) ns9[k] = n9[k] - p->q[k] * (n9[k] - ne9[k]);
        for (int i = 0; i < 9; ++i) {
            double acc = 0.0;
            for (int k = 0; k < 9; ++k) acc += MI9[i][k] * ns9[k];
            go[i] = acc;
        }
        return;
    }
    /* n = N g (dense, Eq. 26) */
    double n[5];
    for (int k = 0; k < 5; ++k) {
        double acc = 0.0;
        for (int i = 0; i < 5; ++i) acc += N5[k][i] * g[i];
        n[k] = acc;
    }
    /* Eq. 28 */
    double neq[5];
    neq[0] = T;
    neq[1] = ux * T;
    neq[2] = uy * T;
    neq[3] = p->varpi * T;
    neq[4] = 0.0;
    /* Eq. 24 with diagonal Q (Eq. 29) */
    double ns[5];
    for (int k = 0; k < 5; ++k) ns[k] = n[k] - p->q[k] * (n[k] - neq[k]);
    /* g* = N^-1 n* (dense, Eq. A2) */
    for (int i = 0; i < 5; ++i) {
        double acc = 0.0;
        for (int k = 0; k < 5; ++k) acc += NI5[i][k] * ns[k];
        go[i] = acc;
    }
}

void orc_collide_node(const orc_params* p, const double f[9], const double* g,
                      double fo[9], double* go) {
    double rho, ux, uy, T, Fx, Fy;
    macroscopic(p, f, g, &rho, &ux, &uy, &T, &Fx, &Fy);
    if (p->collision == COLL_BGK) {
        collide_flow_bgk(p, f, rho, ux, uy, Fx, Fy, fo);
        const double z = p->q[1];
        for (int i = 0; i < model_ng(p); ++i) go[i] = g[i] - z * (g[i] - geq_i(p, i, T, ux, uy));
        return;
    }
    if (p->collision == COLL_ORTHO) collide_flow_ortho(p, f, rho, ux, uy, Fx, Fy, fo);
    else collide_flow_mrt(p, f, rho, ux, uy, Fx, Fy, fo);
    collide_thermal_mrt(p, g, T, ux, uy, go);
}

/* ------------------------------------------------------------------------- */
/* Lattice                                                                    */
/* ------------------------------------------------------------------------- */
static int axis_periodic_x(const orc_params* p) { return p->bc_flow[SIDE_LEFT] == FLOW_PERIODIC; }
static int axis_periodic_y(const orc_params* p) { return p->bc_flow[SIDE_BOTTOM] == FLOW_PERIODIC; }

/* Returns 0 if the parameters describe a consistent lattice. */
int orc_check_params(const orc_params* p) {
    if (p->nx < 1 || p->ny < 1) return -1;
    for (int a = 0; a < 2; ++a) {
        int s0 = 2 * a, s1 = 2 * a + 1;
        int fp0 = p->bc_flow[s0] == FLOW_PERIODIC, fp1 = p->bc_flow[s1] == FLOW_PERIODIC;
        int tp0 = p->bc_temp[s0] == TEMP_PERIODIC, tp1 = p->bc_temp[s1] == TEMP_PERIODIC;
        if (fp0 != fp1 || tp0 != tp1 || fp0 != tp0) return -2;
    }
    int nee = 0, linkwise = 0;
    for (int s = 0; s < 4; ++s) {
        if (p->bc_flow[s] < 0 || p->bc_flow[s] > 2) return -3;
        if (p->bc_temp[s] < 0 || p->bc_temp[s] > 4) return -3;
        int fn = p->bc_flow[s] == FLOW_NEE;
        int tn = p->bc_temp[s] == TEMP_NEE_DIRICHLET || p->bc_temp[s] == TEMP_NEE_ADIABATIC;
        if (fn != tn) return -5;
        nee += fn;
        linkwise += p->bc_flow[s] == FLOW_WALL;
    }
    if (nee && linkwise) return -6;   /* one wall family per lattice */
    if (nee && ((p->bc_flow[SIDE_LEFT] == FLOW_NEE && p->nx < 3) ||
                (p->bc_flow[SIDE_BOTTOM] == FLOW_NEE && p->ny < 3))) return -7;
    if (!(p->rho0 > 0.0)) return -4;
    if (p->model < MODEL_D2Q5 || p->model > MODEL_ISOTHERMAL) return -8;
    if (p->model == MODEL_D2Q9T && !(p->theta == 0.0 || p->theta == 1.0)) return -9;
    if (p->collision < COLL_MRT || p->collision > COLL_ORTHO) return -10;
    return 0;
}

static void apply_nee_to(orc_lattice* L, double* F, double* G);

orc_lattice* orc_create(const orc_params* p) {
    if (orc_check_params(p) != 0) return NULL;
    orc_lattice* L = (orc_lattice*)calloc(1, sizeof(orc_lattice));
    if (!L) return NULL;
    L->p = *p;
    L->ng = model_ng(p);
    size_t n = (size_t)p->nx * (size_t)p->ny;
    size_t ng = L->ng ? (size_t)L->ng : 1;
    L->f = (double*)calloc(n * 9, sizeof(double));
    L->fn = (double*)calloc(n * 9, sizeof(double));
    L->fp = (double*)calloc(n * 9, sizeof(double));
    L->g = (double*)calloc(n * ng, sizeof(double));
    L->gn = (double*)calloc(n * ng, sizeof(double));
    L->gp = (double*)calloc(n * ng, sizeof(double));
    if (!L->f || !L->fn || !L->fp || !L->g || !L->gn || !L->gp) {
        free(L->f); free(L->fn); free(L->fp); free(L->g); free(L->gn); free(L->gp);
        free(L);
        return NULL;
    }
    return L;
}

void orc_destroy(orc_lattice* L) {
    if (!L) return;
    free(L->f); free(L->fn); free(L->fp); free(L->g); free(L->gn); free(L->gp);
    free(L);
}

/* Rest state: fbar_i = f_i^eq(rho0, u=0) (Eq. 22) and g_i = g_i^eq(T, u=0)
 * (Eq. 30 or 31).  T is nx*ny values in [y][x] order, or NULL for T = T0. */
void orc_init_equilibrium(orc_lattice* L, const double* T) {
    const orc_params* p = &L->p;
    const int ng = L->ng;
    size_t n = (size_t)p->nx * (size_t)p->ny;
    for (size_t c = 0; c < n; ++c) {
        double t = T ? T[c] : p->T0;
        for (int i = 0; i < 9; ++i) L->f[c * 9 + i] = W9[i] * p->rho0;
        for (int i = 0; i < ng; ++i) L->g[c * ng + i] = geq_i(p, i, t, 0.0, 0.0);
    }
    apply_nee_to(L, L->f, L->g);   /* NEE wall nodes are always extrapolated */
    L->t = 0;
}

/* State exchange in plane order [i][y][x] (pre-collision at time t). */
void orc_set_state(orc_lattice* L, const double* f, const double* g) {
    size_t n = (size_t)L->p.nx * (size_t)L->p.ny;
    const int ng = L->ng;
    for (size_t c = 0; c < n; ++c) {
        for (int i = 0; i < 9; ++i) L->f[c * 9 + i] = f[(size_t)i * n + c];
        for (int i = 0; i < ng; ++i) L->g[c * ng + i] = g[(size_t)i * n + c];
    }
    apply_nee_to(L, L->f, L->g);
}

void orc_get_state(const orc_lattice* L, double* f, double* g) {
    size_t n = (size_t)L->p.nx * (size_t)L->p.ny;
    const int ng = L->ng;
    for (size_t c = 0; c < n; ++c) {
        for (int i = 0; i < 9; ++i) f[(size_t)i * n + c] = L->f[c * 9 + i];
        for (int i = 0; i < ng; ++i) g[(size_t)i * n + c] = L->g[c * ng + i];
    }
}

int64_t orc_time(const orc_lattice* L) { return L->t; }

static int is_nee(const orc_params* p, int side) { return p->bc_flow[side] == FLOW_NEE; }

/* Non-equilibrium extrapolation (reading R5) on a pre-collision state. */
static void apply_nee_to(orc_lattice* L, double* F, double* G) {
    const orc_params* p = &L->p;
    const int nx = p->nx, ny = p->ny, ng = L->ng;
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            int onL = is_nee(p, SIDE_LEFT) && x == 0, onR = is_nee(p, SIDE_RIGHT) && x == nx - 1;
            int onB = is_nee(p, SIDE_BOTTOM) && y == 0, onT = is_nee(p, SIDE_TOP) && y == ny - 1;
            if (!(onL || onR || onB || onT)) continue;
            int fx = x + (onL ? 1 : (onR ? -1 : 0));
            int fy = y + (onB ? 1 : (onT ? -1 : 0));
            int sx = onL ? SIDE_LEFT : (onR ? SIDE_RIGHT : -1);
            int sy = onB ? SIDE_BOTTOM : (onT ? SIDE_TOP : -1);
            int vside = sy >= 0 ? sy : sx;
            int tside = -1;
            if (sy >= 0 && p->bc_temp[sy] == TEMP_NEE_DIRICHLET) tside = sy;
            else if (sx >= 0 && p->bc_temp[sx] == TEMP_NEE_DIRICHLET) tside = sx;
            const double* ff = F + ((size_t)fy * nx + fx) * 9;
            const double* gf = G + ((size_t)fy * nx + fx) * ng;
            double rho, ux, uy, T, Fx, Fy;
            macroscopic(p, ff, gf, &rho, &ux, &uy, &T, &Fx, &Fy);
            double uwx = p->wall_u[vside][0], uwy = p->wall_u[vside][1];
            double Tb = tside >= 0 ? p->wall_T[tside] : T;
            double* fb = F + ((size_t)y * nx + x) * 9;
            double* gb = G + ((size_t)y * nx + x) * ng;
            for (int i = 0; i < 9; ++i)
                fb[i] = feq_i(p, i, rho, uwx, uwy) + (ff[i] - feq_i(p, i, rho, ux, uy));
            for (int i = 0; i < ng; ++i)
                gb[i] = geq_i(p, i, Tb, uwx, uwy) + (gf[i] - geq_i(p, i, T, ux, uy));
        }
    }
}

/* Push streaming (Eqs. 9, 25) from fp/gp into fn/gn, with link-wise walls
 * (reading R4).  Every (node, direction) slot of the target is written
 * exactly once: either by the neighbour upstream or by the wall rule. */
static void stream_push(orc_lattice* L) {
    const orc_params* p = &L->p;
    const int nx = p->nx, ny = p->ny, ng = L->ng;
    const int px = axis_periodic_x(p), py = axis_periodic_y(p);
    /* rows are independent: every target slot has exactly one writer */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            size_t c = (size_t)y * nx + x;
            for (int i = 0; i < 9; ++i) {
                int tx = x + EX[i], ty = y + EY[i];
                int outx = (tx < 0 || tx >= nx), outy = (ty < 0 || ty >= ny);
                if (outx && px) tx = (tx + nx) % nx;
                if (outy && py) ty = (ty + ny) % ny;
                int wallx = outx && !px, wally = outy && !py;
                if (!wallx && !wally) {
                    L->fn[((size_t)ty * nx + tx) * 9 + i] = L->fp[c * 9 + i];
                } else {
                    int side = wally ? (ty < 0 ? SIDE_BOTTOM : SIDE_TOP)
                                     : (tx < 0 ? SIDE_LEFT : SIDE_RIGHT);
                    if (p->bc_flow[side] == FLOW_NEE) continue;   /* rebuilt by apply_nee */
                    double eu = EX[i] * p->wall_u[side][0] + EY[i] * p->wall_u[side][1];
                    L->fn[c * 9 + OPP9[i]] = L->fp[c * 9 + i] - 6.0 * W9[i] * p->rho0 * eu;
                }
            }
            for (int i = 0; i < ng; ++i) {
                int tx = x + EX[i], ty = y + EY[i];
                int outx = (tx < 0 || tx >= nx), outy = (ty < 0 || ty >= ny);
                if (outx && px) tx = (tx + nx) % nx;
                if (outy && py) ty = (ty + ny) % ny;
                int wallx = outx && !px, wally = outy && !py;
                if (!wallx && !wally) {
                    L->gn[((size_t)ty * nx + tx) * ng + i] = L->gp[c * ng + i];
                } else {
                    int side = wally ? (ty < 0 ? SIDE_BOTTOM : SIDE_TOP)
                                     : (tx < 0 ? SIDE_LEFT : SIDE_RIGHT);
                    if (p->bc_flow[side] == FLOW_NEE) continue;   /* rebuilt by apply_nee */
                    /* anti-bounce-back adds twice the even part of g^eq at
                     * the wall: varpi T_w / 4 per link (Eq. 30) or
                     * w_i T_w [1 + theta (4.5 (e.u_w)^2 - 1.5 u_w^2)] (Eq. 31) */
                    double even;
                    if (p->model == MODEL_D2Q9T) {
                        double eu = EX[i] * p->wall_u[side][0] + EY[i] * p->wall_u[side][1];
                        double usq = p->wall_u[side][0] * p->wall_u[side][0] +
                                     p->wall_u[side][1] * p->wall_u[side][1];
                        even = W9[i] * p->wall_T[side] * (1.0 + p->theta * (4.5 * eu * eu - 1.5 * usq));
                    } else {
                        even = 0.25 * p->varpi * p->wall_T[side];
                    }
                    if (p->bc_temp[side] == TEMP_DIRICHLET)
                        L->gn[c * ng + OPP9[i]] = -L->gp[c * ng + i] + 2.0 * even;
                    else
                        L->gn[c * ng + OPP9[i]] = L->gp[c * ng + i];
                }
            }
        }
    }
}

static void collide_all(orc_lattice* L) {
    size_t n = (size_t)L->p.nx * (size_t)L->p.ny;
    const int ng = L->ng;
#pragma omp parallel for schedule(static)
    for (size_t c = 0; c < n; ++c)
        orc_collide_node(&L->p, L->f + c * 9, L->g + c * ng, L->fp + c * 9, L->gp + c * ng);
}

/* Advance n time steps: collide every node, then push-stream. */
void orc_step(orc_lattice* L, int64_t nsteps) {
    for (int64_t s = 0; s < nsteps; ++s) {
        collide_all(L);
        stream_push(L);
        apply_nee_to(L, L->fn, L->gn);
        double* t;
        t = L->f; L->f = L->fn; L->fn = t;
        t = L->g; L->g = L->gn; L->gn = t;
        L->t += 1;
    }
}

/* Post-collision state of the current time level, plane order, without
 * advancing the lattice. */
void orc_post_collision(orc_lattice* L, double* f, double* g) {
    collide_all(L);
    size_t n = (size_t)L->p.nx * (size_t)L->p.ny;
    const int ng = L->ng;
    for (size_t c = 0; c < n; ++c) {
        for (int i = 0; i < 9; ++i) f[(size_t)i * n + c] = L->fp[c * 9 + i];
        for (int i = 0; i < ng; ++i) g[(size_t)i * n + c] = L->gp[c * ng + i];
    }
}

/* rho, ux, uy, T at time t (Eqs. 18, 19, 27), [y][x] order; NULL skips. */
void orc_moments(const orc_lattice* L, double* rho, double* ux, double* uy, double* T) {
    size_t n = (size_t)L->p.nx * (size_t)L->p.ny;
    for (size_t c = 0; c < n; ++c) {
        double r, u, v, t, fx, fy;
        macroscopic(&L->p, L->f + c * 9, L->g + c * L->ng, &r, &u, &v, &t, &fx, &fy);
        if (rho) rho[c] = r;
        if (ux) ux[c] = u;
        if (uy) uy[c] = v;
        if (T) T[c] = t;
    }
}

/* Local Nusselt number along one Dirichlet wall (Eq. 39 and the local
 * definition before it): Nu = -L (dT/dx_normal-axis)_wall / dT.
 * Link-wise walls sit half a spacing outside the first node; the wall-
 * normal gradient comes from a second-order one-sided fit through T_wall,
 * T(1/2), T(3/2):  dT/dn = (9 T1 - T2 - 8 Tw) / 3  (n into the fluid), and
 * the mean is the midpoint rule over the wall nodes.  NEE walls pass
 * through the first node: dT/dn = (-3 T0 + 4 T1 - T2) / 2 with T0, T1, T2
 * the first three nodes, and the mean is the trapezoidal rule.  On the
 * left/bottom wall d/dx (d/dy) = d/dn; on the right/top it is -d/dn.
 * nu_local gets one value per wall node (ny for left/right, nx for
 * bottom/top) and may be NULL.  Returns 0, or -1 for a bad side. */
static double node_T(const orc_lattice* L, int x, int y) {
    const double* g = L->g + ((size_t)y * L->p.nx + x) * L->ng;
    double t = 0.0;
    for (int i = 0; i < L->ng; ++i) t += g[i];
    return t;
}

int orc_nusselt(const orc_lattice* L, int side, double length, double dT,
                double* nu_local, double* nu_mean, double* nu_max, int32_t* i_max) {
    const orc_params* p = &L->p;
    const int nx = p->nx, ny = p->ny;
    if (side < 0 || side > 3 || L->ng == 0) return -1;
    const int nee = p->bc_temp[side] == TEMP_NEE_DIRICHLET;
    if (p->bc_temp[side] != TEMP_DIRICHLET && !nee) return -1;
    int vertical = (side == SIDE_LEFT || side == SIDE_RIGHT);
    int count = vertical ? ny : nx;
    int depth = vertical ? nx : ny;
    if (depth < (nee ? 3 : 2)) return -1;
    double tw = p->wall_T[side];
    double sign = (side == SIDE_LEFT || side == SIDE_BOTTOM) ? 1.0 : -1.0;
    double sum = 0.0, best = -INFINITY;
    int ibest = -1;
    for (int k = 0; k < count; ++k) {
        double t[3];
        for (int d = 0; d < 3 && d < depth; ++d) {
            int x = vertical ? (side == SIDE_LEFT ? d : nx - 1 - d) : k;
            int y = vertical ? k : (side == SIDE_BOTTOM ? d : ny - 1 - d);
            t[d] = node_T(L, x, y);
        }
        double dtdn = nee ? (-3.0 * t[0] + 4.0 * t[1] - t[2]) / 2.0
                          : (9.0 * t[0] - t[1] - 8.0 * tw) / 3.0;
        double nu = -length * (sign * dtdn) / dT;
        if (nu_local) nu_local[k] = nu;
        sum += (nee && (k == 0 || k == count - 1)) ? 0.5 * nu : nu;
        if (nu > best) { best = nu; ibest = k; }
    }
    if (nu_mean) *nu_mean = nee ? sum / (count - 1) : sum / count;
    if (nu_max) *nu_max = best;
    if (i_max) *i_max = ibest;
    return 0;
}

/* The oracle's own tables, exported so that the tests can compare them
 * with the printed matrices and with the basis construction of Eq. 12. */
void orc_tables(double* m9, double* mi9, double* n5, double* ni5, double* w9,
                int32_t* ex, int32_t* ey) {
    if (m9) memcpy(m9, M9, sizeof(M9));
    if (mi9) memcpy(mi9, MI9, sizeof(MI9));
    if (n5) memcpy(n5, N5, sizeof(N5));
    if (ni5) memcpy(ni5, NI5, sizeof(NI5));
    if (w9) memcpy(w9, W9, sizeof(W9));
    if (ex) for (int i = 0; i < 9; ++i) ex[i] = EX[i];
    if (ey) for (int i = 0; i < 9; ++i) ey[i] = EY[i];
}

size_t orc_params_size(void) { return sizeof(orc_params); }

/* Threads a step uses: 1, or the OpenMP team size in the build with
 * -fopenmp (the same arithmetic; the loops over nodes and rows split
 * across threads, each node's values computed as in the serial build). */
#ifdef _OPENMP
#include <omp.h>
int orc_threads(void) { return omp_get_max_threads(); }
#else
int orc_threads(void) { return 1; }
#endif
