/*
 * lbm_oracle.c -- plain, slow, FP64 reference of the lattice Boltzmann
 * collide-and-stream cycle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle against which the HIP
 * path is checked.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the HIP library: its velocity tables, equilibrium, collision
 * operators, boundary rules and reductions are written out here on their own.
 *
 * Scheme: the two-population "push" formulation (the thread-safe two-array
 * scheme the paper adopts for its GPU port, Sec. 2.3 "Structure-of-array
 * memory layout").  Populations are kept unshifted in FP64, structure of
 * arrays f[i][z][y][x] (x fastest), i in the canonical order below.
 *
 * Physics followed, per function:
 *   - D3Q19 lattice (paper Sec. 3: all validation runs use D3Q19);
 *     D3Q27 is the extension the paper names as future work (Sec. 5).
 *   - BGK with the second-order weighted equilibrium (Sec. 3.1, Sec. 3.2).
 *   - TRT with the "magic" parameter (Sec. 3.3: Berea runs use TRT, which
 *     decouples wall position from the relaxation time).
 *   - Smagorinsky subgrid model (Fig. 3 / Sec. 2.3 list it among the chained
 *     models), in the implicit relaxation-time form.
 *   - Regularized open boundaries on the x planes (Sec. 3.3: the Berea runs
 *     drive the flow by regularized velocity / pressure conditions, after
 *     Latt et al. 2008): the populations entering through the plane are
 *     rebuilt from the imposed velocity (density from mass and normal
 *     momentum balance) or the imposed density (normal velocity likewise),
 *     with the non-equilibrium part of each unknown population taken from
 *     its opposite, then the whole node is regularized and relaxed.
 *   - Recursive regularized collision (the paper's robust model, Sec. 3.1,
 *     3.2): third-order Hermite equilibrium; the second-order non-equilibrium
 *     coefficient is relaxed with 1/tau for its deviatoric part and with 1
 *     for its trace (bulk relaxation fixed to 1, Sec. 3.1), and the
 *     third-order non-equilibrium coefficient follows from it recursively
 *     (after Malaspinas 2015).  Third-order terms use the Hermite polynomials
 *     the lattice supports, projected with the lattice's own weighted inner
 *     product.
 *   - Regularized BGK (the regularized family the paper's robust RR model
 *     belongs to, Sec. 3.1-3.2): the non-equilibrium part is replaced by its
 *     projection on the second-order Hermite polynomials before relaxing
 *     (Latt and Chopard's regularization, textbook form with Guo forcing).
 *   - Standard and modified (moving-wall) bounce-back (Sec. 3 intro: Ladd's
 *     Dirichlet conditions).
 *   - Guo body force (not in the paper; drives the porous case).
 *   - Domain-averaged kinetic energy, Eq. (5).
 *   - Learned eddy-viscosity closure: MLP 7->32->32->1 with BF16 rounding
 *     emulated in software, FP64 accumulation.
 *
 * Parity pins (tests/test_oracle_*.py) tie every function to something
 * other than itself: closed-form moments, exact conservation, analytic
 * Poiseuille / Couette profiles, the z-invariant Taylor-Green decay, single
 * population translation, TRT->BGK and Smagorinsky->BGK reductions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXQ 27
#define ORC_MLP_PARAMS 1359

typedef struct {
    int32_t nx, ny, nz, q;
    double rho0;        /* reference density, also used for the wall term   */
    double tau;         /* BGK / TRT-even relaxation time, tau = 3 nu + 1/2 */
    double trt_lambda;  /* TRT magic parameter                              */
    double smag_cs;     /* Smagorinsky constant                             */
    double force[3];    /* uniform body-force density                       */
    double wall_u[16][3]; /* velocity of moving-wall tags 16..31            */
    double bc_u[3];     /* velocity imposed on velocity-boundary nodes      */
    double bc_rho[2];   /* density imposed on pressure-boundary nodes at    */
                        /* x = 0 ([0]) and x = nx-1 ([1])                   */
    int32_t flags;      /* bit0: skip collision (free streaming, test only) */
    int32_t pad;
    const float *mlp;   /* packed MLP parameters (see below), may be NULL   */
} orc_config;

/* Tag values (fixed interface shared with the C ABI). */
/* Open boundaries: T_VIN velocity at x = 0, T_POUT pressure at x = nx-1,
 * T_PIN pressure at x = 0, T_VOUT velocity at x = nx-1. */
enum { T_SOLID = 0, T_BGK = 1, T_TRT = 2, T_SMAG = 3, T_MLP = 4, T_REG = 5, T_VIN = 6, T_POUT = 7,
       T_PIN = 8, T_VOUT = 9, T_RR = 10, T_WALL0 = 16 };

static int is_fluid(int t) { return t >= 1 && t <= 10; }

/* ------------------------------------------------------------------ tables */
/*
 * Canonical velocity order: rest; +x,+y,+z; the six face diagonals
 * (1,1,0),(1,-1,0),(1,0,1),(1,0,-1),(0,1,1),(0,1,-1); for D3Q27 the four
 * corners (1,1,1),(1,1,-1),(1,-1,1),(1,-1,-1); then the negatives of all
 * of the above in the same order.
 */
static const int first_half[13][3] = {
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
    {1, 1, 0}, {1, -1, 0}, {1, 0, 1}, {1, 0, -1}, {0, 1, 1}, {0, 1, -1},
    {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};

typedef struct {
    int q;
    int c[ORC_MAXQ][3];
    double w[ORC_MAXQ];
    int opp[ORC_MAXQ];
} lattice_t;

static void make_lattice(int q, lattice_t *L) {
    int h = (q - 1) / 2;
    L->q = q;
    L->c[0][0] = L->c[0][1] = L->c[0][2] = 0;
    for (int k = 0; k < h; ++k)
        for (int a = 0; a < 3; ++a) {
            L->c[1 + k][a] = first_half[k][a];
            L->c[1 + h + k][a] = -first_half[k][a];
        }
    for (int i = 0; i < q; ++i) {
        int n2 = L->c[i][0] * L->c[i][0] + L->c[i][1] * L->c[i][1] + L->c[i][2] * L->c[i][2];
        if (q == 19) {
            static const double w19[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0};
            L->w[i] = w19[n2];
        } else {
            static const double w27[4] = {8.0 / 27.0, 2.0 / 27.0, 1.0 / 54.0, 1.0 / 216.0};
            L->w[i] = w27[n2];
        }
    }
    /* opposite index by search, independent of any index formula */
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j)
            if (L->c[j][0] == -L->c[i][0] && L->c[j][1] == -L->c[i][1] && L->c[j][2] == -L->c[i][2])
                L->opp[i] = j;
}

int orc_velocity(int q, int i, int c[3], double *w) {
    lattice_t L;
    if ((q != 19 && q != 27) || i < 0 || i >= q) return -1;
    make_lattice(q, &L);
    c[0] = L.c[i][0]; c[1] = L.c[i][1]; c[2] = L.c[i][2];
    *w = L.w[i];
    return L.opp[i];
}

/* -------------------------------------------------------------- equilibrium */
/* Second-order weighted equilibrium: f_i = w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u). */
static void equilibrium(const lattice_t *L, double rho, const double u[3], double *feq) {
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < L->q; ++i) {
        double cu = L->c[i][0] * u[0] + L->c[i][1] * u[1] + L->c[i][2] * u[2];
        feq[i] = L->w[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* ---------------------------------------------------- third-order Hermite terms */
/*
 * Third-order Hermite polynomials H_abc(c) = c_a c_b c_c - cs^2 (c_a d_bc +
 * c_b d_ac + c_c d_ab), cs^2 = 1/3.  D3Q19 cannot tell H_xxy from H_yzz (and
 * the other two such pairs) apart under its weighted inner product, so the
 * basis is built from the sums and differences of those pairs, which are
 * orthogonal; D3Q27 adds H_xyz.  Each basis polynomial is a signed sum of
 * H_abc; its coefficient for a symmetric tensor T is the same signed sum of
 * the T_abc.  The norms are computed from the lattice.
 */
#define ORC_NB3 7
static const int B3_TERMS[ORC_NB3][2][3] = {
    /* (first term indices), (second term indices); sign from B3_SIGN */
    {{0, 0, 1}, {1, 2, 2}}, {{0, 0, 1}, {1, 2, 2}},   /* H_xxy +- H_yzz */
    {{0, 2, 2}, {0, 1, 1}}, {{0, 2, 2}, {0, 1, 1}},   /* H_xzz +- H_xyy */
    {{1, 1, 2}, {0, 0, 2}}, {{1, 1, 2}, {0, 0, 2}},   /* H_yyz +- H_xxz */
    {{0, 1, 2}, {0, 1, 2}}};                          /* H_xyz (D3Q27)  */
static const double B3_SIGN[ORC_NB3] = {1.0, -1.0, 1.0, -1.0, 1.0, -1.0, 0.0};

static double herm3(const int c[3], const int ix[3]) {
    const double cs2 = 1.0 / 3.0;
    int a = ix[0], b = ix[1], d = ix[2];
    return c[a] * c[b] * c[d] - cs2 * (c[a] * (b == d) + c[b] * (a == d) + c[d] * (a == b));
}

static int basis3_size(int q) { return q == 27 ? 7 : 6; }

static double basis3(int k, const int c[3]) {
    return herm3(c, B3_TERMS[k][0]) + B3_SIGN[k] * herm3(c, B3_TERMS[k][1]);
}

static double basis3_coeff(int k, double T[3][3][3]) {
    const int *a = B3_TERMS[k][0], *b = B3_TERMS[k][1];
    return T[a[0]][a[1]][a[2]] + B3_SIGN[k] * T[b[0]][b[1]][b[2]];
}

/* f_i += w_i sum_k P_k(c_i) coeff_k(T) / <P_k, P_k>_w */
static void add_third_order(const lattice_t *L, double T[3][3][3], double *f) {
    const int nb = basis3_size(L->q);
    for (int k = 0; k < nb; ++k) {
        double nrm = 0.0;
        for (int i = 0; i < L->q; ++i) {
            double p = basis3(k, L->c[i]);
            nrm += L->w[i] * p * p;
        }
        const double a = basis3_coeff(k, T) / nrm;
        for (int i = 0; i < L->q; ++i) f[i] += L->w[i] * basis3(k, L->c[i]) * a;
    }
}

/* Third-order Hermite equilibrium: the second-order one plus the projection
 * of the Maxwellian's third-order coefficient rho u u u. */
static void equilibrium3(const lattice_t *L, double rho, const double u[3], double *feq) {
    equilibrium(L, rho, u, feq);
    double T[3][3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int d = 0; d < 3; ++d) T[a][b][d] = rho * u[a] * u[b] * u[d];
    add_third_order(L, T, feq);
}

void orc_equilibrium3(int q, double rho, const double u[3], double *feq) {
    lattice_t L;
    make_lattice(q, &L);
    equilibrium3(&L, rho, u, feq);
}

void orc_equilibrium(int q, double rho, const double u[3], double *feq) {
    lattice_t L;
    make_lattice(q, &L);
    equilibrium(&L, rho, u, feq);
}

/* --------------------------------------------------------------- MLP closure */
/*
 * Packed parameter vector (floats): W1[32][7], b1[32], W2[32][32], b2[32],
 * W3[32], b3, mean[7], std[7]  (1359 values).  Inputs are the six
 * non-equilibrium stress moments (xx,yy,zz,xy,xz,yz) and rho, z-scored with
 * mean/std in FP32 (x - mean times the FP32 reciprocal of std).  Hidden
 * layers use ReLU; the output passes through softplus and is scaled by the
 * molecular viscosity nu0, giving the eddy viscosity.
 * Inputs, weights and hidden activations are rounded to bfloat16 (round to
 * nearest, ties to even) before each product, as the device does; sums are
 * FP64 here.  Biases stay FP32.
 */
static double bf16_round(double v) {
    float f = (float)v;
    uint32_t b;
    memcpy(&b, &f, 4);
    if ((b & 0x7f800000u) == 0x7f800000u) return (double)f; /* inf/nan as is */
    uint32_t lsb = (b >> 16) & 1u;
    b += 0x7fffu + lsb;
    b &= 0xffff0000u;
    memcpy(&f, &b, 4);
    return (double)f;
}

double orc_bf16(double v) { return bf16_round(v); }

/* Returns nu_t (may be non-finite: caller falls back). */
static double mlp_eddy_viscosity(const float *P, const double feat[7], double nu0) {
    const float *W1 = P, *b1 = P + 224, *W2 = P + 256, *b2 = P + 1280, *W3 = P + 1312;
    const float *b3 = P + 1344, *mean = P + 1345, *sd = P + 1352;
    double x[7], h1[32], h2[32];
    /* z-score in FP32: (x - mean) times the FP32 reciprocal of std */
    for (int k = 0; k < 7; ++k) x[k] = bf16_round(((float)feat[k] - mean[k]) * (1.0f / sd[k]));
    for (int o = 0; o < 32; ++o) {
        double s = 0.0;
        for (int k = 0; k < 7; ++k) s += bf16_round(W1[o * 7 + k]) * x[k];
        s += b1[o];
        h1[o] = bf16_round(s > 0.0 ? s : 0.0);
    }
    for (int o = 0; o < 32; ++o) {
        double s = 0.0;
        for (int k = 0; k < 32; ++k) s += bf16_round(W2[o * 32 + k]) * h1[k];
        s += b2[o];
        h2[o] = bf16_round(s > 0.0 ? s : 0.0);
    }
    double z = 0.0;
    for (int k = 0; k < 32; ++k) z += bf16_round(W3[k]) * h2[k];
    z += b3[0];
    double sp = z > 30.0 ? z : log1p(exp(z));
    return nu0 * sp;
}

double orc_mlp_eddy_viscosity(const float *P, const double feat[7], double nu0) {
    return mlp_eddy_viscosity(P, feat, nu0);
}

/* ---------------------------------------------------------------- collision */
/*
 * Collide one fluid node: fin -> fout (post-collision, pre-streaming).
 * Macroscopic velocity carries half the force (Guo): u = (sum c f + F/2)/rho.
 */
static void collide_node(const orc_config *cfg, const lattice_t *L, int tag,
                         const double *fin, double *fout, double *nu_t_out) {
    const int q = L->q;
    const double *F = cfg->force;
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < q; ++i) {
        rho += fin[i];
        for (int a = 0; a < 3; ++a) j[a] += L->c[i][a] * fin[i];
    }
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * F[a]) / rho;
    double feq[ORC_MAXQ];
    equilibrium(L, rho, u, feq);

    /* Guo source, split in its even and odd parts under c -> -c. */
    double Fev[ORC_MAXQ], Fod[ORC_MAXQ];
    double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    for (int i = 0; i < q; ++i) {
        double cu = L->c[i][0] * u[0] + L->c[i][1] * u[1] + L->c[i][2] * u[2];
        double cF = L->c[i][0] * F[0] + L->c[i][1] * F[1] + L->c[i][2] * F[2];
        Fev[i] = L->w[i] * (9.0 * cu * cF - 3.0 * uF);
        Fod[i] = L->w[i] * 3.0 * cF;
    }

    if (cfg->flags & 1) { /* free streaming: no collision */
        for (int i = 0; i < q; ++i) fout[i] = fin[i];
        return;
    }

    if (tag >= T_VIN && tag <= T_VOUT) {
        /* Open boundary on an x plane.  On the x = 0 plane the populations with
         * c_x = +1 come from outside, on the x = nx-1 plane those with c_x = -1.
         * Mass and x-momentum over the known populations give, with s = -1 at
         * x = 0 and s = +1 at x = nx-1,
         *   rho (1 + s u_x) = sum_{c_x=0} f + 2 sum_{c_x=s} f = K,
         * so a velocity boundary (u imposed) has rho = K / (1 + s u_x) and a
         * pressure boundary (rho imposed, u_y = u_z = 0) has u_x = s (K/rho - 1). */
        const int low = tag == T_VIN || tag == T_PIN;   /* the x = 0 plane */
        const int vel = tag == T_VIN || tag == T_VOUT;  /* velocity imposed */
        const double sg = low ? -1.0 : 1.0;
        double s0 = 0.0, sp = 0.0, sm = 0.0;
        for (int i = 0; i < q; ++i) {
            if (L->c[i][0] == 0) s0 += fin[i];
            else if (L->c[i][0] > 0) sp += fin[i];
            else sm += fin[i];
        }
        const double K = s0 + 2.0 * (low ? sm : sp);
        double rb, ub[3];
        if (vel) {
            for (int a = 0; a < 3; ++a) ub[a] = cfg->bc_u[a];
            rb = K / (1.0 + sg * ub[0]);
        } else {
            rb = cfg->bc_rho[low ? 0 : 1];
            ub[0] = sg * (K / rb - 1.0);
            ub[1] = ub[2] = 0.0;
        }
        double fb[ORC_MAXQ], fe[ORC_MAXQ];
        equilibrium(L, rb, ub, fe);
        for (int i = 0; i < q; ++i) {
            const int unknown = low ? L->c[i][0] > 0 : L->c[i][0] < 0;
            /* unknown: equilibrium plus the opposite population's non-equilibrium part */
            fb[i] = unknown ? fe[i] + (fin[L->opp[i]] - fe[L->opp[i]]) : fin[i];
        }
        /* regularize the completed node, then relax (BGK; its non-equilibrium
         * part is even in c, so a TRT node relaxes the same way) */
        double Pi[3][3] = {{0}};
        for (int i = 0; i < q; ++i) {
            double d = fb[i] - fe[i];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) Pi[a][b] += L->c[i][a] * L->c[i][b] * d;
        }
        const double cs2 = 1.0 / 3.0;
        for (int i = 0; i < q; ++i) {
            double qpi = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    qpi += (L->c[i][a] * L->c[i][b] - (a == b ? cs2 : 0.0)) * Pi[a][b];
            fout[i] = fe[i] + (1.0 - 1.0 / cfg->tau) * L->w[i] / (2.0 * cs2 * cs2) * qpi;
        }
        return;
    }

    double tau = cfg->tau;
    if (tag == T_SMAG || tag == T_MLP) {
        /* Non-equilibrium momentum flux Pi_ab = sum c_a c_b (f - feq). */
        double Pi[3][3] = {{0}};
        for (int i = 0; i < q; ++i) {
            double d = fin[i] - feq[i];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) Pi[a][b] += L->c[i][a] * L->c[i][b] * d;
        }
        double Qn = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Qn += Pi[a][b] * Pi[a][b];
        Qn = sqrt(Qn);
        /* Implicit Smagorinsky: tau_eff solves tau^2 - tau0 tau - (9 sqrt2/2) Cs^2 Q/rho = 0. */
        double cs2 = cfg->smag_cs * cfg->smag_cs;
        double tau_smag = 0.5 * (tau + sqrt(tau * tau + 18.0 * sqrt(2.0) * cs2 * Qn / rho));
        double tau_eff = tau_smag;
        if (tag == T_MLP && cfg->mlp) {
            double nu0 = (tau - 0.5) / 3.0;
            double feat[7] = {Pi[0][0], Pi[1][1], Pi[2][2], Pi[0][1], Pi[0][2], Pi[1][2], rho};
            double nut = mlp_eddy_viscosity(cfg->mlp, feat, nu0);
            if (isfinite(nut) && nut <= 10.0 * nu0) tau_eff = 3.0 * (nu0 + nut) + 0.5;
            if (nu_t_out) *nu_t_out = (tau_eff - 0.5) / 3.0 - nu0;
        } else if (nu_t_out) {
            *nu_t_out = (tau_eff - tau) / 3.0;
        }
        tau = tau_eff;
    }

    if (tag == T_RR) {
        /* Recursive regularized collision with Guo forcing.  As for T_REG the
         * populations read f = feq + f1 - F_i/2 with the momentum flux of f1
         *   Pi1 = sum c c (f - feq3) + (u F + F u)/2
         * (feq3 has the same moments up to second order as feq).  After the
         * collision the second-order non-equilibrium coefficient is
         *   A2 = (1 - 1/tau) dev(Pi1)            (trace relaxed with 1),
         * the third-order one follows recursively,
         *   A3_abc = u_a A2_bc + u_b A2_ac + u_c A2_ab,
         * and f*_i = feq3_i + w_i [Q_i:A2 / (2 cs^4) + third-order projection
         * of A3] + F_i / 2. */
        double fe3[ORC_MAXQ];
        equilibrium3(L, rho, u, fe3);
        double Pi1[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Pi1[a][b] = 0.5 * (u[a] * F[b] + F[a] * u[b]);
        for (int i = 0; i < q; ++i) {
            double d = fin[i] - fe3[i];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) Pi1[a][b] += L->c[i][a] * L->c[i][b] * d;
        }
        const double tr3 = (Pi1[0][0] + Pi1[1][1] + Pi1[2][2]) / 3.0;
        double A2[3][3], A3[3][3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) A2[a][b] = (1.0 - 1.0 / tau) * (Pi1[a][b] - (a == b ? tr3 : 0.0));
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int d = 0; d < 3; ++d) A3[a][b][d] = u[a] * A2[b][d] + u[b] * A2[a][d] + u[d] * A2[a][b];
        const double cs2 = 1.0 / 3.0;
        for (int i = 0; i < q; ++i) {
            double qa = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    qa += (L->c[i][a] * L->c[i][b] - (a == b ? cs2 : 0.0)) * A2[a][b];
            fout[i] = fe3[i] + L->w[i] / (2.0 * cs2 * cs2) * qa + 0.5 * (Fev[i] + Fod[i]);
        }
        add_third_order(L, A3, fout);
    } else if (tag == T_REG) {
        /* Regularized BGK.  With Guo forcing the populations read
         *   f = feq + f1 - F_i/2,
         * f1 the first-order (Chapman-Enskog) non-equilibrium part, whose
         * second moment is Pi1 = sum c c (f - feq) + (u F + F u)/2.  The
         * regularization keeps only the second-order Hermite projection of f1,
         *   f1_i = w_i / (2 cs^4) (c_i c_i - cs^2 I) : Pi1   (cs^2 = 1/3),
         * and BGK with the Guo source on f = feq + f1 - F_i/2 gives
         *   f*_i = feq_i + (1 - 1/tau) f1_i + F_i/2. */
        double Pi1[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Pi1[a][b] = 0.5 * (u[a] * F[b] + F[a] * u[b]);
        for (int i = 0; i < q; ++i) {
            double d = fin[i] - feq[i];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) Pi1[a][b] += L->c[i][a] * L->c[i][b] * d;
        }
        const double cs2 = 1.0 / 3.0;
        for (int i = 0; i < q; ++i) {
            double qpi = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    qpi += (L->c[i][a] * L->c[i][b] - (a == b ? cs2 : 0.0)) * Pi1[a][b];
            double f1 = L->w[i] / (2.0 * cs2 * cs2) * qpi;
            fout[i] = feq[i] + (1.0 - 1.0 / tau) * f1 + 0.5 * (Fev[i] + Fod[i]);
        }
    } else if (tag == T_TRT) {
        double wp = 1.0 / tau;
        double taum = 0.5 + cfg->trt_lambda / (tau - 0.5);
        double wm = 1.0 / taum;
        for (int i = 0; i < q; ++i) {
            int o = L->opp[i];
            double fp = 0.5 * (fin[i] + fin[o]), fm = 0.5 * (fin[i] - fin[o]);
            double ep = 0.5 * (feq[i] + feq[o]), em = 0.5 * (feq[i] - feq[o]);
            fout[i] = fin[i] - wp * (fp - ep) - wm * (fm - em)
                      + (1.0 - 0.5 * wp) * Fev[i] + (1.0 - 0.5 * wm) * Fod[i];
        }
    } else {
        double w = 1.0 / tau;
        for (int i = 0; i < q; ++i)
            fout[i] = fin[i] - w * (fin[i] - feq[i]) + (1.0 - 0.5 * w) * (Fev[i] + Fod[i]);
    }
}

/* Post-collision populations of a single node (unit tests of the operators). */
int orc_collide_node(const orc_config *cfg, int tag, const double *fin, double *fout, double *nu_t) {
    lattice_t L;
    make_lattice(cfg->q, &L);
    if (!is_fluid(tag)) return -1;
    collide_node(cfg, &L, tag, fin, fout, nu_t);
    return 0;
}

/* ------------------------------------------------------------- time stepping */
static int64_t wrap(int64_t v, int64_t n) { return (v % n + n) % n; }

/*
 * Equilibrium initialisation of the fluid nodes from rho, u (either may be
 * NULL: rho0, resp. rest).  u is SoA: u[a*N + cell].  Non-fluid nodes are
 * set to zero (they carry no populations).
 */
void orc_init(const orc_config *cfg, const uint8_t *tags, const double *rho,
              const double *u, double *f) {
    lattice_t L;
    make_lattice(cfg->q, &L);
    int64_t N = (int64_t)cfg->nx * cfg->ny * cfg->nz;
    for (int64_t n = 0; n < N; ++n) {
        double feq[ORC_MAXQ];
        if (is_fluid(tags[n])) {
            double r = rho ? rho[n] : cfg->rho0;
            double v[3] = {u ? u[n] : 0.0, u ? u[N + n] : 0.0, u ? u[2 * N + n] : 0.0};
            equilibrium(&L, r, v, feq);
        } else {
            for (int i = 0; i < L.q; ++i) feq[i] = 0.0;
        }
        for (int i = 0; i < L.q; ++i) f[(int64_t)i * N + n] = feq[i];
    }
}

/*
 * Advance n_steps time steps of collide + push-stream, in place in f
 * (a second buffer is allocated internally).  Every axis is periodic;
 * walls are explicit non-fluid tags.  For a fluid node x and direction i
 * with y = x + c_i:
 *   y fluid     : g_i(y)    = f*_i(x)
 *   y non-fluid : g_opp(i)(x) = f*_i(x) - 6 w_i rho0 (c_i . u_wall(y))
 * Returns 0, or -1 on bad input, -2 on allocation failure.
 */
int orc_run(const orc_config *cfg, const uint8_t *tags, double *f, int64_t n_steps) {
    lattice_t L;
    if (cfg->q != 19 && cfg->q != 27) return -1;
    make_lattice(cfg->q, &L);
    const int64_t nx = cfg->nx, ny = cfg->ny, nz = cfg->nz, N = nx * ny * nz;
    const int q = L.q;
    double *g = (double *)malloc(sizeof(double) * (size_t)q * (size_t)N);
    if (!g) return -2;
    /* non-fluid nodes are never written: carry their values along */
    memcpy(g, f, sizeof(double) * (size_t)q * (size_t)N);
    double *src = f, *dst = g;
    for (int64_t s = 0; s < n_steps; ++s) {
#pragma omp parallel for schedule(static)
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    int64_t n = (z * ny + y) * nx + x;
                    int tag = tags[n];
                    if (!is_fluid(tag)) continue;
                    double fin[ORC_MAXQ], fo[ORC_MAXQ];
                    for (int i = 0; i < q; ++i) fin[i] = src[(int64_t)i * N + n];
                    collide_node(cfg, &L, tag, fin, fo, NULL);
                    for (int i = 0; i < q; ++i) {
                        int64_t xx = wrap(x + L.c[i][0], nx), yy = wrap(y + L.c[i][1], ny);
                        int64_t zz = wrap(z + L.c[i][2], nz);
                        int64_t m = (zz * ny + yy) * nx + xx;
                        int t2 = tags[m];
                        if (is_fluid(t2)) {
                            dst[(int64_t)i * N + m] = fo[i];
                        } else {
                            double cu = 0.0;
                            if (t2 >= T_WALL0 && t2 < T_WALL0 + 16)
                                for (int a = 0; a < 3; ++a) cu += L.c[i][a] * cfg->wall_u[t2 - T_WALL0][a];
                            dst[(int64_t)L.opp[i] * N + n] = fo[i] - 6.0 * L.w[i] * cfg->rho0 * cu;
                        }
                    }
                }
        double *t = src; src = dst; dst = t;
    }
    if (src != f) memcpy(f, src, sizeof(double) * (size_t)q * (size_t)N);
    free(g);
    return 0;
}

/* --------------------------------------------------------------- reductions */
/* Neumaier compensated summation. */
typedef struct { double s, c; } nsum_t;
static void nadd(nsum_t *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static double nval(const nsum_t *a) { return a->s + a->c; }

/*
 * Domain reductions over fluid nodes of the state f (time t, pre-collision):
 * out[0] = sum (rho - rho0)           out[1..3] = sum (j + F/2) = sum rho u
 * out[4..6] = sum u                   out[7] = sum |u|^2 / 2   (Eq. 5 kernel)
 * out[8] = sum rho |u|^2 / 2          out[9] = count of nodes with non-finite rho or u
 * out[10] = number of fluid nodes
 */
void orc_moments(const orc_config *cfg, const uint8_t *tags, const double *f, double *out) {
    lattice_t L;
    make_lattice(cfg->q, &L);
    const int64_t N = (int64_t)cfg->nx * cfg->ny * cfg->nz;
    nsum_t acc[9];
    memset(acc, 0, sizeof acc);
    double bad = 0.0, nf = 0.0;
    for (int64_t n = 0; n < N; ++n) {
        if (!is_fluid(tags[n])) continue;
        nf += 1.0;
        double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < L.q; ++i) {
            double v = f[(int64_t)i * N + n];
            rho += v;
            for (int a = 0; a < 3; ++a) j[a] += L.c[i][a] * v;
        }
        double ju[3], u[3];
        for (int a = 0; a < 3; ++a) {
            ju[a] = j[a] + 0.5 * cfg->force[a];
            u[a] = ju[a] / rho;
        }
        double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        if (!isfinite(rho) || !isfinite(uu)) { bad += 1.0; continue; }
        nadd(&acc[0], rho - cfg->rho0);
        for (int a = 0; a < 3; ++a) { nadd(&acc[1 + a], ju[a]); nadd(&acc[4 + a], u[a]); }
        nadd(&acc[7], 0.5 * uu);
        nadd(&acc[8], 0.5 * rho * uu);
    }
    for (int k = 0; k < 9; ++k) out[k] = nval(&acc[k]);
    out[9] = bad;
    out[10] = nf;
}

/* Density and velocity per node (non-fluid nodes: rho = 0, u = 0). */
void orc_fields(const orc_config *cfg, const uint8_t *tags, const double *f, double *rho, double *u) {
    lattice_t L;
    make_lattice(cfg->q, &L);
    const int64_t N = (int64_t)cfg->nx * cfg->ny * cfg->nz;
    for (int64_t n = 0; n < N; ++n) {
        double r = 0.0, j[3] = {0.0, 0.0, 0.0};
        if (is_fluid(tags[n]))
            for (int i = 0; i < L.q; ++i) {
                double v = f[(int64_t)i * N + n];
                r += v;
                for (int a = 0; a < 3; ++a) j[a] += L.c[i][a] * v;
            }
        rho[n] = r;
        for (int a = 0; a < 3; ++a) u[(int64_t)a * N + n] = r != 0.0 ? (j[a] + 0.5 * cfg->force[a]) / r : 0.0;
    }
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of threads later runs use (timing of the CPU baseline). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
