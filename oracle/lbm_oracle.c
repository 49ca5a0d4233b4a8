/*
 * Plain FP64 CPU oracle of one D3Q19 MRT pseudopotential time step.
 *
 * TEST INFRASTRUCTURE ONLY: called from tests/, the smoke check and the
 * CPU-baseline leg of the benchmark.  It shares no code with the HIP library.
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 *
 * State convention: f[a*N + (z*ny + y)*nx + x] holds fbar_a(x, t) after
 * streaming, i.e. the variable of Eq. (3) at the node it belongs to.
 *
 * One step, every node, in the order of Sec. II:
 *   rho = sum_a fbar_a                                   Eq. (6)
 *   psi(rho)  square-root form with the C-S EOS, or exponential
 *                                                        text after Eq. (15), Eq. (58)
 *   ghost-layer density below/above walls                Eq. (57)
 *   F_m = -G psi(x) sum_a w_a psi(x + e_a) e_a,  F = F_m + rho g
 *                                                        Eq. (15)
 *   rho u = sum_a e_a fbar_a + F/2                       Eq. (6)
 *   m = M fbar (dense)                                   Eqs. (4), (12)
 *   m_eq, S: Eqs. (13), (14) with S_4 from Eq. (16) (non-orthogonal model);
 *            M_orth f_eq and M_orth G for the orthogonal comparison model
 *   m* = m - Lambda (m - m_eq) + (I - Lambda/2) S        Eq. (4), Eq. (11)
 *   fbar* = M^-1 m* (dense)                              Eq. (5), Appendix A
 *   stream fbar_a(x + e_a, t+1) = fbar*_a(x, t)          Eq. (5)
 *   with periodic wrap, or half-way bounce-back at z = -1/2 and z = nz - 1/2.
 *
 * The matrices M and M^-1 and the rate vector are inputs: the caller builds
 * them in exact rational arithmetic from the basis of Eqs. (7)-(10).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19

/* Planted mistakes, compiled only into the variant libraries that the tests
 * build to show that the wetting-layer pins detect them (0 = the oracle):
 * 1 halves phi, 2 takes layer 1 for layer 2, 3 takes phi from layer 2,
 * 4 flips the sign of the phi term.  See compute_rho_psi. */
#ifndef ORACLE_PLANT
#define ORACLE_PLANT 0
#endif

/* Eq. (2), columns in order. */
static const int EX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int EY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int EZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

typedef struct {
    int32_t nx, ny, nz;
    int32_t wall_z;    /* 0 periodic in z; 1 half-way bounce-back walls in z */
    int32_t op;        /* 0 non-orthogonal (Eqs. 13, 14, 16); 1 orthogonal */
    int32_t psi_form;  /* 0 square root with C-S EOS; 1 exponential */
    int32_t nthreads;  /* OpenMP threads (<= 0: runtime default) */
    int32_t reserved;
    double G;
    double eos_a, eos_b, eos_R, eos_T; /* absolute temperature */
    double psi0, rho0;                 /* exponential form */
    double sigma;                      /* Eq. (16) */
    double g[3];                       /* body acceleration, force rho*g */
    double tan_wall;                   /* tan(90 deg - theta_a), Eq. (57) */
    double ghost_rho_min;              /* lower clamp of the ghost density */
    double orth_sig_e, orth_sig_eps;   /* op=1: coefficients of the Eq. (16)
                                          term in the e and eps rows */
    double rates[Q];                   /* diagonal of Lambda */
    double M[Q * Q];                   /* M[k*Q + a] */
    double Minv[Q * Q];                /* Minv[a*Q + k] */
    /* Density-dependent kinematic viscosity (a reading: the paper varies
     * nu_V / nu_L in Sec. IV.D without stating the rule).  nu_ratio <= 0 or
     * == 1: the rates above everywhere.  Otherwise nu_L = (1/s - 1/2)/3 with
     * s the rate of the rows in nu_mask, nu_V = nu_ratio nu_L, and at a node
     * of density rho, nu = nu_V + t (nu_L - nu_V) with
     * t = (rho - visc_rho_V) / (visc_rho_L - visc_rho_V) clamped to [0, 1];
     * those rows then relax at 1 / (3 nu + 1/2) (Eq. (54)). */
    int32_t nu_mask;                   /* bit k set: row k relaxes at s_nu */
    int32_t reserved2;
    double nu_ratio, visc_rho_L, visc_rho_V;
    /* Single-phase runs (G = 0) may also have half-way bounce-back walls at
     * x = -1/2, nx - 1/2 and y = -1/2, ny - 1/2 (the lid-driven cavity of
     * Appendix B).  The face y = ny - 1/2 moves with velocity lid_u
     * (tangential): a population reflected there gains
     * -2 w_a lid_rho (e_a . lid_u) / c_s^2, a the direction that hit it. */
    int32_t wall_x, wall_y;
    double lid_u[3];
    double lid_rho;
    /* Orthogonal model, a reading (the paper names the model without printing
     * it): 0 = m_eq = M_orth f_eq and S = M_orth G as above; 1 = the energy-
     * square and pi rows of the equilibrium set to eps_eq = -475/63 rho |u|^2
     * and pi_eq = 0 (the free parameters of the Gram-Schmidt basis chosen for
     * stability), with their source rows S_eps = 2 (-475/63) F.u, S_pi = 0. */
    int32_t orth_meq;
    int32_t reserved3;
} oracle_params;

static int opp_of(int a) {
    for (int b = 0; b < Q; ++b)
        if (EX[b] == -EX[a] && EY[b] == -EY[a] && EZ[b] == -EZ[a]) return b;
    return -1;
}

static inline int64_t wrap(int64_t i, int64_t n) {
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

/* Pseudopotential psi(rho). Square-root form: sqrt(2 (p_EOS - rho c_s^2) / (G c^2))
 * with c = 1, c_s^2 = 1/3 and the Carnahan-Starling p_EOS of Eq. (58). */
double oracle_psi(const oracle_params *p, double rho) {
    if (p->psi_form == 1) return p->psi0 * exp(-p->rho0 / rho);
    double eta = p->eos_b * rho / 4.0;
    double num = 1.0 + eta + eta * eta - eta * eta * eta;
    double den = (1.0 - eta) * (1.0 - eta) * (1.0 - eta);
    double peos = rho * p->eos_R * p->eos_T * num / den - p->eos_a * rho * rho;
    return sqrt(2.0 * (peos - rho / 3.0) / p->G);
}

/* Velocity-space textbook D3Q19 equilibrium and forcing (weights 1/3, 1/18,
 * 1/36); used only to define the orthogonal model's moments. */
static double wq(int a) { return a == 0 ? 1.0 / 3.0 : (a <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

static void meq_of(const oracle_params *p, double rho, const double u[3], double meq[Q]) {
    double ux = u[0], uy = u[1], uz = u[2];
    double u2 = ux * ux + uy * uy + uz * uz;
    if (p->op == 0) {
        /* Eq. (13) */
        double cs2 = 1.0 / 3.0;
        double phi = rho * cs2 * cs2 * (1.0 - 1.5 * u2);
        meq[0] = rho;
        meq[1] = rho * ux;
        meq[2] = rho * uy;
        meq[3] = rho * uz;
        meq[4] = rho + rho * u2;
        meq[5] = rho * (2.0 * ux * ux - uy * uy - uz * uz);
        meq[6] = rho * (uy * uy - uz * uz);
        meq[7] = rho * ux * uy;
        meq[8] = rho * ux * uz;
        meq[9] = rho * uy * uz;
        meq[10] = rho * cs2 * uy;
        meq[11] = rho * cs2 * ux;
        meq[12] = rho * cs2 * uz;
        meq[13] = rho * cs2 * ux;
        meq[14] = rho * cs2 * uz;
        meq[15] = rho * cs2 * uy;
        meq[16] = phi + rho * cs2 * (ux * ux + uy * uy);
        meq[17] = phi + rho * cs2 * (ux * ux + uz * uz);
        meq[18] = phi + rho * cs2 * (uy * uy + uz * uz);
    } else {
        double feq[Q];
        for (int a = 0; a < Q; ++a) {
            double eu = EX[a] * ux + EY[a] * uy + EZ[a] * uz;
            feq[a] = wq(a) * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * u2);
        }
        for (int k = 0; k < Q; ++k) {
            double s = 0.0;
            for (int a = 0; a < Q; ++a) s += p->M[k * Q + a] * feq[a];
            meq[k] = s;
        }
        if (p->orth_meq == 1) {
            meq[2] = -475.0 / 63.0 * rho * u2; /* eps */
            meq[10] = 0.0;                     /* 3 pi_xx */
            meq[12] = 0.0;                     /* pi_ww */
        }
    }
}

/* Forcing moments. Fm2_over_psi2 = |F_m|^2 / psi^2 for Eq. (16). */
static void source_of(const oracle_params *p, const double u[3], const double F[3],
                      double Fm2_over_psi2, double S[Q]) {
    double ux = u[0], uy = u[1], uz = u[2];
    double Fx = F[0], Fy = F[1], Fz = F[2];
    double Fu = Fx * ux + Fy * uy + Fz * uz;
    if (p->op == 0) {
        /* Eq. (14), with the fifth entry replaced by Eq. (16) */
        double cs2 = 1.0 / 3.0;
        S[0] = 0.0;
        S[1] = Fx;
        S[2] = Fy;
        S[3] = Fz;
        S[4] = 2.0 * Fu + 6.0 * p->sigma * Fm2_over_psi2 / (1.0 / p->rates[4] - 0.5);
        S[5] = 2.0 * (2.0 * Fx * ux - Fy * uy - Fz * uz);
        S[6] = 2.0 * (Fy * uy - Fz * uz);
        S[7] = Fx * uy + Fy * ux;
        S[8] = Fx * uz + Fz * ux;
        S[9] = Fy * uz + Fz * uy;
        S[10] = cs2 * Fy;
        S[11] = cs2 * Fx;
        S[12] = cs2 * Fz;
        S[13] = cs2 * Fx;
        S[14] = cs2 * Fz;
        S[15] = cs2 * Fy;
        S[16] = 2.0 * cs2 * (ux * Fx + uy * Fy);
        S[17] = 2.0 * cs2 * (ux * Fx + uz * Fz);
        S[18] = 2.0 * cs2 * (uy * Fy + uz * Fz);
    } else {
        double G[Q];
        for (int a = 0; a < Q; ++a) {
            double eu = EX[a] * ux + EY[a] * uy + EZ[a] * uz;
            double eF = EX[a] * Fx + EY[a] * Fy + EZ[a] * Fz;
            G[a] = wq(a) * (3.0 * (eF - Fu) + 9.0 * eu * eF);
        }
        for (int k = 0; k < Q; ++k) {
            double s = 0.0;
            for (int a = 0; a < Q; ++a) s += p->M[k * Q + a] * G[a];
            S[k] = s;
        }
        if (p->orth_meq == 1) {
            S[2] = 2.0 * (-475.0 / 63.0) * Fu;
            S[10] = 0.0;
            S[12] = 0.0;
        }
        double c = 6.0 * p->sigma * Fm2_over_psi2;
        S[1] += p->orth_sig_e * c / (1.0 / p->rates[1] - 0.5);
        S[2] += p->orth_sig_eps * c / (1.0 / p->rates[2] - 0.5);
    }
}

/* Interaction-force weights of Eq. (15). */
static double wforce(int a) { return a == 0 ? 0.0 : (a <= 6 ? 1.0 / 6.0 : 1.0 / 12.0); }

typedef struct {
    double *rho;   /* N */
    double *psi;   /* N */
    double *gpsi;  /* 2 * nx * ny ghost psi: [0] below z=0, [1] above z=nz-1 */
} fields_t;

static void compute_rho_psi(const oracle_params *p, const double *f, fields_t *w) {
    const int64_t nx = p->nx, ny = p->ny, nz = p->nz, N = nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double r = 0.0;
        for (int a = 0; a < Q; ++a) r += f[a * N + i];
        w->rho[i] = r;
        w->psi[i] = oracle_psi(p, r);
    }
    if (p->wall_z) {
        /* Eq. (57): ghost density = density two layers away plus phi tan(90-theta),
         * phi the magnitude of the in-plane central difference in the first layer. */
        for (int side = 0; side < 2; ++side) {
            int64_t z1 = side == 0 ? 0 : nz - 1;
            int64_t z2 = side == 0 ? 1 : nz - 2;
#if ORACLE_PLANT == 2
            z2 = z1;
#endif
            int64_t zphi = z1;
#if ORACLE_PLANT == 3
            zphi = z2;
#endif
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    double dx = w->rho[(zphi * ny + y) * nx + wrap(x + 1, nx)] -
                                w->rho[(zphi * ny + y) * nx + wrap(x - 1, nx)];
                    double dy = w->rho[(zphi * ny + wrap(y + 1, ny)) * nx + x] -
                                w->rho[(zphi * ny + wrap(y - 1, ny)) * nx + x];
                    double phi = sqrt(dx * dx + dy * dy);
#if ORACLE_PLANT == 1
                    phi *= 0.5;
#elif ORACLE_PLANT == 4
                    phi = -phi;
#endif
                    double rg = w->rho[(z2 * ny + y) * nx + x] + phi * p->tan_wall;
                    if (rg < p->ghost_rho_min) rg = p->ghost_rho_min;
                    w->gpsi[side * nx * ny + y * nx + x] = oracle_psi(p, rg);
                }
        }
    }
}

/* psi at (x, y, z) with z possibly one layer outside a walled domain. */
static double psi_at(const oracle_params *p, const fields_t *w, int64_t x, int64_t y, int64_t z) {
    const int64_t nx = p->nx, ny = p->ny, nz = p->nz;
    x = wrap(x, nx);
    y = wrap(y, ny);
    if (p->wall_z) {
        if (z < 0) return w->gpsi[y * nx + x];
        if (z >= nz) return w->gpsi[nx * ny + y * nx + x];
    } else {
        z = wrap(z, nz);
    }
    return w->psi[(z * ny + y) * nx + x];
}

/* Relaxation rates at a node of density rho (see nu_ratio above). */
static void local_rates(const oracle_params *p, double rho, double r[Q]) {
    for (int k = 0; k < Q; ++k) r[k] = p->rates[k];
    if (p->nu_ratio <= 0.0 || p->nu_ratio == 1.0) return;
    int k0 = -1;
    for (int k = 0; k < Q; ++k)
        if (p->nu_mask & (1 << k)) {
            k0 = k;
            break;
        }
    if (k0 < 0) return;
    const double nu_L = (1.0 / p->rates[k0] - 0.5) / 3.0;
    const double nu_V = p->nu_ratio * nu_L;
    double t = (rho - p->visc_rho_V) / (p->visc_rho_L - p->visc_rho_V);
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    const double nu = nu_V + t * (nu_L - nu_V);
    const double s = 1.0 / (3.0 * nu + 0.5);
    for (int k = 0; k < Q; ++k)
        if (p->nu_mask & (1 << k)) r[k] = s;
}

/* Collision at one node: fin[19] -> fout[19]; optional macroscopic outputs. */
static void collide_node(const oracle_params *p, const fields_t *w, int64_t x, int64_t y, int64_t z,
                         const double fin[Q], double fout[Q], double *u_out, double *F_out) {
    const int64_t nx = p->nx, ny = p->ny;
    int64_t i = (z * ny + y) * nx + x;
    double rho = w->rho[i];
    double psi = w->psi[i];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int a = 1; a < Q; ++a) {
        double pn = psi_at(p, w, x + EX[a], y + EY[a], z + EZ[a]);
        acc[0] += wforce(a) * pn * EX[a];
        acc[1] += wforce(a) * pn * EY[a];
        acc[2] += wforce(a) * pn * EZ[a];
    }
    double Fm[3], F[3];
    for (int d = 0; d < 3; ++d) {
        Fm[d] = -p->G * psi * acc[d];
        F[d] = Fm[d] + rho * p->g[d];
    }
    double Fm2 = Fm[0] * Fm[0] + Fm[1] * Fm[1] + Fm[2] * Fm[2];
    double Fm2_over_psi2 = Fm2 == 0.0 ? 0.0 : Fm2 / (psi * psi);
    double j[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < Q; ++a) {
        j[0] += EX[a] * fin[a];
        j[1] += EY[a] * fin[a];
        j[2] += EZ[a] * fin[a];
    }
    double u[3];
    for (int d = 0; d < 3; ++d) u[d] = (j[d] + 0.5 * F[d]) / rho;
    double m[Q], meq[Q], S[Q], ms[Q];
    for (int k = 0; k < Q; ++k) {
        double s = 0.0;
        for (int a = 0; a < Q; ++a) s += p->M[k * Q + a] * fin[a];
        m[k] = s;
    }
    meq_of(p, rho, u, meq);
    source_of(p, u, F, Fm2_over_psi2, S);
    double r[Q];
    local_rates(p, rho, r);
    for (int k = 0; k < Q; ++k)
        ms[k] = m[k] - r[k] * (m[k] - meq[k]) + (1.0 - 0.5 * r[k]) * S[k];
    for (int a = 0; a < Q; ++a) {
        double s = 0.0;
        for (int k = 0; k < Q; ++k) s += p->Minv[a * Q + k] * ms[k];
        fout[a] = s;
    }
    if (u_out) memcpy(u_out, u, sizeof(u));
    if (F_out) memcpy(F_out, F, sizeof(F));
}

static int alloc_fields(const oracle_params *p, fields_t *w) {
    int64_t N = (int64_t)p->nx * p->ny * p->nz;
    w->rho = (double *)malloc(sizeof(double) * N);
    w->psi = (double *)malloc(sizeof(double) * N);
    w->gpsi = (double *)malloc(sizeof(double) * 2 * p->nx * p->ny);
    if (!w->rho || !w->psi || !w->gpsi) return -1;
    return 0;
}

static void free_fields(fields_t *w) {
    free(w->rho);
    free(w->psi);
    free(w->gpsi);
}

static int check_params(const oracle_params *p) {
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return -1;
    if (p->wall_z && p->nz < 2) return -1;
    if ((p->wall_x || p->wall_y) && p->G != 0.0) return -1;
    return 0;
}

/* Weight of direction a in the equilibrium's part linear in u: 1/18 axis,
 * 1/36 diagonal (as in the rest state). */
static double wlin(int a) { return a == 0 ? 1.0 / 3.0 : (a <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

#ifdef _OPENMP
#include <omp.h>
static void set_threads(const oracle_params *p) {
    if (p->nthreads > 0) omp_set_num_threads(p->nthreads);
}
#else
static void set_threads(const oracle_params *p) { (void)p; }
#endif

/* nsteps full steps; fin is not modified; fout receives the state after. */
int oracle_step(const oracle_params *p, const double *fin, double *fout, int64_t nsteps) {
    if (check_params(p)) return -1;
    set_threads(p);
    const int64_t nx = p->nx, ny = p->ny, nz = p->nz, N = nx * ny * nz;
    fields_t w;
    if (alloc_fields(p, &w)) return -2;
    double *cur = (double *)malloc(sizeof(double) * Q * N);
    if (!cur) return -2;
    memcpy(cur, fin, sizeof(double) * Q * N);
    int opp[Q];
    for (int a = 0; a < Q; ++a) opp[a] = opp_of(a);
    for (int64_t s = 0; s < nsteps; ++s) {
        compute_rho_psi(p, cur, &w);
#pragma omp parallel for schedule(static)
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    int64_t i = (z * ny + y) * nx + x;
                    double fin_n[Q], fo[Q];
                    for (int a = 0; a < Q; ++a) fin_n[a] = cur[a * N + i];
                    collide_node(p, &w, x, y, z, fin_n, fo, NULL, NULL);
                    /* Eq. (5): streaming to x + e_a; half-way bounce-back when the
                     * target lies beyond a wall, with the moving-lid term when
                     * the wall crossed includes the face y = ny - 1/2. */
                    for (int a = 0; a < Q; ++a) {
                        int64_t tx = x + EX[a], ty = y + EY[a], tz = z + EZ[a];
                        int out_x = p->wall_x && (tx < 0 || tx >= nx);
                        int out_y = p->wall_y && (ty < 0 || ty >= ny);
                        int out_z = p->wall_z && (tz < 0 || tz >= nz);
                        if (out_x || out_y || out_z) {
                            double v = fo[a];
                            if (p->wall_y && ty >= ny) {
                                double eu = EX[a] * p->lid_u[0] + EY[a] * p->lid_u[1] + EZ[a] * p->lid_u[2];
                                v -= 2.0 * wlin(a) * p->lid_rho * eu * 3.0;
                            }
                            fout[opp[a] * N + i] = v;
                        } else {
                            int64_t t = (wrap(tz, nz) * ny + wrap(ty, ny)) * nx + wrap(tx, nx);
                            fout[a * N + t] = fo[a];
                        }
                    }
                }
        memcpy(cur, fout, sizeof(double) * Q * N);
    }
    if (nsteps == 0) memcpy(fout, fin, sizeof(double) * Q * N);
    free(cur);
    free_fields(&w);
    return 0;
}

/* Post-collision values fbar*(x, t) at the listed nodes, computed from the
 * full state at t: the building block for sampled checks on large lattices.
 * out[n*Q + a] for node idx[n]. */
int oracle_collide_nodes(const oracle_params *p, const double *f, int64_t count,
                         const int64_t *idx, double *out) {
    if (check_params(p)) return -1;
    set_threads(p);
    const int64_t nx = p->nx, ny = p->ny, N = (int64_t)p->nx * p->ny * p->nz;
    fields_t w;
    if (alloc_fields(p, &w)) return -2;
    compute_rho_psi(p, f, &w);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < count; ++n) {
        int64_t i = idx[n];
        int64_t x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
        double fin_n[Q];
        for (int a = 0; a < Q; ++a) fin_n[a] = f[a * N + i];
        collide_node(p, &w, x, y, z, fin_n, out + n * Q, NULL, NULL);
    }
    free_fields(&w);
    return 0;
}

/* fbar = M^-1 m_eq(rho, u) at every node (u given as 3 SoA planes). */
int oracle_equilibrium(const oracle_params *p, const double *rho, const double *u, double *f) {
    if (check_params(p)) return -1;
    set_threads(p);
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double uu[3] = {u[i], u[N + i], u[2 * N + i]};
        double meq[Q];
        meq_of(p, rho[i], uu, meq);
        for (int a = 0; a < Q; ++a) {
            double s = 0.0;
            for (int k = 0; k < Q; ++k) s += p->Minv[a * Q + k] * meq[k];
            f[a * N + i] = s;
        }
    }
    return 0;
}

/* Macroscopic fields of the state f: rho, u (Eq. (6), 3 SoA planes), total
 * force F (3 planes), psi and p = rho c_s^2 + G psi^2 / 2.  Any output may be
 * NULL. */
int oracle_fields(const oracle_params *p, const double *f, double *rho_o, double *u_o,
                  double *F_o, double *psi_o, double *p_o) {
    if (check_params(p)) return -1;
    set_threads(p);
    const int64_t nx = p->nx, ny = p->ny, nz = p->nz, N = nx * ny * nz;
    fields_t w;
    if (alloc_fields(p, &w)) return -2;
    compute_rho_psi(p, f, &w);
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t i = (z * ny + y) * nx + x;
                double fin_n[Q], fo[Q], u[3], F[3];
                for (int a = 0; a < Q; ++a) fin_n[a] = f[a * N + i];
                collide_node(p, &w, x, y, z, fin_n, fo, u, F);
                if (rho_o) rho_o[i] = w.rho[i];
                if (psi_o) psi_o[i] = w.psi[i];
                if (p_o) p_o[i] = w.rho[i] / 3.0 + 0.5 * p->G * w.psi[i] * w.psi[i];
                for (int d = 0; d < 3; ++d) {
                    if (u_o) u_o[d * N + i] = u[d];
                    if (F_o) F_o[d * N + i] = F[d];
                }
            }
    free_fields(&w);
    return 0;
}

/* psi(rho) for an array: lets tests pin the EOS through the Maxwell construction. */
int oracle_psi_array(const oracle_params *p, const double *rho, double *psi, int64_t n) {
    for (int64_t i = 0; i < n; ++i) psi[i] = oracle_psi(p, rho[i]);
    return 0;
}

int oracle_abi_version(void) { return 1; }
