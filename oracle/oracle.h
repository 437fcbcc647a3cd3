/* oracle.h -- plain FP64 CPU reference for one lattice update of the
 * multiphase-multicomponent lattice Boltzmann model for self-diffusiophoretic
 * Janus colloids at liquid-liquid interfaces (Palacios, Scagliarini,
 * Pagonabarraga, arXiv:2202.01631).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no source,
 * header, table or helper with the GPU solver; the two agree only on the
 * public data formats documented below (node numbering, D3Q19 direction
 * numbering, the link record), which are interfaces, not arithmetic.
 *
 * Conventions
 *   node index      n = x + nx*(y + ny*z), periodic box, unit spacing, dt = 1
 *   host arrays     FP64, x-fastest; vector fields are structure-of-arrays
 *                   (component a of node n at a*N + n)
 *   D3Q19 numbering 0:(0,0,0)
 *                   1:(+1,0,0) 2:(-1,0,0) 3:(0,+1,0) 4:(0,-1,0) 5:(0,0,+1) 6:(0,0,-1)
 *                   7:(+1,+1,0) 8:(-1,-1,0) 9:(+1,-1,0) 10:(-1,+1,0)
 *                   11:(+1,0,+1) 12:(-1,0,-1) 13:(+1,0,-1) 14:(-1,0,+1)
 *                   15:(0,+1,+1) 16:(0,-1,-1) 17:(0,+1,-1) 18:(0,-1,+1)
 *                   (odd i >= 1 and i+1 are opposite)
 *   link record     (colloid k, fluid node n, direction d, cap) with node
 *                   n + c_d inside colloid k; cap = 1 on the active hemisphere
 *                   (m.n <= 0), or the pattern cell of the link's midpoint for
 *                   a patterned particle.  Canonical order: (k, n, d) ascending.
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny, nz;
    double rho0, tau;            /* tau = 1 gives nu = 1/6 (Sec. II.C) */
    double a, b, kappa, M_psi;   /* f = a/2 psi^2 + b/4 psi^4 + kappa/2 |grad psi|^2 (Eq. 1) */
    double C, E, c_b0, D_c, k_d; /* C/2 (c - c_b0 - E tanh psi)^2 (Eq. 1); Eq. 3a */
    double ext_force[3];         /* uniform body force on the fluid (tests) */
    uint32_t flags;              /* OR_SOLUTE_FORCE, OR_EXPLICIT_COLLOID, OR_CAPILLARY_FORCE,
                                    OR_STRESS_FORM */
    int32_t ch_substeps;         /* psi/c updates per LB step, time step 1/n each
                                    (mu and chi recomputed between them, u held); 0 -> 1 */
    double soft_eps, soft_sigma, soft_nu, soft_hc;
                                 /* soft-sphere repulsion between particles whose surface
                                    gap h is below soft_hc: each takes nu eps sigma^nu
                                    (h^-(nu+1) - hc^-(nu+1)) along the line of centres,
                                    away from the other (h below 0.01 taken as 0.01);
                                    soft_eps = 0: none */
    double lub_hc;               /* normal lubrication between particles whose surface gap
                                    h is below lub_hc (0: none): each takes -6 pi eta
                                    (a_i a_j/(a_i + a_j))^2 (1/h - 1/lub_hc) U_n along the
                                    line of centres, U_n the approach speed at the start of
                                    the step, eta = rho0 (tau - 1/2)/3 (h below 0.1 taken
                                    as 0.1) */
} or_params;

/* options (readings of what the paper leaves open):
 * OR_SOLUTE_FORCE      the solvent also feels -c grad(mu_c), mu_c = C chi
 *                      (off by default: phoresis enters through the slip)
 * OR_EXPLICIT_COLLOID  explicit rigid-body update M X' = M X + F0 - zeta X
 *                      (Ladd) instead of the implicit one
 * OR_CAPILLARY_FORCE   each particle also receives the thermodynamic stress of
 *                      the psi free energy at its boundary links, the share of
 *                      the interfacial force that the solvent force leaves out
 *                      at the particle surface (capillary and wetting forces)
 * OR_STRESS_FORM       (with OR_CAPILLARY_FORCE) the solvent force of the psi
 *                      free energy in divergence form, -div P, P the stress
 *                      above taken at the fluid nodes and P(x) substituted at
 *                      solid neighbours, plus the coupling part -psi grad(mu_c)
 *                      of Eq. 2: the fluid then loses exactly what the particles
 *                      gain at their links, and the pair conserves momentum */
#define OR_SOLUTE_FORCE 1u
#define OR_EXPLICIT_COLLOID 2u
#define OR_CAPILLARY_FORCE 4u
#define OR_STRESS_FORM 8u

#define OR_PATTERN_MAX_BANDS 8
#define OR_PATTERN_MAX_CELLS 64

typedef struct {
    double pos[3], m[3], vel[3], omega[3];
    double radius, alpha_minus, alpha_plus, mu_minus, mu_plus, H, rho_p;
    int32_t fixed;               /* 1: position, orientation and velocities held */
    double cap_cos;              /* the active cap is m.n <= cap_cos, in [-1, 1]; 0 is the
                                    half of Eqs. 5-6 (the paper's Janus particle) */
    double e[3];                 /* second body axis (made orthogonal to m and normalised
                                    on add; any orthogonal axis if zero); turns with m */
    int32_t pat_bands;           /* surface pattern (0: none, the Janus caps above): polar
                                    bands 1..8 of m.n, cut at pat_cos[0 .. bands-2]
                                    (increasing): band b holds pat_cos[b-1] < m.n <=
                                    pat_cos[b] */
    int32_t pat_sectors;         /* azimuthal sectors 1, 2, 4 or 8 of the angle of n about m,
                                    measured from e towards m x e */
    double pat_cos[OR_PATTERN_MAX_BANDS - 1];
    double pat_alpha[OR_PATTERN_MAX_CELLS], pat_mu[OR_PATTERN_MAX_CELLS],
        pat_H[OR_PATTERN_MAX_CELLS];  /* per cell b * sectors + s: production per link
                                         (Eq. 5), phoretic mobility (Eq. 6) and wetting
                                         parameter (Eqs. 8-9) */
    double axial;                /* shape: semi-axis along m of a spheroid whose other two
                                    semi-axes are `radius` (0, or equal to radius: a
                                    sphere) */
} or_colloid;

typedef struct {
    double mass, mom[3], sum_psi, sum_c;
    int64_t n_fluid, n_links, n_active, step;
    int32_t error_bits;
} or_totals;

/* per-step diagnostics of the last completed step (see or_step_diag) */
enum {
    OR_DIAG_SUM_FORCE = 0,  /* 3: sum over fluid nodes of the body force F(x) */
    OR_DIAG_SUM_SRC = 3,    /* 1: total solute emitted this step */
    OR_DIAG_SUM_CHI = 4,    /* 1: sum over fluid nodes of chi(t) */
    OR_DIAG_SUM_DP = 5,     /* 3: momentum handed to all colloids through links (full u_b) */
    OR_DIAG_SUM_TR = 8,     /* 3: momentum handed to all colloids by cover/uncover */
    OR_DIAG_SUM_DMASS = 11, /* 1: mass change from moving-wall terms and uncovering */
    OR_DIAG_N = 12
};

#define OR_OK 0
#define OR_E_INVALID (-1)
#define OR_E_UNSTABLE (-4)
#define OR_E_STATE (-5)

typedef struct or_ctx or_ctx;

int or_create(const or_params *p, or_ctx **out);
int or_destroy(or_ctx *c);
int or_init_fields(or_ctx *c, const double *psi, const double *cc,
                   const double *rho, const double *u);
int or_add_colloids(or_ctx *c, const or_colloid *cols, int32_t n);
int or_step(or_ctx *c, int64_t nsteps);
int or_get_fields(or_ctx *c, double *rho, double *u, double *psi, double *cc);
int or_get_populations(or_ctx *c, double *f);          /* 19*N, plane-major */
int or_set_populations(or_ctx *c, const double *f);
int or_get_aux(or_ctx *c, double *mu, double *force, double *uforced);
int or_get_owner(or_ctx *c, int32_t *owner);           /* -1 fluid, k solid */
int or_get_links(or_ctx *c, int32_t *rec4, int64_t cap, int64_t *n);
/* slip velocity (Eq. 4) of each link as the last step's link loop used it,
 * 3 per link in link-table order; OR_E_STATE when the table has changed
 * size since (a moving particle), OR_E_INVALID when cap < links */
int or_get_link_slip(or_ctx *c, double *slip3, int64_t cap);
int or_observables(or_ctx *c, or_totals *t, or_colloid *out, int32_t n);
int or_colloid_diag(or_ctx *c, int32_t k, double *out40); /* F0[3] T0[3] zeta[36] -> see .c */
int or_step_diag(or_ctx *c, double *out);              /* OR_DIAG_N doubles */
int or_lattice(int32_t *cvec57, double *w19);
int or_set_threads(int32_t n);                         /* per-node loops; results unchanged */
double or_wetting_H(double theta_deg, double kappa, double b);
/* the flat-wall contact angle this lattice realises: Young's cosine for H,
 * and the H giving theta (NaN unless a < 0 < b, kappa > 0 and theta in range) */
double or_lattice_cos(double a, double b, double kappa, double H);
double or_wetting_H_lattice(double theta_deg, double a, double b, double kappa);
double or_solubility_E(double ratio, double c_b0);
const char *or_last_error(const or_ctx *c);

#ifdef __cplusplus
}
#endif
#endif
