/* lb.h -- C ABI of the MI355X (gfx950) lattice update of the
 * multiphase-multicomponent lattice Boltzmann model for self-diffusiophoretic
 * Janus colloids at liquid-liquid interfaces
 * (Palacios, Scagliarini, Pagonabarraga, arXiv:2202.01631).
 *
 * One context = one periodic box resident in GPU memory.  Each lb_step
 * advances it by one time step of the paper's model (Sec. II, Eqs. 1-10):
 *   1. chemical potential mu_psi of Eq. 2, with the wetting condition of
 *      Eqs. 8-9 as a ghost value at particle faces;
 *   2. D3Q19 BGK collision (tau; nu = (tau-1/2)/3, 1/6 at tau = 1, Sec. II.C)
 *      under the free-energy body force F = -psi grad(mu_psi) with the
 *      forcing term of Guo, Zheng and Shi (2002); push streaming;
 *   3. bounce-back on links with the moving-wall term, the wall velocity
 *      being V + Omega x r plus the phoretic slip of Eq. 4 with the Janus
 *      mobility of Eq. 6; momentum exchange summed per particle (Sec. II.B);
 *   4. explicit updates of psi (Cahn-Hilliard, Eq. 3b) and of the solute c
 *      (advection-diffusion with the sink k_d and the Janus production of
 *      Eq. 5 emitted per active link, Eq. 3a);
 *   5. rigid-body update of every particle, implicit in the link drag;
 *   6. particle geometry at the new positions: cover/uncover repair, owner
 *      map, link table.
 *
 * All functions return an lb_status; no exception crosses the ABI.
 * lb_last_error() gives a message for the last failure on a context.
 *
 * Conventions
 *   node index      n = x + nx*(y + ny*z), periodic box, unit spacing, dt = 1.
 *   host arrays     caller-owned, FP64 whatever the storage precision,
 *                   x-fastest; vector fields are structure-of-arrays
 *                   (component a of node n at a*N + n, N = nx*ny*nz).  The
 *                   library copies in and out and keeps no host pointer.
 *   D3Q19 numbering 0:(0,0,0)
 *                   1:(+1,0,0) 2:(-1,0,0) 3:(0,+1,0) 4:(0,-1,0) 5:(0,0,+1) 6:(0,0,-1)
 *                   7:(+1,+1,0) 8:(-1,-1,0) 9:(+1,-1,0) 10:(-1,+1,0)
 *                   11:(+1,0,+1) 12:(-1,0,-1) 13:(+1,0,-1) 14:(-1,0,+1)
 *                   15:(0,+1,+1) 16:(0,-1,-1) 17:(0,+1,-1) 18:(0,-1,+1)
 *                   (odd i >= 1 and i+1 are opposite); weights 1/3, 1/18, 1/36.
 *   links           (particle k, fluid node n, direction d, cap): node n + c_d
 *                   lies strictly inside particle k; cap = 1 when the link
 *                   midpoint is on the active hemisphere m.n <= 0 (Eqs. 5-6),
 *                   or, for a particle with a surface pattern, the pattern
 *                   cell of the midpoint.  Canonical order (k, n, d) ascending.
 *   device memory   the context owns its device state.  If the caller hands
 *                   in an arena (e.g. a torch uint8 tensor), the context only
 *                   borrows it; it must outlive lb_destroy.
 *   streams         work is enqueued on the stream given to lb_create (NULL:
 *                   the default stream).  One context per stream; no internal
 *                   locking.  Calls that return host data synchronise that
 *                   stream.  Large steps with particles also use a second,
 *                   internal stream of default priority, forked from and
 *                   joined back into the context's stream inside each step,
 *                   so the caller sees plain stream order.  On a non-default
 *                   stream, steps are replayed from captured two-step graphs.
 *   call order      lb_create -> lb_init_fields -> [lb_add_colloids] ->
 *                   lb_step* ; violations return LB_E_STATE.
 */
#ifndef LB_H
#define LB_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LB_OK = 0,
    LB_E_INVALID = -1,  /* bad argument or parameter (incl. stability bounds) */
    LB_E_OOM = -2,      /* device allocation failed or arena too small */
    LB_E_DEVICE = -3,   /* HIP runtime error */
    LB_E_UNSTABLE = -4, /* NaN/Inf seen in the FP64 totals */
    LB_E_STATE = -5     /* call order, particle overlap/contact, link overflow */
} lb_status;

typedef enum {
    LB_FP64 = 0,        /* populations, psi, c and arithmetic in FP64 */
    LB_FP32 = 1,        /* populations stored as f_i - w_i rho0 in FP32, FP32 arithmetic */
    LB_FP16_STORAGE = 2 /* (f_i - w_i rho0) * f16_scale stored in IEEE half, FP32 arithmetic */
} lb_precision;

/* error bits reported in lb_totals.error_bits */
#define LB_ERR_NAN 1        /* non-finite FP64 totals */
#define LB_ERR_FAST 2       /* a particle moved 0.5 or more lattice units in one step */
#define LB_ERR_CONTACT 4    /* two particles claim one node, or touch */
#define LB_ERR_LINKS 8      /* link table of a particle overflowed its capacity */

typedef struct {
    int32_t nx, ny, nz;          /* periodic box; nz <= 65535 and one scalar field
                                    (N nodes x 8 bytes in FP64, x 4 otherwise)
                                    below 4 GiB */
    int32_t precision;           /* lb_precision */
    double rho0, tau;            /* rest density, BGK relaxation time (> 1/2) */
    double a, b, kappa, M_psi;   /* f = a/2 psi^2 + b/4 psi^4 + kappa/2 |grad psi|^2, Eq. 1
                                    (the paper's B = a < 0 < A = b); psi mobility */
    double C, E, c_b0, D_c, k_d; /* C/2 (c - c_b0 - E tanh psi)^2 (Eq. 1); solute
                                    diffusivity D_c (= C M_c) and sink rate (Eq. 3a) */
    double ext_force[3];         /* uniform body force on the fluid (0 in the paper) */
    double f16_scale;            /* FP16 storage scale, a power of two; 0 -> 16384 */
    int32_t max_colloids;        /* particle capacity, <= 127 (owner byte); 0 -> 64 */
    uint32_t flags;              /* options, 0 or a combination of the LB_* bits below */
    int32_t ch_substeps;         /* psi/c updates per LB step, 1..64 (0 -> 1): each takes a
                                    time step 1/n with mu and chi recomputed and u held, so
                                    the explicit stability bounds apply to M_psi/n and
                                    (12 D_c + k_d)/n (the paper's M_psi = 0.4 needs 2) */
    double soft_eps, soft_sigma, soft_nu, soft_hc;
                                 /* soft-sphere repulsion for close encounters (soft_eps = 0:
                                    none; else sigma, nu, hc > 0): two particles of a box
                                    whose surface gap h (minimum image) is below hc each take
                                    nu eps sigma^nu (h^-(nu+1) - hc^-(nu+1)) along the line of
                                    centres, away from the other (h below 0.01 taken as
                                    0.01), from the positions at the start of the step, as
                                    part of F0 (the shifted-force form of the potential
                                    eps (sigma/h)^nu) */
    double lub_hc;               /* normal lubrication between particles whose surface gap
                                    h is below lub_hc (0: none, else > 0): each takes
                                    -6 pi eta (a_i a_j/(a_i + a_j))^2 (1/h - 1/lub_hc) U_n
                                    along the line of centres, U_n the approach speed at the
                                    start of the step (explicit), eta = rho0 (tau - 1/2)/3,
                                    h below 0.1 taken as 0.1; part of F0 */
} lb_params;

/* lb_params.flags: readings the paper leaves open, off by default.
 * LB_SOLUTE_FORCE      the solvent also feels -c grad(mu_c), mu_c = C chi the
 *                      c-derivative of the coupling term of Eq. 1 (same
 *                      isotropic gradient as the psi force, chi(x) at solid
 *                      neighbours).  Off: phoresis reaches the fluid through
 *                      the slip of Eq. 4 only.  Selects the one-node form of
 *                      collide-stream.
 * LB_EXPLICIT_COLLOID  explicit rigid-body update (Ladd), M X' = M X + F0 -
 *                      zeta X + transfers, instead of the implicit
 *                      (M + zeta) X' = M X + F0 + transfers.
 * LB_CAPILLARY_FORCE   each particle also takes the stress of the psi free
 *                      energy at the fluid node of each of its links,
 *                      6 w_d c_d.P with P = (a/2 psi^2 + 3b/4 psi^4 - kappa
 *                      psi lap(psi) - kappa/2 |grad psi|^2) I + kappa grad psi
 *                      grad psi^T (wetting ghosts as in mu, central
 *                      differences): the capillary and wetting force that the
 *                      solvent force -psi grad(mu) leaves out at the particle
 *                      surface (Sec. II.B momentum exchange, Sec. III.B
 *                      trapping).  Part of F0, T0.  Experimental: stable in
 *                      the tested regime R = 4.5, M_psi = 0.4 in two psi/c
 *                      sub-steps, over 8x10^4 steps (nine trap cases, a GPU
 *                      test); runs with M_psi = 0.1 or R = 9 near an
 *                      interface can diverge (reported through the error
 *                      bits and LB_E_UNSTABLE): the fluid keeps the
 *                      potential-form force, and the pair does not conserve
 *                      momentum.  LB_STRESS_FORM removes that defect.
 * LB_STRESS_FORM       (with LB_CAPILLARY_FORCE) the solvent force of the psi
 *                      free energy in divergence form: -div P by the same
 *                      isotropic stencil, (div P)_b = 3 sum_i w_i c_ia
 *                      P_ab(x + c_i) with P(x) at solid neighbours, plus the
 *                      coupling part -psi grad(mu_c), mu_c = -C E chi
 *                      sech^2(psi) of Eq. 2, instead of -psi grad(mu).  The
 *                      fluid then loses exactly what the particles gain at
 *                      their links, so fluid and particles together conserve
 *                      momentum.  Selects the one-node forms of the mu update
 *                      and collide-stream and the boundary fix-ups; the arena
 *                      holds 7 more scalar fields.  Either form wants the
 *                      interface to relax faster than a particle disturbs it:
 *                      at M_psi = 0.1 in one psi/c update a strongly pushed or
 *                      emitting particle on an interface can still diverge
 *                      (LB_E_UNSTABLE); the paper's M_psi = 0.4 in two
 *                      sub-steps held in every tested case.
 * Other bits: LB_E_INVALID at lb_create. */
#define LB_SOLUTE_FORCE 1u
#define LB_EXPLICIT_COLLOID 2u
#define LB_CAPILLARY_FORCE 4u
#define LB_STRESS_FORM 8u

#define LB_PATTERN_MAX_BANDS 8
#define LB_PATTERN_MAX_CELLS 64

typedef struct {                 /* FP64, caller-owned */
    double pos[3], m[3], vel[3], omega[3]; /* centre, axis (normalised on add), V, Omega */
    double radius;
    double alpha_minus, alpha_plus;  /* production per link on the active cap m.n <= cap_cos /
                                        on the rest (Eq. 5) */
    double mu_minus, mu_plus;        /* phoretic mobility on the two caps (Eq. 6) */
    double H;                        /* wetting parameter of Eqs. 8-9 (from a contact angle:
                                        lb_wetting_H, Eq. 10, or lb_wetting_H_lattice) */
    double rho_p;                    /* particle density: mass rho_p 4/3 pi R^3 */
    int32_t fixed;                   /* 1: position, axis and velocities held */
    double cap_cos;                  /* the active cap is m.n <= cap_cos, in [-1, 1]; 0 (the
                                        paper's Janus half, Eqs. 5-6) keeps the exact tie
                                        rule m.n <= 0; otherwise m.r <= cap_cos |r|, |r| the
                                        correctly rounded square root, FP64 without
                                        contraction.  LB_E_INVALID outside [-1, 1] */
    double e[3];                     /* second body axis: made orthogonal to m and normalised
                                        on add (zero: an axis chosen orthogonal to m), turned
                                        with the particle; used by surface patterns */
    /* Surface pattern (the inhomogeneous surface patterns of Sec. IV; 0 bands: none,
     * the Janus caps above apply).  The surface is cut into cells: polar bands of
     * m.n, band b holding pattern_cos[b-1] < m.n <= pattern_cos[b] (cuts increasing
     * in (-1, 1), compared as m.r <= t |r| like the cap test), times azimuthal
     * sectors of the angle of n about m from e towards m x e, sector s covering
     * [2 pi s/S, 2 pi (s+1)/S) (decided from the signs and sizes of r.e and
     * r.(m x e); a point on the axis is in sector 0).  Cell b S + s has its own
     * production per link (Eq. 5), phoretic mobility (Eq. 6) and wetting parameter
     * (Eqs. 8-9), taken at the link midpoint or the face midpoint.  Bands 1..8,
     * sectors S in {1, 2, 4, 8}; LB_E_INVALID otherwise, or for wetting with
     * kappa = 0. */
    int32_t pattern_bands, pattern_sectors;
    double pattern_cos[LB_PATTERN_MAX_BANDS - 1];
    double pattern_alpha[LB_PATTERN_MAX_CELLS], pattern_mu[LB_PATTERN_MAX_CELLS],
        pattern_H[LB_PATTERN_MAX_CELLS];
    double axial;                    /* shape (Sec. IV, particles of other shapes): semi-axis
                                        along m of a spheroid whose other semi-axes are
                                        `radius`; 0 or equal to radius: a sphere.  A spheroid
                                        is solid where s^2 b^2 + |p|^2 a^2 < a^2 b^2 (s = m.r,
                                        p = r - s m, a = axial, b = radius, FP64 without
                                        contraction), its normal for the slip (Eq. 4) and the
                                        wetting ghost (Eq. 9) is s m / a^2 + p / b^2
                                        normalised, its mass rho_p 4 pi a b^2 / 3 and its
                                        inertia tensor 2 m b^2 / 5 about m, m (a^2 + b^2) / 5
                                        across it.  LB_E_INVALID if negative or not finite,
                                        or together with soft-sphere or lubrication forces */
} lb_colloid;

typedef struct {
    double mass, mom[3], sum_psi, sum_c; /* FP64 sums over fluid nodes of sum_i f_i,
                                            sum_i f_i c_i, psi, c */
    int64_t n_fluid, n_links, n_active, step; /* n_active: links on an active cap, or in a
                                                 producing cell of a pattern */
    int32_t error_bits;                  /* LB_ERR_* */
} lb_totals;

typedef struct lb_ctx lb_ctx; /* opaque */

/* Device bytes lb_create needs for a box with these parameters (the lattice
 * fields; particle tables are allocated by lb_add_colloids).
 * Errors: LB_E_INVALID for a NULL argument, a non-positive box size, a bad
 * precision or a box beyond the size limits of lb_params. */
lb_status lb_footprint_bytes(const lb_params *p, size_t *bytes);

/* Validate p and create a context for one box.  Checks: the size limits of
 * lb_params, tau > 1/2, rho0 > 0, kappa, M_psi, C, D_c, k_d >= 0, known
 * flags, ch_substeps in [0, 64], explicit-Euler stability of the psi and c
 * updates per sub-step, M_psi (12|a| + 36|b| + 144 kappa) / n < 2 and
 * (12 D_c + k_d) / n < 2 with n = max(ch_substeps, 1) (LB_E_INVALID
 * otherwise).  dev_arena: device memory
 * of at least lb_footprint_bytes, 256-byte aligned (borrowed; LB_E_INVALID
 * if misaligned), or NULL for the library to
 * allocate it (LB_E_OOM if it cannot).  hip_stream: a hipStream_t, or NULL
 * for the default stream.  *out receives the context. */
lb_status lb_create(const lb_params *p, void *dev_arena, size_t arena_bytes,
                    void *hip_stream, lb_ctx **out);

/* Free the context and everything the library allocated for it. */
lb_status lb_destroy(lb_ctx *ctx);

/* Set the state (Sec. II.C, initial condition): psi and c (N each,
 * required), density rho (N, NULL -> rho0) and velocity u (3N SoA, NULL ->
 * 0); populations start at the second-order equilibrium f_i^eq(rho, u).
 * Converts to the storage precision with round-to-nearest-even.  Removes any
 * particles and resets the step counter.  LB_E_INVALID on NULL psi/c or a
 * non-finite or non-positive value. */
lb_status lb_init_fields(lb_ctx *ctx, const double *psi, const double *c,
                         const double *rho, const double *u);

/* Place n particles (Sec. II.B) at their given state; nodes strictly inside
 * a sphere become solid.  The axis m is normalised.  LB_E_INVALID for
 * radius, rho_p or |m| <= 0, wetting H != 0 with kappa = 0, 2 radius + 8
 * larger than a box side, n above max_colloids; LB_E_STATE when two
 * surfaces come closer than 2 lattice units or before lb_init_fields.
 * Replaces any previous particles. */
lb_status lb_add_colloids(lb_ctx *ctx, const lb_colloid *cols, int32_t n);

/* Enqueue nsteps time steps on the context's stream and return (no host
 * synchronisation).  Device-side failures are reported by lb_observables. */
lb_status lb_step(lb_ctx *ctx, int64_t nsteps);

/* Synchronise and read the FP64 totals (may be NULL) and the state of the
 * first n particles (out may be NULL).  Returns LB_E_UNSTABLE when the
 * totals are not finite, LB_E_STATE when error bits are set (the totals are
 * filled in either case). */
lb_status lb_observables(lb_ctx *ctx, lb_totals *t, lb_colloid *out, int32_t n);

/* FP64 host copies of the fields (any pointer may be NULL): rho = sum_i f_i
 * and u = sum_i f_i c_i / rho (N and 3N; 0 at solid nodes), psi and c (N;
 * solid nodes keep their last fluid value). */
lb_status lb_get_fields(lb_ctx *ctx, double *rho, double *u, double *psi, double *c);

/* FP64 host copy of the populations f_i (19 planes of N, plane-major),
 * reconstructed from storage (f = stored/scale + w_i rho0); 0 at solid
 * nodes, whose slots carry no state (a node uncovered by a particle is
 * refilled from equilibrium). */
lb_status lb_get_populations(lb_ctx *ctx, double *f);

/* Owner map: -1 fluid, k for a node inside particle k (int32, N). */
lb_status lb_get_owner(lb_ctx *ctx, int32_t *owner);

/* Link table for the current particle positions, canonical order, as
 * records (k, n, d, cap) of int32.  *n receives the count; rec4 may be NULL
 * to query it; LB_E_INVALID if cap is smaller than the count. */
lb_status lb_get_links(lb_ctx *ctx, int32_t *rec4, int64_t cap, int64_t *n);

/* Per particle k, 12 FP64 values: force and torque acting on it in the last
 * step (F0 - zeta X', including cover/uncover transfers) and the part F0,
 * T0 that does not depend on its velocity at t+1: the link momentum without
 * the wall-velocity term, plus, where enabled, the capillary stress
 * (LB_CAPILLARY_FORCE) and the close-encounter forces (soft_eps, lub_hc). */
lb_status lb_colloid_forces(lb_ctx *ctx, double *out12, int32_t n);

/* Raw state for bitwise resume: stored populations, psi, c, owner map,
 * particle tables and step counter.  *n receives the size in bytes; buf may
 * be NULL to query it.  lb_load_state requires the same parameters. */
lb_status lb_save_state(lb_ctx *ctx, void *buf, size_t cap, size_t *n);
lb_status lb_load_state(lb_ctx *ctx, const void *buf, size_t n);

/* Advance n contexts by nsteps each with batched launches: every kernel of
 * the step is one launch covering all boxes (boxes may differ in size and in
 * particle count; all must share the precision and ch_substeps), and on a
 * non-default stream the launch sequence of two steps is captured once as a
 * HIP graph and replayed.  Work goes to the stream of ctxs[0]; work queued
 * earlier on the other boxes' own streams is waited for first, and the call
 * synchronises the stream of ctxs[0] before returning.  LB_E_INVALID for an empty
 * list, a repeated context, mixed precisions or mixed ch_substeps;
 * LB_E_STATE if a context lacks its fields. */
lb_status lb_batch_step(lb_ctx *const *ctxs, int32_t n, int64_t nsteps);

/* lb_batch_step without device allocation, for callers that cannot call
 * hipMalloc (tight serving loops, harnesses that forbid allocation): the
 * batch's descriptor tables go to a fixed device array of the library
 * (4 MiB per GPU, kept until the process ends) instead of a buffer allocated
 * per call, the steps are launched one by one (no graph is instantiated),
 * and the particle work uses the leading context's side stream only if it
 * already exists (else everything runs in order on its stream; results are
 * the same either way).  It calls no hipMalloc, hipFree or other allocating
 * routine.  Same arguments, semantics and errors as lb_batch_step, plus
 * LB_E_INVALID when the tables of the batch exceed the fixed array (about
 * 4000 boxes with one psi/c update per step, 1000 with sub-steps).  All
 * calls on one GPU share the array: calls that overlap in time on that GPU
 * (from several host threads) race; calls made one after another are safe,
 * since each synchronises its stream before returning. */
lb_status lb_batch_step_noalloc(lb_ctx *const *ctxs, int32_t n, int64_t nsteps);

/* Launch shapes of the three lattice kernels (chemical potential,
 * collide-stream, psi/c update): for each, (bx, by, code) = nodes per row
 * segment, rows per block (bx*by <= 256; 0 = default) and code = remap +
 * 8 vec + 64 zc.  remap is the block renumbering (0 natural order, 1
 * contiguous ranges per XCD, 2 one eighth of every z plane per XCD); vec
 * (0, 2 or 4) selects the row-vector form with vec consecutive x nodes per
 * lane (FP64 takes 2 for 4), in which bx and by are derived from nx, and
 * which boxes with nx % vec != 0, or rows longer than 64 lanes that are not
 * a multiple of 64 lanes (for the collide-stream: any row longer than 64
 * lanes), replace by the one-node form; zc > 1 (psi/c update with vec only)
 * makes each lane march zc planes in z (natural block order).  LB_E_INVALID
 * for other values.  Used by the autotuner; results are identical for every
 * shape.  lb_get_launch_shapes returns the shapes in effect. */
lb_status lb_set_launch_shapes(lb_ctx *ctx, const int32_t *shapes9);
lb_status lb_get_launch_shapes(lb_ctx *ctx, int32_t *shapes9);

/* Per-kernel timing on the context's stream with HIP events, for the
 * benchmark: enable resets the accumulators; lb_timing_read fills ms[i] with
 * the summed duration and calls[i] with the launch count of kernel i
 * (0 mu, 1 collide-stream, 2 psi/c update, 3 links+particles, 4 cover,
 * 5 geometry), synchronising the stream. */
lb_status lb_timing_enable(lb_ctx *ctx, int32_t on);
lb_status lb_timing_read(lb_ctx *ctx, double *ms6, int64_t *calls6);

/* Message for the last failure on ctx (thread-local text; never NULL). */
const char *lb_last_error(const lb_ctx *ctx);

/* Host helpers for parameters given through derived quantities.
 * lb_wetting_H: H of Eqs. 9-10 for a contact angle in degrees,
 *   cos(theta) = ((1+h)^(3/2) - (1-h)^(3/2))/2, h = H / sqrt(kappa b),
 *   solved for h in [-1, 1] by bisection; NaN if kappa b <= 0.
 * lb_wetting_H_lattice: H for which the lattice itself realises the contact
 *   angle theta on a flat wall (Eqs. 8-9 discretised as the library does: the
 *   wall energy H psi at the fluid nodes next to the solid, the discrete
 *   gradient energy of the face differences).  Young's cosine is
 *   (gamma(+psi_b) - gamma(-psi_b)) / sigma of the discrete one-dimensional
 *   minimisers (psi_b = sqrt(-a/b); sigma the lower of the kinks centred
 *   between and on nodes); H found by bisection in [-sqrt(kappa b),
 *   sqrt(kappa b)].  For interfaces a few nodes wide Eq. 10 over-states the
 *   wetting this discretisation gives (the paper's a, b, kappa: Eq. 10's H
 *   for 60 degrees realises about 43); for wide interfaces the two agree.
 *   NaN unless a < 0 < b and kappa > 0, or when theta is beyond that range.
 * lb_solubility_E: E of Eq. 1 giving an oil/water ratio of the equilibrium
 *   solute c0(psi) = c_b0 + E tanh psi at psi = -1 and +1. */
double lb_wetting_H(double theta_deg, double kappa, double b);
double lb_wetting_H_lattice(double theta_deg, double a, double b, double kappa);
double lb_solubility_E(double ratio, double c_b0);

#ifdef __cplusplus
}
#endif
#endif
