/* oracle.c -- plain FP64 CPU reference for one lattice update of the
 * multiphase-multicomponent lattice Boltzmann model for self-diffusiophoretic
 * Janus colloids at liquid-liquid interfaces (Palacios, Scagliarini,
 * Pagonabarraga, arXiv:2202.01631).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the solver.  It is written to be
 * read against the paper: one plain loop per step of the update, FP64
 * throughout, no blocking, fusion or reordering.  Build with
 * -O2 -fno-fast-math -ffp-contract=off so that no multiply-add is fused; the
 * colloid geometry decisions (inside test, cap test) depend on exact FP64
 * rounding.
 *
 * The paper gives the model (Eqs. 1-10) but not its discretisation.  The
 * readings taken here, each marked "reading" below, are:
 *   - solvent: D3Q19, BGK with relaxation time tau (nu = (tau-1/2)/3; tau = 1
 *     gives the paper's nu = 1/6, Sec. II.C), second-order equilibrium, forcing
 *     term of Guo, Zheng and Shi (2002); body force F = -psi grad(mu_psi), the
 *     usual potential form of the free-energy force ("thermohydrodynamic"
 *     model, Sec. I), with the isotropic 18-neighbour lattice gradient;
 *   - psi and c: explicit Euler finite volumes on the lattice, 7-point
 *     Laplacian, central face fluxes for advection (Eq. 3);
 *   - particles: bounce-back on links with the moving-wall term, momentum
 *     exchange (Sec. II.B), implicit velocity update in the manner of
 *     Nguyen and Ladd, cover/uncover repair;
 *   - slip (Eq. 4) added to the wall velocity of every link, with the
 *     concentration gradient taken at the link's fluid node; Janus activity
 *     (Eq. 5) emitted once per active link into its fluid node; Janus mobility
 *     (Eq. 6); tie m.n = 0 on the active cap as Eqs. 5-6 write it;
 *   - wetting (Eqs. 8-9) as a ghost value of psi in the Laplacian at solid
 *     face neighbours, signed so that kappa n.grad(psi) = H with n pointing out
 *     of the particle; contact angle from Eq. 10.
 *
 * Threads: the per-node loops (chemical potential, collision, streaming,
 * psi/c update, owner map) may run on several OpenMP threads; each node's
 * result depends only on its own inputs, and every sum over nodes or links is
 * taken sequentially in node or link order afterwards, so results are
 * bitwise the same for any thread count.
 *
 * Order of one step t -> t+1:
 *   1. mu_psi(t) at fluid nodes                                    (Eq. 2, 9)
 *   2. body force, moments, BGK-Guo collision; pull streaming;
 *      bounce-back on the links of R(t) with wall velocity V + W x r + slip,
 *      momentum exchange accumulated per colloid                 (Sec. II.B, Eq. 4, 6)
 *   3. psi and c updates with u(t), mu(t), chi(t) and emission      (Eq. 3, 5)
 *      (optionally n sub-steps of length 1/n, mu and chi recomputed)
 *   4. colloid update (implicit in V, W; explicit under OR_EXPLICIT_COLLOID),
 *      position and orientation
 *   5. geometry at R(t+1): cover/uncover repair, owner map, link table
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

/* ---------------------------------------------------------------- lattice */
/* D3Q19 velocity set, numbered as documented in oracle.h */
static const int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

static double wt(int i)
{
    if (i == 0) return 1.0 / 3.0;
    if (i <= 6) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

static void cross(const double a[3], const double b[3], double o[3]);

static int opp(int i)
{
    if (i == 0) return 0;
    return (i % 2 == 1) ? i + 1 : i - 1;
}

/* ---------------------------------------------------------------- context */
struct or_ctx {
    or_params p;
    int nx, ny, nz;
    long N;
    double *f, *fs, *fn;          /* pre-collision state f(t), post-collision, f(t+1) */
    double *psi, *cc, *psin, *ccn;
    double *mu, *force, *uf, *src, *chi;
    double *pst, *muc;            /* option OR_STRESS_FORM: stress (6 per node), mu_c */
    int *owner, *owner_new;
    or_colloid *col;
    int ncol;
    double *F0, *T0, *zeta, *trF, *trT, *Flast, *Tlast;
    int *lk, *ln, *ld, *lcap;
    long nl, lcapacity;
    double *lslip;                /* slip of each link in the last link loop */
    long nslip;                   /* links that loop covered (0: none) */
    long step;
    int stage;
    int err;
    double diag[OR_DIAG_N];
    char msg[256];
};

static int fail(or_ctx *c, int code, const char *m)
{
    if (c) snprintf(c->msg, sizeof c->msg, "%s", m);
    return code;
}

static long node(const or_ctx *c, int x, int y, int z)
{
    x = ((x % c->nx) + c->nx) % c->nx;
    y = ((y % c->ny) + c->ny) % c->ny;
    z = ((z % c->nz) + c->nz) % c->nz;
    return x + (long)c->nx * (y + (long)c->ny * z);
}

static void coords(const or_ctx *c, long n, int *x, int *y, int *z)
{
    *x = (int)(n % c->nx);
    *y = (int)((n / c->nx) % c->ny);
    *z = (int)(n / ((long)c->nx * c->ny));
}

/* neighbour of node n along lattice vector i */
static long nbr(const or_ctx *c, long n, int i)
{
    int x, y, z;
    coords(c, n, &x, &y, &z);
    return node(c, x + CX[i], y + CY[i], z + CZ[i]);
}

/* neighbour of node n along -c_i */
static long nbr_back(const or_ctx *c, long n, int i)
{
    int x, y, z;
    coords(c, n, &x, &y, &z);
    return node(c, x - CX[i], y - CY[i], z - CZ[i]);
}

/* ------------------------------------------------------- colloid geometry */
/* minimum-image displacement along one periodic axis of length L */
static double min_image(double d, int L)
{
    double h = 0.5 * (double)L;
    if (d > h) d -= (double)L;
    else if (d < -h) d += (double)L;
    return d;
}

/* displacement from the colloid centre to the point x + s*c_i (s = 0 or 1/2) */
static void disp(const or_ctx *c, const or_colloid *k, int x, int y, int z,
                 int i, double s, double r[3])
{
    r[0] = min_image(((double)x + s * (double)CX[i]) - k->pos[0], c->nx);
    r[1] = min_image(((double)y + s * (double)CY[i]) - k->pos[1], c->ny);
    r[2] = min_image(((double)z + s * (double)CZ[i]) - k->pos[2], c->nz);
}

/* option: a spheroid with semi-axis `axial` along m and `radius` across it
 * (reading: the local surface rules of the model carry over to particles of
 * other shapes, Sec. IV; the spheroid is the shape whose orientation is the
 * axis m the particle already carries).  Spheres keep their own arithmetic. */
static int spheroid(const or_colloid *k)
{
    return k->axial > 0.0 && k->axial != k->radius;
}

/* r split into its part s along m and the rest p across it */
static void split_axis(const or_colloid *k, const double r[3], double *s, double p[3])
{
    double t = k->m[0] * r[0] + k->m[1] * r[1];
    t = t + k->m[2] * r[2];
    *s = t;
    for (int a = 0; a < 3; a++) p[a] = r[a] - t * k->m[a];
}

/* a node is solid when it lies strictly inside the particle (Sec. II.B):
 * |r|^2 < R^2, or for a spheroid s^2/a^2 + |p|^2/b^2 < 1, multiplied out */
static int inside(const or_ctx *c, const or_colloid *k, int x, int y, int z)
{
    double r[3], d2;
    disp(c, k, x, y, z, 0, 0.0, r);
    if (spheroid(k)) {
        double sa, p[3];
        split_axis(k, r, &sa, p);
        double pp = p[0] * p[0] + p[1] * p[1];
        pp = pp + p[2] * p[2];
        const double a2 = k->axial * k->axial, b2 = k->radius * k->radius;
        return sa * sa * b2 + pp * a2 < a2 * b2;
    }
    d2 = r[0] * r[0] + r[1] * r[1];
    d2 = d2 + r[2] * r[2];
    return d2 < k->radius * k->radius;
}

/* outward unit normal for the surface point seen at r from the centre
 * (R9): r/|r| on a sphere; on a spheroid the gradient of
 * s^2/a^2 + |p|^2/b^2, i.e. s m / a^2 + p / b^2, normalised */
static void surface_normal(const or_colloid *k, const double r[3], double n[3])
{
    if (!spheroid(k)) {
        double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        for (int a = 0; a < 3; a++) n[a] = r[a] / rn;
        return;
    }
    double sa, p[3], g[3];
    split_axis(k, r, &sa, p);
    const double a2 = k->axial * k->axial, b2 = k->radius * k->radius;
    for (int a = 0; a < 3; a++) g[a] = (sa / a2) * k->m[a] + p[a] / b2;
    double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    for (int a = 0; a < 3; a++) n[a] = g[a] / gn;
}

/* |e.n| for the lattice axis ax at the surface point seen at r */
static double axis_cos(const or_colloid *k, const double r[3], int ax)
{
    if (!spheroid(k)) {
        double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        return fabs(r[ax]) / rn;
    }
    double n[3];
    surface_normal(k, r, n);
    return fabs(n[ax]);
}

/* active hemisphere of Eqs. 5-6: m.n <= 0, n taken at the link midpoint */
static int on_active_cap(const or_colloid *k, const double r[3])
{
    double md = k->m[0] * r[0] + k->m[1] * r[1];
    md = md + k->m[2] * r[2];
    if (k->cap_cos == 0.0) return md <= 0.0;
    /* option: a cap of any size, m.n <= cap_cos with n = r/|r| (reading: the
     * Janus split of Eqs. 5-6 moved to the polar angle acos(cap_cos)),
     * written as m.r <= cap_cos |r| */
    double rr = r[0] * r[0] + r[1] * r[1];
    rr = rr + r[2] * r[2];
    return md <= k->cap_cos * sqrt(rr);
}

/* option: surface pattern, a reading of the inhomogeneous surface patterns
 * of Sec. IV (the Janus split of Eqs. 5-6 generalised): the surface is cut
 * into cells of polar bands in m.n (cuts pat_cos, increasing, compared as
 * m.r <= t |r| like the cap test) and azimuthal sectors of the angle phi of
 * n about m, measured from the second body axis e towards m x e, in
 * half-open intervals [2 pi s/S, 2 pi (s+1)/S) decided by signs and
 * magnitudes of the two projections (no angle is computed); each cell has
 * its own production, phoretic mobility and wetting parameter.  A particle
 * without a pattern has two cells: 0 the active cap, 1 the rest. */
static int sector_of(double a, double b, int S)
{
    if (S <= 1) return 0;
    /* quadrant of phi = atan2(b, a) in [0, 2 pi); a = b = 0 counts as phi = 0 */
    int q;
    if (a > 0.0 && b >= 0.0) q = 0;
    else if (a <= 0.0 && b > 0.0) q = 1;
    else if (a < 0.0 && b <= 0.0) q = (a == 0.0 && b == 0.0) ? 0 : 2;
    else q = 3;
    if (S == 2) return q < 2 ? 0 : 1;
    if (S == 4) return q;
    /* eighths: turn the quadrant onto the first one, then phi < pi/4 iff y < x */
    double x = a, y = b;
    if (q == 1) { x = b; y = -a; }
    else if (q == 2) { x = -a; y = -b; }
    else if (q == 3) { x = -b; y = a; }
    return 2 * q + (y < x ? 0 : 1);
}

static int surface_cell(const or_colloid *k, const double r[3])
{
    if (k->pat_bands <= 0) return on_active_cap(k, r) ? 0 : 1;
    double md = k->m[0] * r[0] + k->m[1] * r[1];
    md = md + k->m[2] * r[2];
    double rr = r[0] * r[0] + r[1] * r[1];
    rr = rr + r[2] * r[2];
    const double rn = sqrt(rr);
    int band = 0;
    for (int b = 0; b < k->pat_bands - 1; b++)
        if (!(md <= k->pat_cos[b] * rn)) band++;
    double w[3];  /* m x e */
    w[0] = k->m[1] * k->e[2] - k->m[2] * k->e[1];
    w[1] = k->m[2] * k->e[0] - k->m[0] * k->e[2];
    w[2] = k->m[0] * k->e[1] - k->m[1] * k->e[0];
    double a = k->e[0] * r[0] + k->e[1] * r[1];
    a = a + k->e[2] * r[2];
    double b = w[0] * r[0] + w[1] * r[1];
    b = b + w[2] * r[2];
    return band * k->pat_sectors + sector_of(a, b, k->pat_sectors);
}

static double cell_alpha(const or_colloid *k, int cell)
{
    if (k->pat_bands > 0) return k->pat_alpha[cell];
    return cell == 0 ? k->alpha_minus : k->alpha_plus;
}

static double cell_mu(const or_colloid *k, int cell)
{
    if (k->pat_bands > 0) return k->pat_mu[cell];
    return cell == 0 ? k->mu_minus : k->mu_plus;
}

static double cell_H(const or_colloid *k, int cell)
{
    return k->pat_bands > 0 ? k->pat_H[cell] : k->H;
}

/* the 4th entry of a link record: the cap bit, or the cell of a pattern */
static int link_tag(const or_colloid *k, int cell)
{
    return k->pat_bands > 0 ? cell : (cell == 0 ? 1 : 0);
}

/* ------------------------------------------------------------ equilibrium */
static double feq(int i, double rho, const double u[3])
{
    double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return wt(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

/* forcing term of Guo, Zheng and Shi, Phys. Rev. E 65, 046308 (2002) */
static double guo(int i, const double u[3], const double F[3], double tau)
{
    double ci[3] = {(double)CX[i], (double)CY[i], (double)CZ[i]};
    double cu = ci[0] * u[0] + ci[1] * u[1] + ci[2] * u[2];
    double s = 0.0;
    for (int a = 0; a < 3; a++) s += (3.0 * (ci[a] - u[a]) + 9.0 * cu * ci[a]) * F[a];
    return (1.0 - 0.5 / tau) * wt(i) * s;
}

/* ----------------------------------------------------------- allocation */
static void *zalloc(size_t n)
{
    void *p = calloc(n ? n : 1, 1);
    return p;
}

int or_create(const or_params *p, or_ctx **out)
{
    if (!p || !out) return OR_E_INVALID;
    *out = NULL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return OR_E_INVALID;
    if (!(p->tau > 0.5) || !(p->rho0 > 0.0)) return OR_E_INVALID;
    if (p->kappa < 0.0 || p->M_psi < 0.0 || p->D_c < 0.0 || p->k_d < 0.0 || p->C < 0.0)
        return OR_E_INVALID;
    /* explicit-Euler stability of the 7-point schemes for psi and c, per
     * sub-step of length 1/n */
    if (p->ch_substeps < 0 || p->ch_substeps > 64) return OR_E_INVALID;
    const double dt = 1.0 / (p->ch_substeps > 0 ? p->ch_substeps : 1);
    if (dt * p->M_psi * (12.0 * fabs(p->a) + 36.0 * fabs(p->b) + 144.0 * p->kappa) >= 2.0)
        return OR_E_INVALID;
    if (dt * (12.0 * p->D_c + p->k_d) >= 2.0) return OR_E_INVALID;
    if (p->flags & ~(OR_SOLUTE_FORCE | OR_EXPLICIT_COLLOID | OR_CAPILLARY_FORCE | OR_STRESS_FORM))
        return OR_E_INVALID;
    if ((p->flags & OR_STRESS_FORM) && !(p->flags & OR_CAPILLARY_FORCE)) return OR_E_INVALID;
    if (!(p->soft_eps >= 0.0)) return OR_E_INVALID;
    if (p->soft_eps > 0.0 && !(p->soft_sigma > 0.0 && p->soft_nu > 0.0 && p->soft_hc > 0.0))
        return OR_E_INVALID;
    if (!(p->lub_hc >= 0.0)) return OR_E_INVALID;

    or_ctx *c = (or_ctx *)zalloc(sizeof *c);
    if (!c) return OR_E_INVALID;
    c->p = *p;
    c->nx = p->nx;
    c->ny = p->ny;
    c->nz = p->nz;
    c->N = (long)p->nx * p->ny * p->nz;
    long N = c->N;
    c->f = zalloc(sizeof(double) * 19 * N);
    c->fs = zalloc(sizeof(double) * 19 * N);
    c->fn = zalloc(sizeof(double) * 19 * N);
    c->psi = zalloc(sizeof(double) * N);
    c->cc = zalloc(sizeof(double) * N);
    c->psin = zalloc(sizeof(double) * N);
    c->ccn = zalloc(sizeof(double) * N);
    c->mu = zalloc(sizeof(double) * N);
    c->force = zalloc(sizeof(double) * 3 * N);
    c->uf = zalloc(sizeof(double) * 3 * N);
    c->src = zalloc(sizeof(double) * N);
    c->chi = zalloc(sizeof(double) * N);
    c->owner = zalloc(sizeof(int) * N);
    c->owner_new = zalloc(sizeof(int) * N);
    if (p->flags & OR_STRESS_FORM) {
        c->pst = zalloc(sizeof(double) * 6 * N);
        c->muc = zalloc(sizeof(double) * N);
        if (!c->pst || !c->muc) { or_destroy(c); return OR_E_INVALID; }
    }
    if (!c->f || !c->fs || !c->fn || !c->psi || !c->cc || !c->psin || !c->ccn || !c->mu ||
        !c->force || !c->uf || !c->src || !c->chi || !c->owner || !c->owner_new) {
        or_destroy(c);
        return OR_E_INVALID;
    }
    for (long n = 0; n < N; n++) c->owner[n] = -1;
    *out = c;
    return OR_OK;
}

static void free_colloids(or_ctx *c)
{
    free(c->col); free(c->F0); free(c->T0); free(c->zeta); free(c->trF); free(c->trT);
    free(c->Flast); free(c->Tlast);
    free(c->lk); free(c->ln); free(c->ld); free(c->lcap); free(c->lslip);
    c->col = NULL; c->F0 = c->T0 = c->zeta = c->trF = c->trT = c->Flast = c->Tlast = NULL;
    c->lk = c->ln = c->ld = c->lcap = NULL;
    c->lslip = NULL;
    c->ncol = 0; c->nl = 0; c->lcapacity = 0; c->nslip = 0;
}

int or_destroy(or_ctx *c)
{
    if (!c) return OR_OK;
    free(c->f); free(c->fs); free(c->fn); free(c->psi); free(c->cc); free(c->psin);
    free(c->ccn); free(c->mu); free(c->force); free(c->uf); free(c->src); free(c->chi);
    free(c->pst); free(c->muc);
    free(c->owner); free(c->owner_new);
    free_colloids(c);
    free(c);
    return OR_OK;
}

const char *or_last_error(const or_ctx *c) { return c ? c->msg : "null context"; }

/* ------------------------------------------------------------- init */
int or_init_fields(or_ctx *c, const double *psi, const double *cc, const double *rho,
                   const double *u)
{
    if (!c || !psi || !cc) return fail(c, OR_E_INVALID, "psi and c are required");
    long N = c->N;
    for (long n = 0; n < N; n++) {
        double r = rho ? rho[n] : c->p.rho0;
        double v[3] = {0.0, 0.0, 0.0};
        if (u) { v[0] = u[n]; v[1] = u[N + n]; v[2] = u[2 * N + n]; }
        if (!isfinite(psi[n]) || !isfinite(cc[n]) || !isfinite(r) || !(r > 0.0) ||
            !isfinite(v[0]) || !isfinite(v[1]) || !isfinite(v[2]))
            return fail(c, OR_E_INVALID, "non-finite or non-positive initial field");
        for (int i = 0; i < 19; i++) c->f[i * N + n] = feq(i, r, v);
        c->psi[n] = psi[n];
        c->cc[n] = cc[n];
        c->owner[n] = -1;
    }
    free_colloids(c);
    c->step = 0;
    c->err = 0;
    c->stage = 1;
    memset(c->diag, 0, sizeof c->diag);
    return OR_OK;
}

/* ----------------------------------------------------- geometry and links */
/* owner map at the current colloid positions; -1 fluid.  Returns nonzero if
 * two colloids claim one node. */
static int owner_map(or_ctx *c, int *own)
{
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(|:bad)
    for (long n = 0; n < c->N; n++) {
        int x, y, z;
        coords(c, n, &x, &y, &z);
        own[n] = -1;
        for (int k = 0; k < c->ncol; k++) {
            if (inside(c, &c->col[k], x, y, z)) {
                if (own[n] != -1) bad = 1;
                own[n] = k;
            }
        }
    }
    return bad;
}

/* link table in canonical order (k, n, d): fluid node n, n + c_d solid in k */
static void build_links(or_ctx *c)
{
    long *count = zalloc(sizeof(long) * (c->ncol + 1));
    long total = 0;
    for (long n = 0; n < c->N; n++) {
        if (c->owner[n] >= 0) continue;
        for (int d = 1; d < 19; d++) {
            int k = c->owner[nbr(c, n, d)];
            if (k >= 0) { count[k]++; total++; }
        }
    }
    if (total > c->lcapacity) {
        free(c->lk); free(c->ln); free(c->ld); free(c->lcap); free(c->lslip);
        c->lcapacity = total;
        c->lk = zalloc(sizeof(int) * total);
        c->ln = zalloc(sizeof(int) * total);
        c->ld = zalloc(sizeof(int) * total);
        c->lcap = zalloc(sizeof(int) * total);
        c->lslip = zalloc(sizeof(double) * 3 * total);
        c->nslip = 0;
    }
    int same = c->nslip > 0 && total == c->nl; /* table unchanged so far */
    long *off = zalloc(sizeof(long) * (c->ncol + 1));
    for (int k = 1; k <= c->ncol; k++) off[k] = off[k - 1] + count[k - 1];
    for (long n = 0; n < c->N; n++) {
        if (c->owner[n] >= 0) continue;
        int x, y, z;
        coords(c, n, &x, &y, &z);
        for (int d = 1; d < 19; d++) {
            int k = c->owner[nbr(c, n, d)];
            if (k < 0) continue;
            double r[3];
            disp(c, &c->col[k], x, y, z, d, 0.5, r);
            long l = off[k]++;
            if (same && (c->lk[l] != k || c->ln[l] != (int)n || c->ld[l] != d)) same = 0;
            c->lk[l] = k;
            c->ln[l] = (int)n;
            c->ld[l] = d;
            c->lcap[l] = surface_cell(&c->col[k], r);
        }
    }
    if (!same) c->nslip = 0; /* the slip record belongs to the old table */
    c->nl = total;
    free(count);
    free(off);
}

int or_add_colloids(or_ctx *c, const or_colloid *cols, int32_t n)
{
    if (!c) return OR_E_INVALID;
    if (c->stage < 1) return fail(c, OR_E_STATE, "init_fields first");
    if (n < 0 || (n > 0 && !cols)) return fail(c, OR_E_INVALID, "bad colloid array");
    free_colloids(c);
    c->ncol = n;
    c->col = zalloc(sizeof(or_colloid) * (n + 1));
    c->F0 = zalloc(sizeof(double) * 3 * (n + 1));
    c->T0 = zalloc(sizeof(double) * 3 * (n + 1));
    c->zeta = zalloc(sizeof(double) * 36 * (n + 1));
    c->trF = zalloc(sizeof(double) * 3 * (n + 1));
    c->trT = zalloc(sizeof(double) * 3 * (n + 1));
    c->Flast = zalloc(sizeof(double) * 3 * (n + 1));
    c->Tlast = zalloc(sizeof(double) * 3 * (n + 1));
    int L[3] = {c->nx, c->ny, c->nz};
    for (int k = 0; k < n; k++) {
        or_colloid q = cols[k];
        double mm = sqrt(q.m[0] * q.m[0] + q.m[1] * q.m[1] + q.m[2] * q.m[2]);
        if (!(q.radius > 0.0) || !(q.rho_p > 0.0) || !(mm > 0.0))
            return fail(c, OR_E_INVALID, "colloid radius, density and axis must be positive");
        if (!(q.cap_cos >= -1.0 && q.cap_cos <= 1.0))
            return fail(c, OR_E_INVALID, "cap_cos must lie in [-1, 1]");
        if (q.H != 0.0 && !(c->p.kappa > 0.0))
            return fail(c, OR_E_INVALID, "wetting needs kappa > 0");
        if (!(q.axial >= 0.0) || !isfinite(q.axial))
            return fail(c, OR_E_INVALID, "axial semi-axis must be finite and >= 0");
        if (spheroid(&q) && (c->p.soft_eps > 0.0 || c->p.lub_hc > 0.0))
            return fail(c, OR_E_INVALID, "soft-sphere and lubrication forces need spheres");
        if (q.pat_bands < 0 || q.pat_bands > OR_PATTERN_MAX_BANDS)
            return fail(c, OR_E_INVALID, "pattern bands in [0, 8]");
        if (q.pat_bands > 0) {
            const int S = q.pat_sectors;
            if (!(S == 1 || S == 2 || S == 4 || S == 8) || q.pat_bands * S > OR_PATTERN_MAX_CELLS)
                return fail(c, OR_E_INVALID, "pattern sectors 1, 2, 4 or 8");
            for (int b = 0; b < q.pat_bands - 1; b++)
                if (!(q.pat_cos[b] > -1.0 && q.pat_cos[b] < 1.0) ||
                    (b > 0 && !(q.pat_cos[b] > q.pat_cos[b - 1])))
                    return fail(c, OR_E_INVALID, "pattern cuts increasing in (-1, 1)");
            for (int i = 0; i < q.pat_bands * S; i++)
                if (q.pat_H[i] != 0.0 && !(c->p.kappa > 0.0))
                    return fail(c, OR_E_INVALID, "wetting needs kappa > 0");
        }
        const double rb = q.axial > q.radius ? q.axial : q.radius;  /* bounding radius */
        for (int a = 0; a < 3; a++) {
            if (2.0 * rb + 4.0 > (double)L[a])
                return fail(c, OR_E_INVALID, "colloid does not fit in the box");
            q.m[a] /= mm;
            /* positions are kept in [0, L) */
            q.pos[a] = fmod(q.pos[a], (double)L[a]);
            if (q.pos[a] < 0.0) q.pos[a] += (double)L[a];
        }
        /* second body axis: the part of e orthogonal to m, normalised; if that
         * vanishes, the lattice axis least aligned with m crossed into place */
        double em = q.e[0] * q.m[0] + q.e[1] * q.m[1] + q.e[2] * q.m[2];
        double ev[3] = {q.e[0] - em * q.m[0], q.e[1] - em * q.m[1], q.e[2] - em * q.m[2]};
        double ne = sqrt(ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2]);
        if (!(ne > 1e-9)) {
            int j = 0;
            for (int a = 1; a < 3; a++)
                if (fabs(q.m[a]) < fabs(q.m[j])) j = a;
            double ax[3] = {0.0, 0.0, 0.0};
            ax[j] = 1.0;
            double t[3];
            cross(q.m, ax, t);
            cross(t, q.m, ev);  /* (m x ax) x m: ax made orthogonal to m */
            ne = sqrt(ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2]);
        }
        for (int a = 0; a < 3; a++) q.e[a] = ev[a] / ne;
        c->col[k] = q;
    }
    if (owner_map(c, c->owner)) {
        for (long m = 0; m < c->N; m++) c->owner[m] = -1;
        free_colloids(c);
        return fail(c, OR_E_STATE, "colloids overlap");
    }
    /* solid nodes hold the rest populations; they are never read */
    for (long m = 0; m < c->N; m++)
        if (c->owner[m] >= 0)
            for (int i = 0; i < 19; i++) c->f[i * c->N + m] = wt(i) * c->p.rho0;
    build_links(c);
    c->stage = 2;
    return OR_OK;
}

/* --------------------------------------------------------------- one step */
/* wall velocity of colloid k at displacement r: V + Omega x r */
static void rigid_velocity(const or_colloid *k, const double r[3], double u[3])
{
    u[0] = k->vel[0] + (k->omega[1] * r[2] - k->omega[2] * r[1]);
    u[1] = k->vel[1] + (k->omega[2] * r[0] - k->omega[0] * r[2]);
    u[2] = k->vel[2] + (k->omega[0] * r[1] - k->omega[1] * r[0]);
}

static void cross(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* step 1: chemical potential mu_psi of Eq. 2 at fluid nodes.  At a solid face
 * neighbour the Laplacian uses the wetting ghost psi(x) - (H/kappa)|e.n|, the
 * one-sided form of kappa n.grad(psi) = H (Eq. 9, reading: signed, n out of
 * the particle, n taken at the face midpoint). */
static void chemical_potential(or_ctx *c)
{
    const or_params *p = &c->p;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < c->N; n++) {
        if (c->owner[n] >= 0) { c->mu[n] = 0.0; continue; }
        int x, y, z;
        coords(c, n, &x, &y, &z);
        double lap = -6.0 * c->psi[n];
        for (int e = 1; e <= 6; e++) {
            long m = nbr(c, n, e);
            int k = c->owner[m];
            if (k < 0) {
                lap += c->psi[m];
            } else {
                double r[3];
                disp(c, &c->col[k], x, y, z, e, 0.5, r);
                double en = axis_cos(&c->col[k], r, (e - 1) / 2);
                double ghost = c->psi[n];
                if (p->kappa > 0.0)
                    ghost = c->psi[n] - (cell_H(&c->col[k], surface_cell(&c->col[k], r)) / p->kappa) * en;
                lap += ghost;
            }
        }
        double ps = c->psi[n];
        double chi = c->cc[n] - p->c_b0 - p->E * tanh(ps);
        double ch = cosh(ps);
        c->mu[n] = p->a * ps + p->b * ps * ps * ps - p->kappa * lap - p->C * p->E * chi / (ch * ch);
    }
}

/* value of a scalar field at neighbour m of fluid node n, with the node's own
 * value substituted when m is solid (no flux through the particle surface) */
static double hat(const or_ctx *c, const double *fld, long n, long m)
{
    return c->owner[m] < 0 ? fld[m] : fld[n];
}

/* option OR_CAPILLARY_FORCE: thermodynamic stress of the psi part of Eq. 1 at
 * fluid node n,
 *   P = (a/2 psi^2 + 3b/4 psi^4 - kappa psi lap(psi) - kappa/2 |g|^2) I + kappa g g^T,
 * the tensor whose divergence is psi grad(mu) for f = a/2 psi^2 + b/4 psi^4 +
 * kappa/2 |grad psi|^2.  Face neighbours that are solid take the wetting ghost
 * of the chemical potential; g is the central difference over the faces. */
static void stress(const or_ctx *c, long n, double P[3][3])
{
    const or_params *p = &c->p;
    int x, y, z;
    coords(c, n, &x, &y, &z);
    double ph[7];
    for (int e = 1; e <= 6; e++) {
        long m = nbr(c, n, e);
        int k = c->owner[m];
        if (k < 0) {
            ph[e] = c->psi[m];
        } else {
            double r[3];
            disp(c, &c->col[k], x, y, z, e, 0.5, r);
            double en = axis_cos(&c->col[k], r, (e - 1) / 2);
            ph[e] = c->psi[n];
            if (p->kappa > 0.0)
                ph[e] = c->psi[n] - (cell_H(&c->col[k], surface_cell(&c->col[k], r)) / p->kappa) * en;
        }
    }
    double ps = c->psi[n];
    double lap = ph[1] + ph[2] + ph[3] + ph[4] + ph[5] + ph[6] - 6.0 * ps;
    double g[3] = {(ph[1] - ph[2]) / 2.0, (ph[3] - ph[4]) / 2.0, (ph[5] - ph[6]) / 2.0};
    double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    double s = p->a / 2.0 * ps * ps + 3.0 * p->b / 4.0 * ps * ps * ps * ps - p->kappa * ps * lap -
               p->kappa / 2.0 * g2;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) P[a][b] = (a == b ? s : 0.0) + p->kappa * g[a] * g[b];
}

/* step 2: force, moments, collision, streaming and bounce-back on links */
static void collide_stream(or_ctx *c)
{
    const or_params *p = &c->p;
    long N = c->N;
    double sumF[3] = {0.0, 0.0, 0.0};
    const int divform = (p->flags & OR_STRESS_FORM) != 0;
    if (divform) {
        /* option: the stress P (xx, yy, zz, xy, xz, yz) and the coupling part
         * mu_c = -C E chi sech^2(psi) of Eq. 2 at every fluid node */
#pragma omp parallel for schedule(static)
        for (long n = 0; n < N; n++) {
            if (c->owner[n] >= 0) continue;
            double P[3][3];
            stress(c, n, P);
            double *q = &c->pst[6 * n];
            q[0] = P[0][0]; q[1] = P[1][1]; q[2] = P[2][2];
            q[3] = P[0][1]; q[4] = P[0][2]; q[5] = P[1][2];
            double ps = c->psi[n];
            double chi = c->cc[n] - p->c_b0 - p->E * tanh(ps);
            double ch = cosh(ps);
            c->muc[n] = -p->C * p->E * chi / (ch * ch);
        }
    }
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; n++) {
        if (c->owner[n] >= 0) {
            for (int i = 0; i < 19; i++) c->fs[i * N + n] = c->f[i * N + n];
            for (int a = 0; a < 3; a++) { c->force[a * N + n] = 0.0; c->uf[a * N + n] = 0.0; }
            continue;
        }
        /* body force -psi grad(mu), gradient by the isotropic lattice
         * stencil grad(mu) = 3 sum_i w_i c_i mu(x + c_i) (reading: the central
         * 2-point difference makes the explicit force/advection coupling
         * unstable at grid scale when kappa > 0) */
        double gm[3] = {0.0, 0.0, 0.0}, F[3];
        for (int i = 1; i < 19; i++) {
            double mi = hat(c, c->mu, n, nbr(c, n, i));
            gm[0] += wt(i) * CX[i] * mi;
            gm[1] += wt(i) * CY[i] * mi;
            gm[2] += wt(i) * CZ[i] * mi;
        }
        for (int a = 0; a < 3; a++) F[a] = -c->psi[n] * 3.0 * gm[a] + p->ext_force[a];
        if (divform) {
            /* option: -div P by the same isotropic stencil, (div P)_b =
             * 3 sum_i w_i c_ia P_ab(x + c_i), P(x) at solid neighbours, plus
             * -psi grad(mu_c); replaces -psi grad(mu) */
            double dP[3] = {0.0, 0.0, 0.0}, gc[3] = {0.0, 0.0, 0.0};
            for (int i = 1; i < 19; i++) {
                long m = nbr(c, n, i);
                long y = c->owner[m] < 0 ? m : n;
                const double *q = &c->pst[6 * y];
                const double Pm[3][3] = {{q[0], q[3], q[4]}, {q[3], q[1], q[5]}, {q[4], q[5], q[2]}};
                for (int b = 0; b < 3; b++)
                    dP[b] += wt(i) * (CX[i] * Pm[0][b] + CY[i] * Pm[1][b] + CZ[i] * Pm[2][b]);
                gc[0] += wt(i) * CX[i] * c->muc[y];
                gc[1] += wt(i) * CY[i] * c->muc[y];
                gc[2] += wt(i) * CZ[i] * c->muc[y];
            }
            for (int a = 0; a < 3; a++)
                F[a] = -3.0 * dP[a] - c->psi[n] * 3.0 * gc[a] + p->ext_force[a];
        }
        if (p->flags & OR_SOLUTE_FORCE) {
            /* option: the solvent also feels -c grad(mu_c) with mu_c = C chi,
             * the c-derivative of the coupling term of Eq. 1; same stencil,
             * chi(x) at solid neighbours */
            double chi0 = c->cc[n] - p->c_b0 - p->E * tanh(c->psi[n]);
            double gc[3] = {0.0, 0.0, 0.0};
            for (int i = 1; i < 19; i++) {
                long m = nbr(c, n, i);
                double xm = c->owner[m] < 0 ? c->cc[m] - p->c_b0 - p->E * tanh(c->psi[m]) : chi0;
                gc[0] += wt(i) * CX[i] * xm;
                gc[1] += wt(i) * CY[i] * xm;
                gc[2] += wt(i) * CZ[i] * xm;
            }
            for (int a = 0; a < 3; a++) F[a] += -c->cc[n] * p->C * 3.0 * gc[a];
        }
        double rho = 0.0, mom[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < 19; i++) {
            double fi = c->f[i * N + n];
            rho += fi;
            mom[0] += fi * CX[i];
            mom[1] += fi * CY[i];
            mom[2] += fi * CZ[i];
        }
        double u[3];
        for (int a = 0; a < 3; a++) u[a] = (mom[a] + F[a] / 2.0) / rho;
        for (int i = 0; i < 19; i++) {
            double fi = c->f[i * N + n];
            c->fs[i * N + n] = fi - (fi - feq(i, rho, u)) / p->tau + guo(i, u, F, p->tau);
        }
        for (int a = 0; a < 3; a++) { c->force[a * N + n] = F[a]; c->uf[a * N + n] = u[a]; }
    }
    /* summed body force over the fluid nodes, in node order */
    for (long n = 0; n < N; n++)
        if (c->owner[n] < 0)
            for (int a = 0; a < 3; a++) sumF[a] += c->force[a * N + n];
    /* pull streaming from fluid upstream neighbours */
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; n++) {
        if (c->owner[n] >= 0) {
            for (int i = 0; i < 19; i++) c->fn[i * N + n] = c->f[i * N + n];
            continue;
        }
        for (int i = 0; i < 19; i++) {
            long m = nbr_back(c, n, i);
            if (c->owner[m] < 0) c->fn[i * N + n] = c->fs[i * N + m];
        }
    }
    /* bounce-back on links, canonical order; momentum exchange per colloid */
    double sumdp[3] = {0.0, 0.0, 0.0}, dmass = 0.0;
    for (int k = 0; k < c->ncol; k++) {
        for (int a = 0; a < 3; a++) { c->F0[3 * k + a] = 0.0; c->T0[3 * k + a] = 0.0; }
        for (int j = 0; j < 36; j++) c->zeta[36 * k + j] = 0.0;
    }
    for (long n = 0; n < N; n++) c->src[n] = 0.0;
    for (long l = 0; l < c->nl; l++) {
        int k = c->lk[l], d = c->ld[l];
        long n = c->ln[l];
        const or_colloid *q = &c->col[k];
        int x, y, z;
        coords(c, n, &x, &y, &z);
        double r[3], nh[3], g[3], slip[3], ur[3], ub[3];
        disp(c, q, x, y, z, d, 0.5, r);
        surface_normal(q, r, nh);
        /* phoretic slip (Eq. 4) with the Janus mobility of Eq. 6 */
        double mob = cell_mu(q, c->lcap[l]);
        for (int a = 0; a < 3; a++) {
            long mp = nbr(c, n, 1 + 2 * a), mm = nbr(c, n, 2 + 2 * a);
            g[a] = (hat(c, c->cc, n, mp) - hat(c, c->cc, n, mm)) / 2.0;
        }
        double ng = nh[0] * g[0] + nh[1] * g[1] + nh[2] * g[2];
        for (int a = 0; a < 3; a++) slip[a] = mob * (g[a] - nh[a] * ng);
        for (int a = 0; a < 3; a++) c->lslip[3 * l + a] = slip[a];
        rigid_velocity(q, r, ur);
        for (int a = 0; a < 3; a++) ub[a] = ur[a] + slip[a];
        double cd[3] = {(double)CX[d], (double)CY[d], (double)CZ[d]};
        double w = wt(d), fsd = c->fs[d * N + n];
        double cub = cd[0] * ub[0] + cd[1] * ub[1] + cd[2] * ub[2];
        double cus = cd[0] * slip[0] + cd[1] * slip[1] + cd[2] * slip[2];
        c->fn[opp(d) * N + n] = fsd - 6.0 * w * c->p.rho0 * cub;
        /* momentum handed to the colloid: c_d (2 f*_d - 6 w rho0 c_d.u_b) */
        for (int a = 0; a < 3; a++) sumdp[a] += cd[a] * (2.0 * fsd - 6.0 * w * c->p.rho0 * cub);
        dmass += -6.0 * w * c->p.rho0 * cub;
        /* the part of it that does not depend on V and Omega */
        double dp0[3], t0[3], rc[3];
        for (int a = 0; a < 3; a++) dp0[a] = cd[a] * (2.0 * fsd - 6.0 * w * c->p.rho0 * cus);
        if (c->p.flags & OR_CAPILLARY_FORCE) {
            /* option: the stress at the link's fluid node on the link's share
             * of the surface.  For the divergence of a stress with the
             * isotropic stencil, -3 sum_i w_i c_i.P(x + c_i) with P(x)
             * substituted at solid neighbours, the fluid nodes together
             * receive -6 sum_links w_d c_d.P(x); the particle takes the
             * opposite, so that the pair conserves momentum (reading: the
             * proper momentum exchange of Sec. II.B, the capillary force of
             * Sec. III.B) */
            double P[3][3];
            stress(c, n, P);
            for (int b = 0; b < 3; b++)
                dp0[b] += 6.0 * w * (cd[0] * P[0][b] + cd[1] * P[1][b] + cd[2] * P[2][b]);
        }
        cross(r, dp0, t0);
        for (int a = 0; a < 3; a++) { c->F0[3 * k + a] += dp0[a]; c->T0[3 * k + a] += t0[a]; }
        /* drag tensor zeta = sum 6 w rho0 g g^T, g = (c_d, r x c_d) */
        cross(r, cd, rc);
        double gg[6] = {cd[0], cd[1], cd[2], rc[0], rc[1], rc[2]};
        for (int i = 0; i < 6; i++)
            for (int j = 0; j < 6; j++) c->zeta[36 * k + 6 * i + j] += 6.0 * w * c->p.rho0 * gg[i] * gg[j];
        /* Janus activity of Eq. 5, one emission per link into its fluid node */
        c->src[n] += cell_alpha(q, c->lcap[l]);
    }
    for (int a = 0; a < 3; a++) {
        c->diag[OR_DIAG_SUM_FORCE + a] = sumF[a];
        c->diag[OR_DIAG_SUM_DP + a] = sumdp[a];
    }
    c->diag[OR_DIAG_SUM_DMASS] = dmass;
    c->nslip = c->nl;
}

/* step 2b (options, soft_eps > 0 or lub_hc > 0): soft-sphere repulsion and
 * normal lubrication for close encounters.  Soft sphere:
 * (the paper mentions a soft potential for near-contact encounters without
 * giving it).  Reading: the shifted-force soft sphere
 *   U(h) = eps (sigma/h)^nu, force -dU/dh shifted to vanish at the cutoff hc,
 * on the surface gap h = |R_j - R_i| - a_i - a_j (minimum image), added to
 * the velocity-independent force F0 of both particles, from the positions at
 * t.  Lubrication (reading: the normal term of Nguyen and Ladd, explicit in
 * the velocities at t, gap floored at 0.1 for stability): -6 pi eta (a_i
 * a_j/(a_i + a_j))^2 (1/h - 1/lub_hc) U_n along the line of centres.
 * Central: no torque. */
static void soft_contacts(or_ctx *c)
{
    const or_params *p = &c->p;
    if (!(p->soft_eps > 0.0) && !(p->lub_hc > 0.0)) return;
    int L[3] = {c->nx, c->ny, c->nz};
    for (int i = 0; i < c->ncol; i++)
        for (int j = i + 1; j < c->ncol; j++) {
            const or_colloid *a = &c->col[i], *b = &c->col[j];
            double d[3];
            for (int e = 0; e < 3; e++) d[e] = min_image(b->pos[e] - a->pos[e], L[e]);
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double h0 = r - a->radius - b->radius;
            double f = 0.0;
            if (p->soft_eps > 0.0 && h0 < p->soft_hc) {
                double h = h0 < 0.01 ? 0.01 : h0;
                f += p->soft_nu * p->soft_eps * pow(p->soft_sigma, p->soft_nu) *
                     (pow(h, -(p->soft_nu + 1.0)) - pow(p->soft_hc, -(p->soft_nu + 1.0)));
            }
            if (p->lub_hc > 0.0 && h0 < p->lub_hc) {
                /* option: normal lubrication (Nguyen and Ladd), explicit in
                 * the velocities at t; un > 0 when the pair approaches */
                double h = h0 < 0.1 ? 0.1 : h0;
                double un = ((a->vel[0] - b->vel[0]) * d[0] + (a->vel[1] - b->vel[1]) * d[1] +
                             (a->vel[2] - b->vel[2]) * d[2]) / r;
                double ae = a->radius * b->radius / (a->radius + b->radius);
                double eta = p->rho0 * (p->tau - 0.5) / 3.0;
                f += 6.0 * M_PI * eta * ae * ae * (1.0 / h - 1.0 / p->lub_hc) * un;
            }
            /* f > 0 pushes the pair apart */
            for (int e = 0; e < 3; e++) {
                c->F0[3 * i + e] -= f * d[e] / r;
                c->F0[3 * j + e] += f * d[e] / r;
            }
        }
}

/* step 3: Cahn-Hilliard update of psi and advection-diffusion-reaction update
 * of c (Eq. 3), explicit Euler over a time step dt (1, or 1/n for n
 * sub-steps), fluxes through the 6 faces of each node; no flux through faces
 * shared with solid nodes.  The diagnostics sum dt-weighted source and chi. */
static void scalar_update(or_ctx *c, double dt)
{
    const or_params *p = &c->p;
    long N = c->N;
    double sumsrc = 0.0, sumchi = 0.0;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; n++) {
        if (c->owner[n] >= 0) { c->psin[n] = c->psi[n]; c->ccn[n] = c->cc[n]; continue; }
        double ps = c->psi[n], cn = c->cc[n];
        double chi = cn - p->c_b0 - p->E * tanh(ps);
        double adv_psi = 0.0, adv_c = 0.0, dmu = 0.0, dchi = 0.0;
        for (int e = 1; e <= 6; e++) {
            long m = nbr(c, n, e);
            if (c->owner[m] >= 0) continue;
            int a = (e - 1) / 2;
            double sgn = (e % 2 == 1) ? 1.0 : -1.0;
            double ue = 0.5 * (sgn * c->uf[a * N + n] + sgn * c->uf[a * N + m]);
            adv_psi += ue * 0.5 * (ps + c->psi[m]);
            adv_c += ue * 0.5 * (cn + c->cc[m]);
            dmu += c->mu[m] - c->mu[n];
            double chim = c->cc[m] - p->c_b0 - p->E * tanh(c->psi[m]);
            dchi += chim - chi;
        }
        c->psin[n] = ps - dt * adv_psi + dt * p->M_psi * dmu;
        c->ccn[n] = cn - dt * adv_c + dt * p->D_c * dchi + dt * c->src[n] - dt * p->k_d * chi;
        c->chi[n] = chi;
    }
    /* emitted solute and summed chi over the fluid nodes, in node order */
    for (long n = 0; n < N; n++) {
        if (c->owner[n] >= 0) continue;
        sumsrc += dt * c->src[n];
        sumchi += dt * c->chi[n];
    }
    c->diag[OR_DIAG_SUM_SRC] += sumsrc;
    c->diag[OR_DIAG_SUM_CHI] += sumchi;
}

/* solve A x = b for a symmetric positive definite 6x6 A by Gaussian
 * elimination without pivoting (A = M + zeta is SPD) */
static void solve6(double A[36], double b[6], double x[6])
{
    for (int k = 0; k < 6; k++) {
        for (int i = k + 1; i < 6; i++) {
            double l = A[6 * i + k] / A[6 * k + k];
            for (int j = k; j < 6; j++) A[6 * i + j] -= l * A[6 * k + j];
            b[i] -= l * b[k];
        }
    }
    for (int i = 5; i >= 0; i--) {
        double s = b[i];
        for (int j = i + 1; j < 6; j++) s -= A[6 * i + j] * x[j];
        x[i] = s / A[6 * i + i];
    }
}

/* A spheroid's step: mass m = rho_p 4 pi a b^2 / 3, inertia tensor
 * I = I_perp 1 + (I_par - I_perp) m m^T about the centre with I_par =
 * 2 m b^2 / 5 about the axis and I_perp = m (a^2 + b^2) / 5 across it, taken
 * at the axis of the start of the step (the gyroscopic term, second order
 * in Omega, is left out); the same implicit (or explicit) update as a
 * sphere's with M = diag(m, m, m, I). */
static void spheroid_update(const or_colloid *q, const double Z[36], const double Fk[6],
                            const double X[6], int expl, double Xn[6])
{
    const double a = q->axial, b = q->radius;
    const double mass = q->rho_p * (4.0 * M_PI / 3.0) * a * b * b;
    const double ipar = 0.4 * mass * b * b, iperp = 0.2 * mass * (a * a + b * b);
    double M[36];
    for (int i = 0; i < 36; i++) M[i] = 0.0;
    for (int i = 0; i < 3; i++) M[6 * i + i] = mass;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            M[6 * (3 + i) + 3 + j] = (i == j ? iperp : 0.0) + (ipar - iperp) * q->m[i] * q->m[j];
    if (expl) {
        /* M X' = M X + F0 - zeta X: X' = X + M^-1 (F0 - zeta X), with
         * I^-1 = 1/I_perp + (1/I_par - 1/I_perp) m m^T */
        double s[6];
        for (int i = 0; i < 6; i++) {
            s[i] = Fk[i];
            for (int j = 0; j < 6; j++) s[i] -= Z[6 * i + j] * X[j];
        }
        for (int i = 0; i < 3; i++) Xn[i] = X[i] + s[i] / mass;
        const double ms = q->m[0] * s[3] + q->m[1] * s[4] + q->m[2] * s[5];
        for (int i = 0; i < 3; i++)
            Xn[3 + i] = X[3 + i] + s[3 + i] / iperp + (1.0 / ipar - 1.0 / iperp) * q->m[i] * ms;
        return;
    }
    double A[36], bv[6];
    for (int i = 0; i < 36; i++) A[i] = Z[i] + M[i];
    for (int i = 0; i < 6; i++) {
        bv[i] = Fk[i];
        for (int j = 0; j < 6; j++) bv[i] += M[6 * i + j] * X[j];
    }
    solve6(A, bv, Xn);
}

/* step 4: rigid-body update, implicit in the link drag (Nguyen and Ladd):
 * (M + zeta) X' = M X + (F0, T0), X = (V, Omega); R' = R + V';
 * m' = m rotated by the angle |Omega'| about Omega' (Rodrigues). */
static void colloid_update(or_ctx *c)
{
    int L[3] = {c->nx, c->ny, c->nz};
    for (int k = 0; k < c->ncol; k++) {
        or_colloid *q = &c->col[k];
        double *Z = &c->zeta[36 * k];
        double Fk[6], X[6] = {q->vel[0], q->vel[1], q->vel[2], q->omega[0], q->omega[1], q->omega[2]};
        for (int a = 0; a < 3; a++) {
            Fk[a] = c->F0[3 * k + a] + c->trF[3 * k + a];
            Fk[3 + a] = c->T0[3 * k + a] + c->trT[3 * k + a];
        }
        double Xn[6];
        const int expl = (c->p.flags & OR_EXPLICIT_COLLOID) != 0;
        if (q->fixed) {
            for (int i = 0; i < 6; i++) Xn[i] = X[i];
        } else {
            double mass = q->rho_p * (4.0 * M_PI / 3.0) * q->radius * q->radius * q->radius;
            double inertia = 0.4 * mass * q->radius * q->radius;
            double Mv[6] = {mass, mass, mass, inertia, inertia, inertia};
            if (spheroid(q)) {
                spheroid_update(q, Z, Fk, X, expl, Xn);
            } else if (expl) {
                /* option: explicit update (Ladd), M X' = M X + F0 - zeta X */
                for (int i = 0; i < 6; i++) {
                    double s = Fk[i];
                    for (int j = 0; j < 6; j++) s -= Z[6 * i + j] * X[j];
                    Xn[i] = X[i] + s / Mv[i];
                }
            } else {
                double A[36], b[6];
                for (int i = 0; i < 36; i++) A[i] = Z[i];
                for (int i = 0; i < 6; i++) { A[6 * i + i] += Mv[i]; b[i] = Mv[i] * X[i] + Fk[i]; }
                solve6(A, b, Xn);
            }
        }
        /* force and torque actually acting: F0 - zeta X' (implicit), F0 - zeta X
         * (explicit: the links saw the old velocity) */
        for (int i = 0; i < 6; i++) {
            double s = Fk[i];
            for (int j = 0; j < 6; j++) s -= Z[6 * i + j] * (expl ? X[j] : Xn[j]);
            if (i < 3) c->Flast[3 * k + i] = s; else c->Tlast[3 * k + i - 3] = s;
        }
        if (!q->fixed) {
            for (int a = 0; a < 3; a++) {
                q->vel[a] = Xn[a];
                q->omega[a] = Xn[3 + a];
                double r = q->pos[a] + q->vel[a];
                if (r >= (double)L[a]) r -= (double)L[a];
                else if (r < 0.0) r += (double)L[a];
                q->pos[a] = r;
            }
            if (fabs(q->vel[0]) >= 0.5 || fabs(q->vel[1]) >= 0.5 || fabs(q->vel[2]) >= 0.5)
                c->err |= 2;
            double th = sqrt(q->omega[0] * q->omega[0] + q->omega[1] * q->omega[1] + q->omega[2] * q->omega[2]);
            if (th > 0.0) {
                double ax[3] = {q->omega[0] / th, q->omega[1] / th, q->omega[2] / th}, kxm[3];
                cross(ax, q->m, kxm);
                double km = ax[0] * q->m[0] + ax[1] * q->m[1] + ax[2] * q->m[2];
                double cs = cos(th), sn = sin(th), mn[3];
                for (int a = 0; a < 3; a++) mn[a] = q->m[a] * cs + kxm[a] * sn + ax[a] * km * (1.0 - cs);
                double nn = sqrt(mn[0] * mn[0] + mn[1] * mn[1] + mn[2] * mn[2]);
                for (int a = 0; a < 3; a++) q->m[a] = mn[a] / nn;
                /* the second body axis turns the same way, then is made
                 * orthogonal to m again and normalised */
                double kxe[3], en[3];
                cross(ax, q->e, kxe);
                double ke = ax[0] * q->e[0] + ax[1] * q->e[1] + ax[2] * q->e[2];
                for (int a = 0; a < 3; a++) en[a] = q->e[a] * cs + kxe[a] * sn + ax[a] * ke * (1.0 - cs);
                double em = en[0] * q->m[0] + en[1] * q->m[1] + en[2] * q->m[2];
                for (int a = 0; a < 3; a++) en[a] = en[a] - em * q->m[a];
                double ne = sqrt(en[0] * en[0] + en[1] * en[1] + en[2] * en[2]);
                for (int a = 0; a < 3; a++) q->e[a] = en[a] / ne;
            }
        }
        for (int a = 0; a < 3; a++) { c->trF[3 * k + a] = 0.0; c->trT[3 * k + a] = 0.0; }
    }
}

/* step 5: geometry at the new positions.  A node that turns solid hands its
 * fluid momentum to the colloid; a node that turns fluid is refilled with the
 * equilibrium at rho0 and the local rigid-body velocity, the colloid being
 * debited that momentum, and takes psi and c as the mean of its face
 * neighbours that are fluid before and after. */
static void regeometry(or_ctx *c)
{
    long N = c->N;
    double tr[3] = {0.0, 0.0, 0.0}, dmass = 0.0;
    if (owner_map(c, c->owner_new)) c->err |= 4;
    for (long n = 0; n < N; n++) {
        int o = c->owner[n], w = c->owner_new[n];
        if (o == w) continue;
        int x, y, z;
        coords(c, n, &x, &y, &z);
        if (o >= 0 && w >= 0) { c->err |= 4; continue; }
        if (o < 0) {
            const or_colloid *q = &c->col[w];
            double pm[3] = {0.0, 0.0, 0.0}, r[3], t[3], mass = 0.0;
            for (int i = 0; i < 19; i++) {
                double fi = c->fn[i * N + n];
                pm[0] += fi * CX[i];
                pm[1] += fi * CY[i];
                pm[2] += fi * CZ[i];
                mass += fi;
            }
            disp(c, q, x, y, z, 0, 0.0, r);
            cross(r, pm, t);
            for (int a = 0; a < 3; a++) { c->trF[3 * w + a] += pm[a]; c->trT[3 * w + a] += t[a]; tr[a] += pm[a]; }
            dmass -= mass;
        } else {
            const or_colloid *q = &c->col[o];
            double r[3], uw[3], pm[3], t[3];
            disp(c, q, x, y, z, 0, 0.0, r);
            rigid_velocity(q, r, uw);
            for (int i = 0; i < 19; i++) c->fn[i * N + n] = feq(i, c->p.rho0, uw);
            for (int a = 0; a < 3; a++) pm[a] = c->p.rho0 * uw[a];
            cross(r, pm, t);
            for (int a = 0; a < 3; a++) { c->trF[3 * o + a] -= pm[a]; c->trT[3 * o + a] -= t[a]; tr[a] -= pm[a]; }
            dmass += c->p.rho0;
            double sp = 0.0, sc = 0.0;
            int cnt = 0;
            for (int e = 1; e <= 6; e++) {
                long m = nbr(c, n, e);
                if (c->owner[m] < 0 && c->owner_new[m] < 0) { sp += c->psin[m]; sc += c->ccn[m]; cnt++; }
            }
            if (cnt > 0) { c->psin[n] = sp / cnt; c->ccn[n] = sc / cnt; }
        }
    }
    for (long n = 0; n < N; n++) c->owner[n] = c->owner_new[n];
    for (int a = 0; a < 3; a++) c->diag[OR_DIAG_SUM_TR + a] = tr[a];
    c->diag[OR_DIAG_SUM_DMASS] += dmass;
    build_links(c);
}

int or_step(or_ctx *c, int64_t nsteps)
{
    if (!c) return OR_E_INVALID;
    if (c->stage < 1) return fail(c, OR_E_STATE, "init_fields first");
    if (nsteps < 0) return fail(c, OR_E_INVALID, "negative step count");
    const int nsub = c->p.ch_substeps > 0 ? c->p.ch_substeps : 1;
    for (int64_t s = 0; s < nsteps; s++) {
        chemical_potential(c);
        collide_stream(c);
        soft_contacts(c);
        /* psi/c sub-steps: the first from psi(t), c(t) and mu(t); each later
         * one from the previous result, with mu and chi recomputed and u held */
        c->diag[OR_DIAG_SUM_SRC] = 0.0;
        c->diag[OR_DIAG_SUM_CHI] = 0.0;
        for (int j = 0; j < nsub; j++) {
            if (j > 0) {
                double *t;
                t = c->psi; c->psi = c->psin; c->psin = t;
                t = c->cc; c->cc = c->ccn; c->ccn = t;
                chemical_potential(c);
            }
            scalar_update(c, 1.0 / nsub);
        }
        if (c->ncol > 0) {
            colloid_update(c);
            regeometry(c);
        } else {
            for (int a = 0; a < 3; a++) c->diag[OR_DIAG_SUM_TR + a] = 0.0;
        }
        double *t;
        t = c->f; c->f = c->fn; c->fn = t;
        t = c->psi; c->psi = c->psin; c->psin = t;
        t = c->cc; c->cc = c->ccn; c->ccn = t;
        c->step++;
    }
    return OR_OK;
}

/* ------------------------------------------------------------- readback */
int or_get_fields(or_ctx *c, double *rho, double *u, double *psi, double *cc)
{
    if (!c) return OR_E_INVALID;
    long N = c->N;
    for (long n = 0; n < N; n++) {
        double r = 0.0, m[3] = {0.0, 0.0, 0.0};
        if (c->owner[n] < 0) {
            for (int i = 0; i < 19; i++) {
                double fi = c->f[i * N + n];
                r += fi;
                m[0] += fi * CX[i];
                m[1] += fi * CY[i];
                m[2] += fi * CZ[i];
            }
        }
        if (rho) rho[n] = r;
        if (u)
            for (int a = 0; a < 3; a++) u[a * N + n] = (c->owner[n] < 0) ? m[a] / r : 0.0;
        if (psi) psi[n] = c->psi[n];
        if (cc) cc[n] = c->cc[n];
    }
    return OR_OK;
}

int or_get_populations(or_ctx *c, double *f)
{
    if (!c || !f) return OR_E_INVALID;
    memcpy(f, c->f, sizeof(double) * 19 * c->N);
    return OR_OK;
}

int or_set_populations(or_ctx *c, const double *f)
{
    if (!c || !f) return OR_E_INVALID;
    memcpy(c->f, f, sizeof(double) * 19 * c->N);
    return OR_OK;
}

int or_get_aux(or_ctx *c, double *mu, double *force, double *uforced)
{
    if (!c) return OR_E_INVALID;
    if (mu) memcpy(mu, c->mu, sizeof(double) * c->N);
    if (force) memcpy(force, c->force, sizeof(double) * 3 * c->N);
    if (uforced) memcpy(uforced, c->uf, sizeof(double) * 3 * c->N);
    return OR_OK;
}

int or_get_owner(or_ctx *c, int32_t *owner)
{
    if (!c || !owner) return OR_E_INVALID;
    for (long n = 0; n < c->N; n++) owner[n] = c->owner[n];
    return OR_OK;
}

int or_get_links(or_ctx *c, int32_t *rec4, int64_t cap, int64_t *n)
{
    if (!c || !n) return OR_E_INVALID;
    *n = c->nl;
    if (!rec4) return OR_OK;
    if (cap < c->nl) return fail(c, OR_E_INVALID, "link buffer too small");
    for (long l = 0; l < c->nl; l++) {
        rec4[4 * l + 0] = c->lk[l];
        rec4[4 * l + 1] = c->ln[l];
        rec4[4 * l + 2] = c->ld[l];
        rec4[4 * l + 3] = link_tag(&c->col[c->lk[l]], c->lcap[l]);
    }
    return OR_OK;
}

int or_get_link_slip(or_ctx *c, double *slip3, int64_t cap)
{
    if (!c || !slip3) return OR_E_INVALID;
    if (c->nslip == 0 || c->nslip != c->nl)
        return fail(c, OR_E_STATE, "no slip record for the current link table");
    if (cap < c->nl) return fail(c, OR_E_INVALID, "slip buffer too small");
    for (long i = 0; i < 3 * c->nl; i++) slip3[i] = c->lslip[i];
    return OR_OK;
}

int or_observables(or_ctx *c, or_totals *t, or_colloid *out, int32_t n)
{
    if (!c) return OR_E_INVALID;
    if (t) {
        memset(t, 0, sizeof *t);
        long N = c->N;
        for (long m = 0; m < N; m++) {
            if (c->owner[m] >= 0) continue;
            for (int i = 0; i < 19; i++) {
                double fi = c->f[i * N + m];
                t->mass += fi;
                t->mom[0] += fi * CX[i];
                t->mom[1] += fi * CY[i];
                t->mom[2] += fi * CZ[i];
            }
            t->sum_psi += c->psi[m];
            t->sum_c += c->cc[m];
            t->n_fluid++;
        }
        t->n_links = c->nl;
        /* active links: on the active cap, or in a pattern cell that produces */
        for (long l = 0; l < c->nl; l++) {
            const or_colloid *q = &c->col[c->lk[l]];
            t->n_active += q->pat_bands > 0 ? (q->pat_alpha[c->lcap[l]] != 0.0) : (c->lcap[l] == 0);
        }
        t->step = c->step;
        int e = c->err;
        if (!isfinite(t->mass) || !isfinite(t->sum_psi) || !isfinite(t->sum_c)) e |= 1;
        t->error_bits = e;
    }
    if (out) {
        if (n > c->ncol) n = c->ncol;
        for (int k = 0; k < n; k++) out[k] = c->col[k];
    }
    return OR_OK;
}

/* F0[3] T0[3] zeta[36] trF[3] trT[3] Flast[3] Tlast[3]: 54 doubles */
int or_colloid_diag(or_ctx *c, int32_t k, double *out)
{
    if (!c || !out || k < 0 || k >= c->ncol) return OR_E_INVALID;
    int o = 0;
    for (int a = 0; a < 3; a++) out[o++] = c->F0[3 * k + a];
    for (int a = 0; a < 3; a++) out[o++] = c->T0[3 * k + a];
    for (int j = 0; j < 36; j++) out[o++] = c->zeta[36 * k + j];
    for (int a = 0; a < 3; a++) out[o++] = c->trF[3 * k + a];
    for (int a = 0; a < 3; a++) out[o++] = c->trT[3 * k + a];
    for (int a = 0; a < 3; a++) out[o++] = c->Flast[3 * k + a];
    for (int a = 0; a < 3; a++) out[o++] = c->Tlast[3 * k + a];
    return OR_OK;
}

int or_step_diag(or_ctx *c, double *out)
{
    if (!c || !out) return OR_E_INVALID;
    memcpy(out, c->diag, sizeof c->diag);
    return OR_OK;
}

int or_lattice(int32_t *cvec57, double *w19)
{
    for (int i = 0; i < 19; i++) {
        if (cvec57) { cvec57[3 * i] = CX[i]; cvec57[3 * i + 1] = CY[i]; cvec57[3 * i + 2] = CZ[i]; }
        if (w19) w19[i] = wt(i);
    }
    return OR_OK;
}

/* ------------------------------------------------------------- threads */
/* OpenMP threads of the per-node loops (n <= 0: the OpenMP default); returns
 * the count now in effect (1 without OpenMP).  Results do not depend on it. */
int or_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------ parameter maps */
/* Eq. 10: cos(theta) = ((1+h)^(3/2) - (1-h)^(3/2)) / 2 with h = H / sqrt(kappa b),
 * inverted for h in [-1, 1] by bisection (the right side is increasing in h). */
double or_wetting_H(double theta_deg, double kappa, double b)
{
    double target = cos(theta_deg * M_PI / 180.0);
    double lo = -1.0, hi = 1.0;
    for (int it = 0; it < 200; it++) {
        double h = 0.5 * (lo + hi);
        double v = 0.5 * (pow(1.0 + h, 1.5) - pow(1.0 - h, 1.5));
        if (v < target) lo = h; else hi = h;
    }
    return 0.5 * (lo + hi) * sqrt(kappa * b);
}

/* The contact angle the lattice realises (test infrastructure: the reading
 * of Eqs. 8-10 on this lattice).  The wetting ghost of mu_psi is the
 * derivative of
 *   E = sum_nodes [f(psi) - f(psi_b)] + kappa/2 sum_faces (difference)^2
 *       + H * (psi at the fluid nodes next to the wall),
 * so on a flat wall the state is a one-dimensional chain psi_1, psi_2, ...
 * held at a bulk value far away.  Young: cos(theta) = (gamma_+ - gamma_-) /
 * sigma, gamma_s the least E of the chain against bulk s psi_b and sigma the
 * least E of a free interface between -psi_b and +psi_b.  Each minimum by
 * Newton steps on the exact gradient and tridiagonal Hessian, halved until
 * E does not increase. */
static double chain_E(const double *q, int n, double a, double b, double kappa,
                      double H, int wall, double lo, double hi)
{
    double pb2 = -a / b, fb = a / 2.0 * pb2 + b / 4.0 * pb2 * pb2, E = 0.0;
    for (int i = 0; i < n; i++) {
        E += a / 2.0 * q[i] * q[i] + b / 4.0 * q[i] * q[i] * q[i] * q[i] - fb;
        double right = (i + 1 < n) ? q[i + 1] : hi;
        E += kappa / 2.0 * (right - q[i]) * (right - q[i]);
    }
    if (wall) E += H * q[0];
    else E += kappa / 2.0 * (q[0] - lo) * (q[0] - lo);
    return E;
}

static double chain_min(double *q, int n, double a, double b, double kappa, double H,
                        int wall, double lo, double hi)
{
    double *g = malloc(sizeof(double) * n), *dg = malloc(sizeof(double) * n);
    double *step = malloc(sizeof(double) * n), *t = malloc(sizeof(double) * n);
    double *cc = malloc(sizeof(double) * n);
    double E = chain_E(q, n, a, b, kappa, H, wall, lo, hi);
    for (int it = 0; it < 200; it++) {
        double worst = 0.0;
        for (int i = 0; i < n; i++) {
            double left = (i > 0) ? q[i - 1] : lo, right = (i + 1 < n) ? q[i + 1] : hi;
            g[i] = a * q[i] + b * q[i] * q[i] * q[i] + kappa * (q[i] - right);
            dg[i] = a + 3.0 * b * q[i] * q[i] + kappa;
            if (i > 0 || !wall) { g[i] += kappa * (q[i] - left); dg[i] += kappa; }
            if (i == 0 && wall) g[i] += H;
            if (fabs(g[i]) > worst) worst = fabs(g[i]);
        }
        if (worst < 1e-15) break;
        /* solve (tridiag: dg on the diagonal, -kappa beside it) step = -g */
        cc[0] = -kappa / dg[0];
        step[0] = -g[0] / dg[0];
        for (int i = 1; i < n; i++) {
            double den = dg[i] + kappa * cc[i - 1];
            cc[i] = -kappa / den;
            step[i] = (-g[i] + kappa * step[i - 1]) / den;
        }
        for (int i = n - 2; i >= 0; i--) step[i] -= cc[i] * step[i + 1];
        double s = 1.0, Et = E;
        while (s > 1e-12) {
            for (int i = 0; i < n; i++) t[i] = q[i] + s * step[i];
            Et = chain_E(t, n, a, b, kappa, H, wall, lo, hi);
            if (Et <= E) break;
            s /= 2.0;
        }
        if (s <= 1e-12) break;
        for (int i = 0; i < n; i++) q[i] = t[i];
        E = Et;
    }
    free(g); free(dg); free(step); free(t); free(cc);
    return E;
}

double or_lattice_cos(double a, double b, double kappa, double H)
{
    double pb = sqrt(-a / b), w = sqrt(2.0 * kappa / -a);
    int n = (int)(16.0 * w) + 1;
    if (n < 64) n = 64;
    double *q = malloc(sizeof(double) * 2 * n);
    double gp, gm, sigma = 0.0;
    for (int i = 0; i < n; i++) q[i] = pb;
    gp = chain_min(q, n, a, b, kappa, H, 1, 0.0, pb);
    for (int i = 0; i < n; i++) q[i] = -pb;
    gm = chain_min(q, n, a, b, kappa, H, 1, 0.0, -pb);
    for (int centre = 0; centre < 2; centre++) {
        /* kink started between two nodes, then on a node; keep the lower */
        for (int i = 0; i < 2 * n; i++) q[i] = pb * tanh((i - n + 0.5 * centre) / w);
        double s = chain_min(q, 2 * n, a, b, kappa, 0.0, 0, -pb, pb);
        if (centre == 0 || s < sigma) sigma = s;
    }
    free(q);
    return (gp - gm) / sigma;
}

double or_wetting_H_lattice(double theta_deg, double a, double b, double kappa)
{
    if (!(a < 0.0 && b > 0.0 && kappa > 0.0)) return NAN;
    double target = cos(theta_deg * M_PI / 180.0), Hmax = sqrt(kappa * b);
    double lo = -Hmax, hi = Hmax;
    if (target < or_lattice_cos(a, b, kappa, lo) || target > or_lattice_cos(a, b, kappa, hi))
        return NAN;
    for (int it = 0; it < 60; it++) {
        double mid = 0.5 * (lo + hi);
        if (or_lattice_cos(a, b, kappa, mid) < target) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* solubility ratio r = <c>_oil / <c>_water of the equilibrium c0(psi) =
 * c_b0 + E tanh(psi) (Eq. 1) at psi = -1 (oil) and +1 (water):
 * r = (c_b0 - E tanh 1) / (c_b0 + E tanh 1). */
double or_solubility_E(double ratio, double c_b0)
{
    return -c_b0 * (ratio - 1.0) / ((ratio + 1.0) * tanh(1.0));
}
