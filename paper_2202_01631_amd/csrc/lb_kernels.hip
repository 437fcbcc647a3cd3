// lb_kernels.hip -- gfx950 kernels of one time step of the lattice update of
// the multiphase-multicomponent LB model for self-diffusiophoretic Janus
// colloids (arXiv:2202.01631, Sec. II).
//
// Step sequence (cur -> nxt buffers; in large steps with particles the
// boundary fix-ups and the particle kernels run on a side stream beside the
// bulk kernels, see launch_step):
//   k_mu             mu_psi of Eq. 2 at interior nodes (one-node or
//                    row-vector form)
//   k_mu_bnd         per particle box: mu at nodes next to a particle, with
//                    the wetting ghost of Eqs. 8-9
//   k_collide        force -psi grad(mu), moments, BGK-Guo collision, push
//                    streaming with plain (resting-wall) bounce-back (one-node
//                    form, or k_collide_v: row-vector form)
//   k_scalar         psi and c updates of Eq. 3 at interior nodes (one-node,
//                    row-vector or z-marching row-vector form)
//   k_scalar_bnd     per particle box: psi and c next to a particle (no-flux
//                    solid faces, Janus emission of Eq. 5)
//   k_link_partial   per (link chunk, particle): moving-wall and slip
//                    correction of every link (Eqs. 4, 6), FP64 momentum
//                    exchange partials
//   k_colloid_update per particle: partials summed in chunk order, implicit
//                    rigid-body update
//   k_cover          per particle: cover/uncover repair at the new position
//   k_commit         per particle: owner bytes at the new position
//   k_link_count     per particle: boundary bits, link count per chunk
//   k_link_write     per particle: canonical link table
// Lattice kernels run one node per thread or V consecutive x nodes per lane
// over rows in x (coalesced structure-of-arrays access).
#include <utility>

#include "lb_kernels.h"

namespace lbk {

__device__ __forceinline__ int wrap_p(int v, int L) { return v + 1 == L ? 0 : v + 1; }
__device__ __forceinline__ int wrap_m(int v, int L) { return v == 0 ? L - 1 : v - 1; }

// box of global block (or particle) index g: largest j with start[j] <= g
__device__ __forceinline__ int find_box(const int *__restrict__ start, int nbox, int g)
{
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// f(integral_constant<int, I>) for I = 0 .. N-1, expanded at compile time
template <class F, int... I>
__device__ __forceinline__ void static_for_seq(F &f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F> __device__ __forceinline__ void static_for(F &&f)
{
    static_for_seq(f, std::make_integer_sequence<int, N>{});
}

template <class S> __device__ __forceinline__ S s_tanh(S v);
template <> __device__ __forceinline__ double s_tanh<double>(double v) { return tanh(v); }
template <> __device__ __forceinline__ float s_tanh<float>(float v) { return tanhf(v); }

// Store of a row vector by a bulk kernel: nodes next to a particle (owner
// bit 7) are left to the boundary fix-up blocks of the same launch.
template <class S, int V>
__device__ __forceinline__ void st_interior(S *base, unsigned on, const SVec<S, V> &v, unsigned ow)
{
    const unsigned bm = (V == 4) ? 0x80808080u : 0x8080u;
    if (!(ow & bm)) {
        stb((SVec<S, V> *)base, on, v);
        return;
    }
#pragma unroll
    for (int k = 0; k < V; k++)
        if (!(byte_of(ow, k) & OWN_BOUNDARY)) stb(base, on + k * (unsigned)sizeof(S), v.v[k]);
}

// ------------------------------------------------------------------ k_mu
// mu_psi = a psi + b psi^3 - kappa lap(psi) - C E chi (1 - tanh^2 psi),
// chi = c - c_b0 - E tanh psi (Eq. 2; 1/cosh^2 = 1 - tanh^2, cubic factored
// as b psi (psi-1)(psi+1) + (a+b) psi to keep FP32 cancellation small).
// At a solid face neighbour the Laplacian takes the ghost psi - (H/kappa)|e.n|
// (Eq. 9, n through the face midpoint; H of the surface cell there when the
// particle carries a pattern).
// The node arithmetic lives in helpers with contraction off and explicit
// fused forms, so every launch form of a kernel rounds identically.

// psi value the Laplacian takes across face e (x+, x-, y+, y-, z+, z-) of
// fluid node (x, y, z): the neighbour's, or the wetting ghost at a solid one.
// PAT = false: no particle of the box has a surface pattern or another
// shape than a sphere (the forms that treat boundary nodes inside the bulk
// launches; boxes with such particles take the boundary fix-up launches, and
// these forms stay free of that arithmetic and its registers).
template <class S, bool PAT = true>
__device__ __forceinline__ S face_psi(const KParams &p, const DColloid *__restrict__ col,
                                      uint8_t onb, int e, int x, int y, int z, S ps, S pv)
{
#pragma clang fp contract(off)
    const uint8_t om = onb & OWN_SOLID;
    if (!om) return pv;
    const DColloid &q = col[om - 1];
    double r[3];
    const int ax = e >> 1, sg = (e & 1) ? -1 : 1;
    displacement(q, x, y, z, ax == 0 ? sg : 0, ax == 1 ? sg : 0, ax == 2 ? sg : 0, 0.5, p.nx, p.ny,
                 p.nz, r);
    double en;
    if (PAT && is_spheroid(q)) {
        double n[3];
        spheroid_normal(q, r, n);
        en = fabs(n[ax]);
    } else {
        const double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        en = fabs(r[ax]) / rn;
    }
    const double H = (PAT && q.pb > 0) ? q.pH[surface_cell(q, r)] : q.H;
    const double gh = p.kappa > 0.0 ? (H / p.kappa) * en : 0.0;
    return ps - (S)gh;
}

template <class S> __device__ __forceinline__ S lap6(S ps, const S f[6])
{
#pragma clang fp contract(off)
    S l = S(-6) * ps;
#pragma unroll
    for (int e = 0; e < 6; e++) l = l + f[e];
    return l;
}

// chi = c - c_b0 - E tanh psi, the solute's distance from its equilibrium
// c0(psi) (Eq. 1).  In FP32 arithmetic the kernels that need it form it from
// psi and c with this one expression (cheaper than storing and reloading it);
// in FP64, where tanh is dear, the mu pass stores it (chi_stored) and the
// bulk psi/c updates read it back.  Either way the same value.
template <class S> struct ChiStored { static constexpr bool value = sizeof(S) == 8; };
template <class S> __device__ __forceinline__ S chi_of(const KParams &p, S ps, S cn)
{
#pragma clang fp contract(off)
    return fma(-(S)p.E, s_tanh<S>(ps), cn - (S)p.cb0);
}

template <class S>
__device__ __forceinline__ void mu_chi(const KParams &p, S ps, S lap, S cn, S &mu, S &chi)
{
#pragma clang fp contract(off)
    const S a = (S)p.a, b = (S)p.b;
    const S t = s_tanh<S>(ps);
    chi = fma(-(S)p.E, t, cn - (S)p.cb0);  // chi_of, sharing t
    S m = b * ps * (ps - S(1)) * (ps + S(1));
    m = fma(a + b, ps, m);
    m = fma(-(S)p.kappa, lap, m);
    mu = fma(-(S)(p.C * p.E) * chi, fma(-t, t, S(1)), m);
}

// option LB_STRESS_FORM: the stress of the psi free energy at fluid node n,
// P = (a/2 psi^2 + 3b/4 psi^4 - kappa psi lap - kappa/2 |g|^2) 1 + kappa g g^T,
// g the central difference over the faces (pv: x+, x-, y+, y-, z+, z-, with
// the wetting ghosts at solid faces), and mu_c = -C E chi sech^2(psi), the
// coupling part of mu; stored for the divergence-form force of collide-stream
template <class S>
__device__ __forceinline__ void store_stress(const BoxDesc &D, const KParams &p, int n, S ps,
                                             const S pv[6], S cn)
{
    const S lap = lap6<S>(ps, pv);
    const S g[3] = {S(0.5) * (pv[0] - pv[1]), S(0.5) * (pv[2] - pv[3]), S(0.5) * (pv[4] - pv[5])};
    const S kap = (S)p.kappa;
    const S ps2 = ps * ps;
    const S g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    const S sd = S(0.5) * (S)p.a * ps2 + S(0.75) * (S)p.b * ps2 * ps2 - kap * ps * lap -
                 S(0.5) * kap * g2;
    S *__restrict__ P = (S *)D.b.pst;
    const size_t N = (size_t)p.N;
    P[n] = sd + kap * g[0] * g[0];
    P[N + n] = sd + kap * g[1] * g[1];
    P[2 * N + n] = sd + kap * g[2] * g[2];
    P[3 * N + n] = kap * g[0] * g[1];
    P[4 * N + n] = kap * g[0] * g[2];
    P[5 * N + n] = kap * g[1] * g[2];
    const S t = s_tanh<S>(ps);
    const S chi = fma(-(S)p.E, t, cn - (S)p.cb0);
    ((S *)D.b.muc)[n] = -(S)(p.C * p.E) * chi * fma(-t, t, S(1));
}

// mu of fluid node n = (x, y, z) next to a particle: wetting ghost at every
// solid face (and, in the fix-up launches, the stress of LB_STRESS_FORM)
template <class S, bool PAT = true>
__device__ __forceinline__ void mu_bnd_node(const BoxDesc &D, const KParams &p, int n, int x, int y,
                                            int z)
{
    const S *__restrict__ psi = (const S *)D.b.psi;
    const uint8_t *__restrict__ own = D.b.own;
    const int sy = p.nx, sz = p.nx * p.ny;
    const int nb[6] = {n - x + wrap_p(x, p.nx), n - x + wrap_m(x, p.nx),
                       n + (wrap_p(y, p.ny) - y) * sy, n + (wrap_m(y, p.ny) - y) * sy,
                       n + (wrap_p(z, p.nz) - z) * sz, n + (wrap_m(z, p.nz) - z) * sz};
    const S ps = psi[n];
    S pv[6];
#pragma unroll
    for (int e = 0; e < 6; e++)
        pv[e] = face_psi<S, PAT>(p, D.b.col, own[nb[e]], e, x, y, z, ps, psi[nb[e]]);
    S m, c;
    const S cn = ((const S *)D.b.cc)[n];
    mu_chi<S>(p, ps, lap6<S>(ps, pv), cn, m, c);
    ((S *)D.b.mu)[n] = m;
    if (ChiStored<S>::value) ((S *)D.b.chi)[n] = c;
    if (PAT && (p.flags & LB_STRESS_FORM)) store_stress<S>(D, p, n, ps, pv, cn);
}

// one node per thread; ST: some box of the batch has LB_STRESS_FORM (the
// stress is written for those boxes)
template <class S, bool BND, bool ST = false>
__device__ __forceinline__ void mu_one(const BatchArgs &A, const int blk)
{
    const int j = find_box(A.bstart, A.nbox, blk);
    const BoxDesc &D = A.d[j];
    KParams p = D.p;
    p.ls = D.ls[0];
    const S *__restrict__ psi = (const S *)D.b.psi;
    const S *__restrict__ cc = (const S *)D.b.cc;
    const uint8_t *__restrict__ own = D.b.own;
    S *__restrict__ mu = (S *)D.b.mu;
    S *__restrict__ chi_out = (S *)D.b.chi;
    int x, y, z;
    if (!lattice_node(p, blk - A.bstart[j], x, y, z)) return;
    const int sy = p.nx, sz = p.nx * p.ny;
    const int n = x + sy * y + sz * z;
    const int nb[6] = {n - x + wrap_p(x, p.nx), n - x + wrap_m(x, p.nx),
                       n + (wrap_p(y, p.ny) - y) * sy, n + (wrap_m(y, p.ny) - y) * sy,
                       n + (wrap_p(z, p.nz) - z) * sz, n + (wrap_m(z, p.nz) - z) * sz};
    // all loads issued before anything depends on the owner byte
    const uint8_t o = own[n];
    const unsigned on = (unsigned)n * sizeof(S);
    const S ps = ldb(psi, on), cn = ldb(cc, on);
    S pv[6];
#pragma unroll
    for (int e = 0; e < 6; e++) pv[e] = ldb(psi, (unsigned)nb[e] * sizeof(S));
    if (o & OWN_SOLID) {
        stb(mu, on, S(0));
        if (ChiStored<S>::value) stb(chi_out, on, S(0));
        return;
    }
    if (o & OWN_BOUNDARY) {  // here (BND) or in the fix-up launch
        if (BND) mu_bnd_node<S, false>(D, p, n, x, y, z);
        return;
    }
    S m, c;
    mu_chi<S>(p, ps, lap6<S>(ps, pv), cn, m, c);
    stb(mu, on, m);
    if (ChiStored<S>::value) stb(chi_out, on, c);
    if (ST && (p.flags & LB_STRESS_FORM)) store_stress<S>(D, p, n, ps, pv, cn);
}

// Row-vector form: V consecutive x nodes per lane, 8- or 16-byte loads and
// stores, x neighbours exchanged between lanes (the row wraps inside a lane
// group when the group holds the whole row; segment ends of longer rows are
// read directly).  Needs nx % V == 0.
template <class S, int V, bool BND>
__device__ __forceinline__ void mu_vec(const BatchArgs &A, const int blk)
{
    typedef SVec<S, V> Vec;
    typedef typename OwnWord<V>::T OW;
    const int j = find_box(A.bstart, A.nbox, blk);
    const BoxDesc &D = A.d[j];
    KParams p = D.p;
    p.ls = D.ls[0];
    const S *__restrict__ psi = (const S *)D.b.psi;
    const S *__restrict__ cc = (const S *)D.b.cc;
    const uint8_t *__restrict__ own = D.b.own;
    S *__restrict__ mu = (S *)D.b.mu;
    S *__restrict__ chi_out = (S *)D.b.chi;
    int x0, y, z, li, gb;
    if (!vec_node<V>(p, blk - A.bstart[j], x0, y, z, li, gb)) return;
    const int sy = p.nx, sz = p.nx * p.ny;
    const int n0 = x0 + sy * y + sz * z;
    const int nyp = n0 + (wrap_p(y, p.ny) - y) * sy, nym = n0 + (wrap_m(y, p.ny) - y) * sy;
    const int nzp = n0 + (wrap_p(z, p.nz) - z) * sz, nzm = n0 + (wrap_m(z, p.nz) - z) * sz;
    const unsigned on = (unsigned)n0 * sizeof(S);
    const OW ow = ldb((const OW *)own, (unsigned)n0);
    const Vec pc = ldb((const Vec *)psi, on);
    const Vec pyp = ldb((const Vec *)psi, (unsigned)nyp * sizeof(S));
    const Vec pym = ldb((const Vec *)psi, (unsigned)nym * sizeof(S));
    const Vec pzp = ldb((const Vec *)psi, (unsigned)nzp * sizeof(S));
    const Vec pzm = ldb((const Vec *)psi, (unsigned)nzm * sizeof(S));
    const Vec cv = ldb((const Vec *)cc, on);
    const int Ls = p.ls.bx;
    const int srcl = gb + (li == 0 ? Ls - 1 : li - 1), srcr = gb + (li == Ls - 1 ? 0 : li + 1);
    S pl = __shfl(pc.v[V - 1], srcl), pr = __shfl(pc.v[0], srcr);
    if (p.ls.xseg > 1) {
        const int rb = n0 - x0;
        if (li == 0) pl = ldb(psi, (unsigned)(rb + (x0 == 0 ? p.nx - 1 : x0 - 1)) * sizeof(S));
        if (li == Ls - 1) pr = ldb(psi, (unsigned)(rb + (x0 + V == p.nx ? 0 : x0 + V)) * sizeof(S));
    }
    Vec mv, xv;
#pragma unroll
    for (int k = 0; k < V; k++) {
        const uint8_t o = byte_of(ow, k);
        const S ps = pc.v[k];
        const S pv[6] = {k < V - 1 ? pc.v[k + 1] : pr, k > 0 ? pc.v[k - 1] : pl, pyp.v[k], pym.v[k],
                         pzp.v[k], pzm.v[k]};
        S m, c;
        mu_chi<S>(p, ps, lap6<S>(ps, pv), cv.v[k], m, c);
        const bool solid = (o & OWN_SOLID) != 0;
        mv.v[k] = solid ? S(0) : m;
        xv.v[k] = solid ? S(0) : c;
    }
    st_interior<S, V>(mu, on, mv, ow);
    if (ChiStored<S>::value) st_interior<S, V>(chi_out, on, xv, ow);
    if (BND && (ow & ((V == 4) ? 0x80808080u : 0x8080u))) {
        for (int k = 0; k < V; k++)
            if (byte_of(ow, k) & OWN_BOUNDARY) mu_bnd_node<S, false>(D, p, n0 + k, x0 + k, y, z);
    }
}

// ------------------------------------------------------------- k_collide
// Populations are stored shifted, g_i = f_i - w_i rho0 (scaled for FP16).
// rho = rho0 + sum g; j = sum g c; F = -psi grad(mu) (isotropic lattice
// gradient over the 18 neighbours, mu(x) substituted at solid neighbours; the
// central two-point gradient would make the explicit force/advection coupling
// unstable at grid scale) + external force;
// u = (j + F/2)/rho; g*_i = g_i - (g_i - geq_i)/tau + (1 - 1/2tau) w_i
// [3(c_i - u) + 9 (c_i.u) c_i].F with geq_i = w_i [drho + rho(3 c.u +
// 4.5 (c.u)^2 - 1.5 u.u)] (BGK with Guo forcing).  Push: g*_i goes to
// x + c_i, or back into slot opp(i) of x when x + c_i is solid (resting-wall
// bounce-back; the moving-wall and slip terms are added by k_link_partial).
// The node arithmetic lives in helpers with contraction off and explicit
// fused forms, so the one-node and row-vector forms round identically.

// moments and force of one fluid node
template <class S> struct NodeMoments {
    S drho, rho, ux, uy, uz, Fx, Fy, Fz, uu, uF;
};

// g: the 19 populations; mv[1..18]: mu at the neighbours, replaced by
// m0 = mu(x) where bit i of solid is set
template <class S, bool SF = false, bool SP = false>
__device__ __forceinline__ NodeMoments<S> collide_moments(const KParams &p, const S g[19],
                                                          const S mv[19], S m0, unsigned solid,
                                                          S ps, const S *xv = nullptr,
                                                          S x0 = S(0), S cn = S(0),
                                                          const S *fdiv = nullptr)
{
#pragma clang fp contract(off)
    NodeMoments<S> m;
    S drho = S(0), jx = S(0), jy = S(0), jz = S(0);
#pragma unroll
    for (int i = 0; i < 19; i++) {
        drho = drho + g[i];
        if (cx(i)) jx = cx(i) > 0 ? jx + g[i] : jx - g[i];
        if (cy(i)) jy = cy(i) > 0 ? jy + g[i] : jy - g[i];
        if (cz(i)) jz = cz(i) > 0 ? jz + g[i] : jz - g[i];
    }
    if (SP) {
        // single phase: psi = 0, so -psi grad(mu) adds nothing
        m.Fx = (S)p.fx;
        m.Fy = (S)p.fy;
        m.Fz = (S)p.fz;
    } else if (SF && fdiv) {
        // option LB_STRESS_FORM: the divergence-form force, formed by the caller
        m.Fx = fdiv[0] + (S)p.fx;
        m.Fy = fdiv[1] + (S)p.fy;
        m.Fz = fdiv[2] + (S)p.fz;
    } else {
    // grad(mu) = 3 sum_i w_i c_i mu(x + c_i)
    S mi[19];
#pragma unroll
    for (int i = 1; i < 19; i++) mi[i] = mv[i];
    if (solid) {
#pragma unroll
        for (int i = 1; i < 19; i++)
            if (solid & (1u << i)) mi[i] = m0;
    }
    S gx = S(0), gy = S(0), gz = S(0);
#pragma unroll
    for (int i = 1; i < 19; i++) {
        const S wi = (S)(3.0 * wgt(i));
        if (cx(i)) gx = fma(cx(i) > 0 ? wi : -wi, mi[i], gx);
        if (cy(i)) gy = fma(cy(i) > 0 ? wi : -wi, mi[i], gy);
        if (cz(i)) gz = fma(cz(i) > 0 ? wi : -wi, mi[i], gz);
    }
    m.Fx = fma(-ps, gx, (S)p.fx);
    m.Fy = fma(-ps, gy, (S)p.fy);
    m.Fz = fma(-ps, gz, (S)p.fz);
    }
    if (SF) {
        // option: -c grad(mu_c), mu_c = C chi; xv[1..18]: chi at the
        // neighbours, x0 = chi(x) at solid ones; cn = c(x) (0: no term)
        S hx = S(0), hy = S(0), hz = S(0);
#pragma unroll
        for (int i = 1; i < 19; i++) {
            const S wi = (S)(3.0 * wgt(i));
            const S xi = (solid & (1u << i)) ? x0 : xv[i];
            if (cx(i)) hx = fma(cx(i) > 0 ? wi : -wi, xi, hx);
            if (cy(i)) hy = fma(cy(i) > 0 ? wi : -wi, xi, hy);
            if (cz(i)) hz = fma(cz(i) > 0 ? wi : -wi, xi, hz);
        }
        const S cC = -cn * (S)p.C;
        m.Fx = fma(cC, hx, m.Fx);
        m.Fy = fma(cC, hy, m.Fy);
        m.Fz = fma(cC, hz, m.Fz);
    }
    m.drho = drho;
    m.rho = (S)p.rho0 + drho;
    const S ir = S(1) / m.rho;
    m.ux = fma(S(0.5), m.Fx, jx) * ir;
    m.uy = fma(S(0.5), m.Fy, jy) * ir;
    m.uz = fma(S(0.5), m.Fz, jz) * ir;
    m.uu = fma(m.uz, m.uz, fma(m.uy, m.uy, m.ux * m.ux));
    m.uF = fma(m.uz, m.Fz, fma(m.uy, m.Fy, m.ux * m.Fx));
    return m;
}

// post-collision value of population i; om = 1/tau, pref = 1 - 1/(2 tau)
template <class S>
__device__ __forceinline__ S collide_pop(int i, S gi, const NodeMoments<S> &m, S om, S pref)
{
#pragma clang fp contract(off)
    // c_i.u and c_i.F as signed sums (the components of c_i are 0 or +-1),
    // starting from the first nonzero component
    S cu = S(0), cF = S(0);
    bool any = false;
    if (cx(i)) {
        cu = cx(i) > 0 ? m.ux : -m.ux;
        cF = cx(i) > 0 ? m.Fx : -m.Fx;
        any = true;
    }
    if (cy(i)) {
        const S a = cy(i) > 0 ? m.uy : -m.uy, b = cy(i) > 0 ? m.Fy : -m.Fy;
        cu = any ? cu + a : a;
        cF = any ? cF + b : b;
        any = true;
    }
    if (cz(i)) {
        const S a = cz(i) > 0 ? m.uz : -m.uz, b = cz(i) > 0 ? m.Fz : -m.Fz;
        cu = any ? cu + a : a;
        cF = any ? cF + b : b;
    }
    const S w = (S)wgt(i);
    const S q = fma(S(4.5) * cu, cu, fma(S(3), cu, S(-1.5) * m.uu));
    const S geq = w * fma(m.rho, q, m.drho);
    const S fo = fma(S(9) * cu, cF, S(3) * (cF - m.uF));
    return fma(pref * w, fo, fma(-om, gi - geq, gi));
}

// one node per thread; SF: boxes with LB_SOLUTE_FORCE get the -c grad(mu_c)
// term; SP: every box single phase (psi and mu zero everywhere, so the force
// is the external one): psi and mu are not read, with the same results
template <int P, bool SF, bool SP = false>
__global__ __launch_bounds__(256) void k_collide(BatchArgs A)
{
    typedef typename Prec<P>::T T;
    typedef typename Prec<P>::S S;
    const int *bst = A.bstart + (A.nbox + 1);
    const int j = find_box(bst, A.nbox, blockIdx.x);
    const BoxDesc &D = A.d[j];
    KParams p = D.p;
    p.ls = D.ls[1];
    const T *__restrict__ fin = (const T *)D.b.fin;
    T *__restrict__ fout = (T *)D.b.fout;
    const S *__restrict__ psi = (const S *)D.b.psi;
    const S *__restrict__ mu = (const S *)D.b.mu;
    const uint8_t *__restrict__ own = D.b.own;
    S *__restrict__ uout = (S *)D.b.u;
    int x, y, z;
    if (!lattice_node(p, blockIdx.x - bst[j], x, y, z)) return;
    const int sy = p.nx, sz = p.nx * p.ny;
    const int n = x + sy * y + sz * z;
    const size_t N = (size_t)p.N;
    const int xo[3] = {wrap_m(x, p.nx) - x, 0, wrap_p(x, p.nx) - x};
    const int yo[3] = {(wrap_m(y, p.ny) - y) * sy, 0, (wrap_p(y, p.ny) - y) * sy};
    const int zo[3] = {(wrap_m(z, p.nz) - z) * sz, 0, (wrap_p(z, p.nz) - z) * sz};
    // populations and mu neighbours are loaded before anything depends on
    // the owner byte (solid nodes discard them)
    const uint8_t o = own[n];
    const unsigned on = (unsigned)n * sizeof(T);
    S g[19];
#pragma unroll
    for (int i = 0; i < 19; i++) g[i] = ldp(fin + i * N, on, p.inv_scale);
    const unsigned os = (unsigned)n * sizeof(S);
    S m0 = S(0), ps = S(0);
    S mv[19];
#pragma unroll
    for (int i = 0; i < 19; i++) mv[i] = S(0);
    if (!SP) {
        m0 = ldb(mu, os);
        ps = ldb(psi, os);
#pragma unroll
        for (int i = 1; i < 19; i++)
            mv[i] = ldb(mu, (unsigned)(n + xo[cx(i) + 1] + yo[cy(i) + 1] + zo[cz(i) + 1]) *
                                sizeof(S));
    }
    if (o & OWN_SOLID) return;
    // solid neighbours (only boundary nodes have any), as a mask over i
    unsigned solid = 0;
    if (o & OWN_BOUNDARY) {
#pragma unroll
        for (int i = 1; i < 19; i++) {
            const int m = n + xo[cx(i) + 1] + yo[cy(i) + 1] + zo[cz(i) + 1];
            solid |= (ldb(own, (unsigned)m) & OWN_SOLID) ? (1u << i) : 0u;
        }
    }
    S xv[19], x0 = S(0), cn = S(0);
    if (SF) {
#pragma unroll
        for (int i = 0; i < 19; i++) xv[i] = S(0);
        if (p.flags & LB_SOLUTE_FORCE) {
            const S *__restrict__ cc = (const S *)D.b.cc;
            cn = ldb(cc, os);
            x0 = chi_of<S>(p, ps, cn);
#pragma unroll
            for (int i = 1; i < 19; i++) {
                const unsigned om =
                    (unsigned)(n + xo[cx(i) + 1] + yo[cy(i) + 1] + zo[cz(i) + 1]) * sizeof(S);
                xv[i] = chi_of<S>(p, ldb(psi, om), ldb(cc, om));
            }
        }
    }
    // option LB_STRESS_FORM (one-node form only): -div P - psi grad(mu_c),
    // (div P)_b = 3 sum_i w_i c_ia P_ab(x + c_i), P and mu_c of this node at
    // solid neighbours
    S fdiv[3] = {S(0), S(0), S(0)};
    const bool divform = SF && (p.flags & LB_STRESS_FORM);
    if (divform) {
        const S *__restrict__ Pst = (const S *)D.b.pst;
        const S *__restrict__ muc = (const S *)D.b.muc;
        S dx = S(0), dy = S(0), dz = S(0), hx = S(0), hy = S(0), hz = S(0);
#pragma unroll
        for (int i = 1; i < 19; i++) {
            const int m = (solid & (1u << i)) ? n : n + xo[cx(i) + 1] + yo[cy(i) + 1] + zo[cz(i) + 1];
            const S wi = (S)(3.0 * wgt(i));
            const S mc = muc[m];
            if (cx(i)) {
                const S w = cx(i) > 0 ? wi : -wi;
                dx = fma(w, Pst[m], dx);
                dy = fma(w, Pst[3 * N + m], dy);
                dz = fma(w, Pst[4 * N + m], dz);
                hx = fma(w, mc, hx);
            }
            if (cy(i)) {
                const S w = cy(i) > 0 ? wi : -wi;
                dx = fma(w, Pst[3 * N + m], dx);
                dy = fma(w, Pst[N + m], dy);
                dz = fma(w, Pst[5 * N + m], dz);
                hy = fma(w, mc, hy);
            }
            if (cz(i)) {
                const S w = cz(i) > 0 ? wi : -wi;
                dx = fma(w, Pst[4 * N + m], dx);
                dy = fma(w, Pst[5 * N + m], dy);
                dz = fma(w, Pst[2 * N + m], dz);
                hz = fma(w, mc, hz);
            }
        }
        fdiv[0] = fma(-ps, hx, -dx);
        fdiv[1] = fma(-ps, hy, -dy);
        fdiv[2] = fma(-ps, hz, -dz);
    }
    const NodeMoments<S> M = collide_moments<S, SF, SP>(p, g, mv, m0, solid, ps, xv, x0, cn,
                                                        divform ? fdiv : nullptr);
    const S om = (S)p.om;
    const S pref = (S)p.pref;
    // nodes without solid neighbours store along a straight line (FP64
    // keeps the per-direction test: faster there, measured)
    if (sizeof(T) != sizeof(double) && !solid) {
#pragma unroll
        for (int i = 0; i < 19; i++) {
            const int m = n + xo[cx(i) + 1] + yo[cy(i) + 1] + zo[cz(i) + 1];
            stp(fout + i * N, (unsigned)m * sizeof(T), collide_pop<S>(i, g[i], M, om, pref), p.scale);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 19; i++) {
            const S gs = collide_pop<S>(i, g[i], M, om, pref);
            const int m = n + xo[cx(i) + 1] + yo[cy(i) + 1] + zo[cz(i) + 1];
            if (solid & (1u << i))
                stp(fout + opp(i) * N, on, gs, p.scale);
            else
                stp(fout + i * N, (unsigned)m * sizeof(T), gs, p.scale);
        }
    }
    // u as the psi/c update uses it: times the sub-step length (1 by default)
    const S us = (S)p.sub;
    stb(uout, os, M.ux * us);
    stb(uout + N, os, M.uy * us);
    stb(uout + 2 * N, os, M.uz * us);
}

// V consecutive populations of one plane as S values (FP16 storage through
// its 16-bit patterns, scaled as by ldp / stp) and back
template <int V>
__device__ __forceinline__ void ldpv(const double *b, unsigned off, float, double out[V])
{
    const SVec<double, V> w = ldb((const SVec<double, V> *)b, off);
#pragma unroll
    for (int k = 0; k < V; k++) out[k] = w.v[k];
}
template <int V>
__device__ __forceinline__ void ldpv(const float *b, unsigned off, float, float out[V])
{
    const SVec<float, V> w = ldb((const SVec<float, V> *)b, off);
#pragma unroll
    for (int k = 0; k < V; k++) out[k] = w.v[k];
}
template <int V>
__device__ __forceinline__ void ldpv(const __half *b, unsigned off, float inv, float out[V])
{
    const SVec<unsigned short, V> w = ldb((const SVec<unsigned short, V> *)b, off);
#pragma unroll
    for (int k = 0; k < V; k++) out[k] = __half2float(__ushort_as_half(w.v[k])) * inv;
}
template <int V>
__device__ __forceinline__ void stpv(double *b, unsigned off, const double in[V], float)
{
    SVec<double, V> w;
#pragma unroll
    for (int k = 0; k < V; k++) w.v[k] = in[k];
    stb((SVec<double, V> *)b, off, w);
}
template <int V>
__device__ __forceinline__ void stpv(float *b, unsigned off, const float in[V], float)
{
    SVec<float, V> w;
#pragma unroll
    for (int k = 0; k < V; k++) w.v[k] = in[k];
    stb((SVec<float, V> *)b, off, w);
}
template <int V>
__device__ __forceinline__ void stpv(__half *b, unsigned off, const float in[V], float sc)
{
    SVec<unsigned short, V> w;
#pragma unroll
    for (int k = 0; k < V; k++) w.v[k] = __half_as_ushort(__float2half_rn(in[k] * sc));
    stb((SVec<unsigned short, V> *)b, off, w);
}

// Row-vector form: a lane owns V consecutive x nodes and a group of lanes a
// whole row (the host only selects it when nx / V <= 64).  Populations, the
// nine mu rows of the stencil, psi and u move as V-wide accesses.  The push
// is assembled at the destination: for direction i a lane writes the V slots
// of its own x range in row (y + c_iy, z + c_iz), taking the value that
// crosses in from a neighbour lane by a lane exchange, so every store is
// aligned.  A slot is written only when its source node is fluid and does
// not face a solid node along i (the slots the one-node form leaves alone
// stay untouched); lanes with a particle node in reach store element by
// element.  Results equal the one-node form bit for bit.
template <int P, int V>
__global__ __launch_bounds__(256) void k_collide_v(BatchArgs A)
{
    typedef typename Prec<P>::T T;
    typedef typename Prec<P>::S S;
    typedef typename OwnWord<V>::T OW;
    const int *bst = A.bstart + (A.nbox + 1);
    const int j = find_box(bst, A.nbox, blockIdx.x);
    const BoxDesc &D = A.d[j];
    KParams p = D.p;
    p.ls = D.ls[1];
    const T *__restrict__ fin = (const T *)D.b.fin;
    T *__restrict__ fout = (T *)D.b.fout;
    const S *__restrict__ psi = (const S *)D.b.psi;
    const S *__restrict__ mu = (const S *)D.b.mu;
    const uint8_t *__restrict__ own = D.b.own;
    S *__restrict__ uout = (S *)D.b.u;
    int x0, y, z, li, gb;
    if (!vec_node<V>(p, blockIdx.x - bst[j], x0, y, z, li, gb)) return;
    const int sy = p.nx, sz = p.nx * p.ny;
    const int n0 = x0 + sy * y + sz * z;
    const size_t N = (size_t)p.N;
    const int yo[3] = {(wrap_m(y, p.ny) - y) * sy, 0, (wrap_p(y, p.ny) - y) * sy};
    const int zo[3] = {(wrap_m(z, p.nz) - z) * sz, 0, (wrap_p(z, p.nz) - z) * sz};
    const int Ls = p.ls.bx;
    const int srcl = gb + (li == 0 ? Ls - 1 : li - 1), srcr = gb + (li == Ls - 1 ? 0 : li + 1);
    const unsigned on = (unsigned)n0 * sizeof(T), os = (unsigned)n0 * sizeof(S);
    // every load before anything depends on the owner bytes: owner word,
    // populations, the nine mu rows (row r = 3 (dz + 1) + dy + 1), psi
    const OW ow = ldb((const OW *)own, (unsigned)n0);
    S g[V][19];
#pragma unroll
    for (int i = 0; i < 19; i++) {
        S t[V];
        ldpv<V>(fin + i * N, on, p.inv_scale, t);
#pragma unroll
        for (int k = 0; k < V; k++) g[k][i] = t[k];
    }
    SVec<S, V> mr[9];
#pragma unroll
    for (int r = 0; r < 9; r++)
        mr[r] = ldb((const SVec<S, V> *)mu, (unsigned)(n0 + yo[r % 3] + zo[r / 3]) * sizeof(S));
    const SVec<S, V> pv = ldb((const SVec<S, V> *)psi, os);
    // mu just left and right of the lane's range in the five rows that hold
    // x links (dy = 0 or dz = 0)
    S mxl[9], mxr[9];
#pragma unroll
    for (int r = 0; r < 9; r++) {
        if (r % 3 != 1 && r / 3 != 1) continue;
        mxl[r] = __shfl(mr[r].v[V - 1], srcl);
        mxr[r] = __shfl(mr[r].v[0], srcr);
    }
    const unsigned owl = __shfl((unsigned)ow, srcl), owr = __shfl((unsigned)ow, srcr);
    const unsigned bmask = (V == 4) ? 0x80808080u : 0x8080u;
    const unsigned smask_all = (V == 4) ? 0x7f7f7f7fu : 0x7f7fu;
    const bool bnd = ((unsigned)ow & bmask) != 0;
    // owner words of the other eight rows, for boundary lanes only
    unsigned orow[9];
#pragma unroll
    for (int r = 0; r < 9; r++) orow[r] = (unsigned)ow;
    if (bnd) {
#pragma unroll
        for (int r = 0; r < 9; r++)
            if (r != 4) orow[r] = ldb((const OW *)own, (unsigned)(n0 + yo[r % 3] + zo[r / 3]));
    }
    // per node: solid neighbours, mu with substitution, moments
    NodeMoments<S> M[V];
    unsigned smask[V];
#pragma unroll
    for (int k = 0; k < V; k++) {
        unsigned solid = 0;
        if (byte_of(ow, k) & OWN_BOUNDARY) {
#pragma unroll
            for (int i = 1; i < 19; i++) {
                const int r = 3 * (cz(i) + 1) + cy(i) + 1;
                const int kk = k + cx(i);
                uint8_t b;
                if (kk >= 0 && kk < V) {
                    b = byte_of(orow[r], kk);
                } else if (r == 4) {
                    b = kk < 0 ? byte_of(owl, V - 1) : byte_of(owr, 0);
                } else {
                    const int xe = kk < 0 ? (x0 == 0 ? p.nx - 1 : x0 - 1)
                                          : (x0 + V == p.nx ? 0 : x0 + V);
                    b = own[n0 - x0 + xe + yo[r % 3] + zo[r / 3]];
                }
                solid |= (b & OWN_SOLID) ? (1u << i) : 0u;
            }
        }
        smask[k] = solid;
        S mi[19];
#pragma unroll
        for (int i = 1; i < 19; i++) {
            const int r = 3 * (cz(i) + 1) + cy(i) + 1;
            const int kk = k + cx(i);
            mi[i] = kk < 0 ? mxl[r] : (kk >= V ? mxr[r] : mr[r].v[kk]);
        }
        S gk[19];
#pragma unroll
        for (int i = 0; i < 19; i++) gk[i] = g[k][i];
        M[k] = collide_moments<S>(p, gk, mi, mr[4].v[k], solid, pv.v[k]);
    }
    const S om = (S)p.om;
    const S pref = (S)p.pref;
    // sources of this lane's slots: its own nodes and the two nodes next to
    // its range; all fluid away from particles -> whole-vector stores
    const uint8_t oL = byte_of(owl, V - 1), oR = byte_of(owr, 0);
    const bool clean = (unsigned)ow == 0u && oL == 0 && oR == 0;
    const unsigned smL = __shfl(smask[V - 1], srcl), smR = __shfl(smask[0], srcr);
    // the direction loop is expanded at compile time: the unroller leaves
    // loops with lane exchanges under direction-dependent branches rolled
    static_for<19>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        S gs[V];
#pragma unroll
        for (int k = 0; k < V; k++) gs[k] = collide_pop<S>(i, g[k][i], M[k], om, pref);
        // slot k of the destination range takes source k - cx(i)
        S v[V];
        if (cx(i) == 0) {
#pragma unroll
            for (int k = 0; k < V; k++) v[k] = gs[k];
        } else if (cx(i) > 0) {
            v[0] = __shfl(gs[V - 1], srcl);
#pragma unroll
            for (int k = 1; k < V; k++) v[k] = gs[k - 1];
        } else {
#pragma unroll
            for (int k = 0; k < V - 1; k++) v[k] = gs[k + 1];
            v[V - 1] = __shfl(gs[0], srcr);
        }
        const unsigned dst = (unsigned)(n0 + yo[cy(i) + 1] + zo[cz(i) + 1]) * sizeof(T);
        if (clean) {
            stpv<V>(fout + i * N, dst, v, p.scale);
        } else {
#pragma unroll
            for (int k = 0; k < V; k++) {
                const int ks = k - cx(i);
                const uint8_t so = ks < 0 ? oL : (ks >= V ? oR : byte_of(ow, ks));
                const unsigned sm = ks < 0 ? smL : (ks >= V ? smR : smask[ks]);
                if (!(so & OWN_SOLID) && !(sm & (1u << i)))
                    stp(fout + i * N, dst + k * (unsigned)sizeof(T), v[k], p.scale);
            }
            // resting-wall bounce-back of this lane's boundary nodes
            if (i > 0) {
#pragma unroll
                for (int k = 0; k < V; k++)
                    if (smask[k] & (1u << i))
                        stp(fout + opp(i) * N, on + k * (unsigned)sizeof(T), gs[k], p.scale);
            }
        }
    });
    // u at fluid nodes, times the sub-step length (1 by default)
    const S us = (S)p.sub;
    if (!((unsigned)ow & smask_all)) {
        SVec<S, V> w0, w1, w2;
#pragma unroll
        for (int k = 0; k < V; k++) {
            w0.v[k] = M[k].ux * us;
            w1.v[k] = M[k].uy * us;
            w2.v[k] = M[k].uz * us;
        }
        stb((SVec<S, V> *)uout, os, w0);
        stb((SVec<S, V> *)(uout + N), os, w1);
        stb((SVec<S, V> *)(uout + 2 * N), os, w2);
    } else {
#pragma unroll
        for (int k = 0; k < V; k++) {
            if (byte_of(ow, k) & OWN_SOLID) continue;
            const unsigned ok = os + k * (unsigned)sizeof(S);
            stb(uout, ok, M[k].ux * us);
            stb(uout + N, ok, M[k].uy * us);
            stb(uout + 2 * N, ok, M[k].uz * us);
        }
    }
}

// -------------------------------------------------------------- k_scalar
// psi' = psi - sum_e J_e + M sum_e (mu_e - mu),
// c'   = c - sum_e Jc_e + D sum_e (chi_e - chi) + emission - k_d chi,
// J_e = 1/2 (u.e + u_e.e) 1/2 (psi + psi_e) over the 6 faces, nothing
// through faces shared with solid nodes (Eq. 3, explicit Euler, dt = 1).
// Emission: alpha of the cap of each link of the node (Eq. 5).

// face sums of one fluid node; faces in the order x+, x-, y+, y-, z+, z-.
// Returns psi' and the c' partial c - sum Jc + D sum (chi_e - chi).
template <class S>
__device__ __forceinline__ void psi_c_update(const KParams &p, S ps, S cn, S chi, S m0,
                                             const S u0[3], const S um[6], const S pm[6],
                                             const S cm[6], const S mm[6], const S xm[6],
                                             unsigned solid, S &psn, S &cpart)
{
#pragma clang fp contract(off)
    S adv_p = S(0), adv_c = S(0), dmu = S(0), dchi = S(0);
#pragma unroll
    for (int e = 0; e < 6; e++) {
        const bool fl = !(solid & (1u << e));  // no flux through a solid face
        const S us = u0[e >> 1] + um[e];
        const S ue = (e & 1) ? S(-0.5) * us : S(0.5) * us;
        adv_p = fl ? fma(ue, S(0.5) * (ps + pm[e]), adv_p) : adv_p;
        adv_c = fl ? fma(ue, S(0.5) * (cn + cm[e]), adv_c) : adv_c;
        dmu = fl ? dmu + (mm[e] - m0) : dmu;
        dchi = fl ? dchi + (xm[e] - chi) : dchi;
    }
    psn = fma((S)p.M, dmu, ps - adv_p);
    cpart = fma((S)p.D, dchi, cn - adv_c);
}

// Emission of boundary node n = (x, y, z): alpha of the surface cell (the
// cap of a Janus particle) of every link to a solid neighbour, directions in
// ascending order
template <class S, bool PAT = true>
__device__ S emission(const KParams &p, const DColloid *__restrict__ col,
                      const uint8_t *__restrict__ own, int n, int x, int y, int z)
{
#pragma clang fp contract(off)
    const int sy = p.nx, sz = p.nx * p.ny;
    const int xo[3] = {wrap_m(x, p.nx) - x, 0, wrap_p(x, p.nx) - x};
    const int yo[3] = {(wrap_m(y, p.ny) - y) * sy, 0, (wrap_p(y, p.ny) - y) * sy};
    const int zo[3] = {(wrap_m(z, p.nz) - z) * sz, 0, (wrap_p(z, p.nz) - z) * sz};
    // all 18 owner bytes are loaded before any is used
    uint8_t om[19];
#pragma unroll
    for (int d = 1; d < 19; d++)
        om[d] = ldb(own, (unsigned)(n + xo[cx(d) + 1] + yo[cy(d) + 1] + zo[cz(d) + 1])) & OWN_SOLID;
    S src = S(0);
#pragma unroll
    for (int d = 1; d < 19; d++) {
        if (!om[d]) continue;
        const DColloid &q = col[om[d] - 1];
        double r[3];
        displacement(q, x, y, z, cx(d), cy(d), cz(d), 0.5, p.nx, p.ny, p.nz, r);
        const double al = PAT ? cell_alpha(q, surface_cell(q, r)) : (active_cap(q, r) ? q.am : q.ap);
        src = src + (S)(al * p.sub);
    }
    return src;
}

// psi and c of fluid node n = (x, y, z) next to a particle: no flux through
// solid faces, emission of its links
template <class S, bool PAT = true>
__device__ void psic_bnd_node(const BoxDesc &D, const KParams &p, int n, int x, int y, int z)
{
    const S *__restrict__ psi = (const S *)D.b.psi;
    const S *__restrict__ cc = (const S *)D.b.cc;
    const S *__restrict__ mu = (const S *)D.b.mu;
    const S *__restrict__ ua[3] = {(const S *)D.b.u, (const S *)D.b.u + p.N,
                                   (const S *)D.b.u + 2 * (size_t)p.N};
    const uint8_t *__restrict__ own = D.b.own;
    const int sy = p.nx, sz = p.nx * p.ny;
    const int fn[6] = {n - x + wrap_p(x, p.nx), n - x + wrap_m(x, p.nx),
                       n + (wrap_p(y, p.ny) - y) * sy, n + (wrap_m(y, p.ny) - y) * sy,
                       n + (wrap_p(z, p.nz) - z) * sz, n + (wrap_m(z, p.nz) - z) * sz};
    const S ps = psi[n], cn = cc[n], chi = chi_of<S>(p, ps, cn), m0 = mu[n];
    const S u0[3] = {ua[0][n], ua[1][n], ua[2][n]};
    S um[6], pm[6], cm[6], mm[6], xm[6];
    unsigned solid = 0;
#pragma unroll
    for (int e = 0; e < 6; e++) {
        const int m = fn[e];
        um[e] = ua[e >> 1][m];
        pm[e] = psi[m];
        cm[e] = cc[m];
        mm[e] = mu[m];
        xm[e] = chi_of<S>(p, pm[e], cm[e]);
        solid |= (own[m] & OWN_SOLID) ? (1u << e) : 0u;
    }
    S psn, cpart;
    psi_c_update<S>(p, ps, cn, chi, m0, u0, um, pm, cm, mm, xm, solid, psn, cpart);
    ((S *)D.b.psin)[n] = psn;
    ((S *)D.b.ccn)[n] = fma(-(S)p.kd, chi, cpart + emission<S, PAT>(p, D.b.col, own, n, x, y, z));
}

// one node per thread.  SP (every box single phase: psi and mu zero, chi =
// c): psi, mu and chi are not read and psi is not written (it stays zero),
// with the same results for c
template <class S, bool BND, bool SP = false>
__device__ __forceinline__ void psic_one(const BatchArgs &A, const int blk)
{
    const int *bst = A.bstart + 2 * (A.nbox + 1);
    const int j = find_box(bst, A.nbox, blk);
    const BoxDesc &D = A.d[j];
    KParams p = D.p;
    p.ls = D.ls[2];
    const S *__restrict__ psi = (const S *)D.b.psi;
    const S *__restrict__ cc = (const S *)D.b.cc;
    const S *__restrict__ mu = (const S *)D.b.mu;
    const S *__restrict__ ua[3] = {(const S *)D.b.u, (const S *)D.b.u + p.N,
                                   (const S *)D.b.u + 2 * (size_t)p.N};
    const uint8_t *__restrict__ own = D.b.own;
    S *__restrict__ psin = (S *)D.b.psin;
    S *__restrict__ ccn = (S *)D.b.ccn;
    int x, y, z;
    if (!lattice_node(p, blk - bst[j], x, y, z)) return;
    const int sy = p.nx, sz = p.nx * p.ny;
    const int n = x + sy * y + sz * z;
    const int fn[6] = {n - x + wrap_p(x, p.nx), n - x + wrap_m(x, p.nx),
                       n + (wrap_p(y, p.ny) - y) * sy, n + (wrap_m(y, p.ny) - y) * sy,
                       n + (wrap_p(z, p.nz) - z) * sz, n + (wrap_m(z, p.nz) - z) * sz};
    // every field load is issued before anything depends on the owner byte
    const uint8_t o = own[n];
    const unsigned on = (unsigned)n * sizeof(S);
    const S cn = ldb(cc, on);
    constexpr bool CS = ChiStored<S>::value && !SP;
    const S *__restrict__ chiv = (const S *)D.b.chi;
    const S ps = SP ? S(0) : ldb(psi, on), m0 = SP ? S(0) : ldb(mu, on);
    const S chi_l = CS ? ldb(chiv, on) : S(0);
    S xm_l[6];
    const S u0[3] = {ldb(ua[0], on), ldb(ua[1], on), ldb(ua[2], on)};
    S um[6], pm[6], cm[6], mm[6], xm[6];
#pragma unroll
    for (int e = 0; e < 6; e++) {
        const unsigned om = (unsigned)fn[e] * sizeof(S);
        um[e] = ldb(ua[e >> 1], om);
        cm[e] = ldb(cc, om);
        pm[e] = SP ? S(0) : ldb(psi, om);
        mm[e] = SP ? S(0) : ldb(mu, om);
        xm_l[e] = CS ? ldb(chiv, om) : S(0);
    }
    if (o & OWN_SOLID) {
        if (!SP) stb(psin, on, ps);
        stb(ccn, on, cn);
        return;
    }
    if (o & OWN_BOUNDARY) {  // here (BND) or in the fix-up launch
        if (BND) psic_bnd_node<S, false>(D, p, n, x, y, z);
        return;
    }
    // chi read back (FP64) or formed from psi and c (single phase: c itself)
    const S chi = SP ? cn : (CS ? chi_l : chi_of<S>(p, ps, cn));
#pragma unroll
    for (int e = 0; e < 6; e++) xm[e] = SP ? cm[e] : (CS ? xm_l[e] : chi_of<S>(p, pm[e], cm[e]));
    S psn, cpart;
    psi_c_update<S>(p, ps, cn, chi, m0, u0, um, pm, cm, mm, xm, 0u, psn, cpart);
    if (!SP) stb(psin, on, psn);
    stb(ccn, on, fma(-(S)p.kd, chi, cpart));
}

// Row-vector form (as k_mu_v): V consecutive x nodes per lane, x neighbours
// of psi, c, mu, chi and u_x exchanged between lanes.  SP as for psic_one:
// only c and u are read, only c is written.
template <class S, int V, bool BND, bool SP = false>
__device__ __forceinline__ void psic_vec(const BatchArgs &A, const int blk)
{
    typedef SVec<S, V> Vec;
    typedef typename OwnWord<V>::T OW;
    const int *bst = A.bstart + 2 * (A.nbox + 1);
    const int j = find_box(bst, A.nbox, blk);
    const BoxDesc &D = A.d[j];
    KParams p = D.p;
    p.ls = D.ls[2];
    const S *__restrict__ psi = (const S *)D.b.psi;
    const S *__restrict__ cc = (const S *)D.b.cc;
    const S *__restrict__ mu = (const S *)D.b.mu;
    constexpr bool CS = ChiStored<S>::value && !SP;  // chi read back, not formed
    const S *__restrict__ chiv = (const S *)D.b.chi;
    const S *__restrict__ ux = (const S *)D.b.u;
    const S *__restrict__ uy = ux + p.N;
    const S *__restrict__ uz = ux + 2 * (size_t)p.N;
    const uint8_t *__restrict__ own = D.b.own;
    S *__restrict__ psin = (S *)D.b.psin;
    S *__restrict__ ccn = (S *)D.b.ccn;
    // The block's lane groups hold consecutive row segments, so most y
    // neighbour rows are the centre rows of another group of the block:
    // those come from LDS, only rows outside the block from memory.  Every
    // thread reaches the barrier (no early return before it).
    // psi, c, mu, chi, u_y centre vectors (SP: c, u_y)
    constexpr int NS = SP ? 2 : 5;
    __shared__ Vec shr[NS][256];
    auto sf = [](int f) { return SP ? (f == 4 ? 1 : 0) : f; };  // field -> LDS slot
    int x0 = 0, y = 0, z = 0, li = 0, gb = 0;
    const bool live = vec_node<V>(p, blk - bst[j], x0, y, z, li, gb);
    const int sy = p.nx, sz = p.nx * p.ny;
    const int n0 = x0 + sy * y + sz * z;
    const int nb[4] = {n0 + (wrap_p(y, p.ny) - y) * sy, n0 + (wrap_m(y, p.ny) - y) * sy,
                       n0 + (wrap_p(z, p.nz) - z) * sz, n0 + (wrap_m(z, p.nz) - z) * sz};
    // lane holding the same x range of the y +- 1 row, if inside the block
    int src[2] = {-1, -1};
    {
        const int by = p.ls.by, xs = p.ls.xseg;
        const int w = (int)threadIdx.x >> 6, g = gb / p.ls.bx;
        // group slot of this lane in the block; the group of row r, segment
        // s is slot + (r - row) * xseg
        const int slot = w * by + g;
        const int yn[2] = {wrap_p(y, p.ny), wrap_m(y, p.ny)};
#pragma unroll
        for (int e = 0; e < 2; e++) {
            const int st = slot + (yn[e] - y) * xs;
            if (live && st >= 0 && st < 4 * by) src[e] = (st / by) * 64 + (st % by) * p.ls.bx + li;
        }
    }
    const unsigned on = (unsigned)n0 * sizeof(S);
    OW ow = 0;
    Vec c0[4], u0x, u0y, u0z, nbv[4][4], uyp, uym, uzp, uzm;  // nbv: [field][y+, y-, z+, z-]
    if (live) {
        ow = ldb((const OW *)own, (unsigned)n0);
        // centre vectors of the four stencil fields and u, then the rows
        // from memory: z +- 1 always, y +- 1 outside the block
        if (!SP) c0[0] = ldb((const Vec *)psi, on);
        c0[1] = ldb((const Vec *)cc, on);
        if (!SP) c0[2] = ldb((const Vec *)mu, on);
        if (CS) c0[3] = ldb((const Vec *)chiv, on);
        u0x = ldb((const Vec *)ux, on);
        u0y = ldb((const Vec *)uy, on);
        u0z = ldb((const Vec *)uz, on);
#pragma unroll
        for (int e = 0; e < 2; e++) {
            if (src[e] >= 0) continue;
            const unsigned om = (unsigned)nb[e] * sizeof(S);
            if (!SP) nbv[0][e] = ldb((const Vec *)psi, om);
            nbv[1][e] = ldb((const Vec *)cc, om);
            if (!SP) nbv[2][e] = ldb((const Vec *)mu, om);
            if (CS) nbv[3][e] = ldb((const Vec *)chiv, om);
            if (e == 0) uyp = ldb((const Vec *)uy, om);
            else uym = ldb((const Vec *)uy, om);
        }
#pragma unroll
        for (int e = 2; e < 4; e++) {
            const unsigned om = (unsigned)nb[e] * sizeof(S);
            if (!SP) nbv[0][e] = ldb((const Vec *)psi, om);
            nbv[1][e] = ldb((const Vec *)cc, om);
            if (!SP) nbv[2][e] = ldb((const Vec *)mu, om);
            if (CS) nbv[3][e] = ldb((const Vec *)chiv, om);
        }
        uzp = ldb((const Vec *)uz, (unsigned)nb[2] * sizeof(S));
        uzm = ldb((const Vec *)uz, (unsigned)nb[3] * sizeof(S));
        if (!SP && !CS) {
            // chi of the centre vector and of the rows read from memory
#pragma unroll
            for (int k = 0; k < V; k++) c0[3].v[k] = chi_of<S>(p, c0[0].v[k], c0[1].v[k]);
#pragma unroll
            for (int e = 0; e < 4; e++) {
                if (e < 2 && src[e] >= 0) continue;
#pragma unroll
                for (int k = 0; k < V; k++) nbv[3][e].v[k] = chi_of<S>(p, nbv[0][e].v[k], nbv[1][e].v[k]);
            }
        }
#pragma unroll
        for (int f = 0; f < 4; f++)
            if (!SP || f == 1) shr[sf(f)][threadIdx.x] = c0[f];
        shr[sf(4)][threadIdx.x] = u0y;
    }
    __syncthreads();
    if (!live) return;
#pragma unroll
    for (int e = 0; e < 2; e++) {
        if (src[e] < 0) continue;
#pragma unroll
        for (int f = 0; f < 4; f++)
            if (!SP || f == 1) nbv[f][e] = shr[sf(f)][src[e]];
        if (e == 0) uyp = shr[sf(4)][src[e]];
        else uym = shr[sf(4)][src[e]];
    }
    if (SP) {
        // psi and mu zero, chi the solute itself
#pragma unroll
        for (int k = 0; k < V; k++) { c0[0].v[k] = S(0); c0[2].v[k] = S(0); }
        c0[3] = c0[1];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            nbv[0][e] = c0[0];
            nbv[2][e] = c0[0];
            nbv[3][e] = nbv[1][e];
        }
    }
    // x neighbours: last node of the lane on the left, first of the right
    const int Ls = p.ls.bx;
    const int srcl = gb + (li == 0 ? Ls - 1 : li - 1), srcr = gb + (li == Ls - 1 ? 0 : li + 1);
    S fl[5], fr[5];  // psi, c, mu, chi, u_x
#pragma unroll
    for (int f = 0; f < 4; f++) {
        if (SP && f != 1) continue;
        fl[f] = __shfl(c0[f].v[V - 1], srcl);
        fr[f] = __shfl(c0[f].v[0], srcr);
    }
    fl[4] = __shfl(u0x.v[V - 1], srcl);
    fr[4] = __shfl(u0x.v[0], srcr);
    if (p.ls.xseg > 1) {
        const int rb = n0 - x0;
        if (li == 0) {
            const unsigned ol = (unsigned)(rb + (x0 == 0 ? p.nx - 1 : x0 - 1)) * sizeof(S);
            fl[1] = ldb(cc, ol);
            if (!SP) {
                fl[0] = ldb(psi, ol);
                fl[2] = ldb(mu, ol);
                fl[3] = CS ? ldb(chiv, ol) : chi_of<S>(p, fl[0], fl[1]);
            }
            fl[4] = ldb(ux, ol);
        }
        if (li == Ls - 1) {
            const unsigned orr = (unsigned)(rb + (x0 + V == p.nx ? 0 : x0 + V)) * sizeof(S);
            fr[1] = ldb(cc, orr);
            if (!SP) {
                fr[0] = ldb(psi, orr);
                fr[2] = ldb(mu, orr);
                fr[3] = CS ? ldb(chiv, orr) : chi_of<S>(p, fr[0], fr[1]);
            }
            fr[4] = ldb(ux, orr);
        }
    }
    if (SP) {
        fl[0] = fr[0] = fl[2] = fr[2] = S(0);
        fl[3] = fl[1];
        fr[3] = fr[1];
    }
    Vec pnv, cnv;
#pragma unroll
    for (int k = 0; k < V; k++) {
        const uint8_t o = byte_of(ow, k);
        S nbs[4][6];
#pragma unroll
        for (int f = 0; f < 4; f++) {
            nbs[f][0] = k < V - 1 ? c0[f].v[k + 1] : fr[f];
            nbs[f][1] = k > 0 ? c0[f].v[k - 1] : fl[f];
#pragma unroll
            for (int e = 0; e < 4; e++) nbs[f][2 + e] = nbv[f][e].v[k];
        }
        const S um[6] = {k < V - 1 ? u0x.v[k + 1] : fr[4], k > 0 ? u0x.v[k - 1] : fl[4],
                         uyp.v[k], uym.v[k], uzp.v[k], uzm.v[k]};
        const S u0[3] = {u0x.v[k], u0y.v[k], u0z.v[k]};
        S psn, cpart;
        psi_c_update<S>(p, c0[0].v[k], c0[1].v[k], c0[3].v[k], c0[2].v[k], u0, um, nbs[0], nbs[1],
                        nbs[2], nbs[3], 0u, psn, cpart);
        const bool sol = (o & OWN_SOLID) != 0;
        pnv.v[k] = sol ? c0[0].v[k] : psn;
        cnv.v[k] = sol ? c0[1].v[k] : fma(-(S)p.kd, c0[3].v[k], cpart);
    }
    if (!SP) st_interior<S, V>(psin, on, pnv, ow);
    st_interior<S, V>(ccn, on, cnv, ow);
    if (BND && (ow & ((V == 4) ? 0x80808080u : 0x8080u))) {
        for (int k = 0; k < V; k++)
            if (byte_of(ow, k) & OWN_BOUNDARY) psic_bnd_node<S, false>(D, p, n0 + k, x0 + k, y, z);
    }
}

// z-marching row-vector form: each lane also marches zc consecutive planes
// of its row.  psi, c, mu, chi, u_z and the owner bytes of planes z - 1, z,
// z + 1 stay in registers, and the next plane is loaded while the current
// one is computed, so a plane costs its centre loads and the y neighbour
// rows only.  Blocks: bpp blocks per chunk of zc planes, chunks in order.
template <class S, int V, bool BND>
__device__ __forceinline__ void psic_zmarch(const BatchArgs &A, const int blk)
{
    typedef SVec<S, V> Vec;
    typedef typename OwnWord<V>::T OW;
    const int *bst = A.bstart + 2 * (A.nbox + 1);
    const int j = find_box(bst, A.nbox, blk);
    const BoxDesc &D = A.d[j];
    const KParams p = D.p;
    const LaunchShape ls = D.ls[2];
    const S *__restrict__ psi = (const S *)D.b.psi;
    const S *__restrict__ cc = (const S *)D.b.cc;
    const S *__restrict__ mu = (const S *)D.b.mu;
    const S *__restrict__ ux = (const S *)D.b.u;
    const S *__restrict__ uy = ux + p.N;
    const S *__restrict__ uz = ux + 2 * (size_t)p.N;
    const uint8_t *__restrict__ own = D.b.own;
    S *__restrict__ psin = (S *)D.b.psin;
    S *__restrict__ ccn = (S *)D.b.ccn;
    // fields kept over z; chi (slot 3) read back in FP64, else formed from
    // psi and c
    constexpr bool CS = ChiStored<S>::value;
    const S *__restrict__ wf[5] = {psi, cc, mu, CS ? (const S *)D.b.chi : nullptr, uz};
    auto chi_vec = [&](Vec &x, const Vec &ps, const Vec &cv) {
        if (CS) return;
#pragma unroll
        for (int k = 0; k < V; k++) x.v[k] = chi_of<S>(p, ps.v[k], cv.v[k]);
    };
    const int w = (int)threadIdx.x >> 6, l = (int)threadIdx.x & 63;
    const int Ls = ls.bx, g = l / Ls;
    if (g >= ls.by) return;
    const int li = l - g * Ls, gb = g * Ls;
    const int b = blk - bst[j];
    const int chunk = b / ls.bpp;
    const int sg = ((b - chunk * ls.bpp) * 4 + w) * ls.by + g;
    const int y = sg / ls.xseg, seg = sg - y * ls.xseg;
    if (y >= p.ny) return;
    const int x0 = (seg * Ls + li) * V;
    const int z0 = chunk * ls.zc;
    const int z1 = min(z0 + ls.zc, p.nz);
    const int sy = p.nx, sz = p.nx * p.ny;
    const int c0 = x0 + sy * y;
    const int dyp = (wrap_p(y, p.ny) - y) * sy, dym = (wrap_m(y, p.ny) - y) * sy;
    const int srcl = gb + (li == 0 ? Ls - 1 : li - 1), srcr = gb + (li == Ls - 1 ? 0 : li + 1);
    Vec W[5][3];    // [field][z - 1, z, z + 1]
    unsigned WO[3];
    Vec uxc, uyc;   // u_x, u_y of plane z
    {
        const int pl[3] = {wrap_m(z0, p.nz), z0, wrap_p(z0, p.nz)};
#pragma unroll
        for (int s = 0; s < 3; s++) {
            const int n = c0 + sz * pl[s];
#pragma unroll
            for (int f = 0; f < 5; f++)
                if (f != 3 || CS) W[f][s] = ldb((const Vec *)wf[f], (unsigned)n * sizeof(S));
            chi_vec(W[3][s], W[0][s], W[1][s]);
            WO[s] = ldb((const OW *)own, (unsigned)n);
        }
        const unsigned o0 = (unsigned)(c0 + sz * z0) * sizeof(S);
        uxc = ldb((const Vec *)ux, o0);
        uyc = ldb((const Vec *)uy, o0);
    }
    for (int z = z0; z < z1; z++) {
        const int n0 = c0 + sz * z;
        const unsigned on = (unsigned)n0 * sizeof(S);
        // next plane: window fields of z + 2, u_x and u_y of z + 1
        Vec nW[5], nux, nuy;
        unsigned nO = 0;
        if (z + 1 < z1) {
            int z2 = z + 2;
            if (z2 >= p.nz) z2 -= p.nz;
            const int n2 = c0 + sz * z2;
#pragma unroll
            for (int f = 0; f < 5; f++)
                if (f != 3 || CS) nW[f] = ldb((const Vec *)wf[f], (unsigned)n2 * sizeof(S));
            chi_vec(nW[3], nW[0], nW[1]);
            nO = ldb((const OW *)own, (unsigned)n2);
            const unsigned o1 = (unsigned)(c0 + sz * wrap_p(z, p.nz)) * sizeof(S);
            nux = ldb((const Vec *)ux, o1);
            nuy = ldb((const Vec *)uy, o1);
        }
        // y neighbour rows of plane z: psi, c, mu, chi, u_y
        Vec Y[5][2];
        const unsigned oyp = (unsigned)(n0 + dyp) * sizeof(S), oym = (unsigned)(n0 + dym) * sizeof(S);
#pragma unroll
        for (int f = 0; f < 4; f++) {
            if (f == 3 && !CS) continue;
            Y[f][0] = ldb((const Vec *)wf[f], oyp);
            Y[f][1] = ldb((const Vec *)wf[f], oym);
        }
        chi_vec(Y[3][0], Y[0][0], Y[1][0]);
        chi_vec(Y[3][1], Y[0][1], Y[1][1]);
        Y[4][0] = ldb((const Vec *)uy, oyp);
        Y[4][1] = ldb((const Vec *)uy, oym);
        // x neighbours: last node of the lane on the left, first of the right
        S fl[5], fr[5];  // psi, c, mu, chi, u_x
#pragma unroll
        for (int f = 0; f < 4; f++) {
            fl[f] = __shfl(W[f][1].v[V - 1], srcl);
            fr[f] = __shfl(W[f][1].v[0], srcr);
        }
        fl[4] = __shfl(uxc.v[V - 1], srcl);
        fr[4] = __shfl(uxc.v[0], srcr);
        const unsigned ow = WO[1];
        if (ls.xseg > 1) {
            const int rb = n0 - x0;
            if (li == 0) {
                const unsigned ol = (unsigned)(rb + (x0 == 0 ? p.nx - 1 : x0 - 1)) * sizeof(S);
#pragma unroll
                for (int f = 0; f < 3; f++) fl[f] = ldb(wf[f], ol);
                fl[3] = CS ? ldb(wf[3], ol) : chi_of<S>(p, fl[0], fl[1]);
                fl[4] = ldb(ux, ol);
            }
            if (li == Ls - 1) {
                const unsigned orr = (unsigned)(rb + (x0 + V == p.nx ? 0 : x0 + V)) * sizeof(S);
#pragma unroll
                for (int f = 0; f < 3; f++) fr[f] = ldb(wf[f], orr);
                fr[3] = CS ? ldb(wf[3], orr) : chi_of<S>(p, fr[0], fr[1]);
                fr[4] = ldb(ux, orr);
            }
        }
        Vec pnv, cnv;
#pragma unroll
        for (int k = 0; k < V; k++) {
            const uint8_t o = byte_of(ow, k);
            S nbs[4][6];
#pragma unroll
            for (int f = 0; f < 4; f++) {
                nbs[f][0] = k < V - 1 ? W[f][1].v[k + 1] : fr[f];
                nbs[f][1] = k > 0 ? W[f][1].v[k - 1] : fl[f];
                nbs[f][2] = Y[f][0].v[k];
                nbs[f][3] = Y[f][1].v[k];
                nbs[f][4] = W[f][2].v[k];
                nbs[f][5] = W[f][0].v[k];
            }
            const S um[6] = {k < V - 1 ? uxc.v[k + 1] : fr[4], k > 0 ? uxc.v[k - 1] : fl[4],
                             Y[4][0].v[k], Y[4][1].v[k], W[4][2].v[k], W[4][0].v[k]};
            const S u0[3] = {uxc.v[k], uyc.v[k], W[4][1].v[k]};
            S psn, cpart;
            psi_c_update<S>(p, W[0][1].v[k], W[1][1].v[k], W[3][1].v[k], W[2][1].v[k], u0, um,
                            nbs[0], nbs[1], nbs[2], nbs[3], 0u, psn, cpart);
            const bool sol = (o & OWN_SOLID) != 0;
            pnv.v[k] = sol ? W[0][1].v[k] : psn;
            cnv.v[k] = sol ? W[1][1].v[k] : fma(-(S)p.kd, W[3][1].v[k], cpart);
        }
        st_interior<S, V>(psin, on, pnv, ow);
        st_interior<S, V>(ccn, on, cnv, ow);
        if (BND && (ow & ((V == 4) ? 0x80808080u : 0x8080u))) {
            for (int k = 0; k < V; k++)
                if (byte_of(ow, k) & OWN_BOUNDARY) psic_bnd_node<S, false>(D, p, n0 + k, x0 + k, y, z);
        }
        // advance the window
#pragma unroll
        for (int f = 0; f < 5; f++) {
            W[f][0] = W[f][1];
            W[f][1] = W[f][2];
            W[f][2] = nW[f];
        }
        WO[0] = WO[1];
        WO[1] = WO[2];
        WO[2] = nO;
        uxc = nux;
        uyc = nuy;
    }
}

// ------------------------------------------------ block reductions (FP64)
// Fixed-shape reductions: wavefront butterfly, then the waves in order, so
// results do not depend on scheduling.
// Returns, in thread j < NV, the block total of component j (0 elsewhere);
// each thread sums its component over the waves in order.
template <int NV>
__device__ double block_sum(double (&v)[NV], double *lds /* NV * nwaves */)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; j++) {
        double s = v[j];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        v[j] = s;
    }
    __syncthreads();
    if (lane == 0)
        for (int j = 0; j < NV; j++) lds[wave * NV + j] = v[j];
    __syncthreads();
    double t = 0.0;
    if ((int)threadIdx.x < NV) {
        t = lds[threadIdx.x];
        for (int w = 1; w < nw; w++) t += lds[w * NV + threadIdx.x];
    }
    __syncthreads();
    return t;
}

__device__ __forceinline__ int node_of(const KParams &p, int n, int &x, int &y, int &z)
{
    const int sz = p.nx * p.ny;
    z = n / sz;
    const int r = n - z * sz;
    y = r / p.nx;
    x = r - y * p.nx;
    return n;
}

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// ------------------------------------------------------- k_link_partial
// Block (c, k) takes links [c*LINK_THREADS, (c+1)*LINK_THREADS) of particle k.
// For each link (n, d) of k (fluid n, n + c_d in
// k): wall velocity u_b = V + Omega x r + mu_cap (I - nn) grad c(n) with r
// the link midpoint from the centre (Eq. 4, 6); bounced population
// f_opp(d)(n) = f*_d(n) - 6 w_d rho0 c_d.u_b; momentum to the particle
// c_d (2 f*_d - 6 w_d rho0 c_d.u_b), of which the velocity-independent part
// F0 = sum c_d (2 f*_d - 6 w_d rho0 c_d.u_slip) and the drag tensor
// zeta = sum 6 w_d rho0 g g^T, g = (c_d, r x c_d), are accumulated in FP64.
// Then (M + zeta) X' = M X + (F0, T0) + transfers (implicit update),
// R' = R + V', m' = m rotated by |Omega'| about Omega'.
// Option LB_CAPILLARY_FORCE: the stress of the psi free energy at the link's
// fluid node n,
//   P = (a/2 psi^2 + 3b/4 psi^4 - kappa psi lap(psi) - kappa/2 |g|^2) I + kappa g g^T
// (the tensor whose divergence is psi grad(mu)), with the wetting ghost of the
// chemical potential at solid face neighbours and g by central differences
// over the faces, on the link's share of the surface: 6 w_d c_d.P joins the
// momentum the particle takes.  Under the isotropic divergence of a stress
// with P(x) at solid neighbours the fluid nodes together take
// -6 sum_links w_d c_d.P, so fluid and particle exchange it without loss.
template <class S>
__device__ void capillary_link(const KParams &p, const DColloid *__restrict__ col,
                               const uint8_t *__restrict__ own, const S *__restrict__ psi, int n,
                               const int fn[6], int x, int y, int z, double w, const double cd[3],
                               double dp[3])
{
#pragma clang fp contract(off)
    const S ps = psi[n];
    double ph[6];
    for (int e = 0; e < 6; e++) ph[e] = (double)face_psi<S>(p, col, own[fn[e]], e, x, y, z, ps, psi[fn[e]]);
    const double s0 = (double)ps;
    const double lap = ph[0] + ph[1] + ph[2] + ph[3] + ph[4] + ph[5] - 6.0 * s0;
    const double g[3] = {(ph[0] - ph[1]) / 2.0, (ph[2] - ph[3]) / 2.0, (ph[4] - ph[5]) / 2.0};
    const double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    const double sc = p.a / 2.0 * s0 * s0 + 3.0 * p.b / 4.0 * s0 * s0 * s0 * s0 -
                      p.kappa * s0 * lap - p.kappa / 2.0 * g2;
    double P[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) P[a][b] = (a == b ? sc : 0.0) + p.kappa * g[a] * g[b];
    for (int b = 0; b < 3; b++) dp[b] += 6.0 * w * (cd[0] * P[0][b] + cd[1] * P[1][b] + cd[2] * P[2][b]);
}

// Close-encounter pair forces, one thread per particle: on particle k from
// every other particle of its box, the soft-sphere repulsion (soft_eps > 0,
// gap h below soft_hc) nu eps sigma^nu (h^-(nu+1) - hc^-(nu+1)) (h below 0.01
// taken as 0.01) and the normal lubrication (lub_hc > 0, gap below lub_hc)
// 6 pi eta (a_k a_i/(a_k + a_i))^2 (1/h - 1/lub_hc) U_n (h below 0.1 taken as
// 0.1; U_n the approach speed), both along the line of centres, pushing the
// pair apart when positive, into sF for the rigid-body update.  Runs before
// that update rewrites positions and velocities, so all pairs see the state
// at the start of the step.
__global__ __launch_bounds__(64) void k_soft(BatchArgs A, int ncol)
{
#pragma clang fp contract(off)
    const int g = blockIdx.x * 64 + (int)threadIdx.x;
    if (g >= ncol) return;
    const int j = find_box(A.cstart, A.nbox, g);
    const BoxDesc &D = A.d[j];
    const KParams &p = D.p;
    DColloid *__restrict__ col = D.b.col;
    const int k = g - A.cstart[j], nb = A.cstart[j + 1] - A.cstart[j];
    double F[3] = {0.0, 0.0, 0.0};
    if (p.soft_eps > 0.0 || p.lub_hc > 0.0) {
        const DColloid &a = col[k];
        const double eta = p.rho0 * (p.tau - 0.5) / 3.0;
        for (int i = 0; i < nb; i++) {
            if (i == k) continue;
            const DColloid &o = col[i];
            const double d[3] = {min_image(o.pos[0] - a.pos[0], p.nx), min_image(o.pos[1] - a.pos[1], p.ny),
                                 min_image(o.pos[2] - a.pos[2], p.nz)};
            const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            const double h0 = r - a.radius - o.radius;
            double f = 0.0;
            if (p.soft_eps > 0.0 && h0 < p.soft_hc) {
                const double h = h0 < 0.01 ? 0.01 : h0;
                f += p.soft_nu * p.soft_eps * pow(p.soft_sigma, p.soft_nu) *
                     (pow(h, -(p.soft_nu + 1.0)) - pow(p.soft_hc, -(p.soft_nu + 1.0)));
            }
            if (p.lub_hc > 0.0 && h0 < p.lub_hc) {
                const double h = h0 < 0.1 ? 0.1 : h0;
                const double un = ((a.vel[0] - o.vel[0]) * d[0] + (a.vel[1] - o.vel[1]) * d[1] +
                                   (a.vel[2] - o.vel[2]) * d[2]) / r;
                const double ae = a.radius * o.radius / (a.radius + o.radius);
                f += 6.0 * M_PI * eta * ae * ae * (1.0 / h - 1.0 / p.lub_hc) * un;
            }
            for (int e = 0; e < 3; e++) F[e] -= f * d[e] / r;
        }
    }
    for (int e = 0; e < 3; e++) col[k].sF[e] = F[e];
}

template <int P>
__global__ __launch_bounds__(LINK_THREADS) void k_link_partial(BatchArgs A)
{
    typedef typename Prec<P>::T T;
    typedef typename Prec<P>::S S;
    __shared__ double lds[28 * 16];
    const int j = find_box(A.cstart, A.nbox, blockIdx.y);
    const BoxDesc &D = A.d[j];
    const KParams p = D.p;
    DColloid *__restrict__ col = D.b.col;
    const int *__restrict__ lnode = D.b.lnode;
    const uint8_t *__restrict__ ldc = D.b.ldc;
    const int lcap = D.b.lcap;
    T *__restrict__ fout = (T *)D.b.fout;
    const S *__restrict__ cc = (const S *)D.b.cc;
    const uint8_t *__restrict__ own = D.b.own;
    const int k = blockIdx.y - A.cstart[j];
    const DColloid &q = col[k];
    const int nl = min(q.nlinks, lcap);
    const int l0 = blockIdx.x * LINK_THREADS;
    if (l0 >= nl) return;
    const size_t N = (size_t)p.N;
    const double rho0 = p.rho0;
    double acc[28];
#pragma unroll
    for (int jj = 0; jj < 28; jj++) acc[jj] = 0.0;
    const double V[3] = {q.vel[0], q.vel[1], q.vel[2]};
    const double W[3] = {q.omega[0], q.omega[1], q.omega[2]};
    {
        const int l = l0 + threadIdx.x;
        if (l < nl) {
        const int n = lnode[(size_t)k * lcap + l];
        const int dc = ldc[(size_t)k * lcap + l];
        const int d = dc & 31;
        int x, y, z;
        node_of(p, n, x, y, z);
        const int ex = cx(d), ey = cy(d), ez = cz(d);
        double r[3];
        displacement(q, x, y, z, ex, ey, ez, 0.5, p.nx, p.ny, p.nz, r);
        // surface cell from the current axes (the table is rebuilt only on
        // owner changes)
        const int cell = surface_cell(q, r);
        double nh[3];
        if (is_spheroid(q)) {
            spheroid_normal(q, r, nh);
        } else {
            const double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
            for (int a = 0; a < 3; a++) nh[a] = r[a] / rn;
        }
        // grad c at the fluid node, c(x) substituted at solid neighbours
        const int sy = p.nx, sz = p.nx * p.ny;
        const int fn[6] = {n - x + wrap_p(x, p.nx), n - x + wrap_m(x, p.nx),
                           n + (wrap_p(y, p.ny) - y) * sy, n + (wrap_m(y, p.ny) - y) * sy,
                           n + (wrap_p(z, p.nz) - z) * sz, n + (wrap_m(z, p.nz) - z) * sz};
        const double c0 = (double)cc[n];
        double cv[6];
        for (int e = 0; e < 6; e++) cv[e] = (own[fn[e]] & OWN_SOLID) ? c0 : (double)cc[fn[e]];
        const double g[3] = {0.5 * (cv[0] - cv[1]), 0.5 * (cv[2] - cv[3]), 0.5 * (cv[4] - cv[5])};
        const double mob = cell_mu(q, cell);
        const double ng = nh[0] * g[0] + nh[1] * g[1] + nh[2] * g[2];
        double slip[3], ub[3], wr[3];
        for (int a = 0; a < 3; a++) slip[a] = mob * (g[a] - nh[a] * ng);
        cross3(W, r, wr);
        for (int a = 0; a < 3; a++) ub[a] = V[a] + wr[a] + slip[a];
        const double w = wgt(d);
        const size_t slot = (size_t)opp(d) * N + n;
        const S gs = ld_pop(fout, slot, p.inv_scale);
        const double fs = (double)gs + w * rho0;
        const double cub = ex * ub[0] + ey * ub[1] + ez * ub[2];
        const double cus = ex * slip[0] + ey * slip[1] + ez * slip[2];
        st_pop(fout, slot, (S)((double)gs - 6.0 * w * rho0 * cub), p.scale);
        const double mag = 2.0 * fs - 6.0 * w * rho0 * cus;
        double dp[3] = {ex * mag, ey * mag, ez * mag};
        const double cd[3] = {(double)ex, (double)ey, (double)ez};
        if (p.flags & LB_CAPILLARY_FORCE)
            capillary_link<S>(p, col, own, (const S *)D.b.psi, n, fn, x, y, z, w, cd, dp);
        double t[3];
        cross3(r, dp, t);
        double rc[3];
        cross3(r, cd, rc);
        const double gv[6] = {cd[0], cd[1], cd[2], rc[0], rc[1], rc[2]};
        const double coef = 6.0 * w * rho0;
        for (int a = 0; a < 3; a++) { acc[a] += dp[a]; acc[3 + a] += t[a]; }
        int j = 6;
        for (int i1 = 0; i1 < 6; i1++)
            for (int i2 = i1; i2 < 6; i2++) acc[j++] += coef * gv[i1] * gv[i2];
        acc[27] += cell_active(q, cell) ? 1.0 : 0.0;
        }
    }
    const double tot = block_sum<28>(acc, lds);
    if (threadIdx.x < 28)
        D.b.lpart[((size_t)k * D.b.nlchunk_max + blockIdx.x) * 28 + threadIdx.x] = tot;
}

// ------------------------------------------------------ k_colloid_update
// A X = b by Gaussian elimination without pivoting (M + zeta is symmetric
// positive definite)
__device__ void solve6(double A[36], double bb[6], double Xn[6])
{
    for (int c = 0; c < 6; c++)
        for (int i = c + 1; i < 6; i++) {
            const double l = A[6 * i + c] / A[6 * c + c];
            for (int j = c; j < 6; j++) A[6 * i + j] -= l * A[6 * c + j];
            bb[i] -= l * bb[c];
        }
    for (int i = 5; i >= 0; i--) {
        double s = bb[i];
        for (int j = i + 1; j < 6; j++) s -= A[6 * i + j] * Xn[j];
        Xn[i] = s / A[6 * i + i];
    }
}

// A spheroid's step: M = diag(m, m, m, I), I = I_perp 1 + (I_par - I_perp)
// m m^T at the axis of the start of the step (the gyroscopic term, second
// order in Omega, left out); implicit (M + zeta) X' = M X + F, or explicit
// X' = X + M^-1 (F - zeta X) with I^-1 = 1/I_perp + (1/I_par - 1/I_perp) m m^T
__device__ void spheroid_step(const DColloid &q, const double Z[36], const double Fk[6],
                              const double X[6], bool expl, double Xn[6])
{
    double M[36];
    for (int i = 0; i < 36; i++) M[i] = 0.0;
    for (int i = 0; i < 3; i++) M[6 * i + i] = q.mass;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            M[6 * (3 + i) + 3 + j] = (i == j ? q.iperp : 0.0) + (q.ipar - q.iperp) * q.m[i] * q.m[j];
    if (expl) {
        double s[6];
        for (int i = 0; i < 6; i++) {
            s[i] = Fk[i];
            for (int j = 0; j < 6; j++) s[i] -= Z[6 * i + j] * X[j];
        }
        for (int i = 0; i < 3; i++) Xn[i] = X[i] + s[i] / q.mass;
        const double ms = q.m[0] * s[3] + q.m[1] * s[4] + q.m[2] * s[5];
        for (int i = 0; i < 3; i++)
            Xn[3 + i] = X[3 + i] + s[3 + i] / q.iperp + (1.0 / q.ipar - 1.0 / q.iperp) * q.m[i] * ms;
        return;
    }
    double A[36], bb[6];
    for (int i = 0; i < 36; i++) A[i] = Z[i] + M[i];
    for (int i = 0; i < 6; i++) {
        bb[i] = Fk[i];
        for (int j = 0; j < 6; j++) bb[i] += M[6 * i + j] * X[j];
    }
    solve6(A, bb, Xn);
}

// One block per particle: link partials summed in chunk order (FP64), then
// (M + zeta) X' = M X + (F0, T0) + transfers (implicit update),
// R' = R + V', m' = m and e' = e rotated by |Omega'| about Omega' (e' then
// made orthogonal to m' again and normalised).
__global__ __launch_bounds__(64) void k_colloid_update(BatchArgs A)
{
    __shared__ double sacc[28];
    const int j = find_box(A.cstart, A.nbox, blockIdx.x);
    const BoxDesc &D = A.d[j];
    const KParams p = D.p;
    DColloid *__restrict__ col = D.b.col;
    int *__restrict__ err = D.b.err;
    const int k = blockIdx.x - A.cstart[j];
    DColloid &q = col[k];
    const int nl = min(q.nlinks, D.b.lcap);
    const int nch = (nl + LINK_THREADS - 1) / LINK_THREADS;
    if (threadIdx.x < 28) {
        // partials loaded eight chunks at a time (one memory round trip per
        // eight, not per chunk), summed in chunk order
        const double *o = D.b.lpart + (size_t)k * D.b.nlchunk_max * 28 + threadIdx.x;
        double s = 0.0;
        for (int c0 = 0; c0 < nch; c0 += 8) {
            double v[8];
#pragma unroll
            for (int i = 0; i < 8; i++) v[i] = c0 + i < nch ? o[(size_t)(c0 + i) * 28] : 0.0;
#pragma unroll
            for (int i = 0; i < 8; i++)
                if (c0 + i < nch) s += v[i];
        }
        sacc[threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double acc[28];
    for (int a = 0; a < 28; a++) acc[a] = sacc[a];
    if (p.soft_eps > 0.0 || p.lub_hc > 0.0)
        for (int e = 0; e < 3; e++) acc[e] += q.sF[e];  // close-encounter forces join F0
    const double V[3] = {q.vel[0], q.vel[1], q.vel[2]};
    const double W[3] = {q.omega[0], q.omega[1], q.omega[2]};
    double Z[36];
    {
        int j = 6;
        for (int i1 = 0; i1 < 6; i1++)
            for (int i2 = i1; i2 < 6; i2++) { Z[6 * i1 + i2] = acc[j]; Z[6 * i2 + i1] = acc[j]; j++; }
    }
    double Fk[6], X[6] = {V[0], V[1], V[2], W[0], W[1], W[2]}, Xn[6];
    for (int a = 0; a < 3; a++) {
        q.F0[a] = acc[a];
        q.T0[a] = acc[3 + a];
        Fk[a] = acc[a] + q.trF[a];
        Fk[3 + a] = acc[3 + a] + q.trT[a];
    }
    const bool expl = (p.flags & LB_EXPLICIT_COLLOID) != 0;
    if (q.fixed) {
        for (int i = 0; i < 6; i++) Xn[i] = X[i];
    } else if (is_spheroid(q)) {
        spheroid_step(q, Z, Fk, X, expl, Xn);
    } else if (expl) {
        // option: explicit update (Ladd), M X' = M X + F0 + transfers - zeta X
        const double Mv[6] = {q.mass, q.mass, q.mass, q.inertia, q.inertia, q.inertia};
        for (int i = 0; i < 6; i++) {
            double s = Fk[i];
            for (int j = 0; j < 6; j++) s -= Z[6 * i + j] * X[j];
            Xn[i] = X[i] + s / Mv[i];
        }
    } else {
        const double Mv[6] = {q.mass, q.mass, q.mass, q.inertia, q.inertia, q.inertia};
        double A[36], bb[6];
        for (int i = 0; i < 36; i++) A[i] = Z[i];
        for (int i = 0; i < 6; i++) { A[6 * i + i] += Mv[i]; bb[i] = Mv[i] * X[i] + Fk[i]; }
        solve6(A, bb, Xn);
    }
    // force and torque acting: F0 - zeta X' (implicit), F0 - zeta X (explicit)
    for (int i = 0; i < 6; i++) {
        double s = Fk[i];
        for (int j = 0; j < 6; j++) s -= Z[6 * i + j] * (expl ? X[j] : Xn[j]);
        if (i < 3) q.F[i] = s; else q.T[i - 3] = s;
    }
    for (int a = 0; a < 3; a++) { q.trF[a] = 0.0; q.trT[a] = 0.0; }
    if (q.fixed) return;
    const int L[3] = {p.nx, p.ny, p.nz};
    for (int a = 0; a < 3; a++) {
        q.vel[a] = Xn[a];
        q.omega[a] = Xn[3 + a];
        double rr = q.pos[a] + Xn[a];
        if (rr >= (double)L[a]) rr -= (double)L[a];
        else if (rr < 0.0) rr += (double)L[a];
        q.pos[a] = rr;
    }
    if (fabs(Xn[0]) >= 0.5 || fabs(Xn[1]) >= 0.5 || fabs(Xn[2]) >= 0.5) atomicOr(err, LB_ERR_FAST);
    const double th = sqrt(Xn[3] * Xn[3] + Xn[4] * Xn[4] + Xn[5] * Xn[5]);
    if (th > 0.0) {
        const double ax[3] = {Xn[3] / th, Xn[4] / th, Xn[5] / th};
        double kxm[3];
        cross3(ax, q.m, kxm);
        const double km = ax[0] * q.m[0] + ax[1] * q.m[1] + ax[2] * q.m[2];
        const double cs = cos(th), sn = sin(th);
        double mn[3];
        for (int a = 0; a < 3; a++) mn[a] = q.m[a] * cs + kxm[a] * sn + ax[a] * km * (1.0 - cs);
        const double nn = sqrt(mn[0] * mn[0] + mn[1] * mn[1] + mn[2] * mn[2]);
        for (int a = 0; a < 3; a++) q.m[a] = mn[a] / nn;
        double kxe[3];
        cross3(ax, q.e, kxe);
        const double ke = ax[0] * q.e[0] + ax[1] * q.e[1] + ax[2] * q.e[2];
        double en[3];
        for (int a = 0; a < 3; a++) en[a] = q.e[a] * cs + kxe[a] * sn + ax[a] * ke * (1.0 - cs);
        const double em = en[0] * q.m[0] + en[1] * q.m[1] + en[2] * q.m[2];
        for (int a = 0; a < 3; a++) en[a] = en[a] - em * q.m[a];
        const double ne = sqrt(en[0] * en[0] + en[1] * en[1] + en[2] * en[2]);
        for (int a = 0; a < 3; a++) q.e[a] = en[a] / ne;
    }
}

// ---------------------------------------------------- particle geometry
// The geometry kernels run on a grid (chunk, particle): block (c, k) handles
// bounding-box nodes [c*GCHUNK, (c+1)*GCHUNK) of particle k, visited in
// ascending node order, so that per-particle results are assembled in a fixed
// order whatever the block scheduling.
struct BoxIter {
    AxisBox bx, by, bz;
    int total, nchunk;
};

__device__ __forceinline__ BoxIter box_of(const DColloid &q, const KParams &p)
{
    BoxIter b;
    const double rb = bound_radius(q);
    b.bx = axis_box(q.pos[0], rb, p.nx);
    b.by = axis_box(q.pos[1], rb, p.ny);
    b.bz = axis_box(q.pos[2], rb, p.nz);
    b.total = b.bx.count * b.by.count * b.bz.count;
    b.nchunk = (b.total + GCHUNK - 1) / GCHUNK;
    return b;
}

__device__ __forceinline__ int box_node(const BoxIter &b, int t, const KParams &p, int &x, int &y,
                                        int &z)
{
    const int ix = t % b.bx.count, iy = (t / b.bx.count) % b.by.count,
              iz = t / (b.bx.count * b.by.count);
    x = b.bx.at(ix);
    y = b.by.at(iy);
    z = b.bz.at(iz);
    return x + p.nx * (y + p.ny * z);
}

// ------------------------------------------------------- boundary fix-ups
// The bulk mu and psi/c blocks skip the fluid nodes next to a particle.  These
// blocks recompute the fluid nodes next to a particle (owner bit 7).
// Fix-up block (particle, section): it scans BND_SCAN * GCHUNK nodes of the
// particle's bounding box, gathers the boundary nodes among them in LDS and
// works through that list with all lanes busy.  Only these nodes have solid
// neighbours, so the wetting ghost (Eq. 9), the no-flux faces and the
// emission (Eq. 5) live here, off the bulk kernels' register budget.  A
// node inside two boxes is recomputed twice with identical results.

// boundary nodes (box indices) of this block's section, in any order
__device__ __forceinline__ int gather_boundary(const BoxIter &B, const KParams &p,
                                               const uint8_t *__restrict__ own, int sec, int *list,
                                               int &cnt)
{
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < BND_SCAN; r++) {
        const int t = (sec * BND_SCAN + r) * GCHUNK + (int)threadIdx.x;
        if (t < B.total) {
            int x, y, z;
            if (own[box_node(B, t, p, x, y, z)] & OWN_BOUNDARY) list[atomicAdd(&cnt, 1)] = t;
        }
    }
    __syncthreads();
    return cnt;
}
template <class S, bool PAT>
__device__ __forceinline__ void mu_fix(const BatchArgs &A, const int blk)
{
    const int gk = blk / A.nsec, sec = blk - gk * A.nsec;
    const int j = find_box(A.cstart, A.nbox, gk);
    const BoxDesc &D = A.d[j];
    const KParams p = D.p;
    __shared__ int list[BND_SCAN * GCHUNK];
    __shared__ int cnt;
    const BoxIter B = box_of(D.b.col[gk - A.cstart[j]], p);
    if (sec * BND_SCAN * GCHUNK >= B.total) return;  // whole block
    const int count = gather_boundary(B, p, D.b.own, sec, list, cnt);
    for (int i = threadIdx.x; i < count; i += GCHUNK) {
        int x, y, z;
        const int n = box_node(B, list[i], p, x, y, z);
        mu_bnd_node<S, PAT>(D, p, n, x, y, z);
    }
}

template <class S, bool PAT>
__device__ __forceinline__ void psic_fix(const BatchArgs &A, const int blk)
{
    const int gk = blk / A.nsec, sec = blk - gk * A.nsec;
    const int j = find_box(A.cstart, A.nbox, gk);
    const BoxDesc &D = A.d[j];
    const KParams p = D.p;
    __shared__ int list[BND_SCAN * GCHUNK];
    __shared__ int cnt;
    const BoxIter B = box_of(D.b.col[gk - A.cstart[j]], p);
    if (sec * BND_SCAN * GCHUNK >= B.total) return;  // whole block
    const int count = gather_boundary(B, p, D.b.own, sec, list, cnt);
    for (int i = threadIdx.x; i < count; i += GCHUNK) {
        int x, y, z;
        const int n = box_node(B, list[i], p, x, y, z);
        psic_bnd_node<S, PAT>(D, p, n, x, y, z);
    }
}

// ------------------------------------------------ mu and psi/c launches
// Bulk launches (V = 1: one node per thread; 2, 4: row vectors; ZM:
// z-marching row vectors) and the boundary fix-up launch, grid A.nsec
// blocks per particle.  Bulk and fix-up blocks write disjoint nodes, so the
// two launches of an update may run side by side on two streams.  With BND
// the bulk launch does the boundary nodes itself (small steps, where a
// separate fix-up launch would cost more than it saves).
template <class S, int V, bool BND, bool ST = false>
__global__ __launch_bounds__(256) void k_mu(BatchArgs A)
{
    if (V == 1) mu_one<S, BND, ST>(A, blockIdx.x);
    else mu_vec<S, (V > 1 ? V : 2), BND>(A, blockIdx.x);
}

// PAT: some particle of the batch carries a surface pattern or is not a
// sphere (the form without that arithmetic keeps a smaller register budget)
template <class S, bool PAT>
__global__ __launch_bounds__(GCHUNK) void k_mu_bnd(BatchArgs A)
{
    mu_fix<S, PAT>(A, blockIdx.x);
}

template <class S, int V, bool ZM, bool BND, bool SP = false>
__global__ __launch_bounds__(256) void k_scalar(BatchArgs A)
{
    if (V == 1) psic_one<S, BND, SP>(A, blockIdx.x + A.boff);
    else if (ZM) psic_zmarch<S, (V > 1 ? V : 2), BND>(A, blockIdx.x + A.boff);
    else psic_vec<S, (V > 1 ? V : 2), BND, SP>(A, blockIdx.x + A.boff);
}

template <class S, bool PAT>
__global__ __launch_bounds__(GCHUNK) void k_scalar_bnd(BatchArgs A)
{
    psic_fix<S, PAT>(A, blockIdx.x);
}

// ------------------------------------------------------------- k_cover
// At the new position: a fluid node now inside hands its momentum
// sum_i f_i c_i to the particle; a node of this particle now outside is
// refilled with f^eq(rho0, V + Omega x r) (the particle is debited
// rho0 (V + Omega x r)) and takes psi, c as the mean of its face neighbours
// that are fluid before and after.  Per-block FP64 partial transfers and an
// owner-change flag go to cpart[k][c]; k_commit sums them in chunk order.
template <int P>
__global__ __launch_bounds__(GCHUNK) void k_cover(BatchArgs A)
{
    typedef typename Prec<P>::T T;
    typedef typename Prec<P>::S S;
    __shared__ double lds[6 * 16];
    const int j = find_box(A.cstart, A.nbox, blockIdx.y);
    const BoxDesc &D = A.d[j];
    const KParams p = D.p;
    const DColloid *__restrict__ col = D.b.col;
    T *__restrict__ f = (T *)D.b.fout;
    S *__restrict__ psi = (S *)D.b.psin;
    S *__restrict__ cc = (S *)D.b.ccn;
    const uint8_t *__restrict__ own = D.b.own;
    double *__restrict__ cpart = D.b.cpart;
    const int nchunk_max = D.b.nchunk_max;
    int *__restrict__ err = D.b.err;
    const int k = blockIdx.y - A.cstart[j], c = blockIdx.x;
    const DColloid &q = col[k];
    const BoxIter B = box_of(q, p);
    if (c >= B.nchunk) return;
    const size_t N = (size_t)p.N;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int changed = 0;
    const int sy = p.nx, sz = p.nx * p.ny;
    const int t = c * GCHUNK + threadIdx.x;
    if (t < B.total) {
        int x, y, z;
        const int n = box_node(B, t, p, x, y, z);
        const int old = own[n] & OWN_SOLID;
        const bool ins = inside(q, x, y, z, p.nx, p.ny, p.nz);
        if (ins != (old == k + 1)) changed = 1;
        if (ins && old == 0) {
            double pm[3] = {0.0, 0.0, 0.0}, r[3], tq[3];
            for (int i = 1; i < 19; i++) {
                const double gi = (double)ld_pop(f, i * N + n, p.inv_scale);
                pm[0] += cx(i) * gi;
                pm[1] += cy(i) * gi;
                pm[2] += cz(i) * gi;
            }
            displacement(q, x, y, z, 0, 0, 0, 0.0, p.nx, p.ny, p.nz, r);
            cross3(r, pm, tq);
            for (int a = 0; a < 3; a++) { acc[a] += pm[a]; acc[3 + a] += tq[a]; }
        } else if (ins && old != k + 1) {
            atomicOr(err, LB_ERR_CONTACT);
        } else if (!ins && old == k + 1) {
            double r[3], uw[3], tq[3], pm[3];
            displacement(q, x, y, z, 0, 0, 0, 0.0, p.nx, p.ny, p.nz, r);
            cross3(q.omega, r, uw);
            for (int a = 0; a < 3; a++) uw[a] += q.vel[a];
            const double uu = uw[0] * uw[0] + uw[1] * uw[1] + uw[2] * uw[2];
            for (int i = 0; i < 19; i++) {
                const double cu = cx(i) * uw[0] + cy(i) * uw[1] + cz(i) * uw[2];
                const double geq = wgt(i) * p.rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
                st_pop(f, i * N + n, (S)geq, p.scale);
            }
            for (int a = 0; a < 3; a++) pm[a] = p.rho0 * uw[a];
            cross3(r, pm, tq);
            for (int a = 0; a < 3; a++) { acc[a] -= pm[a]; acc[3 + a] -= tq[a]; }
            const int fn[6] = {n - x + wrap_p(x, p.nx), n - x + wrap_m(x, p.nx),
                               n + (wrap_p(y, p.ny) - y) * sy, n + (wrap_m(y, p.ny) - y) * sy,
                               n + (wrap_p(z, p.nz) - z) * sz, n + (wrap_m(z, p.nz) - z) * sz};
            const int fx[6] = {wrap_p(x, p.nx), wrap_m(x, p.nx), x, x, x, x};
            const int fy[6] = {y, y, wrap_p(y, p.ny), wrap_m(y, p.ny), y, y};
            const int fz[6] = {z, z, z, z, wrap_p(z, p.nz), wrap_m(z, p.nz)};
            double sp = 0.0, sc = 0.0;
            int cnt = 0;
            for (int e = 0; e < 6; e++) {
                if ((own[fn[e]] & OWN_SOLID) == 0 && !inside(q, fx[e], fy[e], fz[e], p.nx, p.ny, p.nz)) {
                    sp += (double)psi[fn[e]];
                    sc += (double)cc[fn[e]];
                    cnt++;
                }
            }
            if (cnt > 0) { psi[n] = (S)(sp / cnt); cc[n] = (S)(sc / cnt); }
        }
    }
    const int any = __syncthreads_or(changed);
    const double tot = block_sum<6>(acc, lds);
    if (threadIdx.x < 7)
        cpart[((size_t)k * nchunk_max + c) * 8 + threadIdx.x] =
            threadIdx.x < 6 ? tot : (any ? 1.0 : 0.0);
}

// ------------------------------------------------------------- k_commit
// Owner bytes at the new position (inside -> k+1, left behind -> fluid), only
// for particles whose owner map changed.  Block (0, k) also adds the chunk
// partial transfers to the particle in chunk order and records the flag.
__global__ __launch_bounds__(GCHUNK) void k_commit(BatchArgs A)
{
    const int j = find_box(A.cstart, A.nbox, blockIdx.y);
    const BoxDesc &D = A.d[j];
    const KParams p = D.p;
    DColloid *__restrict__ col = D.b.col;
    uint8_t *__restrict__ own = D.b.own;
    const double *__restrict__ cpart = D.b.cpart;
    const int nchunk_max = D.b.nchunk_max;
    const int k = blockIdx.y - A.cstart[j], c = blockIdx.x;
    DColloid &q = col[k];
    const BoxIter B = box_of(q, p);
    if (c >= B.nchunk) return;
    const double *cp = cpart + (size_t)k * nchunk_max * 8;
    // change flags of all chunks, loaded in parallel
    int flag = 0;
    for (int jj = threadIdx.x; jj < B.nchunk; jj += blockDim.x) flag |= cp[8 * jj + 6] != 0.0;
    const int any = __syncthreads_or(flag);
    if (c == 0) {
        // transfers summed in chunk order: thread a < 6 sums component a
        if (threadIdx.x < 6) {
            const int a = threadIdx.x;
            double s = 0.0;
            for (int jj = 0; jj < B.nchunk; jj++) s += cp[8 * jj + a];
            if (a < 3) q.trF[a] += s; else q.trT[a - 3] += s;
        }
        if (threadIdx.x == 0) q.changed = any;
    }
    if (!any) return;
    const int t = c * GCHUNK + threadIdx.x;
    if (t >= B.total) return;
    int x, y, z;
    const int n = box_node(B, t, p, x, y, z);
    const bool ins = inside(q, x, y, z, p.nx, p.ny, p.nz);
    const uint8_t o = own[n];
    if (ins) {
        if ((o & OWN_SOLID) != k + 1) own[n] = (uint8_t)(k + 1);
    } else if ((o & OWN_SOLID) == k + 1) {
        own[n] = 0;
    }
}

// ----------------------------------------------------- k_link_count/write
// Boundary bits and the link table of particle k in canonical order
// (ascending node, then direction): k_link_count stores the 18-bit mask of
// directions linked to k for every box node and the link count per chunk;
// k_link_write places each chunk after the counts of the chunks before it.
// Without an owner change the node set, the directions and the boundary bits
// are unchanged and both kernels return; the cap bit is recomputed where it
// is used.
__device__ int block_exclusive_scan(int v, int *lds, int &total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int s = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(s, off, 64);
        if (lane >= off) s += t;
    }
    if (lane == 63) lds[wave] = s;
    __syncthreads();
    int base = 0;
    for (int w = 0; w < wave; w++) base += lds[w];
    total = 0;
    for (int w = 0; w < nw; w++) total += lds[w];
    __syncthreads();
    return base + s - v;
}

__global__ __launch_bounds__(GCHUNK) void k_link_count(BatchArgs A)
{
    __shared__ int lds[16];
    const int j = find_box(A.cstart, A.nbox, blockIdx.y);
    const BoxDesc &D = A.d[j];
    const KParams p = D.p;
    const DColloid *__restrict__ col = D.b.col;
    uint8_t *__restrict__ own = D.b.own;
    uint32_t *__restrict__ lmask = D.b.lmask;
    const int bbmax = D.b.bbmax;
    int *__restrict__ ccount = D.b.ccount;
    const int nchunk_max = D.b.nchunk_max;
    const int k = blockIdx.y - A.cstart[j], c = blockIdx.x;
    const DColloid &q = col[k];
    if (!q.changed) return;
    const BoxIter B = box_of(q, p);
    if (c >= B.nchunk) return;
    const int t = c * GCHUNK + threadIdx.x;
    int cnt = 0;
    if (t < B.total) {
        int x, y, z;
        const int n = box_node(B, t, p, x, y, z);
        uint32_t mask = 0;
        const uint8_t o = own[n];
        if ((o & OWN_SOLID) == 0) {
            bool bnd = false;
            const int sy = p.nx, sz = p.nx * p.ny;
            const int xs[3] = {wrap_m(x, p.nx), x, wrap_p(x, p.nx)};
            const int ys[3] = {wrap_m(y, p.ny), y, wrap_p(y, p.ny)};
            const int zs[3] = {wrap_m(z, p.nz), z, wrap_p(z, p.nz)};
            for (int d = 1; d < 19; d++) {
                const int m = xs[cx(d) + 1] + sy * ys[cy(d) + 1] + sz * zs[cz(d) + 1];
                const int om = own[m] & OWN_SOLID;
                if (om) bnd = true;
                if (om == k + 1) { mask |= 1u << d; cnt++; }
            }
            const uint8_t want = bnd ? OWN_BOUNDARY : 0;
            if (o != want) own[n] = want;
        }
        lmask[(size_t)k * bbmax + t] = mask;
    }
    int tot;
    block_exclusive_scan(cnt, lds, tot);
    if (threadIdx.x == 0) ccount[(size_t)k * nchunk_max + c] = tot;
}

__global__ __launch_bounds__(GCHUNK) void k_link_write(BatchArgs A)
{
    __shared__ int lds[16];
    __shared__ int sbase;
    const int j = find_box(A.cstart, A.nbox, blockIdx.y);
    const BoxDesc &D = A.d[j];
    const KParams p = D.p;
    DColloid *__restrict__ col = D.b.col;
    const uint32_t *__restrict__ lmask = D.b.lmask;
    const int bbmax = D.b.bbmax;
    const int *__restrict__ ccount = D.b.ccount;
    const int nchunk_max = D.b.nchunk_max;
    int *__restrict__ lnode = D.b.lnode;
    uint8_t *__restrict__ ldc = D.b.ldc;
    const int lcap = D.b.lcap;
    int *__restrict__ err = D.b.err;
    const int k = blockIdx.y - A.cstart[j], c = blockIdx.x;
    DColloid &q = col[k];
    if (!q.changed) return;
    const BoxIter B = box_of(q, p);
    if (c >= B.nchunk) return;
    {
        // links in the chunks before this one, and in all chunks (block sums)
        const int *cnts = ccount + (size_t)k * nchunk_max;
        int before = 0, all = 0;
        for (int jj = threadIdx.x; jj < B.nchunk; jj += blockDim.x) {
            const int v = cnts[jj];
            all += v;
            if (jj < c) before += v;
        }
        int tb, ta;
        block_exclusive_scan(before, lds, tb);
        block_exclusive_scan(all, lds, ta);
        if (threadIdx.x == 0) {
            sbase = tb;
            if (c == 0) {
                q.nlinks = ta;
                if (ta > lcap) atomicOr(err, LB_ERR_LINKS);
            }
        }
        __syncthreads();
    }
    const int t = c * GCHUNK + threadIdx.x;
    const uint32_t mask = t < B.total ? lmask[(size_t)k * bbmax + t] : 0u;
    int tot;
    const int off = block_exclusive_scan(__popc(mask), lds, tot);
    if (!mask) return;
    int x, y, z;
    const int n = box_node(B, t, p, x, y, z);
    int l = sbase + off;
    for (int d = 1; d < 19; d++) {
        if (!(mask & (1u << d))) continue;
        if (l < lcap) {
            lnode[(size_t)k * lcap + l] = n;
            ldc[(size_t)k * lcap + l] = (uint8_t)d;
        }
        l++;
    }
}

// --------------------------------------------------------------- k_init
template <int P>
__global__ __launch_bounds__(256) void k_init(KParams p, const double *__restrict__ psi0,
                                              const double *__restrict__ c0,
                                              const double *__restrict__ rho0,
                                              const double *__restrict__ u0,
                                              typename Prec<P>::T *__restrict__ f,
                                              typename Prec<P>::S *__restrict__ psi,
                                              typename Prec<P>::S *__restrict__ cc,
                                              uint8_t *__restrict__ own)
{
    typedef typename Prec<P>::S S;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= p.N) return;
    const size_t N = (size_t)p.N;
    const double r = rho0 ? rho0[n] : p.rho0;
    const double ux = u0 ? u0[n] : 0.0, uy = u0 ? u0[N + n] : 0.0, uz = u0 ? u0[2 * N + n] : 0.0;
    const double uu = ux * ux + uy * uy + uz * uz;
    for (int i = 0; i < 19; i++) {
        const double cu = cx(i) * ux + cy(i) * uy + cz(i) * uz;
        const double geq = wgt(i) * (r * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu) - p.rho0);
        st_pop(f, i * N + n, (S)geq, p.scale);
    }
    psi[n] = (S)psi0[n];
    cc[n] = (S)c0[n];
    own[n] = 0;
}

// ------------------------------------------------------------ k_reduce
// FP64 totals over fluid nodes: sum_i f_i, sum_i f_i c_i, psi, c, count.
template <int P>
__global__ __launch_bounds__(256) void k_reduce(KParams p, const typename Prec<P>::T *__restrict__ f,
                                                const typename Prec<P>::S *__restrict__ psi,
                                                const typename Prec<P>::S *__restrict__ cc,
                                                const uint8_t *__restrict__ own,
                                                double *__restrict__ part)
{
    __shared__ double lds[7 * 16];
    const size_t N = (size_t)p.N;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < p.N; n += gridDim.x * blockDim.x) {
        if (own[n] & OWN_SOLID) continue;
        double m = p.rho0, jx = 0.0, jy = 0.0, jz = 0.0;
        for (int i = 0; i < 19; i++) {
            const double g = (double)ld_pop(f, i * N + n, p.inv_scale);
            m += g;
            jx += cx(i) * g;
            jy += cy(i) * g;
            jz += cz(i) * g;
        }
        v[0] += m;
        v[1] += jx;
        v[2] += jy;
        v[3] += jz;
        v[4] += (double)psi[n];
        v[5] += (double)cc[n];
        v[6] += 1.0;
    }
    const double tot = block_sum<7>(v, lds);
    if (threadIdx.x < 7) part[blockIdx.x * 7 + threadIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_reduce_final(const double *__restrict__ part, int nblocks,
                                                      double *__restrict__ out)
{
    __shared__ double lds[7 * 16];
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        for (int j = 0; j < 7; j++) v[j] += part[b * 7 + j];
    const double tot = block_sum<7>(v, lds);
    if (threadIdx.x < 7) out[threadIdx.x] = tot;
}

// ------------------------------------------------------------ k_fields
template <int P>
__global__ __launch_bounds__(256) void k_fields(KParams p, const typename Prec<P>::T *__restrict__ f,
                                                const typename Prec<P>::S *__restrict__ psi,
                                                const typename Prec<P>::S *__restrict__ cc,
                                                const uint8_t *__restrict__ own,
                                                double *__restrict__ out /* 6N: rho u psi c */,
                                                double *__restrict__ fout /* 19N or null */)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= p.N) return;
    const size_t N = (size_t)p.N;
    double m = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    const bool fluid = (own[n] & OWN_SOLID) == 0;
    for (int i = 0; i < 19; i++) {
        const double g = (double)ld_pop(f, i * N + n, p.inv_scale);
        if (fout) fout[i * N + n] = fluid ? g + wgt(i) * p.rho0 : 0.0;
        m += g;
        jx += cx(i) * g;
        jy += cy(i) * g;
        jz += cz(i) * g;
    }
    if (!out) return;
    m += p.rho0;
    out[n] = fluid ? m : 0.0;
    out[N + n] = fluid ? jx / m : 0.0;
    out[2 * N + n] = fluid ? jy / m : 0.0;
    out[3 * N + n] = fluid ? jz / m : 0.0;
    out[4 * N + n] = (double)psi[n];
    out[5 * N + n] = (double)cc[n];
}

// ------------------------------------------------------------ launchers
void finish_shape(LaunchShape &ls, int nx, int ny, int nz, int ssize, bool whole_rows)
{
    if (ls.vec > 1) {
        const int V = (ssize == 8 && ls.vec > 2) ? 2 : ls.vec;
        const int W = nx / V;
        if ((V == 2 || V == 4) && nx % V == 0 && (W <= 64 || (W % 64 == 0 && !whole_rows))) {
            // row-vector launch: groups of Ls lanes per row segment, 64 / Ls
            // groups per wavefront, four wavefronts per block
            ls.vec = V;
            ls.bx = W < 64 ? W : 64;
            ls.by = 64 / ls.bx;
            ls.xseg = W / ls.bx;
            const long long segs = (long long)ny * nz * ls.xseg, per = 4LL * ls.by;
            ls.nblocks = (int)((segs + per - 1) / per);
            ls.bpp = 0;
            if (ls.zc > 1) {
                // z-marching: blocks over (row group, chunk of zc planes)
                if (ls.zc > nz) ls.zc = nz;
                ls.remap = 0;
                ls.bpp = (int)(((long long)ny * ls.xseg + per - 1) / per);
                ls.nblocks = ls.bpp * ((nz + ls.zc - 1) / ls.zc);
                return;
            }
            ls.zc = 0;
            if (ls.remap == 2) {
                const long long pp = (long long)ny * ls.xseg;
                if (pp % per == 0 && (pp / per) % 8 == 0) ls.bpp = (int)(pp / per);
                else ls.remap = 0;
            }
            return;
        }
        ls.bx = 0;  // not available for this box: default one-node shape
        ls.by = 0;
    }
    ls.vec = 0;
    ls.zc = 0;
    if (ls.bx <= 0 || ls.bx > 256) ls.bx = nx < 256 ? nx : 256;
    if (ls.bx > nx) ls.bx = nx;
    if (ls.by <= 0) ls.by = ls.bx >= 256 ? 1 : 256 / ls.bx;
    if (ls.bx * ls.by > 256) ls.by = 256 / ls.bx;  // the kernels' launch bound
    if (ls.by < 1) ls.by = 1;
    ls.xseg = (nx + ls.bx - 1) / ls.bx;
    const long long rows = (long long)ny * nz;
    ls.nblocks = (int)(ls.xseg * ((rows + ls.by - 1) / ls.by));
    ls.bpp = 0;
    if (ls.remap == 2) {
        // plane-wise renumbering needs whole planes per block row and
        // blocks per plane divisible by 8
        if (ny % ls.by == 0 && (ls.xseg * (ny / ls.by)) % 8 == 0) ls.bpp = ls.xseg * (ny / ls.by);
        else ls.remap = 0;
    }
}

// The link table write goes to stream sw (the next step's bulk mu and
// collide-stream kernels read owner bytes and boundary bits, which
// k_link_count finishes, but not the table).
static void launch_geometry_tail(const Batch &B, hipStream_t s, hipStream_t sw)
{
    const dim3 g(B.nchunk_max, B.ncol);
    k_commit<<<g, GCHUNK, 0, s>>>(B.args);
    k_link_count<<<g, GCHUNK, 0, s>>>(B.args);
    k_link_write<<<g, GCHUNK, 0, sw>>>(B.args);
}

// One step.  With a side stream (and particles, no per-kernel timing, and
// at least SIDE_MIN_NODES nodes, below which the fork and join cost more
// than they hide) the particle work runs beside the bulk lattice kernels:
// the mu fix-up
// beside the bulk mu update, and the psi/c fix-up, the link pass and the
// rigid-body update beside the bulk psi/c update.  Fork and join go through
// events, so a captured graph holds them as parallel branches.  The bulk
// kernels touch neither the boundary nodes nor the particle records, and
// the side work touches no node the bulk kernels write.
constexpr long long SIDE_MIN_NODES = 1LL << 22;

template <int P>
void launch_step(const Batch &B, hipStream_t s, const SideStream *side, TimingHook *tm,
                 bool defer_links)
{
    typedef typename Prec<P>::S S;
    constexpr int V4 = sizeof(S) == 4 ? 4 : 2;  // FP64 scalars: 2 per 16-byte access
    // split: boundary nodes in fix-up launches (on the side stream if par);
    // psi/c sub-steps keep everything in order on s
    const bool split = B.ncol > 0 && (B.nodes >= SIDE_MIN_NODES || B.special);
    const bool par = split && side && !tm && B.nsub <= 1;
    hipStream_t ss = par ? side->s : s;
    const dim3 gfix(B.args.nfix);
    const int vm = B.vec[0] == 4 ? 4 : (B.vec[0] == 2 ? 2 : 1);
    const bool bi = B.ncol > 0 && !split;  // boundary nodes inline
    auto mu = [&](const BatchArgs &a) {
        if (B.nopsi) return;  // single phase: mu stays 0
        if (split && B.special) k_mu_bnd<S, true><<<gfix, GCHUNK, 0, ss>>>(a);
        else if (split) k_mu_bnd<S, false><<<gfix, GCHUNK, 0, ss>>>(a);
        if (B.stress) k_mu<S, 1, false, true><<<B.nblocks[0], 256, 0, s>>>(a);
        else if (vm == 4 && bi) k_mu<S, V4, true><<<B.nblocks[0], 256, 0, s>>>(a);
        else if (vm == 4) k_mu<S, V4, false><<<B.nblocks[0], 256, 0, s>>>(a);
        else if (vm == 2 && bi) k_mu<S, 2, true><<<B.nblocks[0], 256, 0, s>>>(a);
        else if (vm == 2) k_mu<S, 2, false><<<B.nblocks[0], 256, 0, s>>>(a);
        else if (bi) k_mu<S, 1, true><<<B.nblocks[0], 256, 0, s>>>(a);
        else k_mu<S, 1, false><<<B.nblocks[0], 256, 0, s>>>(a);
    };
    if (tm) tm->begin(0, s);
    if (par) {
        hipEventRecord(side->ev[0], s);
        hipStreamWaitEvent(ss, side->ev[0], 0);
    }
    mu(B.args);
    if (par) {
        hipEventRecord(side->ev[1], ss);
        hipStreamWaitEvent(s, side->ev[1], 0);
    }
    if (tm) tm->end(0, s);
    if (tm) tm->begin(1, s);
    if (B.solute_force || B.stress) k_collide<P, true><<<B.nblocks[1], 256, 0, s>>>(B.args);
    else if (B.nopsi && B.vec[1] <= 1) k_collide<P, false, true><<<B.nblocks[1], 256, 0, s>>>(B.args);
    else if (B.vec[1] == 4) k_collide_v<P, V4><<<B.nblocks[1], 256, 0, s>>>(B.args);
    else if (B.vec[1] == 2) k_collide_v<P, 2><<<B.nblocks[1], 256, 0, s>>>(B.args);
    else k_collide<P, false><<<B.nblocks[1], 256, 0, s>>>(B.args);
    if (tm) tm->end(1, s);
    if (tm) tm->begin(2, s);
    if (par) {
        hipEventRecord(side->ev[2], s);
        hipStreamWaitEvent(ss, side->ev[2], 0);
    }
    // sub-step 0 reads the state at t and writes the pair its table names
    BatchArgs a0 = B.args;
    if (B.nsub > 1) a0.d = B.dsub[0];
    // the link pass first on the side stream: its few blocks take CUs before
    // the bulk psi/c update fills them (it reads the state at t, like the
    // boundary psi/c fix-up after it, and writes neither's inputs)
    const bool early_links = par && B.ncol > 0;
    if (early_links) {
        if (B.soft) k_soft<<<(B.ncol + 63) / 64, 64, 0, ss>>>(B.args, B.ncol);
        k_link_partial<P><<<dim3(B.nlchunk_max, B.ncol), LINK_THREADS, 0, ss>>>(B.args);
    }
    if (split && B.special) k_scalar_bnd<S, true><<<gfix, GCHUNK, 0, ss>>>(a0);
    else if (split) k_scalar_bnd<S, false><<<gfix, GCHUNK, 0, ss>>>(a0);
    const int vs = B.vec[2] == 4 ? 4 : (B.vec[2] == 2 ? 2 : 1);
    auto scalar = [&](const dim3 gs, const BatchArgs &a) {
        if (B.nopsi && !B.zmarch) {
            // single phase: c and u only
            if (vs == 4) {
                if (bi) k_scalar<S, V4, false, true, true><<<gs, 256, 0, s>>>(a);
                else k_scalar<S, V4, false, false, true><<<gs, 256, 0, s>>>(a);
            } else if (vs == 2) {
                if (bi) k_scalar<S, 2, false, true, true><<<gs, 256, 0, s>>>(a);
                else k_scalar<S, 2, false, false, true><<<gs, 256, 0, s>>>(a);
            } else {
                if (bi) k_scalar<S, 1, false, true, true><<<gs, 256, 0, s>>>(a);
                else k_scalar<S, 1, false, false, true><<<gs, 256, 0, s>>>(a);
            }
            return;
        }
        if (vs == 4 && B.zmarch) {
            if (bi) k_scalar<S, V4, true, true><<<gs, 256, 0, s>>>(a);
            else k_scalar<S, V4, true, false><<<gs, 256, 0, s>>>(a);
        } else if (vs == 2 && B.zmarch) {
            if (bi) k_scalar<S, 2, true, true><<<gs, 256, 0, s>>>(a);
            else k_scalar<S, 2, true, false><<<gs, 256, 0, s>>>(a);
        } else if (vs == 4) {
            if (bi) k_scalar<S, V4, false, true><<<gs, 256, 0, s>>>(a);
            else k_scalar<S, V4, false, false><<<gs, 256, 0, s>>>(a);
        } else if (vs == 2) {
            if (bi) k_scalar<S, 2, false, true><<<gs, 256, 0, s>>>(a);
            else k_scalar<S, 2, false, false><<<gs, 256, 0, s>>>(a);
        } else {
            if (bi) k_scalar<S, 1, false, true><<<gs, 256, 0, s>>>(a);
            else k_scalar<S, 1, false, false><<<gs, 256, 0, s>>>(a);
        }
    };
    if (par && B.nblocks[2] >= 2) {
        // two launches of half the blocks each: the side-stream kernels
        // queued meanwhile are dispatched between the halves instead of
        // after the whole grid (measured: step -12 us FP32, -15 us FP16)
        const int h = B.nblocks[2] / 2;
        BatchArgs a2 = B.args;
        a2.boff = h;
        scalar(dim3(h), B.args);
        scalar(dim3(B.nblocks[2] - h), a2);
    } else {
        scalar(dim3(B.nblocks[2]), a0);
    }
    if (tm) tm->end(2, s);
    // later sub-steps: mu and chi of the previous result, then its update,
    // from whichever pair sub-step j-1 wrote (the next-state pair when
    // n-1-(j-1) is even) into the other
    for (int j = 1; j < B.nsub; j++) {
        BatchArgs a = B.args;
        a.d = B.dsub[(B.nsub - j) % 2 == 0 ? 1 : 2];
        if (tm) tm->begin(0, s);
        mu(a);
        if (tm) tm->end(0, s);
        if (tm) tm->begin(2, s);
        if (split && B.special) k_scalar_bnd<S, true><<<gfix, GCHUNK, 0, s>>>(a);
        else if (split) k_scalar_bnd<S, false><<<gfix, GCHUNK, 0, s>>>(a);
        scalar(dim3(B.nblocks[2]), a);
        if (tm) tm->end(2, s);
    }
    if (B.ncol <= 0) return;
    if (tm) tm->begin(3, s);
    if (!early_links) {
        if (B.soft) k_soft<<<(B.ncol + 63) / 64, 64, 0, ss>>>(B.args, B.ncol);
        k_link_partial<P><<<dim3(B.nlchunk_max, B.ncol), LINK_THREADS, 0, ss>>>(B.args);
    }
    k_colloid_update<<<B.ncol, 64, 0, ss>>>(B.args);
    if (par) {
        hipEventRecord(side->ev[3], ss);
        hipStreamWaitEvent(s, side->ev[3], 0);
    }
    if (tm) tm->end(3, s);
    if (tm) tm->begin(4, s);
    k_cover<P><<<dim3(B.nchunk_max, B.ncol), GCHUNK, 0, s>>>(B.args);
    if (tm) tm->end(4, s);
    if (tm) tm->begin(5, s);
    if (par && defer_links) {
        // the link table write of this step runs beside the next step's bulk
        // mu update; the next step's side work is ordered after it and
        // joined before its collide-stream, ahead of the link pass
        const dim3 g(B.nchunk_max, B.ncol);
        k_commit<<<g, GCHUNK, 0, s>>>(B.args);
        k_link_count<<<g, GCHUNK, 0, s>>>(B.args);
        hipEventRecord(side->ev[4], s);
        hipStreamWaitEvent(ss, side->ev[4], 0);
        k_link_write<<<g, GCHUNK, 0, ss>>>(B.args);
    } else {
        launch_geometry_tail(B, s, s);
    }
    if (tm) tm->end(5, s);
}

// geometry at placement: no transfer, every particle marked changed
__global__ void k_mark_placed(BatchArgs A)
{
    const int j = find_box(A.cstart, A.nbox, blockIdx.x);
    const BoxDesc &D = A.d[j];
    const int k = blockIdx.x - A.cstart[j];
    for (int c = threadIdx.x; c < D.b.nchunk_max; c += blockDim.x) {
        double *o = D.b.cpart + ((size_t)k * D.b.nchunk_max + c) * 8;
        for (int a = 0; a < 8; a++) o[a] = 0.0;
        o[6] = 1.0;
    }
}

void launch_geometry(const Batch &B, hipStream_t s)
{
    if (B.ncol <= 0) return;
    k_mark_placed<<<B.ncol, 64, 0, s>>>(B.args);
    launch_geometry_tail(B, s, s);
}

template <int P>
void launch_init(const KParams &p, const double *psi0, const double *c0, const double *rho0,
                 const double *u0, void *f, void *psi, void *cc, uint8_t *own, hipStream_t s)
{
    typedef typename Prec<P>::T T;
    typedef typename Prec<P>::S S;
    k_init<P><<<(p.N + 255) / 256, 256, 0, s>>>(p, psi0, c0, rho0, u0, (T *)f, (S *)psi, (S *)cc, own);
}

template <int P>
void launch_reduce(const KParams &p, const void *f, const void *psi, const void *cc,
                   const uint8_t *own, double *part, int nblocks, double *out, hipStream_t s)
{
    typedef typename Prec<P>::T T;
    typedef typename Prec<P>::S S;
    k_reduce<P><<<nblocks, 256, 0, s>>>(p, (const T *)f, (const S *)psi, (const S *)cc, own, part);
    k_reduce_final<<<1, 256, 0, s>>>(part, nblocks, out);
}

template <int P>
void launch_fields(const KParams &p, const void *f, const void *psi, const void *cc,
                   const uint8_t *own, double *out, double *fout, hipStream_t s)
{
    typedef typename Prec<P>::T T;
    typedef typename Prec<P>::S S;
    k_fields<P><<<(p.N + 255) / 256, 256, 0, s>>>(p, (const T *)f, (const S *)psi, (const S *)cc,
                                                  own, out, fout);
}

#define LB_INSTANTIATE(P)                                                                          \
    template void launch_step<P>(const Batch &, hipStream_t, const SideStream *, TimingHook *,      \
                                 bool);                                                             \
    template void launch_init<P>(const KParams &, const double *, const double *, const double *,   \
                                 const double *, void *, void *, void *, uint8_t *, hipStream_t);   \
    template void launch_reduce<P>(const KParams &, const void *, const void *, const void *,       \
                                   const uint8_t *, double *, int, double *, hipStream_t);          \
    template void launch_fields<P>(const KParams &, const void *, const void *, const void *,       \
                                   const uint8_t *, double *, double *, hipStream_t);

LB_INSTANTIATE(LB_FP64)
LB_INSTANTIATE(LB_FP32)
LB_INSTANTIATE(LB_FP16_STORAGE)

}  // namespace lbk
