// lb_kernels.hip -- gfx950 kernels of one time step of the lattice update of
// the multiphase-multicomponent LB model for self-diffusiophoretic Janus
// colloids (arXiv:2202.01631, Sec. II).
//
// Step sequence on one stream (cur -> nxt buffers):
//   k_mu             mu_psi of Eq. 2 with the wetting ghost of Eqs. 8-9
//   k_collide        force -psi grad(mu), moments, BGK-Guo collision, push
//                    streaming with plain (resting-wall) bounce-back
//   k_scalar         psi and c updates of Eq. 3 with Janus emission (Eq. 5)
//   k_link_partial   per (link chunk, particle): moving-wall and slip
//                    correction of every link (Eqs. 4, 6), FP64 momentum
//                    exchange partials
//   k_colloid_update per particle: partials summed in chunk order, implicit
//                    rigid-body update
//   k_cover          per particle: cover/uncover repair at the new position
//   k_commit         per particle: owner bytes at the new position
//   k_links          per particle: boundary bits and canonical link table
// Lattice kernels use one thread per node, 64-wide rows in x (one wavefront
// per row segment, coalesced structure-of-arrays access).
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

template <class S> __device__ __forceinline__ S s_tanh(S v);
template <> __device__ __forceinline__ double s_tanh<double>(double v) { return tanh(v); }
template <> __device__ __forceinline__ float s_tanh<float>(float v) { return tanhf(v); }

// ------------------------------------------------------------------ k_mu
// Also stores chi = c - c_b0 - E tanh psi for the solute update.
// mu_psi = a psi + b psi^3 - kappa lap(psi) - C E chi (1 - tanh^2 psi),
// chi = c - c_b0 - E tanh psi (Eq. 2; 1/cosh^2 = 1 - tanh^2, cubic factored
// as b psi (psi-1)(psi+1) + (a+b) psi to keep FP32 cancellation small).
// At a solid face neighbour the Laplacian takes the ghost psi - (H/kappa)|e.n|
// (Eq. 9, n through the face midpoint).
template <class S>
__global__ __launch_bounds__(256) void k_mu(BatchArgs A)
{
    const int j = find_box(A.bstart, A.nbox, blockIdx.x);
    const BoxDesc &D = A.d[j];
    KParams p = D.p;
    p.ls = D.ls[0];
    const S *__restrict__ psi = (const S *)D.b.psi;
    const S *__restrict__ cc = (const S *)D.b.cc;
    const uint8_t *__restrict__ own = D.b.own;
    const DColloid *__restrict__ col = D.b.col;
    S *__restrict__ mu = (S *)D.b.mu;
    S *__restrict__ chi_out = (S *)D.b.chi;
    int x, y, z;
    if (!lattice_node(p, blockIdx.x - A.bstart[j], x, y, z)) return;
    const int sy = p.nx, sz = p.nx * p.ny;
    const int n = x + sy * y + sz * z;
    const uint8_t o = own[n];
    if (o & OWN_SOLID) { mu[n] = S(0); chi_out[n] = S(0); return; }
    const int nb[6] = {n - x + wrap_p(x, p.nx), n - x + wrap_m(x, p.nx),
                       n + (wrap_p(y, p.ny) - y) * sy, n + (wrap_m(y, p.ny) - y) * sy,
                       n + (wrap_p(z, p.nz) - z) * sz, n + (wrap_m(z, p.nz) - z) * sz};
    const S ps = psi[n];
    S pv[6];
#pragma unroll
    for (int e = 0; e < 6; e++) pv[e] = psi[nb[e]];
    S lap = S(-6) * ps;
    if (o & OWN_BOUNDARY) {
#pragma unroll
        for (int e = 0; e < 6; e++) {
            const uint8_t om = own[nb[e]] & OWN_SOLID;
            if (!om) {
                lap += pv[e];
            } else {
                const DColloid &q = col[om - 1];
                double r[3];
                const int ax = e >> 1, sg = (e & 1) ? -1 : 1;
                displacement(q, x, y, z, ax == 0 ? sg : 0, ax == 1 ? sg : 0, ax == 2 ? sg : 0, 0.5,
                             p.nx, p.ny, p.nz, r);
                const double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
                const double en = fabs(r[ax]) / rn;
                const double gh = p.kappa > 0.0 ? (q.H / p.kappa) * en : 0.0;
                lap += ps - (S)gh;
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < 6; e++) lap += pv[e];
    }
    const S a = (S)p.a, b = (S)p.b;
    const S t = s_tanh<S>(ps);
    const S chi = cc[n] - (S)p.cb0 - (S)p.E * t;
    mu[n] = b * ps * (ps - S(1)) * (ps + S(1)) + (a + b) * ps - (S)p.kappa * lap -
            (S)(p.C * p.E) * chi * (S(1) - t * t);
    chi_out[n] = chi;
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
// bounce-back; the moving-wall and slip terms are added by k_links_colloid).
template <int P>
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
    const uint8_t o = own[n];
    if (o & OWN_SOLID) return;
    const bool bnd = (o & OWN_BOUNDARY) != 0;
    const size_t N = (size_t)p.N;
    const int xo[3] = {wrap_m(x, p.nx) - x, 0, wrap_p(x, p.nx) - x};
    const int yo[3] = {(wrap_m(y, p.ny) - y) * sy, 0, (wrap_p(y, p.ny) - y) * sy};
    const int zo[3] = {(wrap_m(z, p.nz) - z) * sz, 0, (wrap_p(z, p.nz) - z) * sz};

    S g[19];
#pragma unroll
    for (int i = 0; i < 19; i++) g[i] = ld_pop(fin, i * N + n, p.inv_scale);
    S drho = S(0), jx = S(0), jy = S(0), jz = S(0);
#pragma unroll
    for (int i = 0; i < 19; i++) {
        drho += g[i];
        if (cx(i)) jx += cx(i) > 0 ? g[i] : -g[i];
        if (cy(i)) jy += cy(i) > 0 ? g[i] : -g[i];
        if (cz(i)) jz += cz(i) > 0 ? g[i] : -g[i];
    }
    // solid neighbours (only boundary nodes have any), as a mask over i
    unsigned solid = 0;
    if (bnd) {
#pragma unroll
        for (int i = 1; i < 19; i++) {
            const int m = n + xo[cx(i) + 1] + yo[cy(i) + 1] + zo[cz(i) + 1];
            solid |= (own[m] & OWN_SOLID) ? (1u << i) : 0u;
        }
    }
    // body force -psi grad(mu), isotropic lattice gradient
    // grad(mu) = 3 sum_i w_i c_i mu(x + c_i), mu(x) at solid neighbours
    const S m0 = mu[n];
    S gx = S(0), gy = S(0), gz = S(0);
#pragma unroll
    for (int i = 1; i < 19; i++) {
        const int m = n + xo[cx(i) + 1] + yo[cy(i) + 1] + zo[cz(i) + 1];
        S mi = mu[m];
        if (solid & (1u << i)) mi = m0;
        const S wi = (S)(3.0 * wgt(i));
        if (cx(i)) gx += cx(i) > 0 ? wi * mi : -wi * mi;
        if (cy(i)) gy += cy(i) > 0 ? wi * mi : -wi * mi;
        if (cz(i)) gz += cz(i) > 0 ? wi * mi : -wi * mi;
    }
    const S ps = psi[n];
    const S Fx = -ps * gx + (S)p.fx;
    const S Fy = -ps * gy + (S)p.fy;
    const S Fz = -ps * gz + (S)p.fz;
    const S rho = (S)p.rho0 + drho;
    const S ir = S(1) / rho;
    const S ux = (jx + S(0.5) * Fx) * ir;
    const S uy = (jy + S(0.5) * Fy) * ir;
    const S uz = (jz + S(0.5) * Fz) * ir;
    const S uu = ux * ux + uy * uy + uz * uz;
    const S uF = ux * Fx + uy * Fy + uz * Fz;
    const S om = (S)(1.0 / p.tau);
    const S pref = (S)(1.0 - 0.5 / p.tau);
#pragma unroll
    for (int i = 0; i < 19; i++) {
        const S w = (S)wgt(i);
        const S cu = (S)cx(i) * ux + (S)cy(i) * uy + (S)cz(i) * uz;
        const S cF = (S)cx(i) * Fx + (S)cy(i) * Fy + (S)cz(i) * Fz;
        const S geq = w * (drho + rho * (S(3) * cu + S(4.5) * cu * cu - S(1.5) * uu));
        const S gs = g[i] - om * (g[i] - geq) + pref * w * (S(3) * (cF - uF) + S(9) * cu * cF);
        if (i == 0) {
            st_pop(fout, (size_t)n, gs, p.scale);
        } else {
            const int m = n + xo[cx(i) + 1] + yo[cy(i) + 1] + zo[cz(i) + 1];
            if (solid & (1u << i))
                st_pop(fout, opp(i) * N + n, gs, p.scale);
            else
                st_pop(fout, i * N + m, gs, p.scale);
        }
    }
    uout[n] = ux;
    uout[N + n] = uy;
    uout[2 * N + n] = uz;
}

// -------------------------------------------------------------- k_scalar
// psi' = psi - sum_e J_e + M sum_e (mu_e - mu),
// c'   = c - sum_e Jc_e + D sum_e (chi_e - chi) + emission - k_d chi,
// J_e = 1/2 (u.e + u_e.e) 1/2 (psi + psi_e) over the 6 faces, nothing
// through faces shared with solid nodes (Eq. 3, explicit Euler, dt = 1).
// Emission: alpha of the cap of each link of the node (Eq. 5).
template <class S>
__global__ __launch_bounds__(256) void k_scalar(BatchArgs A)
{
    const int *bst = A.bstart + 2 * (A.nbox + 1);
    const int j = find_box(bst, A.nbox, blockIdx.x);
    const BoxDesc &D = A.d[j];
    KParams p = D.p;
    p.ls = D.ls[2];
    const S *__restrict__ psi = (const S *)D.b.psi;
    const S *__restrict__ cc = (const S *)D.b.cc;
    const S *__restrict__ mu = (const S *)D.b.mu;
    const S *__restrict__ chiv = (const S *)D.b.chi;
    const S *__restrict__ u = (const S *)D.b.u;
    const uint8_t *__restrict__ own = D.b.own;
    const DColloid *__restrict__ col = D.b.col;
    S *__restrict__ psin = (S *)D.b.psin;
    S *__restrict__ ccn = (S *)D.b.ccn;
    int x, y, z;
    if (!lattice_node(p, blockIdx.x - bst[j], x, y, z)) return;
    const int sy = p.nx, sz = p.nx * p.ny;
    const int n = x + sy * y + sz * z;
    const uint8_t o = own[n];
    const S ps = psi[n], cn = cc[n];
    if (o & OWN_SOLID) { psin[n] = ps; ccn[n] = cn; return; }
    const bool bnd = (o & OWN_BOUNDARY) != 0;
    const size_t N = (size_t)p.N;
    const int xo[3] = {wrap_m(x, p.nx) - x, 0, wrap_p(x, p.nx) - x};
    const int yo[3] = {(wrap_m(y, p.ny) - y) * sy, 0, (wrap_p(y, p.ny) - y) * sy};
    const int zo[3] = {(wrap_m(z, p.nz) - z) * sz, 0, (wrap_p(z, p.nz) - z) * sz};
    const int fn[6] = {n + xo[2], n + xo[0], n + yo[2], n + yo[0], n + zo[2], n + zo[0]};
    const S chi = chiv[n];
    const S m0 = mu[n];
    const S u0[3] = {u[n], u[N + n], u[2 * N + n]};
    // all neighbour loads issued together; solid faces masked afterwards
    S um[6], pm[6], cm[6], mm[6], xm[6];
#pragma unroll
    for (int e = 0; e < 6; e++) {
        const int m = fn[e];
        um[e] = u[(e >> 1) * N + m];
        pm[e] = psi[m];
        cm[e] = cc[m];
        mm[e] = mu[m];
        xm[e] = chiv[m];
    }
    unsigned solid = 0;
    if (bnd) {
#pragma unroll
        for (int e = 0; e < 6; e++) solid |= (own[fn[e]] & OWN_SOLID) ? (1u << e) : 0u;
    }
    S adv_p = S(0), adv_c = S(0), dmu = S(0), dchi = S(0);
#pragma unroll
    for (int e = 0; e < 6; e++) {
        const bool fl = !(solid & (1u << e));  // no flux through a solid face
        const int ax = e >> 1;
        const S ue = (e & 1) ? S(-0.5) * (u0[ax] + um[e]) : S(0.5) * (u0[ax] + um[e]);
        adv_p += fl ? ue * (S(0.5) * (ps + pm[e])) : S(0);
        adv_c += fl ? ue * (S(0.5) * (cn + cm[e])) : S(0);
        dmu += fl ? mm[e] - m0 : S(0);
        dchi += fl ? xm[e] - chi : S(0);
    }
    S src = S(0);
    if (bnd) {
        for (int d = 1; d < 19; d++) {
            const int m = n + xo[cx(d) + 1] + yo[cy(d) + 1] + zo[cz(d) + 1];
            const uint8_t om = own[m] & OWN_SOLID;
            if (!om) continue;
            const DColloid &q = col[om - 1];
            double r[3];
            displacement(q, x, y, z, cx(d), cy(d), cz(d), 0.5, p.nx, p.ny, p.nz, r);
            src += (S)(active_cap(q, r) ? q.am : q.ap);
        }
    }
    psin[n] = ps - adv_p + (S)p.M * dmu;
    ccn[n] = cn - adv_c + (S)p.D * dchi + src - (S)p.kd * chi;
}

// ----------------------------------------------------------- k_scalar_zm
// The same update with each thread marching zc consecutive planes of one
// (x, y) column: the z - 1, z, z + 1 values of psi, c, mu, chi and u_z stay
// in registers, so a node costs five plane loads fewer than in k_scalar.
// Blocks of (bx, by) columns; block b covers x segment b % xseg, row group
// (b / xseg) % ygroups and z chunk b / (xseg * ygroups).
template <class S>
__global__ __launch_bounds__(256) void k_scalar_zm(BatchArgs A)
{
    const int *bst = A.bstart + 2 * (A.nbox + 1);
    const int j = find_box(bst, A.nbox, blockIdx.x);
    const BoxDesc &D = A.d[j];
    const KParams p = D.p;
    const LaunchShape ls = D.ls[2];
    const S *__restrict__ psi = (const S *)D.b.psi;
    const S *__restrict__ cc = (const S *)D.b.cc;
    const S *__restrict__ mu = (const S *)D.b.mu;
    const S *__restrict__ chiv = (const S *)D.b.chi;
    const S *__restrict__ u = (const S *)D.b.u;
    const uint8_t *__restrict__ own = D.b.own;
    const DColloid *__restrict__ col = D.b.col;
    S *__restrict__ psin = (S *)D.b.psin;
    S *__restrict__ ccn = (S *)D.b.ccn;
    const int b = blockIdx.x - bst[j];
    const int ygroups = (p.ny + ls.by - 1) / ls.by;
    const int tx = (int)threadIdx.x % ls.bx, ty = (int)threadIdx.x / ls.bx;
    if (ty >= ls.by) return;
    const int seg = b % ls.xseg, rest = b / ls.xseg;
    const int x = seg * ls.bx + tx, y = (rest % ygroups) * ls.by + ty;
    const int z0 = (rest / ygroups) * ls.zc;
    if (x >= p.nx || y >= p.ny || z0 >= p.nz) return;
    const int z1 = min(z0 + ls.zc, p.nz);
    const int sy = p.nx, sz = p.nx * p.ny;
    const size_t N = (size_t)p.N;
    const int xm = wrap_m(x, p.nx) - x, xp = wrap_p(x, p.nx) - x;
    const int ym = (wrap_m(y, p.ny) - y) * sy, yp = (wrap_p(y, p.ny) - y) * sy;
    const int col0 = x + sy * y;
    // rolling window along z: index 0 = z - 1, 1 = z, 2 = z + 1
    S wp[3], wc[3], wm[3], wx[3], wu[3];
    uint8_t wo[3];
    {
        const int zb = wrap_m(z0, p.nz);
        const int nb = col0 + sz * zb, n0 = col0 + sz * z0;
        wp[0] = psi[nb]; wc[0] = cc[nb]; wm[0] = mu[nb]; wx[0] = chiv[nb]; wu[0] = u[2 * N + nb];
        wo[0] = own[nb];
        wp[1] = psi[n0]; wc[1] = cc[n0]; wm[1] = mu[n0]; wx[1] = chiv[n0]; wu[1] = u[2 * N + n0];
        wo[1] = own[n0];
    }
    for (int z = z0; z < z1; z++) {
        const int n = col0 + sz * z;
        const int zn = wrap_p(z, p.nz);
        const int na = col0 + sz * zn;
        wp[2] = psi[na]; wc[2] = cc[na]; wm[2] = mu[na]; wx[2] = chiv[na]; wu[2] = u[2 * N + na];
        wo[2] = own[na];
        const uint8_t o = wo[1];
        const S ps = wp[1], cn = wc[1];
        if (o & OWN_SOLID) {
            psin[n] = ps;
            ccn[n] = cn;
        } else {
            const bool bnd = (o & OWN_BOUNDARY) != 0;
            const int fn[4] = {n + xp, n + xm, n + yp, n + ym};
            S um[6], pm[6], cm[6], mm[6], xmv[6];
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int m = fn[e];
                um[e] = u[(e >> 1) * N + m];
                pm[e] = psi[m];
                cm[e] = cc[m];
                mm[e] = mu[m];
                xmv[e] = chiv[m];
            }
            um[4] = wu[2]; pm[4] = wp[2]; cm[4] = wc[2]; mm[4] = wm[2]; xmv[4] = wx[2];
            um[5] = wu[0]; pm[5] = wp[0]; cm[5] = wc[0]; mm[5] = wm[0]; xmv[5] = wx[0];
            const S chi = wx[1], m0 = wm[1];
            const S u0[3] = {u[n], u[N + n], wu[1]};
            unsigned solid = 0;
            if (bnd) {
#pragma unroll
                for (int e = 0; e < 4; e++) solid |= (own[fn[e]] & OWN_SOLID) ? (1u << e) : 0u;
                solid |= (wo[2] & OWN_SOLID) ? 16u : 0u;
                solid |= (wo[0] & OWN_SOLID) ? 32u : 0u;
            }
            S adv_p = S(0), adv_c = S(0), dmu = S(0), dchi = S(0);
#pragma unroll
            for (int e = 0; e < 6; e++) {
                const bool fl = !(solid & (1u << e));
                const int ax = e >> 1;
                const S ue = (e & 1) ? S(-0.5) * (u0[ax] + um[e]) : S(0.5) * (u0[ax] + um[e]);
                adv_p += fl ? ue * (S(0.5) * (ps + pm[e])) : S(0);
                adv_c += fl ? ue * (S(0.5) * (cn + cm[e])) : S(0);
                dmu += fl ? mm[e] - m0 : S(0);
                dchi += fl ? xmv[e] - chi : S(0);
            }
            S src = S(0);
            if (bnd) {
                const int xo[3] = {xm, 0, xp}, yo[3] = {ym, 0, yp};
                const int zo[3] = {(wrap_m(z, p.nz) - z) * sz, 0, (zn - z) * sz};
                for (int d = 1; d < 19; d++) {
                    const int m = n + xo[cx(d) + 1] + yo[cy(d) + 1] + zo[cz(d) + 1];
                    const uint8_t om = own[m] & OWN_SOLID;
                    if (!om) continue;
                    const DColloid &q = col[om - 1];
                    double r[3];
                    displacement(q, x, y, z, cx(d), cy(d), cz(d), 0.5, p.nx, p.ny, p.nz, r);
                    src += (S)(active_cap(q, r) ? q.am : q.ap);
                }
            }
            psin[n] = ps - adv_p + (S)p.M * dmu;
            ccn[n] = cn - adv_c + (S)p.D * dchi + src - (S)p.kd * chi;
        }
        wp[0] = wp[1]; wc[0] = wc[1]; wm[0] = wm[1]; wx[0] = wx[1]; wu[0] = wu[1]; wo[0] = wo[1];
        wp[1] = wp[2]; wc[1] = wc[2]; wm[1] = wm[2]; wx[1] = wx[2]; wu[1] = wu[2]; wo[1] = wo[2];
    }
}

// ------------------------------------------------ block reductions (FP64)
// Fixed-shape reductions: wavefront butterfly, then the waves in order, so
// results do not depend on scheduling.
template <int NV>
__device__ void block_sum(double (&v)[NV], double *lds /* NV * nwaves */)
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
    if (threadIdx.x == 0) {
        for (int j = 0; j < NV; j++) {
            double s = lds[j];
            for (int w = 1; w < nw; w++) s += lds[w * NV + j];
            v[j] = s;
        }
    }
    __syncthreads();
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
        // cap from the current axis (the table is rebuilt only on owner changes)
        const bool cap = active_cap(q, r);
        const double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        const double nh[3] = {r[0] / rn, r[1] / rn, r[2] / rn};
        // grad c at the fluid node, c(x) substituted at solid neighbours
        const int sy = p.nx, sz = p.nx * p.ny;
        const int fn[6] = {n - x + wrap_p(x, p.nx), n - x + wrap_m(x, p.nx),
                           n + (wrap_p(y, p.ny) - y) * sy, n + (wrap_m(y, p.ny) - y) * sy,
                           n + (wrap_p(z, p.nz) - z) * sz, n + (wrap_m(z, p.nz) - z) * sz};
        const double c0 = (double)cc[n];
        double cv[6];
        for (int e = 0; e < 6; e++) cv[e] = (own[fn[e]] & OWN_SOLID) ? c0 : (double)cc[fn[e]];
        const double g[3] = {0.5 * (cv[0] - cv[1]), 0.5 * (cv[2] - cv[3]), 0.5 * (cv[4] - cv[5])};
        const double mob = cap ? q.mum : q.mup;
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
        const double dp[3] = {ex * mag, ey * mag, ez * mag};
        double t[3];
        cross3(r, dp, t);
        const double cd[3] = {(double)ex, (double)ey, (double)ez};
        double rc[3];
        cross3(r, cd, rc);
        const double gv[6] = {cd[0], cd[1], cd[2], rc[0], rc[1], rc[2]};
        const double coef = 6.0 * w * rho0;
        for (int a = 0; a < 3; a++) { acc[a] += dp[a]; acc[3 + a] += t[a]; }
        int j = 6;
        for (int i1 = 0; i1 < 6; i1++)
            for (int i2 = i1; i2 < 6; i2++) acc[j++] += coef * gv[i1] * gv[i2];
        acc[27] += cap ? 1.0 : 0.0;
        }
    }
    block_sum<28>(acc, lds);
    if (threadIdx.x == 0) {
        double *o = D.b.lpart + ((size_t)k * D.b.nlchunk_max + blockIdx.x) * 28;
        for (int a = 0; a < 28; a++) o[a] = acc[a];
    }
}

// ------------------------------------------------------ k_colloid_update
// One block per particle: link partials summed in chunk order (FP64), then
// (M + zeta) X' = M X + (F0, T0) + transfers (implicit update),
// R' = R + V', m' = m rotated by |Omega'| about Omega'.
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
        const double *o = D.b.lpart + (size_t)k * D.b.nlchunk_max * 28 + threadIdx.x;
        double s = 0.0;
        for (int c = 0; c < nch; c++) s += o[(size_t)c * 28];
        sacc[threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double acc[28];
    for (int a = 0; a < 28; a++) acc[a] = sacc[a];
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
    if (q.fixed) {
        for (int i = 0; i < 6; i++) Xn[i] = X[i];
    } else {
        const double Mv[6] = {q.mass, q.mass, q.mass, q.inertia, q.inertia, q.inertia};
        double A[36], bb[6];
        for (int i = 0; i < 36; i++) A[i] = Z[i];
        for (int i = 0; i < 6; i++) { A[6 * i + i] += Mv[i]; bb[i] = Mv[i] * X[i] + Fk[i]; }
        // Gaussian elimination without pivoting (M + zeta is symmetric positive definite)
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
    for (int i = 0; i < 6; i++) {
        double s = Fk[i];
        for (int j = 0; j < 6; j++) s -= Z[6 * i + j] * Xn[j];
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
    b.bx = axis_box(q.pos[0], q.radius, p.nx);
    b.by = axis_box(q.pos[1], q.radius, p.ny);
    b.bz = axis_box(q.pos[2], q.radius, p.nz);
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
    block_sum<6>(acc, lds);
    if (threadIdx.x == 0) {
        double *o = cpart + ((size_t)k * nchunk_max + c) * 8;
        for (int a = 0; a < 6; a++) o[a] = acc[a];
        o[6] = any ? 1.0 : 0.0;
    }
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
        double r[3];
        displacement(q, x, y, z, cx(d), cy(d), cz(d), 0.5, p.nx, p.ny, p.nz, r);
        const bool cap = active_cap(q, r);
        if (l < lcap) {
            lnode[(size_t)k * lcap + l] = n;
            ldc[(size_t)k * lcap + l] = (uint8_t)(d | (cap ? 0x80 : 0));
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
    block_sum<7>(v, lds);
    if (threadIdx.x == 0)
        for (int j = 0; j < 7; j++) part[blockIdx.x * 7 + j] = v[j];
}

__global__ __launch_bounds__(256) void k_reduce_final(const double *__restrict__ part, int nblocks,
                                                      double *__restrict__ out)
{
    __shared__ double lds[7 * 16];
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        for (int j = 0; j < 7; j++) v[j] += part[b * 7 + j];
    block_sum<7>(v, lds);
    if (threadIdx.x == 0)
        for (int j = 0; j < 7; j++) out[j] = v[j];
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
        if (fout) fout[i * N + n] = g + wgt(i) * p.rho0;
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
void finish_shape(LaunchShape &ls, int nx, int ny, int nz)
{
    if (ls.bx <= 0 || ls.bx > 256) ls.bx = nx < 256 ? nx : 256;
    if (ls.bx > nx) ls.bx = nx;
    if (ls.by <= 0) ls.by = ls.bx >= 256 ? 1 : 256 / ls.bx;
    if (ls.bx * ls.by > 256) ls.by = 256 / ls.bx;  // the kernels' launch bound
    if (ls.by < 1) ls.by = 1;
    ls.xseg = (nx + ls.bx - 1) / ls.bx;
    const long long rows = (long long)ny * nz;
    ls.nblocks = (int)(ls.xseg * ((rows + ls.by - 1) / ls.by));
    ls.bpp = 0;
    if (ls.zc > 0) {
        // z-marching launch: blocks over (x segment, row group in y, z chunk)
        if (ls.zc > nz) ls.zc = nz;
        ls.remap = 0;
        ls.nblocks = ls.xseg * ((ny + ls.by - 1) / ls.by) * ((nz + ls.zc - 1) / ls.zc);
        return;
    }
    if (ls.remap == 2) {
        // plane-wise renumbering needs whole planes per block row and
        // blocks per plane divisible by 8
        if (ny % ls.by == 0 && (ls.xseg * (ny / ls.by)) % 8 == 0) ls.bpp = ls.xseg * (ny / ls.by);
        else ls.remap = 0;
    }
}

static void launch_geometry_tail(const Batch &B, hipStream_t s)
{
    const dim3 g(B.nchunk_max, B.ncol);
    k_commit<<<g, GCHUNK, 0, s>>>(B.args);
    k_link_count<<<g, GCHUNK, 0, s>>>(B.args);
    k_link_write<<<g, GCHUNK, 0, s>>>(B.args);
}

template <int P> void launch_step(const Batch &B, hipStream_t s, TimingHook *tm)
{
    typedef typename Prec<P>::S S;
    if (tm) tm->begin(0, s);
    k_mu<S><<<B.nblocks[0], 256, 0, s>>>(B.args);
    if (tm) tm->end(0, s);
    if (tm) tm->begin(1, s);
    k_collide<P><<<B.nblocks[1], 256, 0, s>>>(B.args);
    if (tm) tm->end(1, s);
    if (tm) tm->begin(2, s);
    if (B.scalar_zm)
        k_scalar_zm<S><<<B.nblocks[2], 256, 0, s>>>(B.args);
    else
        k_scalar<S><<<B.nblocks[2], 256, 0, s>>>(B.args);
    if (tm) tm->end(2, s);
    if (B.ncol <= 0) return;
    if (tm) tm->begin(3, s);
    k_link_partial<P><<<dim3(B.nlchunk_max, B.ncol), LINK_THREADS, 0, s>>>(B.args);
    k_colloid_update<<<B.ncol, 64, 0, s>>>(B.args);
    if (tm) tm->end(3, s);
    if (tm) tm->begin(4, s);
    k_cover<P><<<dim3(B.nchunk_max, B.ncol), GCHUNK, 0, s>>>(B.args);
    if (tm) tm->end(4, s);
    if (tm) tm->begin(5, s);
    launch_geometry_tail(B, s);
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
    launch_geometry_tail(B, s);
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
    template void launch_step<P>(const Batch &, hipStream_t, TimingHook *);                          \
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
