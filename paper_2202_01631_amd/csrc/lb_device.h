// lb_device.h -- device-side building blocks of the lattice update: D3Q19
// constants, storage precisions, kernel parameter block, particle record and
// FP64 particle geometry.  Included by the kernel and host translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "lb.h"

namespace lbk {

// ------------------------------------------------------------------ D3Q19
// Lattice vectors as constexpr functions: in fully unrolled loops they fold
// to immediates, so the collision carries no table loads.
__host__ __device__ constexpr int cx(int i)
{
    return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1
           : ((i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0);
}
__host__ __device__ constexpr int cy(int i)
{
    return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1
           : ((i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0);
}
__host__ __device__ constexpr int cz(int i)
{
    return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1
           : ((i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0);
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr double wgt(int i)
{
    return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// Owner byte per node: bits 0-6 hold k+1 for a node inside particle k
// (0 = fluid); bit 7 marks a fluid node with a solid node among its 18
// neighbours, the only nodes where bounce-back, wetting ghosts, no-flux
// faces and emission can occur.
constexpr uint8_t OWN_SOLID = 0x7f;
constexpr int GCHUNK = 256;        // bounding-box nodes per geometry block
constexpr int LINK_THREADS = 512;  // threads per particle in the link kernel
constexpr int BND_SCAN = 4;        // geometry chunks a boundary fix-up block scans
constexpr uint8_t OWN_BOUNDARY = 0x80;
constexpr int MAX_COLLOIDS = 127;

// ------------------------------------------------------- storage precision
template <int P> struct Prec;
template <> struct Prec<LB_FP64> { typedef double T; typedef double S; };
template <> struct Prec<LB_FP32> { typedef float T; typedef float S; };
template <> struct Prec<LB_FP16_STORAGE> { typedef __half T; typedef float S; };

__device__ __forceinline__ double ld_pop(const double *p, size_t i, float) { return p[i]; }
__device__ __forceinline__ float ld_pop(const float *p, size_t i, float) { return p[i]; }
__device__ __forceinline__ float ld_pop(const __half *p, size_t i, float inv)
{
    return __half2float(p[i]) * inv;
}
__device__ __forceinline__ void st_pop(double *p, size_t i, double v, float) { p[i] = v; }
__device__ __forceinline__ void st_pop(float *p, size_t i, float v, float) { p[i] = v; }
__device__ __forceinline__ void st_pop(__half *p, size_t i, float v, float sc)
{
    p[i] = __float2half_rn(v * sc);
}

// Access through a uniform base pointer and a 32-bit byte offset: the
// compiler emits global loads and stores with a scalar base and one 32-bit
// vector offset, shared by every field indexed alike (instead of a 64-bit
// vector address per field and neighbour).  Boxes are limited to scalar
// fields below 4 GiB, so byte offsets fit in 32 bits.
template <class T> __device__ __forceinline__ T ldb(const T *base, unsigned off)
{
    return *(const T *)((const char *)base + off);
}
template <class T> __device__ __forceinline__ void stb(T *base, unsigned off, T v)
{
    *(T *)((char *)base + off) = v;
}

// the same for populations (FP16 storage scaled on the way in and out)
__device__ __forceinline__ double ldp(const double *b, unsigned off, float) { return ldb(b, off); }
__device__ __forceinline__ float ldp(const float *b, unsigned off, float) { return ldb(b, off); }
__device__ __forceinline__ float ldp(const __half *b, unsigned off, float inv)
{
    return __half2float(ldb(b, off)) * inv;
}
__device__ __forceinline__ void stp(double *b, unsigned off, double v, float) { stb(b, off, v); }
__device__ __forceinline__ void stp(float *b, unsigned off, float v, float) { stb(b, off, v); }
__device__ __forceinline__ void stp(__half *b, unsigned off, float v, float sc)
{
    stb(b, off, __float2half_rn(v * sc));
}

// --------------------------------------------------------- parameter block
// Shape of a lattice launch: blocks of (bx, by) threads cover an x segment
// of bx nodes in by consecutive rows (rows = (y, z) flattened).
struct LaunchShape {
    int bx, by, remap;         // remap: XCD-aware block renumbering (0 off, 1, 2)
    int xseg, nblocks, bpp;    // derived: segments per row, blocks, blocks per z plane
                               // (marching: blocks per chunk of zc planes)
    int vec;                   // > 1: row-vector form, vec consecutive x nodes per lane
    int zc;                    // > 1 (row-vector psi/c update): planes marched per lane
};

struct KParams {
    int nx, ny, nz, N;         // N = nx*ny*nz < 2^31
    LaunchShape ls;            // shape of the current lattice launch
    double rho0, tau, a, b, kappa, M, C, E, cb0, D, kd;
    double om, pref;           // 1/tau and 1 - 1/(2 tau), formed once on the host
    double sub;                // psi/c sub-step length 1/n (M, D, kd above already carry it):
                               // scales the emission and the stored advection velocity
    double soft_eps, soft_sigma, soft_nu, soft_hc;  // soft-sphere repulsion (eps 0: none)
    double lub_hc;             // normal lubrication cutoff (0: none)
    double fx, fy, fz;
    float scale, inv_scale;    // FP16 storage scale and its inverse (1 otherwise)
    unsigned flags;            // LB_SOLUTE_FORCE, LB_EXPLICIT_COLLOID, LB_CAPILLARY_FORCE
};

// ---------------------------------------------------------- particle record
struct DColloid {
    double pos[3], m[3], vel[3], omega[3];
    double radius, am, ap, mum, mup, H, rho_p, mass, inertia;
    double trF[3], trT[3];     // pending cover/uncover transfer, used next step
    double F[3], T[3];         // force and torque acting in the last step
    double F0[3], T0[3];       // velocity-independent link momentum of the last step
    int fixed, nlinks, nactive, changed;  // changed: owner map moved this step
    double capc;               // active cap m.n <= capc (0: the Janus half)
    double sF[3];              // soft-sphere force of this step (when the box has it)
    double e[3];               // second body axis (orthogonal to m), turns with it
    int pb, ps;                // surface pattern: bands (0: none), sectors
    double pcos[LB_PATTERN_MAX_BANDS - 1];  // band cuts in m.n, increasing
    double palpha[LB_PATTERN_MAX_CELLS], pmu[LB_PATTERN_MAX_CELLS], pH[LB_PATTERN_MAX_CELLS];
    double axial;              // spheroid: semi-axis along m (0 or radius: a sphere)
    double ipar, iperp;        // spheroid: moments of inertia about m and across it
};

// -------------------------------------------------------- particle geometry
// FP64 with no contraction: the inside test and the cap test must resolve
// exact ties the same way everywhere.
__host__ __device__ inline double min_image(double d, int L)
{
#pragma clang fp contract(off)
    const double h = 0.5 * (double)L;
    if (d > h) d -= (double)L;
    else if (d < -h) d += (double)L;
    return d;
}

// displacement from the centre to node (x,y,z) + s*(ex,ey,ez), s in {0, 1/2}
__host__ __device__ inline void displacement(const DColloid &q, int x, int y, int z, int ex, int ey,
                                             int ez, double s, int nx, int ny, int nz, double r[3])
{
#pragma clang fp contract(off)
    r[0] = min_image(((double)x + s * (double)ex) - q.pos[0], nx);
    r[1] = min_image(((double)y + s * (double)ey) - q.pos[1], ny);
    r[2] = min_image(((double)z + s * (double)ez) - q.pos[2], nz);
}

// a spheroid (semi-axis axial along m, radius across it); spheres keep
// their own arithmetic
__host__ __device__ inline bool is_spheroid(const DColloid &q)
{
    return q.axial > 0.0 && q.axial != q.radius;
}

// half-width of the particle's bounding box
__host__ __device__ inline double bound_radius(const DColloid &q)
{
    return q.axial > q.radius ? q.axial : q.radius;
}

// r split into its part s along m and the rest p across it
__host__ __device__ inline double split_axis(const DColloid &q, const double r[3], double p[3])
{
#pragma clang fp contract(off)
    double s = q.m[0] * r[0] + q.m[1] * r[1];
    s = s + q.m[2] * r[2];
    for (int a = 0; a < 3; a++) p[a] = r[a] - s * q.m[a];
    return s;
}

// strictly inside the particle: |r|^2 < R^2, or s^2 b^2 + |p|^2 a^2 < a^2 b^2
__host__ __device__ inline bool inside(const DColloid &q, int x, int y, int z, int nx, int ny, int nz)
{
#pragma clang fp contract(off)
    double r[3];
    displacement(q, x, y, z, 0, 0, 0, 0.0, nx, ny, nz, r);
    if (is_spheroid(q)) {
        double p[3];
        const double s = split_axis(q, r, p);
        double pp = p[0] * p[0] + p[1] * p[1];
        pp = pp + p[2] * p[2];
        const double a2 = q.axial * q.axial, b2 = q.radius * q.radius;
        return s * s * b2 + pp * a2 < a2 * b2;
    }
    double d2 = r[0] * r[0] + r[1] * r[1];
    d2 = d2 + r[2] * r[2];
    return d2 < q.radius * q.radius;
}

// outward unit normal of a spheroid for the surface point seen at r: the
// gradient s m / a^2 + p / b^2 of its implicit function, normalised
__host__ __device__ inline void spheroid_normal(const DColloid &q, const double r[3], double n[3])
{
    double p[3], g[3];
    const double s = split_axis(q, r, p);
    const double a2 = q.axial * q.axial, b2 = q.radius * q.radius;
    for (int a = 0; a < 3; a++) g[a] = (s / a2) * q.m[a] + p[a] / b2;
    const double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    for (int a = 0; a < 3; a++) n[a] = g[a] / gn;
}

// active hemisphere m.n <= 0, n through the link midpoint (Eqs. 5-6)
__host__ __device__ inline bool active_cap(const DColloid &q, const double r[3])
{
#pragma clang fp contract(off)
    double md = q.m[0] * r[0] + q.m[1] * r[1];
    md = md + q.m[2] * r[2];
    if (q.capc == 0.0) return md <= 0.0;
    // a cap of any size: m.r <= capc |r| (correctly rounded square root)
    double rr = r[0] * r[0] + r[1] * r[1];
    rr = rr + r[2] * r[2];
    return md <= q.capc * sqrt(rr);
}

// Surface cell of the point at displacement r from the centre: with a
// pattern, band (cuts compared as m.r <= t |r|, as the cap test) times
// sectors plus the azimuthal sector of r about m, counted from e towards
// m x e in half-open intervals decided by signs and sizes of the two
// projections; without one, 0 on the active cap and 1 elsewhere.  FP64, no
// contraction: link tables are compared bit for bit.
__host__ __device__ inline int azimuth_sector(double a, double b, int S)
{
    if (S <= 1) return 0;
    int q;  // quadrant of the angle atan2(b, a) in [0, 2 pi); a = b = 0 is angle 0
    if (a > 0.0 && b >= 0.0) q = 0;
    else if (a <= 0.0 && b > 0.0) q = 1;
    else if (a < 0.0 && b <= 0.0) q = (a == 0.0 && b == 0.0) ? 0 : 2;
    else q = 3;
    if (S == 2) return q < 2 ? 0 : 1;
    if (S == 4) return q;
    // eighths: the quadrant turned onto the first, whose lower half is y < x
    double x = a, y = b;
    if (q == 1) { x = b; y = -a; }
    else if (q == 2) { x = -a; y = -b; }
    else if (q == 3) { x = -b; y = a; }
    return 2 * q + (y < x ? 0 : 1);
}

__host__ __device__ inline int surface_cell(const DColloid &q, const double r[3])
{
#pragma clang fp contract(off)
    if (q.pb <= 0) return active_cap(q, r) ? 0 : 1;
    double md = q.m[0] * r[0] + q.m[1] * r[1];
    md = md + q.m[2] * r[2];
    double rr = r[0] * r[0] + r[1] * r[1];
    rr = rr + r[2] * r[2];
    const double rn = sqrt(rr);
    int band = 0;
    for (int b = 0; b < q.pb - 1; b++)
        if (!(md <= q.pcos[b] * rn)) band++;
    const double w[3] = {q.m[1] * q.e[2] - q.m[2] * q.e[1], q.m[2] * q.e[0] - q.m[0] * q.e[2],
                         q.m[0] * q.e[1] - q.m[1] * q.e[0]};
    double a = q.e[0] * r[0] + q.e[1] * r[1];
    a = a + q.e[2] * r[2];
    double b = w[0] * r[0] + w[1] * r[1];
    b = b + w[2] * r[2];
    return band * q.ps + azimuth_sector(a, b, q.ps);
}

// production, phoretic mobility and wetting parameter of a surface cell
__host__ __device__ inline double cell_alpha(const DColloid &q, int cell)
{
    return q.pb > 0 ? q.palpha[cell] : (cell == 0 ? q.am : q.ap);
}
__host__ __device__ inline double cell_mu(const DColloid &q, int cell)
{
    return q.pb > 0 ? q.pmu[cell] : (cell == 0 ? q.mum : q.mup);
}
__host__ __device__ inline double cell_H(const DColloid &q, int cell)
{
    return q.pb > 0 ? q.pH[cell] : q.H;
}
// active link: on the active cap, or in a pattern cell that produces
__host__ __device__ inline bool cell_active(const DColloid &q, int cell)
{
    return q.pb > 0 ? q.palpha[cell] != 0.0 : cell == 0;
}

// Particle bounding box along one axis, with the node coordinates visited in
// ascending wrapped order: element t of the sorted list is
// wrap(lo + (t + shift) % count).
struct AxisBox {
    int lo, count, shift, L;
    __host__ __device__ int at(int t) const
    {
        int v = lo + (t + shift) % count;
        v %= L;
        return v < 0 ? v + L : v;
    }
};

__host__ __device__ inline AxisBox axis_box(double c, double radius, int L)
{
    AxisBox b;
    int lo = (int)floor(c - radius) - 3;
    int hi = (int)floor(c + radius) + 3;
    int count = hi - lo + 1;
    if (count >= L) { lo = 0; count = L; }
    b.lo = lo;
    b.count = count;
    b.L = L;
    int l = lo % L;
    if (l < 0) l += L;
    // index in range order of the first element in ascending wrapped order
    int first = 0;
    if (l + count > L) first = L - l;
    b.shift = first % count;
    return b;
}

// Lattice launch geometry.  With bx = nx (rows up to 256 nodes) a block owns
// whole rows, so every shifted store of the push streaming completes the
// cache lines of its row inside one block.  With remap on, blocks are
// renumbered XCD-aware: the hardware sends workgroup i to XCD i % 8, and each
// XCD receives a contiguous range of blocks, so the halo rows a block reads
// were mostly loaded by blocks of the same XCD (same L2).
__device__ __forceinline__ int block_order(const LaunchShape &ls, int i)
{
    int b = i;
    if (ls.remap == 1) {
        // contiguous block ranges per XCD
        const int q = ls.nblocks >> 3, r = ls.nblocks & 7;
        const int xcd = i & 7, slot = i >> 3;
        b = (xcd < r) ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
    } else if (ls.remap == 2) {
        // one eighth of every z plane per XCD, planes in order: the eight XCDs
        // sweep a plane together (no address-range camping) and the z +- 1
        // rows of a block belong to its own XCD
        const int bpp = ls.bpp, G = bpp >> 3;
        const int xcd = i & 7, slot = i >> 3;
        b = (slot / G) * bpp + xcd * G + (slot % G);
    }
    return b;
}

__device__ __forceinline__ bool lattice_node(const KParams &p, int i, int &x, int &y, int &z)
{
    const int b = block_order(p.ls, i);
    // 256 threads per block, read as (bx, by) for this box: boxes of a batch
    // may use different shapes within one launch
    const int tx = (int)threadIdx.x % p.ls.bx, ty = (int)threadIdx.x / p.ls.bx;
    if (ty >= p.ls.by) return false;
    const int seg = b % p.ls.xseg, grp = b / p.ls.xseg;
    x = seg * p.ls.bx + tx;
    const int row = grp * p.ls.by + ty;
    if (x >= p.nx || row >= p.ny * p.nz) return false;
    z = row / p.ny;
    y = row - z * p.ny;
    return true;
}

// Row-vector launch (vec = V > 1): lane li of a group of bx lanes covers the
// V consecutive nodes x0 .. x0 + V - 1 of one row segment (xseg segments per
// row); a wavefront holds by = 64 / bx groups, a block four wavefronts.
// Returns false for lanes without nodes, always whole groups, so exchanges
// between the lanes of a live group stay inside live lanes.
template <int V>
__device__ __forceinline__ bool vec_node(const KParams &p, int i, int &x0, int &y, int &z, int &li,
                                         int &gb)
{
    const int b = block_order(p.ls, i);
    const int w = (int)threadIdx.x >> 6, l = (int)threadIdx.x & 63;
    const int Ls = p.ls.bx, g = l / Ls;
    if (g >= p.ls.by) return false;
    li = l - g * Ls;
    gb = g * Ls;
    const int sg = (b * 4 + w) * p.ls.by + g;
    const int row = sg / p.ls.xseg, seg = sg - row * p.ls.xseg;
    if (row >= p.ny * p.nz) return false;
    z = row / p.ny;
    y = row - z * p.ny;
    x0 = (seg * Ls + li) * V;
    return true;
}

// V consecutive scalars moved as one 8- or 16-byte access
template <class S, int V> struct alignas(sizeof(S) * V) SVec { S v[V]; };
template <int V> struct OwnWord;
template <> struct OwnWord<2> { typedef uint16_t T; };
template <> struct OwnWord<4> { typedef uint32_t T; };
__device__ __forceinline__ uint8_t byte_of(unsigned w, int k) { return (uint8_t)(w >> (8 * k)); }

}  // namespace lbk
