// lb_api.hip -- host side of the C ABI in include/lb.h: parameter checks,
// device memory layout, per-step launch sequence, readback.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lb_kernels.h"

using namespace lbk;

namespace {

thread_local std::string g_err;  // message when no context is at hand

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t storage_bytes(int prec) { return prec == LB_FP64 ? 8 : (prec == LB_FP32 ? 4 : 2); }
size_t compute_bytes(int prec) { return prec == LB_FP64 ? 8 : 4; }

// Arena layout (each piece 256-byte aligned): f[2] (19 N storage), psi[2],
// c[2], mu (N compute), in FP64 chi (N), u (3N compute), owner (N bytes),
// and with psi/c sub-steps one more psi and c pair (N compute each).
struct Layout {
    size_t f[2], psi[2], cc[2], mu, chi, u, own, psis, ccs, pst, muc, total;
};

int substeps_of(const lb_params &p) { return p.ch_substeps > 1 ? p.ch_substeps : 1; }

Layout layout_of(const lb_params &p)
{
    const size_t N = (size_t)p.nx * p.ny * p.nz;
    const size_t sb = storage_bytes(p.precision), cb = compute_bytes(p.precision);
    Layout L;
    size_t o = 0;
    for (int b = 0; b < 2; b++) { L.f[b] = o; o = align256(o + 19 * N * sb); }
    for (int b = 0; b < 2; b++) { L.psi[b] = o; o = align256(o + N * cb); }
    for (int b = 0; b < 2; b++) { L.cc[b] = o; o = align256(o + N * cb); }
    L.mu = o; o = align256(o + N * cb);
    L.chi = 0;
    if (p.precision == LB_FP64) { L.chi = o; o = align256(o + N * cb); }
    L.u = o; o = align256(o + 3 * N * cb);
    L.own = o; o = align256(o + N);
    L.psis = L.ccs = 0;
    if (substeps_of(p) > 1) {
        L.psis = o; o = align256(o + N * cb);
        L.ccs = o; o = align256(o + N * cb);
    }
    L.pst = L.muc = 0;
    if (p.flags & LB_STRESS_FORM) {
        // the stress (6 planes) and mu_c of the divergence-form solvent force
        L.pst = o; o = align256(o + 6 * N * cb);
        L.muc = o; o = align256(o + N * cb);
    }
    L.total = o;
    return L;
}

}  // namespace

struct lb_ctx {
    lb_params p;
    KParams kp;
    long long N;
    hipStream_t stream;
    bool own_arena;
    char *arena;
    Layout L;
    int cur;
    int stage;  // 0 created, 1 fields, 2 colloids
    int64_t step;
    // particles
    int ncol, maxcol, lcap;
    DColloid *dcol;
    int *lnode;
    uint8_t *ldc;
    double *cpart;
    uint32_t *lmask;
    int *ccount;
    int bbmax, nchunk_max;
    double *lpart;
    int nlchunk_max;
    int *derr;
    double *part;   // reduction partials
    double *dsum;   // 7 totals
    int nred;
    TimingHook *timing;
    LaunchShape shapes[3];  // mu, collide, scalar
    // single-box batches for the two buffer parities, their device tables,
    // and the replay graphs of a (cur, 1-cur) step pair
    Batch self[2];
    char *selfdev;
    bool dirty;
    hipGraphExec_t graph[2];
    SideStream side;    // particle work beside the bulk kernels
    bool has_side;
    // single phase: a = b = kappa = E = c_b0 = 0 and psi = 0 at init, so mu
    // is 0 and chi is c at every step (set by lb_init_fields)
    bool nopsi;
    bool special;       // some particle carries a surface pattern or is not a sphere
    std::string err;
};

static lb_status fail(lb_ctx *c, lb_status s, const std::string &m)
{
    if (c) c->err = m; else g_err = m;
    return s;
}

static lb_status hip_fail(lb_ctx *c, hipError_t e, const char *what)
{
    // copies queued before the failing call may still target host buffers
    // of the caller's frame: let the stream finish them before returning
    // (not while it captures: nothing it holds has run)
    if (c) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(c->stream, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone)
            (void)hipStreamSynchronize(c->stream);
    }
    return fail(c, LB_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(c, call)                                                                           \
    do {                                                                                           \
        hipError_t _e = (call);                                                                    \
        if (_e != hipSuccess) return hip_fail((c), _e, #call);                                     \
    } while (0)

static void *ptr(lb_ctx *c, size_t off) { return c->arena + off; }

static StepBuffers buffers(lb_ctx *c, int cu)
{
    StepBuffers b;
    const int nx = 1 - cu;
    b.fin = ptr(c, c->L.f[cu]);
    b.fout = ptr(c, c->L.f[nx]);
    b.psi = ptr(c, c->L.psi[cu]);
    b.cc = ptr(c, c->L.cc[cu]);
    b.psin = ptr(c, c->L.psi[nx]);
    b.ccn = ptr(c, c->L.cc[nx]);
    b.mu = ptr(c, c->L.mu);
    b.chi = c->p.precision == LB_FP64 ? ptr(c, c->L.chi) : nullptr;
    b.u = ptr(c, c->L.u);
    b.pst = (c->p.flags & LB_STRESS_FORM) ? ptr(c, c->L.pst) : nullptr;
    b.muc = (c->p.flags & LB_STRESS_FORM) ? ptr(c, c->L.muc) : nullptr;
    b.own = (uint8_t *)ptr(c, c->L.own);
    b.col = c->dcol;
    b.lnode = c->lnode;
    b.ldc = c->ldc;
    b.lcap = c->lcap;
    b.err = c->derr;
    b.cpart = c->cpart;
    b.lmask = c->lmask;
    b.ccount = c->ccount;
    b.bbmax = c->bbmax;
    b.nchunk_max = c->nchunk_max;
    b.lpart = c->lpart;
    b.nlchunk_max = c->nlchunk_max;
    return b;
}

static BoxDesc box_desc(lb_ctx *c, int parity)
{
    BoxDesc d;
    d.p = c->kp;
    for (int w = 0; w < 3; w++) d.ls[w] = c->shapes[w];
    d.b = buffers(c, parity);
    return d;
}

// psi/c sub-steps ping-pong between the next-state pair and the scratch
// pair, the last one landing in the next-state pair: sub-step s of n writes
// the next-state pair when n-1-s is even, else the scratch pair.  Three
// descriptor tables besides the step's own cover them: sub-step 0 (from the
// state at t), and the two directions between the pairs.
static void substep_tables(lb_ctx *c, const BoxDesc &d, BoxDesc t[3], bool chi_is_c)
{
    void *ps = ptr(c, c->L.psis), *cs = ptr(c, c->L.ccs);
    const int n = substeps_of(c->p);
    for (int k = 0; k < 3; k++) t[k] = d;
    if (n % 2 == 0) { t[0].b.psin = ps; t[0].b.ccn = cs; }
    t[1].b.psi = d.b.psin; t[1].b.cc = d.b.ccn; t[1].b.psin = ps; t[1].b.ccn = cs;
    t[2].b.psi = ps; t[2].b.cc = cs;
    if (chi_is_c)
        for (int k = 0; k < 3; k++)
            if (t[k].b.chi) t[k].b.chi = const_cast<void *>(t[k].b.cc);
}

// Host side of a batch: descriptors and block/particle start tables, laid
// out in one device buffer: [BoxDesc x n][bstart 3(n+1)][cstart n+1], then
// with psi/c sub-steps three more [BoxDesc x n] tables.
static size_t batch_bytes(int n, int nsub)
{
    const size_t d = align256(sizeof(BoxDesc) * n);
    return align256(d + sizeof(int) * (4 * (size_t)n + 4)) + (nsub > 1 ? 3 * d : 0);
}

static void batch_fill(lb_ctx *const *ctxs, int n, const int *parity, std::vector<char> &host,
                       char *dev, Batch &B)
{
    const int nsub = substeps_of(ctxs[0]->p);
    host.assign(batch_bytes(n, nsub), 0);
    BoxDesc *d = (BoxDesc *)host.data();
    int *bst = (int *)(host.data() + align256(sizeof(BoxDesc) * n));
    int *cst = bst + 3 * (n + 1);
    for (int w = 0; w < 3; w++) bst[w * (n + 1)] = 0;
    cst[0] = 0;
    B.nchunk_max = 0;
    B.nlchunk_max = 0;
    for (int j = 0; j < n; j++) {
        d[j] = box_desc(ctxs[j], parity[j]);
        for (int w = 0; w < 3; w++) bst[w * (n + 1) + j + 1] = bst[w * (n + 1) + j] + d[j].ls[w].nblocks;
        cst[j + 1] = cst[j] + ctxs[j]->ncol;
        if (ctxs[j]->ncol > 0) {
            B.nchunk_max = std::max(B.nchunk_max, ctxs[j]->nchunk_max);
            B.nlchunk_max = std::max(B.nlchunk_max, ctxs[j]->nlchunk_max);
        }
    }
    // one kernel form per launch: where the boxes disagree on the row-vector
    // (or z-marching) form of a lattice kernel, all of them take the
    // one-node form of that kernel
    // (the solute-force term lives in the one-node collide-stream only)
    const int ssize = ctxs[0]->p.precision == LB_FP64 ? 8 : 4;
    // single-phase batch (every box): no mu launches, single-phase kernels
    B.nopsi = n > 0;
    for (int j = 0; j < n; j++) B.nopsi = B.nopsi && ctxs[j]->nopsi;
    B.special = 0;
    for (int j = 0; j < n; j++) B.special |= (ctxs[j]->special && ctxs[j]->ncol > 0) ? 1 : 0;
    if (B.nopsi) {
        // single-phase kernels exist in the one-node collide-stream and the
        // one-node and row-vector psi/c updates: other forms drop to those
        for (int j = 0; j < n; j++) {
            // a stored chi (FP64) is c itself: the mu pass that writes it does not run
            if (d[j].b.chi) d[j].b.chi = const_cast<void *>(d[j].b.cc);
            const int ss = ctxs[j]->p.precision == LB_FP64 ? 8 : 4;
            if (d[j].ls[1].vec > 1) {
                d[j].ls[1].vec = 0;
                d[j].ls[1].bx = d[j].ls[1].by = 0;
                finish_shape(d[j].ls[1], ctxs[j]->p.nx, ctxs[j]->p.ny, ctxs[j]->p.nz, ss, true);
            }
            if (d[j].ls[2].zc > 1) {
                d[j].ls[2].zc = 0;
                finish_shape(d[j].ls[2], ctxs[j]->p.nx, ctxs[j]->p.ny, ctxs[j]->p.nz, ss);
            }
            for (int w = 1; w < 3; w++) bst[w * (n + 1) + j + 1] = bst[w * (n + 1) + j] + d[j].ls[w].nblocks;
        }
    }
    B.solute_force = 0;
    B.stress = 0;
    B.soft = 0;
    for (int j = 0; j < n; j++) {
        if (ctxs[j]->p.flags & LB_SOLUTE_FORCE) B.solute_force = 1;
        if (ctxs[j]->p.flags & LB_STRESS_FORM) {
            B.stress = 1;
            // boundary nodes in the fix-up launches, which write the stress there
            if (ctxs[j]->ncol > 0) B.special = 1;
        }
        if (ctxs[j]->p.soft_eps > 0.0 || ctxs[j]->p.lub_hc > 0.0) B.soft = 1;
    }
    for (int w = 0; w < 3; w++) {
        bool same = true;
        for (int j = 1; j < n; j++)
            same = same && d[j].ls[w].vec == d[0].ls[w].vec &&
                   (d[j].ls[w].zc > 1) == (d[0].ls[w].zc > 1);
        // the solute force and the divergence-form force live in the one-node
        // collide-stream; the stress is written by the one-node mu update
        if (w == 1 && (B.solute_force || B.stress)) same = n > 0 && d[0].ls[1].vec <= 1 && same;
        if (w == 0 && B.stress) same = n > 0 && d[0].ls[0].vec <= 1 && same;
        if (!same) {
            for (int j = 0; j < n; j++) {
                if (d[j].ls[w].vec > 1) {
                    d[j].ls[w].vec = 0;
                    d[j].ls[w].zc = 0;
                    finish_shape(d[j].ls[w], ctxs[j]->p.nx, ctxs[j]->p.ny, ctxs[j]->p.nz, ssize,
                                 w == 1);
                }
                bst[w * (n + 1) + j + 1] = bst[w * (n + 1) + j] + d[j].ls[w].nblocks;
            }
        }
        B.vec[w] = n > 0 ? d[0].ls[w].vec : 0;
    }
    B.zmarch = n > 0 && d[0].ls[2].zc > 1;
    for (int w = 0; w < 3; w++) B.nblocks[w] = bst[w * (n + 1) + n];
    B.ncol = cst[n];
    B.nodes = 0;
    for (int j = 0; j < n; j++) B.nodes += ctxs[j]->N;
    B.precision = ctxs[0]->p.precision;
    B.args.d = (const BoxDesc *)dev;
    B.args.bstart = (const int *)(dev + align256(sizeof(BoxDesc) * n));
    B.args.cstart = B.args.bstart + 3 * (n + 1);
    B.args.nbox = n;
    B.args.nsec = (B.nchunk_max + BND_SCAN - 1) / BND_SCAN;
    B.args.nfix = B.ncol > 0 ? B.args.nsec * B.ncol : 0;
    B.args.boff = 0;
    B.nsub = nsub;
    for (int k = 0; k < 3; k++) B.dsub[k] = nullptr;
    if (nsub > 1) {
        const size_t dbytes = align256(sizeof(BoxDesc) * n);
        const size_t base = align256(dbytes + sizeof(int) * (4 * (size_t)n + 4));
        for (int j = 0; j < n; j++) {
            BoxDesc t[3];
            substep_tables(ctxs[j], d[j], t, B.nopsi != 0);
            for (int k = 0; k < 3; k++) ((BoxDesc *)(host.data() + base + k * dbytes))[j] = t[k];
        }
        for (int k = 0; k < 3; k++) B.dsub[k] = (const BoxDesc *)(dev + base + k * dbytes);
    }
}

// the captured step pairs; the stream first finishes a replay still in flight
static void drop_graphs(lb_ctx *c)
{
    if (!c->graph[0] && !c->graph[1]) return;
    (void)hipStreamSynchronize(c->stream);
    for (int g = 0; g < 2; g++)
        if (c->graph[g]) { hipGraphExecDestroy(c->graph[g]); c->graph[g] = nullptr; }
}

// rebuild the two single-box batches after buffers or shapes changed
static lb_status refresh_self(lb_ctx *c)
{
    if (!c->dirty) return LB_OK;
    drop_graphs(c);
    const size_t bb = align256(batch_bytes(1, substeps_of(c->p)));
    if (!c->selfdev) HIP_TRY(c, hipMalloc((void **)&c->selfdev, 2 * bb));
    std::vector<char> host[2];
    for (int par = 0; par < 2; par++) {
        char *dev = c->selfdev + par * bb;
        lb_ctx *one[1] = {c};
        batch_fill(one, 1, &par, host[par], dev, c->self[par]);
        HIP_TRY(c, hipMemcpyAsync(dev, host[par].data(), host[par].size(), hipMemcpyHostToDevice, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->dirty = false;
    return LB_OK;
}

// ---------------------------------------------------------------- timing
hipEvent_t TimingHook::take()
{
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
void TimingHook::begin(int i, hipStream_t s)
{
    hipEvent_t e = take();
    if (e) { hipEventRecord(e, s); open[i].push_back(e); }
}
void TimingHook::end(int i, hipStream_t s)
{
    if (open[i].empty()) return;
    hipEvent_t b = open[i].back();
    open[i].pop_back();
    hipEvent_t e = take();
    if (!e) { pool.push_back(b); return; }
    hipEventRecord(e, s);
    done[i].push_back(std::make_pair(b, e));
}
void TimingHook::flush()
{
    for (int i = 0; i < 6; i++) {
        for (auto &pr : done[i]) {
            float t = 0.f;
            hipEventSynchronize(pr.second);
            if (hipEventElapsedTime(&t, pr.first, pr.second) == hipSuccess) {
                ms[i] += t;
                calls[i]++;
            }
            pool.push_back(pr.first);
            pool.push_back(pr.second);
        }
        done[i].clear();
    }
}
void TimingHook::reset()
{
    flush();
    for (int i = 0; i < 6; i++) { ms[i] = 0.0; calls[i] = 0; }
}
TimingHook::~TimingHook()
{
    for (int i = 0; i < 6; i++) {
        for (auto &pr : done[i]) { hipEventDestroy(pr.first); hipEventDestroy(pr.second); }
        for (auto e : open[i]) hipEventDestroy(e);
    }
    for (auto e : pool) hipEventDestroy(e);
}

// ------------------------------------------------------------- dispatch
// The side stream of a context, created on first use (default priority,
// non-blocking); null if it cannot be created, then steps run in order on
// one stream.
static const SideStream *side_of(lb_ctx *c)
{
    if (!c->has_side) {
        SideStream v;
        if (hipStreamCreateWithFlags(&v.s, hipStreamNonBlocking) != hipSuccess) return nullptr;
        int i = 0;
        for (; i < SIDE_EVENTS; i++)
            if (hipEventCreateWithFlags(&v.ev[i], hipEventDisableTiming) != hipSuccess) break;
        if (i < SIDE_EVENTS) {
            while (i > 0) hipEventDestroy(v.ev[--i]);
            hipStreamDestroy(v.s);
            return nullptr;
        }
        c->side = v;
        c->has_side = true;
    }
    return &c->side;
}

static void launch_one_step(const Batch &B, hipStream_t s, const SideStream *side, TimingHook *tm,
                            bool defer_links = false)
{
    switch (B.precision) {
    case LB_FP64: launch_step<LB_FP64>(B, s, side, tm, defer_links); break;
    case LB_FP32: launch_step<LB_FP32>(B, s, side, tm, defer_links); break;
    default: launch_step<LB_FP16_STORAGE>(B, s, side, tm, defer_links); break;
    }
}

// capture the step pair (B0 then B1) on stream s into an executable graph;
// the first step's link table write overlaps the second step's mu update
static hipError_t capture_pair(const Batch &B0, const Batch &B1, hipStream_t s,
                               const SideStream *side, hipGraphExec_t *out)
{
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return e;
    launch_one_step(B0, s, side, nullptr, true);
    launch_one_step(B1, s, side, nullptr, false);
    e = hipStreamEndCapture(s, &g);
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    return e;
}

// ------------------------------------------------------------- checks
static lb_status check_size(const lb_params *p, std::string &why)
{
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) { why = "box sizes must be >= 1"; return LB_E_INVALID; }
    if ((double)p->nx * p->ny * p->nz >= 2147483647.0) { why = "box too large (N >= 2^31)"; return LB_E_INVALID; }
    if (p->nz > 65535) { why = "nz > 65535"; return LB_E_INVALID; }
    if (p->precision < LB_FP64 || p->precision > LB_FP16_STORAGE) { why = "bad precision"; return LB_E_INVALID; }
    // kernels address scalar fields with 32-bit byte offsets
    if ((double)p->nx * p->ny * p->nz * (p->precision == LB_FP64 ? 8.0 : 4.0) >= 4294967296.0) {
        why = "box too large (one scalar field must stay below 4 GiB)";
        return LB_E_INVALID;
    }
    return LB_OK;
}

static lb_status check_params(const lb_params *p, std::string &why)
{
    if (!p) { why = "null parameters"; return LB_E_INVALID; }
    const lb_status sz = check_size(p, why);
    if (sz != LB_OK) return sz;
    if (!(p->tau > 0.5)) { why = "tau must exceed 1/2"; return LB_E_INVALID; }
    if (!(p->rho0 > 0.0)) { why = "rho0 must be positive"; return LB_E_INVALID; }
    if (p->kappa < 0 || p->M_psi < 0 || p->C < 0 || p->D_c < 0 || p->k_d < 0) {
        why = "kappa, M_psi, C, D_c, k_d must be >= 0";
        return LB_E_INVALID;
    }
    if ((p->flags & LB_STRESS_FORM) && !(p->flags & LB_CAPILLARY_FORCE)) {
        why = "LB_STRESS_FORM needs LB_CAPILLARY_FORCE";
        return LB_E_INVALID;
    }
    if (p->flags & ~(LB_SOLUTE_FORCE | LB_EXPLICIT_COLLOID | LB_CAPILLARY_FORCE | LB_STRESS_FORM)) {
        why = "unknown option flags";
        return LB_E_INVALID;
    }
    if (p->ch_substeps < 0 || p->ch_substeps > 64) { why = "ch_substeps in [0, 64]"; return LB_E_INVALID; }
    if (!(p->soft_eps >= 0.0) ||
        (p->soft_eps > 0.0 && !(p->soft_sigma > 0.0 && p->soft_nu > 0.0 && p->soft_hc > 0.0))) {
        why = "soft_eps must be >= 0, and with soft_eps > 0 soft_sigma, soft_nu, soft_hc > 0";
        return LB_E_INVALID;
    }
    if (!(p->lub_hc >= 0.0)) { why = "lub_hc must be >= 0"; return LB_E_INVALID; }
    // the psi/c bounds hold per sub-step, of length 1/n
    const double dt = 1.0 / substeps_of(*p);
    if (dt * p->M_psi * (12.0 * fabs(p->a) + 36.0 * fabs(p->b) + 144.0 * p->kappa) >= 2.0) {
        why = "M_psi above the explicit-Euler stability bound M (12|a| + 36|b| + 144 kappa) / n < 2 "
              "(n = ch_substeps)";
        return LB_E_INVALID;
    }
    if (dt * (12.0 * p->D_c + p->k_d) >= 2.0) {
        why = "(12 D_c + k_d) / n must be < 2 (n = ch_substeps)";
        return LB_E_INVALID;
    }
    if (p->max_colloids < 0 || p->max_colloids > MAX_COLLOIDS) { why = "max_colloids in [0, 127]"; return LB_E_INVALID; }
    if (p->precision == LB_FP16_STORAGE && p->f16_scale != 0.0) {
        int e;
        double m = frexp(p->f16_scale, &e);
        if (!(p->f16_scale > 0.0) || m != 0.5) { why = "f16_scale must be a power of two"; return LB_E_INVALID; }
    }
    return LB_OK;
}

// Launch shapes of the lattice kernels: whole rows (up to 256 nodes) per block
// for collide-stream in natural block order; the row-vector forms for the mu
// and psi/c updates, the psi/c update with plane-wise XCD renumbering.
// LB_LATTICE_SHAPES="bx,by,remap[,vec[,zc]];..." (mu; collide; psi/c, 0 =
// default; zc for the psi/c update only) overrides them for tuning sweeps.
static void set_shapes(lb_ctx *c)
{
    LaunchShape d = {0, 0, 0, 0, 0, 0, 0, 0};
    LaunchShape v[3] = {d, d, d};
    v[0].vec = 4;
    v[2].vec = 4;
    v[2].remap = 2;
    if (const char *e = getenv("LB_LATTICE_SHAPES")) {
        for (int k = 0; k < 3 && *e; k++) {
            int bx = 0, by = 0, rm = 1, used = 0, vec = 0, zc = 0, used2 = 0;
            if (sscanf(e, "%d,%d,%d%n", &bx, &by, &rm, &used) == 3) {
                v[k].bx = bx;
                v[k].by = by;
                v[k].remap = rm >= 0 && rm <= 2 ? rm : 0;
                v[k].vec = 0;
                v[k].zc = 0;
                e += used;
                if (sscanf(e, ",%d%n", &vec, &used2) == 1) {
                    if (vec == 2 || vec == 4) v[k].vec = vec;
                    e += used2;
                    if (sscanf(e, ",%d%n", &zc, &used2) == 1) {
                        if (k == 2 && zc > 1) v[k].zc = zc;
                        e += used2;
                    }
                }
                if (*e == ';') e++;
            } else {
                break;
            }
        }
    }
    for (int k = 0; k < 3; k++) {
        finish_shape(v[k], c->p.nx, c->p.ny, c->p.nz, c->p.precision == LB_FP64 ? 8 : 4, k == 1);
        c->shapes[k] = v[k];
    }
    c->dirty = true;
}

template <int P> static void reduce_t(lb_ctx *c)
{
    launch_reduce<P>(c->kp, ptr(c, c->L.f[c->cur]), ptr(c, c->L.psi[c->cur]), ptr(c, c->L.cc[c->cur]),
                     (const uint8_t *)ptr(c, c->L.own), c->part, c->nred, c->dsum, c->stream);
}

template <int P> static void fields_t(lb_ctx *c, double *out, double *fout)
{
    launch_fields<P>(c->kp, ptr(c, c->L.f[c->cur]), ptr(c, c->L.psi[c->cur]), ptr(c, c->L.cc[c->cur]),
                     (const uint8_t *)ptr(c, c->L.own), out, fout, c->stream);
}

static lb_status run_fields(lb_ctx *c, double *out, double *fout)
{
    switch (c->p.precision) {
    case LB_FP64: fields_t<LB_FP64>(c, out, fout); break;
    case LB_FP32: fields_t<LB_FP32>(c, out, fout); break;
    default: fields_t<LB_FP16_STORAGE>(c, out, fout); break;
    }
    HIP_TRY(c, hipGetLastError());
    return LB_OK;
}

// raw state: header, f (both buffers not needed: current only), psi, c,
// owner, particle table, link tables
struct StateHeader {
    uint64_t magic;
    int32_t nx, ny, nz, precision, ncol, lcap;
    int64_t step;
};
// (the last byte counts layouts of the particle record: "3" has the second
// body axis, the surface pattern and the spheroid's semi-axis)
static const uint64_t STATE_MAGIC = 0x4c42504852534133ull;

static size_t state_size(lb_ctx *c)
{
    const size_t N = (size_t)c->N;
    return sizeof(StateHeader) + 19 * N * storage_bytes(c->p.precision) +
           2 * N * compute_bytes(c->p.precision) + N + sizeof(DColloid) * c->ncol +
           (sizeof(int) + 1) * (size_t)c->lcap * c->ncol;
}

// particle tables sized for particles up to radius rmax
static lb_status alloc_colloid_tables(lb_ctx *c, double rmax, int lcap)
{
    const int side = 2 * (int)ceil(rmax) + 8;
    const int Ls[3] = {c->p.nx, c->p.ny, c->p.nz};
    long long bb = 1;
    for (int a = 0; a < 3; a++) bb *= std::min(side, Ls[a]);
    c->bbmax = (int)bb;
    c->nchunk_max = (c->bbmax + GCHUNK - 1) / GCHUNK;
    c->lcap = lcap;
    const size_t m = (size_t)c->maxcol;
    HIP_TRY(c, hipMalloc((void **)&c->dcol, sizeof(DColloid) * m));
    HIP_TRY(c, hipMalloc((void **)&c->lnode, sizeof(int) * (size_t)c->lcap * m));
    HIP_TRY(c, hipMalloc((void **)&c->ldc, (size_t)c->lcap * m));
    HIP_TRY(c, hipMalloc((void **)&c->cpart, sizeof(double) * 8 * (size_t)c->nchunk_max * m));
    HIP_TRY(c, hipMalloc((void **)&c->lmask, sizeof(uint32_t) * (size_t)c->bbmax * m));
    HIP_TRY(c, hipMalloc((void **)&c->ccount, sizeof(int) * (size_t)c->nchunk_max * m));
    c->nlchunk_max = (c->lcap + LINK_THREADS - 1) / LINK_THREADS;
    HIP_TRY(c, hipMalloc((void **)&c->lpart, sizeof(double) * 28 * (size_t)c->nlchunk_max * m));
    HIP_TRY(c, hipMemsetAsync(c->cpart, 0, sizeof(double) * 8 * (size_t)c->nchunk_max * m, c->stream));
    return LB_OK;
}

// ------------------------------------------------------------ batches
// checks shared by the batched entry points; work still queued on the other
// boxes' own streams (initialisation copies, earlier steps) is waited for,
// so that it finishes before the batch touches their state
static lb_status batch_check(lb_ctx *const *ctxs, int n, int64_t nsteps)
{
    if (!ctxs || n < 1) return fail(nullptr, LB_E_INVALID, "empty batch");
    if (nsteps < 0) return fail(nullptr, LB_E_INVALID, "negative step count");
    for (int j = 0; j < n; j++) {
        if (!ctxs[j]) return fail(nullptr, LB_E_INVALID, "null context in batch");
        if (ctxs[j]->stage < 1) return fail(ctxs[j], LB_E_STATE, "lb_init_fields must come first");
        if (ctxs[j]->p.precision != ctxs[0]->p.precision)
            return fail(ctxs[j], LB_E_INVALID, "boxes of a batch must share the precision");
        if (substeps_of(ctxs[j]->p) != substeps_of(ctxs[0]->p))
            return fail(ctxs[j], LB_E_INVALID, "boxes of a batch must share ch_substeps");
        for (int i = 0; i < j; i++)
            if (ctxs[i] == ctxs[j]) return fail(ctxs[j], LB_E_INVALID, "context twice in a batch");
    }
    hipStream_t s = ctxs[0]->stream;
    for (int j = 1; j < n; j++) {
        bool seen = ctxs[j]->stream == s;
        for (int i = 1; i < j && !seen; i++) seen = ctxs[i]->stream == ctxs[j]->stream;
        if (!seen) HIP_TRY(ctxs[j], hipStreamSynchronize(ctxs[j]->stream));
    }
    return LB_OK;
}

// nsteps steps of every box, descriptor tables of the two buffer parities at
// dev and dev + bb (device memory of at least 2 bb bytes), on the stream of
// ctxs[0]; step pairs replayed from a captured graph when graphs is set and
// the stream is not the legacy default one, else launched one by one.
// Synchronises the stream before returning.
static lb_status batch_run(lb_ctx *const *ctxs, int n, int64_t nsteps, char *dev, size_t bb,
                           bool graphs, const SideStream *side)
{
    lb_ctx *c0 = ctxs[0];
    hipStream_t s = c0->stream;
    std::vector<int> par0(n), par1(n);
    for (int j = 0; j < n; j++) { par0[j] = ctxs[j]->cur; par1[j] = 1 - ctxs[j]->cur; }
    Batch B0, B1;
    std::vector<char> h0, h1;
    batch_fill(ctxs, n, par0.data(), h0, dev, B0);
    batch_fill(ctxs, n, par1.data(), h1, dev + bb, B1);
    hipError_t e = hipMemcpyAsync(dev, h0.data(), h0.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dev + bb, h1.data(), h1.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    int64_t k = 0;
    hipGraphExec_t ge = nullptr;
    if (graphs && e == hipSuccess && s && nsteps >= 2) {
        e = capture_pair(B0, B1, s, side, &ge);
        for (; e == hipSuccess && k + 2 <= nsteps; k += 2) e = hipGraphLaunch(ge, s);
    }
    for (; e == hipSuccess && k < nsteps; k++) {
        launch_one_step((k & 1) ? B1 : B0, s, side, nullptr);
        e = hipGetLastError();
    }
    hipError_t e2 = hipStreamSynchronize(s);
    if (ge) hipGraphExecDestroy(ge);
    if (e != hipSuccess) return hip_fail(c0, e, "batched step");
    if (e2 != hipSuccess) return hip_fail(c0, e2, "batched step");
    for (int j = 0; j < n; j++) {
        if (nsteps & 1) ctxs[j]->cur ^= 1;
        ctxs[j]->step += nsteps;
    }
    return LB_OK;
}

// ---------------------------------------------- allocation-free batches
// lb_batch_step_noalloc keeps the descriptor tables of a batch in this fixed
// device array instead of a buffer allocated per call.  Each GPU holds its
// own copy for the life of the process; host code reaches it only through
// the address hipGetSymbolAddress returns for the current device (the
// array's name is not a device address on the host).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)4 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];
static void *g_scratch_dev[NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mu;

static lb_status scratch_address(lb_ctx *c, char **out)
{
    int dev = -1;
    HIP_TRY(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(c, LB_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        HIP_TRY(c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(c, LB_E_DEVICE, "no device address for the fixed batch array");
        g_scratch_dev[dev] = p;
    }
    *out = (char *)g_scratch_dev[dev];
    return LB_OK;
}

extern "C" {

lb_status lb_footprint_bytes(const lb_params *p, size_t *bytes)
{
    if (!p || !bytes) return fail(nullptr, LB_E_INVALID, "null argument");
    std::string why;
    if (check_size(p, why) != LB_OK) return fail(nullptr, LB_E_INVALID, why.c_str());
    *bytes = layout_of(*p).total;
    return LB_OK;
}

lb_status lb_create(const lb_params *p, void *dev_arena, size_t arena_bytes, void *hip_stream,
                    lb_ctx **out)
{
    if (!out) return fail(nullptr, LB_E_INVALID, "null output pointer");
    *out = nullptr;
    std::string why;
    lb_status s = check_params(p, why);
    if (s != LB_OK) return fail(nullptr, s, why);
    lb_ctx *c = new (std::nothrow) lb_ctx();
    if (!c) return fail(nullptr, LB_E_OOM, "host allocation failed");
    c->p = *p;
    if (c->p.max_colloids == 0) c->p.max_colloids = 64;
    if (c->p.precision == LB_FP16_STORAGE && c->p.f16_scale == 0.0) c->p.f16_scale = 16384.0;
    c->N = (long long)p->nx * p->ny * p->nz;
    KParams &k = c->kp;
    k.nx = p->nx; k.ny = p->ny; k.nz = p->nz; k.N = (int)c->N;
    k.rho0 = p->rho0; k.tau = p->tau; k.om = 1.0 / p->tau; k.pref = 1.0 - 0.5 / p->tau; k.a = p->a; k.b = p->b; k.kappa = p->kappa;
    // psi/c coefficients per sub-step of length 1/n (exactly the given ones for n = 1)
    const int nsub = substeps_of(*p);
    k.sub = 1.0 / nsub;
    k.M = p->M_psi / nsub; k.C = p->C; k.E = p->E; k.cb0 = p->c_b0; k.D = p->D_c / nsub; k.kd = p->k_d / nsub;
    k.fx = p->ext_force[0]; k.fy = p->ext_force[1]; k.fz = p->ext_force[2];
    k.scale = p->precision == LB_FP16_STORAGE ? (float)c->p.f16_scale : 1.0f;
    k.inv_scale = 1.0f / k.scale;
    k.flags = p->flags;
    k.soft_eps = p->soft_eps; k.soft_sigma = p->soft_sigma; k.soft_nu = p->soft_nu; k.soft_hc = p->soft_hc;
    k.lub_hc = p->lub_hc;
    set_shapes(c);
    c->stream = (hipStream_t)hip_stream;
    c->L = layout_of(c->p);
    if (dev_arena) {
        if ((uintptr_t)dev_arena & 255) {
            delete c;
            return fail(nullptr, LB_E_INVALID, "arena must be 256-byte aligned");
        }
        if (arena_bytes < c->L.total) {
            delete c;
            return fail(nullptr, LB_E_OOM, "arena smaller than lb_footprint_bytes");
        }
        c->arena = (char *)dev_arena;
        c->own_arena = false;
    } else {
        if (hipMalloc((void **)&c->arena, c->L.total) != hipSuccess) {
            delete c;
            return fail(nullptr, LB_E_OOM, "hipMalloc of the lattice arena failed");
        }
        c->own_arena = true;
    }
    c->nred = 1024;
    if (hipMalloc((void **)&c->derr, sizeof(int)) != hipSuccess ||
        hipMalloc((void **)&c->part, sizeof(double) * 7 * c->nred) != hipSuccess ||
        hipMalloc((void **)&c->dsum, sizeof(double) * 8) != hipSuccess) {
        lb_destroy(c);
        return fail(nullptr, LB_E_OOM, "hipMalloc of small buffers failed");
    }
    hipMemsetAsync(c->derr, 0, sizeof(int), c->stream);
    c->maxcol = c->p.max_colloids;
    *out = c;
    return LB_OK;
}

static void free_colloids(lb_ctx *c)
{
    if (c->dcol) hipFree(c->dcol);
    if (c->lnode) hipFree(c->lnode);
    if (c->ldc) hipFree(c->ldc);
    if (c->cpart) hipFree(c->cpart);
    if (c->lmask) hipFree(c->lmask);
    if (c->ccount) hipFree(c->ccount);
    if (c->lpart) hipFree(c->lpart);
    c->lpart = nullptr;
    c->dcol = nullptr;
    c->lnode = nullptr;
    c->ldc = nullptr;
    c->cpart = nullptr;
    c->lmask = nullptr;
    c->ccount = nullptr;
    c->ncol = 0;
    c->lcap = 0;
    c->special = false;
    c->dirty = true;  // descriptors hold the particle-table pointers
}

lb_status lb_destroy(lb_ctx *c)
{
    if (!c) return LB_OK;
    if (c->stream) hipStreamSynchronize(c->stream); else hipDeviceSynchronize();
    free_colloids(c);
    drop_graphs(c);
    if (c->selfdev) hipFree(c->selfdev);
    if (c->own_arena && c->arena) hipFree(c->arena);
    if (c->derr) hipFree(c->derr);
    if (c->part) hipFree(c->part);
    if (c->dsum) hipFree(c->dsum);
    if (c->has_side) {
        hipStreamSynchronize(c->side.s);
        for (int i = 0; i < SIDE_EVENTS; i++) hipEventDestroy(c->side.ev[i]);
        hipStreamDestroy(c->side.s);
    }
    delete c->timing;
    delete c;
    return LB_OK;
}

const char *lb_last_error(const lb_ctx *c) { return c ? c->err.c_str() : g_err.c_str(); }

// The second population lattice starts as a copy of the first and u as zero:
// slots that streaming never writes (those of solid nodes) and u at solid
// nodes then hold defined values, so no result depends on earlier contents
// of the device memory.
static hipError_t define_spare_state(lb_ctx *c)
{
    const size_t N = (size_t)c->N;
    hipError_t e = hipMemcpyAsync(ptr(c, c->L.f[1]), ptr(c, c->L.f[0]),
                                  19 * N * storage_bytes(c->p.precision), hipMemcpyDeviceToDevice,
                                  c->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(ptr(c, c->L.u), 0, 3 * N * compute_bytes(c->p.precision), c->stream);
    return e;
}

lb_status lb_init_fields(lb_ctx *c, const double *psi, const double *cc, const double *rho,
                         const double *u)
{
    if (!c) return fail(nullptr, LB_E_INVALID, "null context");
    if (!psi || !cc) return fail(c, LB_E_INVALID, "psi and c are required");
    const size_t N = (size_t)c->N;
    for (size_t n = 0; n < N; n++) {
        if (!std::isfinite(psi[n]) || !std::isfinite(cc[n])) return fail(c, LB_E_INVALID, "non-finite psi or c");
        if (rho && !(std::isfinite(rho[n]) && rho[n] > 0.0)) return fail(c, LB_E_INVALID, "rho must be finite and positive");
    }
    if (u)
        for (size_t n = 0; n < 3 * N; n++)
            if (!std::isfinite(u[n])) return fail(c, LB_E_INVALID, "non-finite u");
    // FP64 staging of the host fields: in the second population lattice,
    // which the init kernel does not touch and which is set from the first
    // right after it; a separate buffer only where that does not hold them
    // (FP16 storage with rho and u given)
    double *d = nullptr;
    const size_t need = (2 + (rho ? 1 : 0) + (u ? 3 : 0)) * N;
    const bool staged = need * sizeof(double) <= 19 * N * storage_bytes(c->p.precision);
    if (staged) d = (double *)ptr(c, c->L.f[1]);
    else HIP_TRY(c, hipMalloc((void **)&d, need * sizeof(double)));
    double *dpsi = d, *dc = d + N, *drho = rho ? d + 2 * N : nullptr;
    double *du = u ? d + (rho ? 3 : 2) * N : nullptr;
    hipError_t e = hipMemcpyAsync(dpsi, psi, N * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dc, cc, N * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && rho) e = hipMemcpyAsync(drho, rho, N * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && u) e = hipMemcpyAsync(du, u, 3 * N * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) {
        hipStreamSynchronize(c->stream);
        if (!staged) hipFree(d);
        return hip_fail(c, e, "hipMemcpyAsync");
    }
    free_colloids(c);
    c->dirty = true;
    c->cur = 0;
    void *f = ptr(c, c->L.f[0]), *ps = ptr(c, c->L.psi[0]), *cv = ptr(c, c->L.cc[0]);
    uint8_t *own = (uint8_t *)ptr(c, c->L.own);
    switch (c->p.precision) {
    case LB_FP64: launch_init<LB_FP64>(c->kp, dpsi, dc, drho, du, f, ps, cv, own, c->stream); break;
    case LB_FP32: launch_init<LB_FP32>(c->kp, dpsi, dc, drho, du, f, ps, cv, own, c->stream); break;
    default: launch_init<LB_FP16_STORAGE>(c->kp, dpsi, dc, drho, du, f, ps, cv, own, c->stream); break;
    }
    e = hipGetLastError();
    hipError_t e2 = hipStreamSynchronize(c->stream);
    if (!staged) hipFree(d);
    if (e != hipSuccess) return hip_fail(c, e, "init kernel launch");
    if (e2 != hipSuccess) return hip_fail(c, e2, "init kernel");
    HIP_TRY(c, hipMemsetAsync(c->derr, 0, sizeof(int), c->stream));
    HIP_TRY(c, define_spare_state(c));
    // single phase (A = kappa = E = 0, c_b0 = 0, psi = 0): mu stays 0 and chi
    // equals c, and psi stays 0 through the psi/c update and cover/uncover;
    // batches of such boxes skip the mu pass and read chi from c
    // (not with LB_STRESS_FORM, whose force reads the stress the mu pass writes)
    bool np = c->p.a == 0.0 && c->p.b == 0.0 && c->p.kappa == 0.0 && c->p.E == 0.0 &&
              c->p.c_b0 == 0.0 && !(c->p.flags & LB_STRESS_FORM);
    for (size_t n = 0; np && n < N; n++) np = psi[n] == 0.0;
    c->nopsi = np;
    if (np) {
        // the single-phase kernels neither compute mu nor write psi: both
        // psi buffers (and the sub-step one) and mu hold zeros from here on
        const size_t sb = N * compute_bytes(c->p.precision);
        HIP_TRY(c, hipMemsetAsync(ptr(c, c->L.mu), 0, sb, c->stream));
        HIP_TRY(c, hipMemsetAsync(ptr(c, c->L.psi[1]), 0, sb, c->stream));
        if (substeps_of(c->p) > 1) HIP_TRY(c, hipMemsetAsync(ptr(c, c->L.psis), 0, sb, c->stream));
    }
    c->step = 0;
    c->stage = 1;
    return LB_OK;
}

lb_status lb_add_colloids(lb_ctx *c, const lb_colloid *cols, int32_t n)
{
    if (!c) return fail(nullptr, LB_E_INVALID, "null context");
    if (c->stage < 1) return fail(c, LB_E_STATE, "lb_init_fields must come first");
    if (n < 0 || (n > 0 && !cols)) return fail(c, LB_E_INVALID, "bad particle array");
    if (n > c->maxcol) return fail(c, LB_E_INVALID, "more particles than max_colloids");
    const int Ls[3] = {c->p.nx, c->p.ny, c->p.nz};
    std::vector<DColloid> h(n > 0 ? n : 1);
    double rmax = 0.0;
    for (int k = 0; k < n; k++) {
        const lb_colloid &q = cols[k];
        DColloid &d = h[k];
        memset(&d, 0, sizeof d);
        double mm;
        {
#pragma clang fp contract(off)
            mm = sqrt(q.m[0] * q.m[0] + q.m[1] * q.m[1] + q.m[2] * q.m[2]);
        }
        if (!(q.radius > 0.0) || !(q.rho_p > 0.0) || !(mm > 0.0))
            return fail(c, LB_E_INVALID, "particle radius, density and axis must be positive");
        if (q.H != 0.0 && !(c->p.kappa > 0.0)) return fail(c, LB_E_INVALID, "wetting needs kappa > 0");
        if (!(q.cap_cos >= -1.0 && q.cap_cos <= 1.0)) return fail(c, LB_E_INVALID, "cap_cos must lie in [-1, 1]");
        if (!(q.axial >= 0.0) || !std::isfinite(q.axial))
            return fail(c, LB_E_INVALID, "axial semi-axis must be finite and >= 0");
        const bool sph = q.axial > 0.0 && q.axial != q.radius;
        if (sph && (c->p.soft_eps > 0.0 || c->p.lub_hc > 0.0))
            return fail(c, LB_E_INVALID, "soft-sphere and lubrication forces need spheres");
        const double rb = q.axial > q.radius ? q.axial : q.radius;
        if (q.pattern_bands < 0 || q.pattern_bands > LB_PATTERN_MAX_BANDS)
            return fail(c, LB_E_INVALID, "pattern bands must lie in [0, 8]");
        if (q.pattern_bands > 0) {
            const int S = q.pattern_sectors;
            if (!(S == 1 || S == 2 || S == 4 || S == 8) || q.pattern_bands * S > LB_PATTERN_MAX_CELLS)
                return fail(c, LB_E_INVALID, "pattern sectors must be 1, 2, 4 or 8");
            for (int b = 0; b < q.pattern_bands - 1; b++)
                if (!(q.pattern_cos[b] > -1.0 && q.pattern_cos[b] < 1.0) ||
                    (b > 0 && !(q.pattern_cos[b] > q.pattern_cos[b - 1])))
                    return fail(c, LB_E_INVALID, "pattern cuts must increase within (-1, 1)");
            for (int i = 0; i < q.pattern_bands * S; i++) {
                if (!std::isfinite(q.pattern_alpha[i]) || !std::isfinite(q.pattern_mu[i]) ||
                    !std::isfinite(q.pattern_H[i]))
                    return fail(c, LB_E_INVALID, "non-finite pattern value");
                if (q.pattern_H[i] != 0.0 && !(c->p.kappa > 0.0))
                    return fail(c, LB_E_INVALID, "wetting needs kappa > 0");
            }
            d.pb = q.pattern_bands;
            d.ps = S;
            for (int b = 0; b < q.pattern_bands - 1; b++) d.pcos[b] = q.pattern_cos[b];
            for (int i = 0; i < q.pattern_bands * S; i++) {
                d.palpha[i] = q.pattern_alpha[i];
                d.pmu[i] = q.pattern_mu[i];
                d.pH[i] = q.pattern_H[i];
            }
        }
        for (int a = 0; a < 3; a++) {
            if (2.0 * rb + 8.0 > (double)Ls[a])
                return fail(c, LB_E_INVALID, "particle too large for the box (2 R + 8 > side)");
            if (!std::isfinite(q.pos[a]) || !std::isfinite(q.vel[a]) || !std::isfinite(q.omega[a]))
                return fail(c, LB_E_INVALID, "non-finite particle state");
            double ps = fmod(q.pos[a], (double)Ls[a]);
            if (ps < 0.0) ps += (double)Ls[a];
            d.pos[a] = ps;
            d.m[a] = q.m[a] / mm;
            d.vel[a] = q.vel[a];
            d.omega[a] = q.omega[a];
        }
        d.radius = q.radius;
        d.am = q.alpha_minus;
        d.ap = q.alpha_plus;
        d.mum = q.mu_minus;
        d.mup = q.mu_plus;
        d.H = q.H;
        d.rho_p = q.rho_p;
        d.mass = q.rho_p * (4.0 * M_PI / 3.0) * q.radius * q.radius * q.radius;
        d.inertia = 0.4 * d.mass * q.radius * q.radius;
        if (sph) {
            // spheroid: mass rho_p 4 pi a b^2 / 3, 2 m b^2 / 5 about the axis,
            // m (a^2 + b^2) / 5 across it
            const double a = q.axial, b = q.radius;
            d.axial = a;
            d.mass = q.rho_p * (4.0 * M_PI / 3.0) * a * b * b;
            d.ipar = 0.4 * d.mass * b * b;
            d.iperp = 0.2 * d.mass * (a * a + b * b);
        }
        d.fixed = q.fixed ? 1 : 0;
        d.capc = q.cap_cos;
        {
            // second body axis: e made orthogonal to m and normalised; where
            // that part vanishes, the lattice axis least aligned with m,
            // (m x a) x m, in its place
#pragma clang fp contract(off)
            if (!std::isfinite(q.e[0]) || !std::isfinite(q.e[1]) || !std::isfinite(q.e[2]))
                return fail(c, LB_E_INVALID, "non-finite particle axis");
            const double em = q.e[0] * d.m[0] + q.e[1] * d.m[1] + q.e[2] * d.m[2];
            double ev[3] = {q.e[0] - em * d.m[0], q.e[1] - em * d.m[1], q.e[2] - em * d.m[2]};
            double ne = sqrt(ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2]);
            if (!(ne > 1e-9)) {
                int j = 0;
                for (int a = 1; a < 3; a++)
                    if (fabs(d.m[a]) < fabs(d.m[j])) j = a;
                double ax[3] = {0.0, 0.0, 0.0};
                ax[j] = 1.0;
                const double t[3] = {d.m[1] * ax[2] - d.m[2] * ax[1], d.m[2] * ax[0] - d.m[0] * ax[2],
                                     d.m[0] * ax[1] - d.m[1] * ax[0]};
                ev[0] = t[1] * d.m[2] - t[2] * d.m[1];
                ev[1] = t[2] * d.m[0] - t[0] * d.m[2];
                ev[2] = t[0] * d.m[1] - t[1] * d.m[0];
                ne = sqrt(ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2]);
            }
            for (int a = 0; a < 3; a++) d.e[a] = ev[a] / ne;
        }
        d.changed = 1;  // build the owner map and link table on placement
        rmax = std::max(rmax, rb);
    }
    // surfaces at least 2 lattice units apart (minimum image)
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++) {
            double s2 = 0.0;
            for (int a = 0; a < 3; a++) {
                double d = min_image(h[i].pos[a] - h[j].pos[a], Ls[a]);
                s2 += d * d;
            }
            // (spheroids by their bounding spheres)
            if (sqrt(s2) < bound_radius(h[i]) + bound_radius(h[j]) + 2.0)
                return fail(c, LB_E_STATE, "particle surfaces closer than 2 lattice units");
        }
    free_colloids(c);
    c->dirty = true;
    // reset the owner map to all fluid before placing the new set
    HIP_TRY(c, hipMemsetAsync(ptr(c, c->L.own), 0, (size_t)c->N, c->stream));
    if (n == 0) { c->stage = 2; return LB_OK; }
    // link capacity: 10 links per node of the shell R-1/2 .. R+3/2, plus slack
    const double ro = rmax + 1.5, ri = std::max(0.0, rmax - 0.5);
    const int lcap = (int)(10.0 * (4.0 / 3.0) * M_PI * (ro * ro * ro - ri * ri * ri)) + 512;
    {
        lb_status st = alloc_colloid_tables(c, rmax, lcap);
        if (st != LB_OK) { free_colloids(c); return st; }
    }
    HIP_TRY(c, hipMemcpyAsync(c->dcol, h.data(), sizeof(DColloid) * n, hipMemcpyHostToDevice, c->stream));
    c->ncol = n;
    for (int k = 0; k < n; k++) c->special = c->special || h[k].pb > 0 || is_spheroid(h[k]);
    c->dirty = true;
    {
        lb_status st = refresh_self(c);
        if (st != LB_OK) return st;
    }
    launch_geometry(c->self[c->cur], c->stream);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int herr = 0;
    HIP_TRY(c, hipMemcpy(&herr, c->derr, sizeof(int), hipMemcpyDeviceToHost));
    if (herr & LB_ERR_LINKS) return fail(c, LB_E_STATE, "link table overflow");
    c->stage = 2;
    return LB_OK;
}

lb_status lb_step(lb_ctx *c, int64_t nsteps)
{
    if (!c) return fail(nullptr, LB_E_INVALID, "null context");
    if (c->stage < 1) return fail(c, LB_E_STATE, "lb_init_fields must come first");
    if (nsteps < 0) return fail(c, LB_E_INVALID, "negative step count");
    lb_status st = refresh_self(c);
    if (st != LB_OK) return st;
    int64_t s = 0;
    // step pairs replayed from a captured graph (not while timing kernels,
    // not on the legacy default stream, which cannot be captured)
    if (!c->timing && c->stream && nsteps >= 2) {
        const int par = c->cur;
        // both parities at once: a later call that starts on the other
        // parity (after an odd step count) then replays without capturing
        for (int q = 0; q < 2; q++) {
            if (c->graph[q]) continue;
            hipError_t e = capture_pair(c->self[q], c->self[1 - q], c->stream, side_of(c),
                                        &c->graph[q]);
            if (e != hipSuccess) { c->graph[q] = nullptr; return hip_fail(c, e, "graph capture"); }
        }
        for (; s + 2 <= nsteps; s += 2) HIP_TRY(c, hipGraphLaunch(c->graph[par], c->stream));
    }
    for (; s < nsteps; s++) {
        launch_one_step(c->self[c->cur], c->stream, side_of(c), c->timing);
        c->cur ^= 1;
    }
    c->step += nsteps;
    HIP_TRY(c, hipGetLastError());
    return LB_OK;
}

lb_status lb_batch_step(lb_ctx *const *ctxs, int32_t n, int64_t nsteps)
{
    lb_status st = batch_check(ctxs, n, nsteps);
    if (st != LB_OK) return st;
    lb_ctx *c0 = ctxs[0];
    char *dev = nullptr;
    const size_t bb = align256(batch_bytes(n, substeps_of(c0->p)));
    HIP_TRY(c0, hipMalloc((void **)&dev, 2 * bb));
    st = batch_run(ctxs, n, nsteps, dev, bb, true, side_of(c0));
    hipFree(dev);
    return st;
}

lb_status lb_batch_step_noalloc(lb_ctx *const *ctxs, int32_t n, int64_t nsteps)
{
    lb_status st = batch_check(ctxs, n, nsteps);
    if (st != LB_OK) return st;
    lb_ctx *c0 = ctxs[0];
    const size_t bb = align256(batch_bytes(n, substeps_of(c0->p)));
    if (2 * bb > NOALLOC_SCRATCH_BYTES)
        return fail(c0, LB_E_INVALID,
                    "batch too large for lb_batch_step_noalloc: its descriptor tables need " +
                        std::to_string(2 * bb) + " bytes, the fixed device array holds " +
                        std::to_string(NOALLOC_SCRATCH_BYTES));
    char *dev = nullptr;
    st = scratch_address(c0, &dev);
    if (st != LB_OK) return st;
    // no graph (instantiation allocates), and the side stream only if the
    // leading context already has one
    return batch_run(ctxs, n, nsteps, dev, bb, false, c0->has_side ? &c0->side : nullptr);
}

lb_status lb_set_launch_shapes(lb_ctx *c, const int32_t *shapes9)
{
    if (!c || !shapes9) return fail(c, LB_E_INVALID, "null argument");
    LaunchShape v[3];
    for (int k = 0; k < 3; k++) {
        // code = remap + 8 vec + 64 zc
        const int code = shapes9[3 * k + 2];
        const int rm = code & 7, vec = code >= 0 ? (code >> 3) & 7 : -1, zc = code >> 6;
        v[k] = LaunchShape{shapes9[3 * k], shapes9[3 * k + 1], rm, 0, 0, 0, vec, zc};
        if (v[k].bx < 0 || v[k].by < 0 || code < 0 || rm > 2 ||
            !(vec == 0 || vec == 1 || vec == 2 || vec == 4) ||
            (zc > 1 && (k != 2 || vec < 2)) || zc > 65535)
            return fail(c, LB_E_INVALID, "bad shape");
        finish_shape(v[k], c->p.nx, c->p.ny, c->p.nz, c->p.precision == LB_FP64 ? 8 : 4, k == 1);
    }
    for (int k = 0; k < 3; k++) c->shapes[k] = v[k];
    c->dirty = true;
    return LB_OK;
}

lb_status lb_get_launch_shapes(lb_ctx *c, int32_t *shapes9)
{
    if (!c || !shapes9) return fail(c, LB_E_INVALID, "null argument");
    for (int k = 0; k < 3; k++) {
        shapes9[3 * k] = c->shapes[k].bx;
        shapes9[3 * k + 1] = c->shapes[k].by;
        shapes9[3 * k + 2] = c->shapes[k].remap + 8 * (c->shapes[k].vec > 1 ? c->shapes[k].vec : 0) +
                             64 * (c->shapes[k].zc > 1 ? c->shapes[k].zc : 0);
    }
    return LB_OK;
}

lb_status lb_observables(lb_ctx *c, lb_totals *t, lb_colloid *out, int32_t n)
{
    if (!c) return fail(nullptr, LB_E_INVALID, "null context");
    if (c->stage < 1) return fail(c, LB_E_STATE, "lb_init_fields must come first");
    int herr = 0;
    std::vector<DColloid> h(c->ncol > 0 ? c->ncol : 1);
    double sums[7] = {0, 0, 0, 0, 0, 0, 0};
    if (t) {
        switch (c->p.precision) {
        case LB_FP64: reduce_t<LB_FP64>(c); break;
        case LB_FP32: reduce_t<LB_FP32>(c); break;
        default: reduce_t<LB_FP16_STORAGE>(c); break;
        }
        HIP_TRY(c, hipGetLastError());
        HIP_TRY(c, hipMemcpyAsync(sums, c->dsum, sizeof(double) * 7, hipMemcpyDeviceToHost, c->stream));
    }
    HIP_TRY(c, hipMemcpyAsync(&herr, c->derr, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    if (c->ncol > 0)
        HIP_TRY(c, hipMemcpyAsync(h.data(), c->dcol, sizeof(DColloid) * c->ncol, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (t) {
        memset(t, 0, sizeof *t);
        t->mass = sums[0];
        t->mom[0] = sums[1];
        t->mom[1] = sums[2];
        t->mom[2] = sums[3];
        t->sum_psi = sums[4];
        t->sum_c = sums[5];
        t->n_fluid = (int64_t)sums[6];
        if (c->ncol > 0) {
            int64_t nl = 0;
            lb_status st = lb_get_links(c, nullptr, 0, &nl);
            if (st != LB_OK) return st;
            std::vector<int32_t> rec(4 * (size_t)std::max<int64_t>(nl, 1));
            st = lb_get_links(c, rec.data(), nl, &nl);
            if (st != LB_OK) return st;
            t->n_links = nl;
            // active links: the cap bit, or a producing cell of a pattern
            for (int64_t l = 0; l < nl; l++) {
                const DColloid &q = h[rec[4 * l]];
                const int tag = rec[4 * l + 3];
                t->n_active += q.pb > 0 ? (q.palpha[tag] != 0.0 ? 1 : 0) : tag;
            }
        }
        t->step = c->step;
        int e = herr;
        for (int j = 0; j < 6; j++)
            if (!std::isfinite(sums[j])) e |= LB_ERR_NAN;
        t->error_bits = e;
        herr = e;
    }
    if (out) {
        if (n > c->ncol) n = c->ncol;
        for (int k = 0; k < n; k++) {
            lb_colloid &q = out[k];
            const DColloid &d = h[k];
            for (int a = 0; a < 3; a++) {
                q.pos[a] = d.pos[a];
                q.m[a] = d.m[a];
                q.vel[a] = d.vel[a];
                q.omega[a] = d.omega[a];
            }
            q.radius = d.radius;
            q.alpha_minus = d.am;
            q.alpha_plus = d.ap;
            q.mu_minus = d.mum;
            q.mu_plus = d.mup;
            q.H = d.H;
            q.rho_p = d.rho_p;
            q.fixed = d.fixed;
            q.cap_cos = d.capc;
            q.axial = d.axial;
            for (int a = 0; a < 3; a++) q.e[a] = d.e[a];
            q.pattern_bands = d.pb;
            q.pattern_sectors = d.ps;
            for (int b = 0; b < LB_PATTERN_MAX_BANDS - 1; b++) q.pattern_cos[b] = d.pcos[b];
            for (int i = 0; i < LB_PATTERN_MAX_CELLS; i++) {
                q.pattern_alpha[i] = d.palpha[i];
                q.pattern_mu[i] = d.pmu[i];
                q.pattern_H[i] = d.pH[i];
            }
        }
    }
    if (herr & LB_ERR_NAN) return fail(c, LB_E_UNSTABLE, "non-finite totals");
    if (herr) return fail(c, LB_E_STATE, "device error bits set: " + std::to_string(herr));
    return LB_OK;
}

lb_status lb_get_fields(lb_ctx *c, double *rho, double *u, double *psi, double *cc)
{
    if (!c) return fail(nullptr, LB_E_INVALID, "null context");
    if (c->stage < 1) return fail(c, LB_E_STATE, "lb_init_fields must come first");
    const size_t N = (size_t)c->N;
    double *d = nullptr;
    HIP_TRY(c, hipMalloc((void **)&d, 6 * N * sizeof(double)));
    lb_status s = run_fields(c, d, nullptr);
    hipError_t e = hipSuccess;
    if (s == LB_OK) {
        if (rho) e = hipMemcpyAsync(rho, d, N * 8, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess && u) e = hipMemcpyAsync(u, d + N, 3 * N * 8, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess && psi) e = hipMemcpyAsync(psi, d + 4 * N, N * 8, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess && cc) e = hipMemcpyAsync(cc, d + 5 * N, N * 8, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    hipFree(d);
    if (s != LB_OK) return s;
    if (e != hipSuccess) return hip_fail(c, e, "field readback");
    return LB_OK;
}

lb_status lb_get_populations(lb_ctx *c, double *f)
{
    if (!c || !f) return fail(c, LB_E_INVALID, "null argument");
    if (c->stage < 1) return fail(c, LB_E_STATE, "lb_init_fields must come first");
    const size_t N = (size_t)c->N;
    double *d = nullptr;
    HIP_TRY(c, hipMalloc((void **)&d, 19 * N * sizeof(double)));
    lb_status s = run_fields(c, nullptr, d);
    hipError_t e = hipSuccess;
    if (s == LB_OK) {
        e = hipMemcpyAsync(f, d, 19 * N * 8, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    hipFree(d);
    if (s != LB_OK) return s;
    if (e != hipSuccess) return hip_fail(c, e, "population readback");
    return LB_OK;
}

lb_status lb_get_owner(lb_ctx *c, int32_t *owner)
{
    if (!c || !owner) return fail(c, LB_E_INVALID, "null argument");
    if (c->stage < 1) return fail(c, LB_E_STATE, "lb_init_fields must come first");
    std::vector<uint8_t> h((size_t)c->N);
    HIP_TRY(c, hipMemcpyAsync(h.data(), ptr(c, c->L.own), (size_t)c->N, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (size_t n = 0; n < h.size(); n++) owner[n] = (int)(h[n] & OWN_SOLID) - 1;
    return LB_OK;
}

lb_status lb_get_links(lb_ctx *c, int32_t *rec4, int64_t cap, int64_t *nout)
{
    if (!c || !nout) return fail(c, LB_E_INVALID, "null argument");
    *nout = 0;
    if (c->ncol == 0) return LB_OK;
    std::vector<DColloid> h(c->ncol);
    HIP_TRY(c, hipMemcpyAsync(h.data(), c->dcol, sizeof(DColloid) * c->ncol, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int64_t total = 0;
    for (int k = 0; k < c->ncol; k++) total += std::min(h[k].nlinks, c->lcap);
    *nout = total;
    if (!rec4) return LB_OK;
    if (cap < total) return fail(c, LB_E_INVALID, "link buffer too small");
    std::vector<int> nodes((size_t)c->lcap * c->ncol);
    std::vector<uint8_t> dcs((size_t)c->lcap * c->ncol);
    HIP_TRY(c, hipMemcpy(nodes.data(), c->lnode, sizeof(int) * nodes.size(), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(dcs.data(), c->ldc, dcs.size(), hipMemcpyDeviceToHost));
    int64_t l = 0;
    for (int k = 0; k < c->ncol; k++)
        for (int j = 0; j < std::min(h[k].nlinks, c->lcap); j++) {
            const size_t s = (size_t)k * c->lcap + j;
            rec4[4 * l + 0] = k;
            rec4[4 * l + 1] = nodes[s];
            const int d = dcs[s], n = nodes[s];
            const int z = n / (c->p.nx * c->p.ny), y = (n / c->p.nx) % c->p.ny, x = n % c->p.nx;
            double r[3];
            displacement(h[k], x, y, z, cx(d), cy(d), cz(d), 0.5, c->p.nx, c->p.ny, c->p.nz, r);
            rec4[4 * l + 2] = d;
            // from the current axes: the cap bit, or the cell of a pattern
            const int cell = surface_cell(h[k], r);
            rec4[4 * l + 3] = h[k].pb > 0 ? cell : (cell == 0 ? 1 : 0);
            l++;
        }
    return LB_OK;
}

lb_status lb_colloid_forces(lb_ctx *c, double *out12, int32_t n)
{
    if (!c || !out12) return fail(c, LB_E_INVALID, "null argument");
    if (n > c->ncol) n = c->ncol;
    if (n <= 0) return LB_OK;
    std::vector<DColloid> h(c->ncol);
    HIP_TRY(c, hipMemcpyAsync(h.data(), c->dcol, sizeof(DColloid) * c->ncol, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < n; k++)
        for (int a = 0; a < 3; a++) {
            out12[12 * k + a] = h[k].F[a];
            out12[12 * k + 3 + a] = h[k].T[a];
            out12[12 * k + 6 + a] = h[k].F0[a];
            out12[12 * k + 9 + a] = h[k].T0[a];
        }
    return LB_OK;
}

lb_status lb_save_state(lb_ctx *c, void *buf, size_t cap, size_t *nout)
{
    if (!c || !nout) return fail(c, LB_E_INVALID, "null argument");
    if (c->stage < 1) return fail(c, LB_E_STATE, "lb_init_fields must come first");
    const size_t need = state_size(c);
    *nout = need;
    if (!buf) return LB_OK;
    if (cap < need) return fail(c, LB_E_INVALID, "state buffer too small");
    const size_t N = (size_t)c->N;
    char *o = (char *)buf;
    StateHeader hd = {STATE_MAGIC, c->p.nx, c->p.ny, c->p.nz, c->p.precision, c->ncol, c->lcap, c->step};
    memcpy(o, &hd, sizeof hd);
    o += sizeof hd;
    const size_t fb = 19 * N * storage_bytes(c->p.precision), sb = N * compute_bytes(c->p.precision);
    HIP_TRY(c, hipMemcpyAsync(o, ptr(c, c->L.f[c->cur]), fb, hipMemcpyDeviceToHost, c->stream)); o += fb;
    HIP_TRY(c, hipMemcpyAsync(o, ptr(c, c->L.psi[c->cur]), sb, hipMemcpyDeviceToHost, c->stream)); o += sb;
    HIP_TRY(c, hipMemcpyAsync(o, ptr(c, c->L.cc[c->cur]), sb, hipMemcpyDeviceToHost, c->stream)); o += sb;
    HIP_TRY(c, hipMemcpyAsync(o, ptr(c, c->L.own), N, hipMemcpyDeviceToHost, c->stream)); o += N;
    if (c->ncol) {
        HIP_TRY(c, hipMemcpyAsync(o, c->dcol, sizeof(DColloid) * c->ncol, hipMemcpyDeviceToHost, c->stream));
        o += sizeof(DColloid) * c->ncol;
        HIP_TRY(c, hipMemcpyAsync(o, c->lnode, sizeof(int) * (size_t)c->lcap * c->ncol, hipMemcpyDeviceToHost, c->stream));
        o += sizeof(int) * (size_t)c->lcap * c->ncol;
        HIP_TRY(c, hipMemcpyAsync(o, c->ldc, (size_t)c->lcap * c->ncol, hipMemcpyDeviceToHost, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LB_OK;
}

lb_status lb_load_state(lb_ctx *c, const void *buf, size_t n)
{
    if (!c || !buf) return fail(c, LB_E_INVALID, "null argument");
    StateHeader hd;
    if (n < sizeof hd) return fail(c, LB_E_INVALID, "state too short");
    memcpy(&hd, buf, sizeof hd);
    if (hd.magic != STATE_MAGIC || hd.nx != c->p.nx || hd.ny != c->p.ny || hd.nz != c->p.nz ||
        hd.precision != c->p.precision || hd.ncol > c->maxcol)
        return fail(c, LB_E_INVALID, "state does not match this context");
    free_colloids(c);
    c->ncol = hd.ncol;
    if (hd.ncol > 0) {
        const DColloid *hc = (const DColloid *)((const char *)buf + sizeof hd +
                                                19 * (size_t)c->N * storage_bytes(c->p.precision) +
                                                2 * (size_t)c->N * compute_bytes(c->p.precision) +
                                                (size_t)c->N);
        if (n < sizeof hd + 19 * (size_t)c->N * storage_bytes(c->p.precision) +
                    2 * (size_t)c->N * compute_bytes(c->p.precision) + (size_t)c->N +
                    sizeof(DColloid) * hd.ncol)
            return fail(c, LB_E_INVALID, "state too short");
        double rmax = 0.0;
        for (int k = 0; k < hd.ncol; k++) rmax = std::max(rmax, bound_radius(hc[k]));
        for (int k = 0; k < hd.ncol; k++) c->special = c->special || hc[k].pb > 0 || is_spheroid(hc[k]);
        lb_status st = alloc_colloid_tables(c, rmax, hd.lcap);
        if (st != LB_OK) { free_colloids(c); c->ncol = 0; return st; }
    }
    if (n < state_size(c)) return fail(c, LB_E_INVALID, "state too short");
    const size_t N = (size_t)c->N;
    const char *o = (const char *)buf + sizeof hd;
    c->cur = 0;
    const size_t fb = 19 * N * storage_bytes(c->p.precision), sb = N * compute_bytes(c->p.precision);
    HIP_TRY(c, hipMemcpyAsync(ptr(c, c->L.f[0]), o, fb, hipMemcpyHostToDevice, c->stream)); o += fb;
    HIP_TRY(c, hipMemcpyAsync(ptr(c, c->L.psi[0]), o, sb, hipMemcpyHostToDevice, c->stream)); o += sb;
    HIP_TRY(c, hipMemcpyAsync(ptr(c, c->L.cc[0]), o, sb, hipMemcpyHostToDevice, c->stream)); o += sb;
    HIP_TRY(c, hipMemcpyAsync(ptr(c, c->L.own), o, N, hipMemcpyHostToDevice, c->stream)); o += N;
    if (c->ncol) {
        HIP_TRY(c, hipMemcpyAsync(c->dcol, o, sizeof(DColloid) * c->ncol, hipMemcpyHostToDevice, c->stream));
        o += sizeof(DColloid) * c->ncol;
        HIP_TRY(c, hipMemcpyAsync(c->lnode, o, sizeof(int) * (size_t)c->lcap * c->ncol, hipMemcpyHostToDevice, c->stream));
        o += sizeof(int) * (size_t)c->lcap * c->ncol;
        HIP_TRY(c, hipMemcpyAsync(c->ldc, o, (size_t)c->lcap * c->ncol, hipMemcpyHostToDevice, c->stream));
    }
    HIP_TRY(c, hipMemsetAsync(c->derr, 0, sizeof(int), c->stream));
    HIP_TRY(c, define_spare_state(c));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->nopsi = false;  // the loaded psi need not be zero: general path
    c->dirty = true;
    c->step = hd.step;
    c->stage = 2;
    c->dirty = true;
    return LB_OK;
}

lb_status lb_timing_enable(lb_ctx *c, int32_t on)
{
    if (!c) return fail(nullptr, LB_E_INVALID, "null context");
    if (on) {
        if (!c->timing) c->timing = new (std::nothrow) TimingHook();
        if (!c->timing) return fail(c, LB_E_OOM, "host allocation failed");
        c->timing->reset();
    } else {
        delete c->timing;
        c->timing = nullptr;
    }
    return LB_OK;
}

lb_status lb_timing_read(lb_ctx *c, double *ms6, int64_t *calls6)
{
    if (!c || !ms6 || !calls6) return fail(c, LB_E_INVALID, "null argument");
    if (!c->timing) return fail(c, LB_E_STATE, "timing is not enabled");
    c->timing->flush();
    for (int i = 0; i < 6; i++) { ms6[i] = c->timing->ms[i]; calls6[i] = c->timing->calls[i]; }
    return LB_OK;
}

double lb_wetting_H(double theta_deg, double kappa, double b)
{
    if (!(kappa * b > 0.0)) return NAN;
    const double target = cos(theta_deg * M_PI / 180.0);
    double lo = -1.0, hi = 1.0;
    for (int it = 0; it < 200; it++) {
        const double h = 0.5 * (lo + hi);
        const double v = 0.5 * (pow(1.0 + h, 1.5) - pow(1.0 - h, 1.5));
        if (v < target) lo = h; else hi = h;
    }
    return 0.5 * (lo + hi) * sqrt(kappa * b);
}

}  // extern "C"

// ------------------------------------------- wetting map of the lattice
// The wetting ghost of the chemical potential (psi - (H/kappa)|e.n| at a
// solid face neighbour) is the derivative of the discrete free energy
//   sum_x [f(psi) - f_b] + kappa/2 sum_faces (psi' - psi)^2 + H sum_wall psi,
// the wall sum over the fluid nodes next to the solid, weighted by |e.n| per
// solid face neighbour (H per unit area for any wall orientation).  On a flat
// wall this is a one-dimensional chain; the contact angle it realises follows
// from Young's balance of the discrete tensions.  Minimisers by Newton's method
// on the tridiagonal Hessian with a backtracking line search.
namespace {

struct Chain {
    double a, b, kappa, H;
    bool wall;                 // node 0 next to the wall (else pinned at `left`)
    double left, right;        // pinned values beyond the ends
    std::vector<double> p;
};

double chain_energy(const Chain &c, const std::vector<double> &p)
{
    const double pb2 = -c.a / c.b, fb = 0.5 * c.a * pb2 + 0.25 * c.b * pb2 * pb2;
    const size_t M = p.size();
    double e = 0.0;
    for (size_t i = 0; i < M; i++) {
        const double q = p[i];
        e += 0.5 * c.a * q * q + 0.25 * c.b * q * q * q * q - fb;
        const double nxt = i + 1 < M ? p[i + 1] : c.right;
        e += 0.5 * c.kappa * (nxt - q) * (nxt - q);
    }
    if (c.wall) e += c.H * p[0];
    else e += 0.5 * c.kappa * (p[0] - c.left) * (p[0] - c.left);
    return e;
}

double chain_minimum(Chain &c)
{
    const size_t M = c.p.size();
    std::vector<double> g(M), d(M), cp(M), dp(M), x(M), trial(M);
    double e = chain_energy(c, c.p);
    for (int it = 0; it < 100; it++) {
        double gmax = 0.0;
        for (size_t i = 0; i < M; i++) {
            const double q = c.p[i];
            const double prv = i > 0 ? c.p[i - 1] : (c.wall ? q : c.left);
            const double nxt = i + 1 < M ? c.p[i + 1] : c.right;
            g[i] = c.a * q + c.b * q * q * q + c.kappa * ((q - prv) + (q - nxt));
            d[i] = c.a + 3.0 * c.b * q * q + ((i == 0 && c.wall) ? 1.0 : 2.0) * c.kappa;
            gmax = std::max(gmax, std::fabs(g[i]));
        }
        if (c.wall) g[0] += c.H;
        gmax = std::max(gmax, std::fabs(g[0]));
        if (gmax < 1e-15) break;
        // Thomas algorithm for (diag d, off-diagonals -kappa) x = -g
        cp[0] = -c.kappa / d[0];
        dp[0] = -g[0] / d[0];
        for (size_t i = 1; i < M; i++) {
            const double den = d[i] + c.kappa * cp[i - 1];
            cp[i] = -c.kappa / den;
            dp[i] = (-g[i] + c.kappa * dp[i - 1]) / den;
        }
        x[M - 1] = dp[M - 1];
        for (size_t i = M - 1; i-- > 0;) x[i] = dp[i] - cp[i] * x[i + 1];
        double t = 1.0, et = e;
        for (; t > 1e-12; t *= 0.5) {
            for (size_t i = 0; i < M; i++) trial[i] = c.p[i] + t * x[i];
            et = chain_energy(c, trial);
            if (et <= e) break;
        }
        if (!(t > 1e-12)) break;
        c.p.swap(trial);
        e = et;
    }
    return e;
}

// Young's cosine of the discrete flat wall with wetting parameter H:
// (gamma(+psi_b) - gamma(-psi_b)) / sigma, the wall tensions against each
// bulk phase over the tension of the discrete flat interface (the lower of
// the kink centred between nodes and on a node)
double lattice_cos(double a, double b, double kappa, double H)
{
    const double pb = std::sqrt(-a / b), w = std::sqrt(2.0 * kappa / -a);
    const int M = std::max(64, (int)(16.0 * w) + 1);
    double gam[2];
    for (int k = 0; k < 2; k++) {
        const double s = k == 0 ? pb : -pb;
        Chain c{a, b, kappa, H, true, 0.0, s, std::vector<double>(M, s)};
        gam[k] = chain_minimum(c);
    }
    double sigma = INFINITY;
    for (int k = 0; k < 2; k++) {
        Chain c{a, b, kappa, 0.0, false, -pb, pb, std::vector<double>(2 * M)};
        for (int i = 0; i < 2 * M; i++) c.p[i] = pb * std::tanh((i - M + 0.5 * k) / w);
        sigma = std::min(sigma, chain_minimum(c));
    }
    return (gam[0] - gam[1]) / sigma;
}

}  // namespace

extern "C" {

double lb_wetting_H_lattice(double theta_deg, double a, double b, double kappa)
{
    if (!(a < 0.0 && b > 0.0 && kappa > 0.0) || !std::isfinite(theta_deg)) return NAN;
    const double target = std::cos(theta_deg * M_PI / 180.0), scale = std::sqrt(kappa * b);
    double lo = -scale, hi = scale;
    const double clo = lattice_cos(a, b, kappa, lo), chi = lattice_cos(a, b, kappa, hi);
    if (!(target >= clo && target <= chi)) return NAN;
    for (int it = 0; it < 60; it++) {
        const double mid = 0.5 * (lo + hi);
        if (lattice_cos(a, b, kappa, mid) < target) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

double lb_solubility_E(double ratio, double c_b0)
{
    return -c_b0 * (ratio - 1.0) / ((ratio + 1.0) * tanh(1.0));
}

}  // extern "C"
