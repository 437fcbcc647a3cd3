// lb_kernels.h -- host-side launch interface of the lattice-update kernels.
#pragma once
#include <utility>
#include <vector>

#include "lb_device.h"

namespace lbk {

// Device buffers one step reads and writes (cur -> nxt).
struct StepBuffers {
    const void *fin;
    void *fout;
    const void *psi, *cc;   // state at t
    void *psin, *ccn;       // state at t+1
    void *mu, *chi, *u;     // derived fields of step t (chi stored in FP64 only)
    void *pst, *muc;        // LB_STRESS_FORM: stress (6 planes xx yy zz xy xz yz) and mu_c
    uint8_t *own;
    DColloid *col;
    int *lnode;
    uint8_t *ldc;
    int lcap;
    int *err;
    double *cpart;      // per (particle, chunk): 6 transfer partials + change flag
    uint32_t *lmask;    // per (particle, box node): directions linked to the particle
    int *ccount;        // per (particle, chunk): links in the chunk
    int bbmax, nchunk_max;
    double *lpart;      // per (particle, link chunk): 28 FP64 link-momentum partials
    int nlchunk_max;
};

// One box of a batched launch: parameters, per-kernel lattice launch shapes
// (mu, collide, scalar) and the buffers of the step it takes.
struct BoxDesc {
    KParams p;
    LaunchShape ls[3];
    StepBuffers b;
};

// Device-side view of a batch: box descriptors, the first block of each box
// in each of the three lattice launches (3 x (nbox+1)), and the first global
// particle index of each box (nbox+1).
struct BatchArgs {
    const BoxDesc *d;
    const int *bstart;
    const int *cstart;
    int nbox;
    int nsec;   // boundary fix-up blocks per particle
    int nfix;   // blocks of a boundary fix-up launch
    int boff;   // first block of a partial launch of a lattice kernel (0: whole grid)
};

// Host-side batch: device tables plus launch extents.
struct Batch {
    BatchArgs args;
    int nblocks[3];   // blocks of the mu, collide, scalar launches
    int ncol;         // particles over all boxes
    int nchunk_max;   // geometry chunks of the largest particle box
    int nlchunk_max;  // link chunks of the largest link table
    int precision;
    int vec[3];       // row-vector form of each lattice launch (all boxes of the batch)
    int zmarch;       // z-marching form of the psi/c update (all boxes of the batch)
    long long nodes;  // lattice nodes over all boxes
    int solute_force; // some box has LB_SOLUTE_FORCE (one-node collide-stream with the term)
    int stress;       // some box has LB_STRESS_FORM (one-node mu and collide-stream, fix-ups)
    int nsub;         // psi/c sub-steps per step (all boxes of the batch)
    int soft;         // some box has soft-sphere repulsion (k_soft runs)
    int nopsi;        // every box single phase: no mu launches, single-phase kernels
    int special;      // some particle carries a surface pattern or is not a sphere:
                      // boundary nodes always in the fix-up launches (the inline forms
                      // have neither the cell arithmetic nor the spheroid normal)
    // with nsub > 1: descriptor tables of sub-step 0 (state at t -> its
    // target), next-state -> scratch and scratch -> next-state psi/c pairs
    const BoxDesc *dsub[3];
};

// Optional per-kernel HIP-event timing (groups 0..5: mu, collide, scalar,
// links+particles, cover, geometry).
struct TimingHook {
    std::vector<hipEvent_t> pool;            // free events
    std::vector<hipEvent_t> open[6];         // begin events awaiting their end
    std::vector<std::pair<hipEvent_t, hipEvent_t>> done[6];
    double ms[6] = {0, 0, 0, 0, 0, 0};
    long long calls[6] = {0, 0, 0, 0, 0, 0};
    hipEvent_t take();
    void begin(int i, hipStream_t s);
    void end(int i, hipStream_t s);
    void flush();   // waits for recorded events, accumulates, recycles
    void reset();
    ~TimingHook();
};

// derive the launch extents of a shape; ssize = bytes of a scalar field value;
// whole_rows: a row-vector shape must keep each row in one lane group (the
// row-vector collide-stream), else the shape falls back to one node per
// thread
void finish_shape(LaunchShape &ls, int nx, int ny, int nz, int ssize, bool whole_rows = false);

// Second stream for the particle work of a step, with the events of its
// forks and joins.
constexpr int SIDE_EVENTS = 5;
struct SideStream {
    hipStream_t s;
    hipEvent_t ev[SIDE_EVENTS];
};

// one time step of every box of the batch (all boxes share the precision P);
// side may be null (everything in order on s).  defer_links: the link table
// write of the step's tail may stay on the side stream, unjoined; the caller
// guarantees that another step follows on s (its side-stream work is ordered
// after it and joined before its collide-stream).
template <int P>
void launch_step(const Batch &B, hipStream_t s, const SideStream *side, TimingHook *tm,
                 bool defer_links = false);
// particle geometry at placement (owner map, boundary bits, link tables)
void launch_geometry(const Batch &B, hipStream_t s);

template <int P>
void launch_init(const KParams &p, const double *psi0, const double *c0, const double *rho0,
                 const double *u0, void *f, void *psi, void *cc, uint8_t *own, hipStream_t s);
template <int P>
void launch_reduce(const KParams &p, const void *f, const void *psi, const void *cc,
                   const uint8_t *own, double *part, int nblocks, double *out, hipStream_t s);
template <int P>
void launch_fields(const KParams &p, const void *f, const void *psi, const void *cc,
                   const uint8_t *own, double *out, double *fout, hipStream_t s);

}  // namespace lbk
