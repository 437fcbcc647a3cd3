// hip_cpu.cpp -- CPU stand-in for the HIP runtime calls made by the library's
// host code.  TEST INFRASTRUCTURE ONLY (see include/hip/hip_runtime.h): it is
// linked with the host-only, sanitizer-instrumented build of the library so
// that the ABI's call sequences (create, init, particles, batched steps with
// graph capture, readback, destroy) can be checked for memory and lifetime
// errors without a GPU.  Kernels are not executed: a launch only checks its
// configuration and its stream.  Asynchronous copies and fills are not done
// when they are issued but at the next point where the caller may rely on
// them (a stream, event or device synchronisation, a synchronous copy, a
// free): a host buffer released before its asynchronous copy has run is then
// read or written after its release, which AddressSanitizer reports.
//
// What is checked (a violation prints "hostcheck:" and aborts):
//   * device memory: every copy and fill lies inside one live allocation;
//     hipFree takes only live allocations (device memory is host memory, so
//     AddressSanitizer also sees any host-side overrun);
//   * streams and events: every use is of a live object (destroyed objects
//     are poisoned and freed, so a later use is a heap-use-after-free);
//   * capture: a stream joins a capture by waiting on an event recorded in
//     it; at the end of the capture every joined stream must have been waited
//     on after its last captured work (no unjoined fork), no synchronisation
//     or copy may run on a capturing stream;
//   * graphs: launched only while instantiated, on a live stream that is not
//     capturing; an executable graph is destroyed only after its last launch
//     is known complete (its stream, an event recorded after it or the device
//     synchronised, or a free, which waits for the device).
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <vector>

#include <hip/hip_runtime.h>

namespace {

constexpr uint64_t STREAM_MAGIC = 0x53545245414d2121ull, EVENT_MAGIC = 0x4556454e54212121ull,
                   GRAPH_MAGIC = 0x4752415048212121ull, EXEC_MAGIC = 0x4558454321212121ull;

// Built on first use: the library's load-time registration of its
// __device__ variables can run before this file's static constructors.
// Never destroyed, so calls during process exit still find them.
std::recursive_mutex &mutex_instance()
{
    static std::recursive_mutex *m = new std::recursive_mutex;
    return *m;
}
std::map<uintptr_t, size_t> &memory_registry()  // live device allocations
{
    static std::map<uintptr_t, size_t> *m = new std::map<uintptr_t, size_t>;
    return *m;
}
#define g_mu mutex_instance()
#define g_mem memory_registry()
hipError_t g_last = hipSuccess;
size_t g_registered_vars = 0;  // entries of g_mem that are __device__ variables

[[noreturn]] void die(const char *what)
{
    fprintf(stderr, "hostcheck: %s\n", what);
    fflush(stderr);
    abort();
}

struct Capture;

// asynchronous copies and fills not yet done, in issue order
struct Pending {
    void *dst;
    const void *src;  // null: a fill with value v
    size_t n;
    int v;
};
std::vector<Pending> &pending_work()
{
    static std::vector<Pending> *q = new std::vector<Pending>;
    return *q;
}

// do every pending copy and fill (issue order is one valid order of the
// streams' work; doing other streams' work early only hides errors)
void drain()
{
    std::vector<Pending> q;
    q.swap(pending_work());
    for (const Pending &w : q) {
        if (w.src) memmove(w.dst, w.src, w.n);
        else memset(w.dst, w.v, w.n);
    }
}

}  // namespace

struct ihipStream_t {
    uint64_t magic;
    Capture *cap;        // capture this stream takes part in, or null
    long ops;            // work items enqueued (captured or not)
    long joined_at;      // ops count at the last join back into the origin
    long synced;         // ops count known complete (synchronised)
};

struct ihipEvent_t {
    uint64_t magic;
    ihipStream_t *src;   // stream of the last record (null: default stream)
    long seq;            // its ops count at that record
    Capture *cap;        // capture the record belongs to, or null
};

struct ihipGraph {
    uint64_t magic;
    long nodes;
};

struct hipGraphExec {
    uint64_t magic;
    long nodes;
    ihipStream_t *launch_stream;  // stream of the last launch not known complete, or null
    long launch_ops;              // that stream's ops count after the launch
    bool unknown;                 // launched on a stream destroyed before it was synchronised
};

namespace {

struct Capture {
    ihipStream_t *origin;
    std::set<ihipStream_t *> members;
    long nodes;
};

std::set<ihipStream_t *> &live_streams()
{
    static std::set<ihipStream_t *> *s = new std::set<ihipStream_t *>;
    return *s;
}
std::set<hipGraphExec *> &live_execs()
{
    static std::set<hipGraphExec *> *s = new std::set<hipGraphExec *>;
    return *s;
}

// everything issued so far is complete
void device_synced()
{
    for (ihipStream_t *q : live_streams()) q->synced = q->ops;
    for (hipGraphExec *x : live_execs()) { x->launch_stream = nullptr; x->unknown = false; }
}


void check_stream(hipStream_t s, const char *what)
{
    if (s && s->magic != STREAM_MAGIC) die(what);
}

void check_event(hipEvent_t e, const char *what)
{
    if (!e || e->magic != EVENT_MAGIC) die(what);
}

// inside one live allocation?
void check_range(const void *p, size_t n, const char *what)
{
    const uintptr_t a = (uintptr_t)p;
    auto it = g_mem.upper_bound(a);
    if (it == g_mem.begin()) die(what);
    --it;
    if (a < it->first || a + n > it->first + it->second) die(what);
}

bool is_device(const void *p)
{
    const uintptr_t a = (uintptr_t)p;
    auto it = g_mem.upper_bound(a);
    if (it == g_mem.begin()) return false;
    --it;
    return a >= it->first && a < it->first + it->second;
}

// one unit of work on s (a kernel, a copy, a fill, an event record)
void enqueue(hipStream_t s)
{
    if (!s) return;
    s->ops++;
    if (s->cap) s->cap->nodes++;
}

thread_local std::vector<std::pair<dim3, dim3>> t_cfg;
thread_local std::vector<hipStream_t> t_cfg_stream;

}  // namespace

extern "C" {

hipError_t hipMalloc(void **p, size_t n)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    if (!p) die("hipMalloc: null output");
    void *q = calloc(n ? n : 1, 1);
    if (!q) { *p = nullptr; return g_last = hipErrorOutOfMemory; }
    g_mem[(uintptr_t)q] = n ? n : 1;
    *p = q;
    return hipSuccess;
}

hipError_t hipFree(void *p)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    if (!p) return hipSuccess;
    auto it = g_mem.find((uintptr_t)p);
    if (it == g_mem.end()) die("hipFree of memory that is not a live device allocation");
    drain();  // hipFree waits for the device's work
    device_synced();
    it = g_mem.find((uintptr_t)p);
    g_mem.erase(it);
    free(p);
    return hipSuccess;
}

static hipError_t copy(void *dst, const void *src, size_t n, hipMemcpyKind k, hipStream_t s,
                       const char *who, bool sync)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    check_stream(s, "copy on a destroyed stream");
    if (s && s->cap) die("copy on a capturing stream");
    if (k == hipMemcpyHostToDevice || k == hipMemcpyDeviceToDevice) check_range(dst, n, who);
    if (k == hipMemcpyDeviceToHost || k == hipMemcpyDeviceToDevice) check_range(src, n, who);
    if (k == hipMemcpyHostToDevice && is_device(src)) die("host-to-device copy from device memory");
    if (k == hipMemcpyDeviceToHost && is_device(dst)) die("device-to-host copy into device memory");
    if (!sync) {
        if (n) pending_work().push_back(Pending{dst, src, n, 0});
    } else {
        drain();
        if (n) memmove(dst, src, n);
    }
    enqueue(s);
    return hipSuccess;
}

hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind k)
{
    return copy(dst, src, n, k, nullptr, "hipMemcpy outside a device allocation", true);
}

hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind k, hipStream_t s)
{
    return copy(dst, src, n, k, s, "hipMemcpyAsync outside a device allocation", false);
}

hipError_t hipMemsetAsync(void *dst, int v, size_t n, hipStream_t s)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    check_stream(s, "hipMemsetAsync on a destroyed stream");
    if (s && s->cap) die("hipMemsetAsync on a capturing stream");
    check_range(dst, n, "hipMemsetAsync outside a device allocation");
    if (n) pending_work().push_back(Pending{dst, nullptr, n, v});
    enqueue(s);
    return hipSuccess;
}

hipError_t hipDeviceSynchronize(void)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    drain();
    device_synced();
    return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t s)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    check_stream(s, "hipStreamSynchronize on a destroyed stream");
    if (s && s->cap) die("hipStreamSynchronize on a capturing stream");
    drain();
    if (s) {
        s->synced = s->ops;
        for (hipGraphExec *x : live_execs())
            if (x->launch_stream == s) x->launch_stream = nullptr;
    }
    return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    ihipStream_t *q = new ihipStream_t();
    q->magic = STREAM_MAGIC;
    live_streams().insert(q);
    *s = q;
    return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t s)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    check_stream(s, "hipStreamDestroy of a destroyed stream");
    if (!s) die("hipStreamDestroy of the default stream");
    if (s->cap) die("hipStreamDestroy of a capturing stream");
    // launches on it not known complete stay unknown (the device still runs them)
    for (hipGraphExec *x : live_execs())
        if (x->launch_stream == s) { x->launch_stream = nullptr; x->unknown = true; }
    live_streams().erase(s);
    s->magic = 0;
    delete s;
    return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    ihipEvent_t *q = new ihipEvent_t();
    q->magic = EVENT_MAGIC;
    *e = q;
    return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t *e) { return hipEventCreateWithFlags(e, 0); }

hipError_t hipEventDestroy(hipEvent_t e)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    check_event(e, "hipEventDestroy of a destroyed event");
    e->magic = 0;
    delete e;
    return hipSuccess;
}

hipError_t hipEventSynchronize(hipEvent_t e)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    check_event(e, "hipEventSynchronize of a destroyed event");
    if (e->cap) die("hipEventSynchronize of an event recorded in a capture");
    drain();
    if (e->src && live_streams().count(e->src)) {
        if (e->src->synced < e->seq) e->src->synced = e->seq;
        for (hipGraphExec *x : live_execs())
            if (x->launch_stream == e->src && x->launch_ops <= e->seq) x->launch_stream = nullptr;
    }
    return hipSuccess;
}

hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    check_event(a, "hipEventElapsedTime of a destroyed event");
    check_event(b, "hipEventElapsedTime of a destroyed event");
    *ms = 0.0f;
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    check_event(e, "hipEventRecord of a destroyed event");
    check_stream(s, "hipEventRecord on a destroyed stream");
    e->src = s;
    e->seq = s ? s->ops : 0;
    e->cap = s ? s->cap : nullptr;
    return hipSuccess;
}

hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    check_stream(s, "hipStreamWaitEvent on a destroyed stream");
    check_event(e, "hipStreamWaitEvent on a destroyed event");
    if (e->cap) {
        if (!s) die("default stream joins a capture");
        if (s->cap && s->cap != e->cap) die("stream waits on an event of another capture");
        if (!s->cap) {  // fork: s joins the capture
            s->cap = e->cap;
            e->cap->members.insert(s);
            s->joined_at = s->ops;
        }
        // join: the source stream's work up to the record is now ordered before s
        if (e->src && e->src != s && e->seq == e->src->ops) e->src->joined_at = e->src->ops;
    }
    return hipSuccess;
}

hipError_t hipStreamIsCapturing(hipStream_t s, hipStreamCaptureStatus *st)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    check_stream(s, "hipStreamIsCapturing on a destroyed stream");
    if (!st) die("hipStreamIsCapturing with a null argument");
    *st = (s && s->cap) ? hipStreamCaptureStatusActive : hipStreamCaptureStatusNone;
    return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    if (!s) return g_last = hipErrorStreamCaptureUnsupported;
    check_stream(s, "hipStreamBeginCapture on a destroyed stream");
    if (s->cap) die("nested capture");
    Capture *c = new Capture();
    c->origin = s;
    c->nodes = 0;
    c->members.insert(s);
    s->cap = c;
    return hipSuccess;
}

hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    check_stream(s, "hipStreamEndCapture on a destroyed stream");
    if (!s || !s->cap || s->cap->origin != s) die("hipStreamEndCapture without a capture");
    Capture *c = s->cap;
    bool unjoined = false;
    for (ihipStream_t *m : c->members) {
        check_stream(m, "a stream of the capture was destroyed during it");
        if (m != s && m->joined_at != m->ops) unjoined = true;
        m->cap = nullptr;
    }
    ihipGraph *q = new ihipGraph();
    q->magic = GRAPH_MAGIC;
    q->nodes = c->nodes;
    delete c;
    if (unjoined) {
        delete q;
        *g = nullptr;
        die("capture ended with a forked stream not joined back");
    }
    *g = q;
    return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, hipGraphNode_t *, char *, size_t)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    if (!g || g->magic != GRAPH_MAGIC) die("hipGraphInstantiate of a destroyed graph");
    hipGraphExec *q = new hipGraphExec();
    q->magic = EXEC_MAGIC;
    q->nodes = g->nodes;
    live_execs().insert(q);
    *x = q;
    return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t g)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    if (!g || g->magic != GRAPH_MAGIC) die("hipGraphDestroy of a destroyed graph");
    g->magic = 0;
    delete g;
    return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t x)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    if (!x || x->magic != EXEC_MAGIC) die("hipGraphExecDestroy of a destroyed graph");
    if (x->launch_stream || x->unknown)
        die("hipGraphExecDestroy of a graph whose last launch is not known complete");
    live_execs().erase(x);
    x->magic = 0;
    delete x;
    return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    if (!x || x->magic != EXEC_MAGIC) die("hipGraphLaunch of a destroyed graph");
    check_stream(s, "hipGraphLaunch on a destroyed stream");
    if (s && s->cap) die("hipGraphLaunch on a capturing stream");
    if (!s) die("hipGraphLaunch on the default stream");
    enqueue(s);
    x->launch_stream = s;
    x->launch_ops = s->ops;
    return hipSuccess;
}

hipError_t hipGetLastError(void)
{
    hipError_t e = g_last;
    g_last = hipSuccess;
    return e;
}

hipError_t hipGetDevice(int *d)
{
    if (!d) die("hipGetDevice with a null argument");
    *d = 0;
    return hipSuccess;
}

hipError_t hipGetSymbolAddress(void **p, const void *sym)
{
    if (!p || !sym) die("hipGetSymbolAddress with a null argument");
    *p = const_cast<void *>(sym);
    return hipSuccess;
}

const char *hipGetErrorString(hipError_t e)
{
    switch (e) {
    case hipSuccess: return "hipSuccess";
    case hipErrorOutOfMemory: return "hipErrorOutOfMemory";
    case hipErrorStreamCaptureUnsupported: return "hipErrorStreamCaptureUnsupported";
    default: return "hipError";
    }
}

unsigned __hipPushCallConfiguration(dim3 g, dim3 b, size_t, hipStream_t s)
{
    t_cfg.push_back(std::make_pair(g, b));
    t_cfg_stream.push_back(s);
    return 0;
}

hipError_t __hipPopCallConfiguration(dim3 *g, dim3 *b, size_t *shm, hipStream_t *s)
{
    if (t_cfg.empty()) die("launch configuration stack empty");
    *g = t_cfg.back().first;
    *b = t_cfg.back().second;
    *shm = 0;
    *s = t_cfg_stream.back();
    t_cfg.pop_back();
    t_cfg_stream.pop_back();
    return hipSuccess;
}

hipError_t hipLaunchKernel(const void *, dim3 g, dim3 b, void **, size_t, hipStream_t s)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    check_stream(s, "kernel launch on a destroyed stream");
    if (g.x == 0 || g.y == 0 || g.z == 0) die("kernel launch with an empty grid");
    if (g.y > 65535 || g.z > 65535) die("kernel launch with grid y or z above 65535");
    if ((unsigned long long)b.x * b.y * b.z > 1024 || b.x == 0) die("kernel launch with a bad block");
    enqueue(s);
    return hipSuccess;
}

// registration entry points that clang's host-side HIP code calls at load
void **__hipRegisterFatBinary(const void *) { static void *h = nullptr; return &h; }
void __hipRegisterFunction(void **, const void *, char *, const char *, int, void *, void *,
                           void *, void *, int *) {}
// a __device__ variable: its host shadow stands for the device copy
void __hipRegisterVar(void **, char *var, char *, const char *, int, size_t size, int, int)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    g_mem[(uintptr_t)var] = size;
    g_registered_vars++;
}
void __hipUnregisterFatBinary(void **) {}

// for the harness: live device allocations, and a stream it can hand to the
// library as a caller-owned one
size_t hostcheck_live_allocations(void)
{
    std::lock_guard<std::recursive_mutex> l(g_mu);
    return g_mem.size() - g_registered_vars;
}

}  // extern "C"
