// Host-only stand-in for the HIP runtime calls the library makes, for the CPU sanitizer check of the
// library's host code (tests/test_host_sanitizer.py); test infrastructure, not linked into the library.
// Device memory is calloc'd host memory kept in a registry, so that copies and frees are checked against
// live allocations; streams, events and graphs are bookkeeping objects (capture forks and joins tracked);
// kernel launches check their shape and do nothing. Calls that HIP forbids while a stream is capturing
// (allocation, synchronization, host copies) are reported as errors.
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>

struct ihipStream_t {
    int capturing = 0;       // 0 none, else capture id
    int origin = 0;          // 1 on the stream that began the capture
    long ops = 0;            // work enqueued during the current capture
    long joined_at = 0;      // ops covered by an event some other capturing stream waited on
};
struct ihipEvent_t {
    int captured_in = 0;     // capture id of the stream it was last recorded on (0: not capturing)
    bool recorded = false;
    ihipStream_t* src = nullptr;
    long ops = 0;
};
struct ihipGraph { int id; };
struct hipGraphExec { int id; };

static std::mutex mu;
static std::map<char*, size_t> allocs;
static std::set<ihipStream_t*> streams;
static std::set<ihipEvent_t*> events;
static std::set<ihipGraph*> graphs;
static std::set<hipGraphExec*> execs;
static int next_capture = 1;
static long n_launch = 0, n_bad = 0, n_capture = 0, n_glaunch = 0, n_inst = 0, n_streams = 0;

static void bad(const char* what) {
    ++n_bad;
    fprintf(stderr, "[hip-stub] ERROR: %s\n", what);
}
static bool any_capturing() {
    for (auto* s : streams)
        if (s->capturing) return true;
    return false;
}
// a device pointer range [p, p + n) must lie in one live allocation; returns false for host memory
static bool dev_range(const void* p, size_t n, const char* what) {
    char* c = (char*)p;
    auto it = allocs.upper_bound(c);
    if (it == allocs.begin()) return false;
    --it;
    if (c >= it->first && c < it->first + it->second) {
        if (c + n > it->first + it->second) {
            char msg[256];
            snprintf(msg, sizeof msg, "%s: range of %zu bytes at offset %zu past an allocation of %zu", what, n,
                     (size_t)(c - it->first), it->second);
            bad(msg);
        }
        return true;
    }
    return false;
}
static ihipStream_t null_stream;
static ihipStream_t* S(hipStream_t s) { return s ? s : &null_stream; }
static bool valid_stream(hipStream_t s) { return s == nullptr || streams.count(s); }

extern "C" {

hipError_t hipMalloc(void** p, size_t n) {
    std::lock_guard<std::mutex> g(mu);
    if (any_capturing()) bad("hipMalloc while a stream is capturing");
    if (n == 0) { *p = nullptr; return hipSuccess; }
    void* q = calloc(1, n);
    if (!q) return hipErrorOutOfMemory;
    allocs[(char*)q] = n;
    *p = q;
    return hipSuccess;
}
hipError_t hipFree(void* p) {
    std::lock_guard<std::mutex> g(mu);
    if (any_capturing()) bad("hipFree while a stream is capturing");
    if (!p) return hipSuccess;
    auto it = allocs.find((char*)p);
    if (it == allocs.end()) { bad("hipFree of a pointer that is not a live allocation"); return hipErrorInvalidValue; }
    allocs.erase(it);
    free(p);
    return hipSuccess;
}
static hipError_t copy(void* dst, const void* src, size_t n, hipMemcpyKind kind, const char* what) {
    const bool dd = dev_range(dst, n, what), sd = dev_range(src, n, what);
    if ((kind == hipMemcpyHostToDevice || kind == hipMemcpyDeviceToDevice) && !dd && n) bad("copy to a non-device pointer");
    if ((kind == hipMemcpyDeviceToHost || kind == hipMemcpyDeviceToDevice) && !sd && n) bad("copy from a non-device pointer");
    if (n) memmove(dst, src, n);
    return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind kind) {
    std::lock_guard<std::mutex> g(mu);
    if (any_capturing()) bad("synchronous hipMemcpy while a stream is capturing");
    return copy(dst, src, n, kind, "hipMemcpy");
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind kind, hipStream_t s) {
    std::lock_guard<std::mutex> g(mu);
    if (!valid_stream(s)) bad("hipMemcpyAsync on a destroyed stream");
    if (S(s)->capturing && kind != hipMemcpyDeviceToDevice) bad("host copy recorded into a capture");
    if (!S(s)->capturing && any_capturing() && s == nullptr) bad("null-stream copy while capturing");
    if (S(s)->capturing) ++S(s)->ops;
    return copy(dst, src, n, kind, "hipMemcpyAsync");
}
hipError_t hipMemGetInfo(size_t* f, size_t* t) {
    *f = 200ull << 30;
    *t = 288ull << 30;
    return hipSuccess;
}
hipError_t hipStreamCreate(hipStream_t* s) {
    std::lock_guard<std::mutex> g(mu);
    *s = new ihipStream_t();
    ++n_streams;
    streams.insert(*s);
    return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) { return hipStreamCreate(s); }
hipError_t hipStreamDestroy(hipStream_t s) {
    std::lock_guard<std::mutex> g(mu);
    if (!streams.count(s)) { bad("hipStreamDestroy of an unknown stream"); return hipErrorInvalidValue; }
    if (s->capturing) bad("hipStreamDestroy of a capturing stream");
    streams.erase(s);
    delete s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
    std::lock_guard<std::mutex> g(mu);
    if (!valid_stream(s)) bad("hipStreamSynchronize on a destroyed stream");
    if (any_capturing()) bad("hipStreamSynchronize while a stream is capturing");
    return hipSuccess;
}
hipError_t hipDeviceSynchronize() {
    std::lock_guard<std::mutex> g(mu);
    if (any_capturing()) bad("hipDeviceSynchronize while a stream is capturing");
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
    std::lock_guard<std::mutex> g(mu);
    if (!valid_stream(s)) bad("hipStreamWaitEvent on a destroyed stream");
    if (!events.count(e)) { bad("hipStreamWaitEvent on an unknown event"); return hipErrorInvalidValue; }
    if (e->captured_in) {
        if (S(s)->capturing && S(s)->capturing != e->captured_in) bad("wait joins two different captures");
        if (!S(s)->capturing) {                                   // fork: the stream joins the capture
            S(s)->capturing = e->captured_in;
            S(s)->ops = 0;
            S(s)->joined_at = 0;
        }
        if (e->src && e->src != S(s) && e->ops > e->src->joined_at) e->src->joined_at = e->ops;
    } else if (S(s)->capturing) {
        // waiting on an event recorded outside the capture is allowed (an external dependency)
    }
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    std::lock_guard<std::mutex> g(mu);
    if (!valid_stream(s) || s == nullptr) { bad("capture on the null or a destroyed stream"); return hipErrorInvalidValue; }
    if (s->capturing) { bad("hipStreamBeginCapture on a capturing stream"); return hipErrorIllegalState; }
    s->capturing = next_capture++;
    ++n_capture;
    s->origin = 1;
    s->ops = 0;
    s->joined_at = 0;
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* gr) {
    std::lock_guard<std::mutex> g(mu);
    if (!valid_stream(s) || !s || !s->capturing || !s->origin) { bad("hipStreamEndCapture without a capture"); return hipErrorIllegalState; }
    const int id = s->capturing;
    for (auto* o : streams)
        if (o != s && o->capturing == id && o->ops > o->joined_at) {
            char msg[160];
            snprintf(msg, sizeof msg, "capture ended with a forked stream not joined back (%ld ops, joined at %ld)",
                     o->ops, o->joined_at);
            bad(msg);
        }
    for (auto* o : streams)
        if (o->capturing == id) { o->capturing = 0; o->origin = 0; o->ops = 0; o->joined_at = 0; }
    for (auto* e : events)
        if (e->captured_in == id) e->captured_in = 0;
    auto* G = new ihipGraph{id};
    graphs.insert(G);
    *gr = G;
    return hipSuccess;
}
hipError_t hipStreamIsCapturing(hipStream_t s, hipStreamCaptureStatus* st) {
    std::lock_guard<std::mutex> g(mu);
    if (!valid_stream(s)) bad("hipStreamIsCapturing on a destroyed stream");
    *st = S(s)->capturing ? hipStreamCaptureStatusActive : hipStreamCaptureStatusNone;
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
    std::lock_guard<std::mutex> g(mu);
    *e = new ihipEvent_t();
    events.insert(*e);
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
    std::lock_guard<std::mutex> g(mu);
    if (!events.count(e)) { bad("hipEventDestroy of an unknown event"); return hipErrorInvalidValue; }
    events.erase(e);
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    std::lock_guard<std::mutex> g(mu);
    if (!events.count(e)) { bad("hipEventRecord of an unknown event"); return hipErrorInvalidValue; }
    if (!valid_stream(s)) bad("hipEventRecord on a destroyed stream");
    if (!S(s)->capturing && any_capturing() && s == nullptr) bad("null-stream event record while capturing");
    e->captured_in = S(s)->capturing;
    e->recorded = true;
    e->src = S(s);
    e->ops = S(s)->ops;
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
    std::lock_guard<std::mutex> g(mu);
    if (!events.count(e)) { bad("hipEventSynchronize of an unknown event"); return hipErrorInvalidValue; }
    if (any_capturing()) bad("hipEventSynchronize while a stream is capturing");
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
    std::lock_guard<std::mutex> g(mu);
    if (!events.count(a) || !events.count(b)) { bad("hipEventElapsedTime of an unknown event"); return hipErrorInvalidValue; }
    if (!a->recorded || !b->recorded) bad("hipEventElapsedTime of an event never recorded");
    *ms = 1.0f;
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t gr, hipGraphNode_t*, char*, size_t) {
    std::lock_guard<std::mutex> g(mu);
    if (!graphs.count(gr)) { bad("hipGraphInstantiate of an unknown graph"); return hipErrorInvalidValue; }
    ++n_inst;
    auto* X = new hipGraphExec{gr->id};
    execs.insert(X);
    *x = X;
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
    std::lock_guard<std::mutex> g(mu);
    if (!execs.count(x)) { bad("hipGraphLaunch of an unknown executable graph"); return hipErrorInvalidValue; }
    ++n_glaunch;
    if (!valid_stream(s)) bad("hipGraphLaunch on a destroyed stream");
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
    std::lock_guard<std::mutex> g(mu);
    if (!execs.count(x)) { bad("hipGraphExecDestroy of an unknown executable graph"); return hipErrorInvalidValue; }
    execs.erase(x);
    delete x;
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t gr) {
    std::lock_guard<std::mutex> g(mu);
    if (!graphs.count(gr)) { bad("hipGraphDestroy of an unknown graph"); return hipErrorInvalidValue; }
    graphs.erase(gr);
    delete gr;
    return hipSuccess;
}
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
    *v = a == hipDeviceAttributeMultiprocessorCount ? 256 : 0;
    return hipSuccess;
}
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "hip-stub error"; }
hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* nb, const void*, int, size_t) {
    *nb = 2;
    return hipSuccess;
}
static char* symbol_mem = nullptr;
hipError_t hipGetSymbolAddress(void** p, const void*) {
    std::lock_guard<std::mutex> g(mu);
    if (!symbol_mem) {
        symbol_mem = (char*)calloc(1, 64ull << 20);
        allocs[symbol_mem] = 64ull << 20;
    }
    *p = symbol_mem;
    return hipSuccess;
}

static dim3 cfg_grid, cfg_block;
static size_t cfg_shm;
static hipStream_t cfg_stream;
hipError_t __hipPushCallConfiguration(dim3 grid, dim3 block, size_t shm, hipStream_t s) {
    cfg_grid = grid; cfg_block = block; cfg_shm = shm; cfg_stream = s;
    return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3* grid, dim3* block, size_t* shm, hipStream_t* s) {
    *grid = cfg_grid; *block = cfg_block; *shm = cfg_shm; *s = cfg_stream;
    return hipSuccess;
}
hipError_t hipLaunchKernel(const void*, dim3 grid, dim3 block, void**, size_t shm, hipStream_t s) {
    std::lock_guard<std::mutex> g(mu);
    ++n_launch;
    if (!valid_stream(s)) bad("kernel launched on a destroyed stream");
    if (grid.x == 0 || grid.y == 0 || grid.z == 0) bad("kernel launched with an empty grid");
    if ((unsigned long)block.x * block.y * block.z > 1024 || block.x == 0) bad("kernel launched with a bad block");
    if (shm > 160 * 1024) bad("kernel launched with too much dynamic LDS");
    if (!S(s)->capturing && any_capturing() && s == nullptr) bad("null-stream launch while capturing");
    if (S(s)->capturing) ++S(s)->ops;
    return hipSuccess;
}
void** __hipRegisterFatBinary(const void*) {
    static void* handle = nullptr;
    return &handle;
}
void __hipRegisterFunction(void**, const void*, char*, const char*, unsigned int, uint3*, uint3*, dim3*, dim3*, int*) {}
void __hipRegisterVar(void**, void*, char*, char*, int, size_t, int, int) {}
void __hipUnregisterFatBinary(void**) {}

long hip_stub_launches() { return n_launch; }
void hip_stub_report() {
    printf("[hip-stub] captures %ld, instantiations %ld, graph launches %ld, streams created %ld\n", n_capture,
            n_inst, n_glaunch, n_streams);
}
long hip_stub_errors() { return n_bad; }
size_t hip_stub_live_allocs() { return allocs.size(); }
}
