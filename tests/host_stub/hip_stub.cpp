// A stand-in for the HIP runtime, for checking the library's host code on a machine without a
// GPU (built with AddressSanitizer and UBSan together with a host-only build of the library).
//
// Device memory is host memory, tracked so that every copy is range-checked against a live
// allocation; kernel launches are validated (non-empty grid, block and dynamic LDS limits, no
// launch configuration left unconsumed) and counted but run nothing; graph capture is tracked
// (a copy or a synchronisation during a capture is an error); event timings are pseudo-random,
// which walks the autotuner through its choices.  Any violation aborts with a message.
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

namespace {

std::mutex mu;
std::map<char *, size_t> dev_allocs;     // device allocations (and the scratch symbol)
std::map<char *, size_t> pinned_allocs;  // pinned host allocations
std::map<const void *, size_t> vars;     // registered device variables
hipError_t last = hipSuccess;
unsigned long long rng = 88172645463325252ull;
long long n_launch = 0, n_alloc = 0, n_free = 0;
bool capturing = false;
size_t lds_limit = 65536;

struct Cfg {
    dim3 g, b;
    size_t sh;
    hipStream_t s;
};
std::vector<Cfg> cfgs;

[[noreturn]] void die(const char *msg, const void *p = nullptr, size_t n = 0) {
    fprintf(stderr, "HIP STUB VIOLATION: %s (%p, %zu)\n", msg, p, n);
    fflush(stderr);
    abort();
}

bool inside(const std::map<char *, size_t> &m, const void *p, size_t n) {
    std::lock_guard<std::mutex> l(mu);
    char *c = (char *)p;
    auto it = m.upper_bound(c);
    if (it == m.begin()) return false;
    --it;
    return c >= it->first && c + n <= it->first + it->second;
}

struct Obj {
    int tag;
};

}  // namespace

// ------------------------------------------------------------------ registration (host-only objects)
extern "C" {
void **__hipRegisterFatBinary(const void *) {
    static void *h = nullptr;
    return &h;
}
void __hipUnregisterFatBinary(void **) {}
void __hipRegisterFunction(void **, const void *, char *, const char *, unsigned int, void *, void *, dim3 *, dim3 *,
                           int *) {}
void __hipRegisterVar(void **, char *var, char *, const char *, int, size_t size, int, int) {
    std::lock_guard<std::mutex> l(mu);
    vars[var] = size;
}
long long hip_stub_launches() { return n_launch; }
long long hip_stub_allocations() { return n_alloc + n_free; }
}

// ------------------------------------------------------------------ launches
hipError_t __hipPushCallConfiguration(dim3 g, dim3 b, size_t sh, hipStream_t s) {
    cfgs.push_back({g, b, sh, s});
    return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3 *g, dim3 *b, size_t *sh, hipStream_t *s) {
    if (cfgs.empty()) die("launch configuration popped without a push");
    const Cfg c = cfgs.back();
    cfgs.pop_back();
    *g = c.g;
    *b = c.b;
    *sh = c.sh;
    *s = c.s;
    return hipSuccess;
}
hipError_t hipLaunchKernel(const void *f, dim3 g, dim3 b, void **args, size_t sh, hipStream_t) {
    if (!f || !args) die("launch of a null kernel or without arguments");
    if (!cfgs.empty()) die("launch configuration left on the stack", nullptr, cfgs.size());
    const unsigned long long blocks = (unsigned long long)g.x * g.y * g.z;
    const unsigned threads = b.x * b.y * b.z;
    if (blocks == 0) die("launch with an empty grid");
    if (g.y > 65535 || g.z > 65535) die("grid y or z above 65535", nullptr, g.y);
    if (threads == 0 || threads > 1024) die("block size outside [1, 1024]", nullptr, threads);
    if (blocks * threads >= (1ull << 32)) die("2^32 or more work items", nullptr, blocks);
    if (sh > lds_limit) die("dynamic LDS above the budget", nullptr, sh);
    ++n_launch;
    return hipSuccess;
}
hipError_t hipGetLastError() {
    const hipError_t e = last;
    last = hipSuccess;
    return e;
}
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "stub error"; }

// ------------------------------------------------------------------ device
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetDevice(int *d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipGetDeviceCount(int *c) {
    *c = 1;
    return hipSuccess;
}
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600 *p, int) {
    memset(p, 0, sizeof(*p));
    strcpy(p->name, "host stub");
    p->multiProcessorCount = 256;
    p->warpSize = 64;
    p->totalGlobalMem = 288ull << 30;
    p->sharedMemPerBlock = 160 * 1024;
    return hipSuccess;
}
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *n, const void *, int, size_t lds) {
    *n = lds > 32768 ? 1 : 4;
    return hipSuccess;
}

// ------------------------------------------------------------------ memory
hipError_t hipMalloc(void **p, size_t n) {
    if (capturing) die("allocation during a graph capture");
    const size_t cap = (n + 255) / 256 * 256 + 256;
    void *q = aligned_alloc(256, cap);
    memset(q, 0, cap);
    std::lock_guard<std::mutex> l(mu);
    dev_allocs[(char *)q] = n;
    ++n_alloc;
    *p = q;
    return hipSuccess;
}
hipError_t hipFree(void *p) {
    if (!p) return hipSuccess;
    std::lock_guard<std::mutex> l(mu);
    auto it = dev_allocs.find((char *)p);
    if (it == dev_allocs.end()) die("hipFree of a pointer that is not a live allocation", p);
    dev_allocs.erase(it);
    ++n_free;
    free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t n, unsigned) {
    void *q = malloc(n);
    std::lock_guard<std::mutex> l(mu);
    pinned_allocs[(char *)q] = n;
    ++n_alloc;
    *p = q;
    return hipSuccess;
}
hipError_t hipHostFree(void *p) {
    std::lock_guard<std::mutex> l(mu);
    auto it = pinned_allocs.find((char *)p);
    if (it == pinned_allocs.end()) die("hipHostFree of a pointer that is not a pinned allocation", p);
    pinned_allocs.erase(it);
    ++n_free;
    free(p);
    return hipSuccess;
}
static hipError_t copy(void *dst, const void *src, size_t n, hipMemcpyKind k) {
    if (n == 0) return hipSuccess;
    if (capturing) die("copy during a graph capture", dst, n);
    if (k == hipMemcpyHostToDevice && !inside(dev_allocs, dst, n)) die("host-to-device copy outside device memory", dst, n);
    if (k == hipMemcpyDeviceToHost && !inside(dev_allocs, src, n)) die("device-to-host copy outside device memory", src, n);
    if (k == hipMemcpyDeviceToDevice && (!inside(dev_allocs, src, n) || !inside(dev_allocs, dst, n)))
        die("device-to-device copy outside device memory", dst, n);
    memcpy(dst, src, n);
    return hipSuccess;
}
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind k) { return copy(d, s, n, k); }
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t) {
    if (k == hipMemcpyHostToDevice && !inside(pinned_allocs, s, n)) die("asynchronous upload from pageable memory", s, n);
    if (k == hipMemcpyDeviceToHost && n > 4096 && !inside(pinned_allocs, d, n))
        fprintf(stderr, "hip stub note: asynchronous download of %zu bytes to pageable memory\n", n);
    return copy(d, s, n, k);
}
hipError_t hipGetSymbolAddress(void **p, const void *sym) {
    std::lock_guard<std::mutex> l(mu);
    auto it = vars.find(sym);
    const size_t n = it == vars.end() ? (size_t)64 << 20 : it->second;  // host-only objects register none
    void *q = aligned_alloc(256, (n + 255) / 256 * 256);
    dev_allocs[(char *)q] = n;
    *p = q;
    return hipSuccess;
}

// ------------------------------------------------------------------ streams, events, graphs
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
    *s = (hipStream_t) new Obj{1};
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    delete (Obj *)s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) {
    if (capturing) die("stream synchronisation during a graph capture");
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t e, unsigned) {
    if (!e) die("wait on a null event");
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) {
    *e = (hipEvent_t) new Obj{2};
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
    delete (Obj *)e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
    if (!e) die("record of a null event");
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
    if (!e) die("query of a null event");
    // work is sometimes still pending on a real device: report it now and then, so that the
    // callers' paths for an unfinished upload (a new staging buffer, a wait) run too
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return rng % 3 == 0 ? hipErrorNotReady : hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
    if (!e) die("synchronisation on a null event");
    if (capturing) die("event synchronisation during a graph capture");
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
    if (!a || !b) die("elapsed time of a null event");
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    *ms = 1.f + (float)(rng % 1000) / 1000.f;
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) {
    if (capturing) die("nested graph capture");
    capturing = true;
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) {
    if (!capturing) die("end of a capture that did not begin");
    capturing = false;
    *g = (hipGraph_t) new Obj{3};
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, hipGraphNode_t *, char *, size_t) {
    if (!g) die("instantiation of a null graph");
    *x = (hipGraphExec_t) new Obj{4};
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    delete (Obj *)g;
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
    delete (Obj *)x;
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t) {
    if (!x) die("launch of a null graph");
    if (capturing) die("graph launch during a capture");
    return hipSuccess;
}
