// A host-only stand-in for the HIP runtime, linked with the library's objects
// in place of the real runtime (kernels are registered but never run) so that the request
// server's threads, admission, failure paths and clean-up run on the CPU
// under AddressSanitizer.  Device memory is host memory, copies are memcpy,
// kernel launches and graph replays do nothing.
//
// Kernel launches are logged by name (mock_launch_log).  Two behaviours are
// scripted:
//  * a 96-byte device-to-host copy is the CG solver reading its scalar state
//    (10 doubles, 4 int32): it reads back a converged state, so every solve
//    takes the capture -> replay -> confirm path and ends;
//  * MOCK_FAIL_COPY_EVERY=N makes every N-th host-to-device copy fail
//    (matrix uploads, request inputs), so that uploads fail part-way through
//    and requests fail while buffers are being filled.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

namespace {
thread_local int t_device = 0;

// host stub -> registered device name, and the names of launched kernels.
// Constructed on first use: the compiler's registration hooks run from other
// objects' static constructors, possibly before this file's globals exist.
struct Registry {
    std::mutex mu;
    std::map<const void *, std::string> names;
    std::string log;
};
Registry &registry() {
    static Registry *r = new Registry();
    return *r;
}

void record_launch(const void *f) {
    Registry &g = registry();
    std::lock_guard<std::mutex> lk(g.mu);
    auto it = g.names.find(f);
    g.log += it == g.names.end() ? std::string("?") : it->second;
    g.log += '\n';
}
std::atomic<long> n_h2d{0};

long fail_every() {
    static const long v = [] {
        const char *s = std::getenv("MOCK_FAIL_COPY_EVERY");
        return s ? std::atol(s) : 0L;
    }();
    return v;
}

void copy_bytes(void *d, const void *s, size_t n) {
    if (n) std::memcpy(d, s, n);
}
}  // namespace

extern "C" {
hipError_t hipMalloc(void **p, size_t n) {
    *p = std::calloc(1, n ? n : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipMallocAsync(void **p, size_t n, hipStream_t) { return hipMalloc(p, n); }
hipError_t hipFree(void *p) {
    std::free(p);
    return hipSuccess;
}
hipError_t hipFreeAsync(void *p, hipStream_t) { return hipFree(p); }
hipError_t hipHostMalloc(void **p, size_t n, unsigned int) { return hipMalloc(p, n); }
hipError_t hipHostFree(void *p) { return hipFree(p); }

static bool injected_failure(hipMemcpyKind k) {
    const long every = fail_every();
    return every > 0 && k == hipMemcpyHostToDevice && ++n_h2d % every == 0;
}

hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind k) {
    if (injected_failure(k)) return hipErrorOutOfMemory;
    copy_bytes(d, s, n);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t) {
    if (injected_failure(k)) return hipErrorOutOfMemory;
    copy_bytes(d, s, n);
    if (k == hipMemcpyDeviceToHost && n == 96) {  // the CG scalar state
        double *v = static_cast<double *>(d);
        v[0] = 1.0;  // rho
        v[5] = 1.0;  // |b|^2
        v[6] = 0.5;  // tol^2 |b|^2
        v[7] = 0.1;  // true residual^2
        int32_t *w = reinterpret_cast<int32_t *>(v + 10);
        w[0] = 3;  // iterations
        w[2] = 1;  // done
        w[3] = 1;  // converged
    }
    return hipSuccess;
}
hipError_t hipMemset(void *d, int v, size_t n) {
    std::memset(d, v, n);
    return hipSuccess;
}
hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t) { return hipMemset(d, v, n); }

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int) {
    *s = reinterpret_cast<hipStream_t>(new int(1));
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    delete reinterpret_cast<int *>(s);
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipExtStreamCreateWithCUMask(hipStream_t *s, uint32_t, const uint32_t *) {
    return hipStreamCreateWithFlags(s, 0);
}
hipError_t hipDeviceSynchronize(void) { return hipSuccess; }
hipError_t hipHostGetDevicePointer(void **d, void *h, unsigned int) {
    *d = h;
    return hipSuccess;
}
// events exist but time nothing: every interval reads zero
hipError_t hipEventCreate(hipEvent_t *e) {
    *e = reinterpret_cast<hipEvent_t>(new int(4));
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
    delete reinterpret_cast<int *>(e);
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned int) { return hipEventCreate(e); }
hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) {
    *ms = 0.0f;
    return hipSuccess;
}
hipError_t hipGetDevice(int *d) {
    *d = t_device;
    return hipSuccess;
}
hipError_t hipSetDevice(int d) {
    t_device = d;
    return hipSuccess;
}
hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipPointerGetAttributes(hipPointerAttribute_t *a, const void *p) {  // all memory is "device" here
    *a = hipPointerAttribute_t{};
    a->type = hipMemoryTypeDevice;
    a->devicePointer = const_cast<void *>(p);
    return hipSuccess;
}
const char *hipGetErrorString(hipError_t) { return "mock runtime error"; }
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t, int) {
    *v = 256;
    return hipSuccess;
}
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *n, const void *, int, size_t) {
    *n = 8;
    return hipSuccess;
}
hipError_t hipFuncSetAttribute(const void *, hipFuncAttribute, int) { return hipSuccess; }
// a device variable's address is its host shadow here (device memory is host memory)
hipError_t hipGetSymbolAddress(void **p, const void *symbol) {
    *p = const_cast<void *>(symbol);
    return hipSuccess;
}
// kernel launches are recorded by the device name the compiler registered
// for the host stub (mock_launch_log), so a driver can check which kernels a
// call launched
hipError_t hipLaunchKernel(const void *f, dim3, dim3, void **, size_t, hipStream_t) {
    record_launch(f);
    return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) {
    *g = reinterpret_cast<hipGraph_t>(new int(2));
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t, hipGraphNode_t *, char *, size_t) {
    *e = reinterpret_cast<hipGraphExec_t>(new int(3));
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
    delete reinterpret_cast<int *>(e);
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    delete reinterpret_cast<int *>(g);
    return hipSuccess;
}

// registration hooks that compiler-generated host code calls
void **__hipRegisterFatBinary(const void *) {
    static void *handle = nullptr;
    return &handle;
}
void __hipRegisterFunction(void **, const void *host, char *, const char *name, unsigned int, void *, void *, dim3 *,
                           dim3 *, int *) {
    Registry &g = registry();
    std::lock_guard<std::mutex> lk(g.mu);
    g.names[host] = name ? name : "";
}

// Mangled device names of the kernels launched since the last call, one per
// line; the log is cleared.  The returned buffer is valid until the next call.
const char *mock_launch_log(void) {
    static std::string out;
    Registry &g = registry();
    std::lock_guard<std::mutex> lk(g.mu);
    out.swap(g.log);
    g.log.clear();
    return out.c_str();
}
void __hipUnregisterFatBinary(void **) {}
void __hipRegisterVar(void **, void *, char *, const char *, int, size_t, int, int) {}
hipError_t __hipPushCallConfiguration(dim3, dim3, size_t, hipStream_t) { return hipSuccess; }
hipError_t __hipPopCallConfiguration(dim3 *, dim3 *, size_t *, hipStream_t *) { return hipSuccess; }
}
