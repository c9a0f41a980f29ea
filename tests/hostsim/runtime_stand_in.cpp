// Test double of the HIP runtime (see hip/hip_runtime_api.h in this folder).
#include <hip/hip_runtime_api.h>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
static int dummy_obj;
// With HOSTSIM_STREAM set, every stream handle that reaches the runtime must
// be NULL or exactly that value: a handle cut to 32 bits on its way through
// the binding aborts the run.
void hostsim_check_stream(hipStream_t s)
{
    static const char* want = std::getenv("HOSTSIM_STREAM");
    if (!want || !s) return;
    const unsigned long long w = std::strtoull(want, nullptr, 0);
    if ((unsigned long long)(uintptr_t)s != w) {
        std::fprintf(stderr, "hostsim: stream handle %p reached the runtime, expected %#llx\n", (void*)s, w);
        std::abort();
    }
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
hipError_t hipMalloc(void** p, size_t n) { *p = std::malloc(n ? n : 1); return *p ? hipSuccess : hipErrorOutOfMemory; }
hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
hipError_t hipHostMalloc(void** p, size_t n, unsigned) { *p = std::malloc(n ? n : 1); return *p ? hipSuccess : hipErrorOutOfMemory; }
hipError_t hipHostFree(void* p) { std::free(p); return hipSuccess; }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { std::memcpy(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t st) { hostsim_check_stream(st); std::memcpy(d, s, n); return hipSuccess; }
hipError_t hipMemset(void* p, int v, size_t n) { std::memset(p, v, n); return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t st) { hostsim_check_stream(st); return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = (hipEvent_t)&dummy_obj; return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = (hipEvent_t)&dummy_obj; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t st) { hostsim_check_stream(st); return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0.f; return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t st, hipStreamCaptureMode) { hostsim_check_stream(st); return hipSuccess; }
hipError_t hipStreamIsCapturing(hipStream_t st, hipStreamCaptureStatus* s) { hostsim_check_stream(st); *s = hipStreamCaptureStatusNone; return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t st, hipEvent_t, unsigned int) { hostsim_check_stream(st); return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) { *g = (hipGraph_t)&dummy_obj; return hipSuccess; }
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t, hipGraphNode_t*, char*, size_t) { *x = (hipGraphExec_t)&dummy_obj; return hipSuccess; }
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t st) { hostsim_check_stream(st); return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "fake"; }
hipError_t hipGetLastError() { return hipSuccess; }
