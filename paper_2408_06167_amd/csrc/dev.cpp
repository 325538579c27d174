// dev.cpp -- the library's HIP runtime calls, with a CPU-only dry-run mode
// (BM_DRY_RUN=1) that keeps every launch check but touches no GPU.
#include <atomic>
#include <cstdlib>
#include <cstring>

#include "bm_internal.hpp"

namespace bm {
namespace dev {

namespace {
thread_local int g_sizing = 0;
}

bool sizing() { return g_sizing > 0; }
SizingScope::SizingScope() { ++g_sizing; }
SizingScope::~SizingScope() { --g_sizing; }

bool dry() {
  static const bool d = [] {
    const char* e = std::getenv("BM_DRY_RUN");
    return e && e[0] == '1';
  }();
  return d;
}

hipError_t malloc_raw(void** p, size_t bytes) {
  if (dry()) {
    *p = std::malloc(bytes ? bytes : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

hipError_t free(void* p) {
  if (dry()) {
    std::free(p);
    return hipSuccess;
  }
  return hipFree(p);
}

hipError_t memcpy(void* d, const void* s, size_t bytes, hipMemcpyKind k) {
  if (dry()) {
    std::memmove(d, s, bytes);
    return hipSuccess;
  }
  return hipMemcpy(d, s, bytes, k);
}

hipError_t memcpy_async(void* d, const void* s, size_t bytes, hipMemcpyKind k, hipStream_t st) {
  if (sizing()) return hipSuccess;
  if (dry()) {
    std::memmove(d, s, bytes);
    return hipSuccess;
  }
  return hipMemcpyAsync(d, s, bytes, k, st);
}

hipError_t stream_sync(hipStream_t s) { return dry() || sizing() ? hipSuccess : hipStreamSynchronize(s); }
hipError_t device_sync() { return dry() ? hipSuccess : hipDeviceSynchronize(); }

hipError_t stream_create(hipStream_t* s) {
  if (dry()) {
    static std::atomic<uintptr_t> next{0x1000};
    *s = (hipStream_t)(next += 16);
    return hipSuccess;
  }
  return hipStreamCreateWithFlags(s, hipStreamNonBlocking);
}

hipError_t stream_destroy(hipStream_t s) { return dry() ? hipSuccess : hipStreamDestroy(s); }

hipError_t set_device(int d) { return dry() ? hipSuccess : hipSetDevice(d); }

hipError_t event_create(hipEvent_t* e, bool timing) {
  if (dry()) {
    static std::atomic<uintptr_t> next{0x100000};
    *e = (hipEvent_t)(next += 16);
    return hipSuccess;
  }
  return timing ? hipEventCreate(e) : hipEventCreateWithFlags(e, hipEventDisableTiming);
}

hipError_t event_destroy(hipEvent_t e) { return dry() ? hipSuccess : hipEventDestroy(e); }
hipError_t event_record(hipEvent_t e, hipStream_t s) {
  return dry() || sizing() ? hipSuccess : hipEventRecord(e, s);
}
hipError_t event_sync(hipEvent_t e) { return dry() ? hipSuccess : hipEventSynchronize(e); }

hipError_t event_elapsed(float* ms, hipEvent_t a, hipEvent_t b) {
  if (dry()) {
    *ms = 0.f;
    return hipSuccess;
  }
  return hipEventElapsedTime(ms, a, b);
}

hipError_t event_query(hipEvent_t e) { return dry() ? hipSuccess : hipEventQuery(e); }
hipError_t last_error() { return dry() || sizing() ? hipSuccess : hipGetLastError(); }

hipError_t begin_capture(hipStream_t s) {
  return dry() ? hipSuccess : hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
}

hipError_t end_capture(hipStream_t s, hipGraph_t* g) {
  if (dry()) {
    *g = (hipGraph_t)0x1;
    return hipSuccess;
  }
  return hipStreamEndCapture(s, g);
}

hipError_t graph_instantiate(hipGraphExec_t* e, hipGraph_t g) {
  if (dry()) {
    static std::atomic<uintptr_t> next{0x200000};
    *e = (hipGraphExec_t)(next += 16);
    return hipSuccess;
  }
  return hipGraphInstantiate(e, g, nullptr, nullptr, 0);
}

hipError_t graph_destroy(hipGraph_t g) { return dry() ? hipSuccess : hipGraphDestroy(g); }
hipError_t graph_launch(hipGraphExec_t e, hipStream_t s) { return dry() ? hipSuccess : hipGraphLaunch(e, s); }

}  // namespace dev
}  // namespace bm
