// Stand-in runtime: allocation registry and range checks (host-logic test).
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <execinfo.h>
#include <unistd.h>
static std::map<uintptr_t, size_t>& reg() { static std::map<uintptr_t, size_t> r; return r; }
static std::mutex& mu() { static std::mutex m; return m; }
void emu_check(const void* p, size_t bytes, const char* what) {
  if (bytes == 0) return;
  std::lock_guard<std::mutex> lk(mu());
  uintptr_t a = reinterpret_cast<uintptr_t>(p);
  auto it = reg().upper_bound(a);
  if (it != reg().begin()) {
    --it;
    if (a >= it->first && a + bytes <= it->first + it->second) return;
    std::fprintf(stderr, "EMU OOB: %s [%p, +%zu) vs allocation [%p, +%zu)\n", what, p, bytes, (void*)it->first, it->second);
  } else {
    std::fprintf(stderr, "EMU OOB: %s [%p, +%zu) before any allocation\n", what, p, bytes);
  }
  void* bt[32];
  int nbt = backtrace(bt, 32);
  backtrace_symbols_fd(bt, nbt, 2);
  std::abort();
}
static void* alloc(size_t bytes) {
  void* p = std::malloc(bytes ? bytes : 1);
  std::memset(p, 0xA5, bytes);
  std::lock_guard<std::mutex> lk(mu());
  reg()[reinterpret_cast<uintptr_t>(p)] = bytes;
  return p;
}
static void release(void* p) {
  if (!p) return;
  { std::lock_guard<std::mutex> lk(mu());
    auto it = reg().find(reinterpret_cast<uintptr_t>(p));
    if (it == reg().end()) { std::fprintf(stderr, "EMU: free of unknown %p\n", p); std::abort(); }
    reg().erase(it); }
  std::free(p);
}
hipError_t hipMalloc(void** p, size_t bytes) { *p = alloc(bytes); return hipSuccess; }
hipError_t hipFree(void* p) { release(p); return hipSuccess; }
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) { *p = alloc(bytes); return hipSuccess; }
hipError_t hipHostFree(void* p) { release(p); return hipSuccess; }
hipError_t hipHostGetDevicePointer(void** d, void* h, unsigned) { emu_check(h, 1, "host pointer"); *d = h; return hipSuccess; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t bytes, hipMemcpyKind k, hipStream_t) {
  if (k != hipMemcpyDeviceToHost) emu_check(d, bytes, "memcpy dst");
  if (k != hipMemcpyHostToDevice) emu_check(s, bytes, "memcpy src");
  std::memmove(d, s, bytes); return hipSuccess; }
hipError_t hipMemcpy(void* d, const void* s, size_t bytes, hipMemcpyKind k) { return hipMemcpyAsync(d, s, bytes, k, nullptr); }
namespace kpp {
void emu_note_memset(const void* d);
}
hipError_t hipMemsetAsync(void* d, int v, size_t bytes, hipStream_t) {
  emu_check(d, bytes, "memset");
  std::memset(d, v, bytes);
  kpp::emu_note_memset(d);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
// launches run synchronously: a stream is always idle
hipError_t hipStreamQuery(hipStream_t) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* st, unsigned) { *st = reinterpret_cast<hipStream_t>(new char[8]); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t st) { delete[] reinterpret_cast<char*>(st); return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = reinterpret_cast<hipEvent_t>(new char[8]); return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete[] reinterpret_cast<char*>(e); return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0.01f; return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) { p->multiProcessorCount = 256; return hipSuccess; }
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) { *v = 100000; return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "emu error"; }
