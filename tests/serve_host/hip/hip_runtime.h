// Host stand-in (tests only) for the parts of the HIP runtime that serve.cpp calls.  Copies are
// queued per stream and run when the stream is synchronized (or by a later device
// operation on that stream), so a source buffer freed or reused before then is read
// after the fact, which AddressSanitizer reports.
#pragma once
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>
typedef int hipError_t;
constexpr hipError_t hipSuccess = 0;
enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2 };
constexpr unsigned hipHostMallocDefault = 0, hipStreamNonBlocking = 1;
struct StubCopy { void* dst; const void* src; size_t n; };
struct StubStream { std::mutex mu; std::vector<StubCopy> q; };
typedef StubStream* hipStream_t;
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = new StubStream(); return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t s) {
  std::lock_guard<std::mutex> lk(s->mu);
  for (auto& c : s->q) std::memcpy(c.dst, c.src, c.n);
  s->q.clear();
  return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s) { hipStreamSynchronize(s); delete s; return hipSuccess; }
inline hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t s) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->q.push_back({dst, src, n});
  return hipSuccess;
}
inline hipError_t hipHostMalloc(void** p, size_t n, unsigned) { *p = std::malloc(n); return *p ? hipSuccess : 1; }
inline hipError_t hipHostFree(void* p) { std::free(p); return hipSuccess; }
