// A stand-in for the HIP runtime calls the library's host code makes, on
// host memory, for CPU tests of that code (tests/test_server_model.py).
// "Device" memory is host memory. Work on a stream is deferred as on a GPU:
// asynchronous copies and kernel stand-ins (fake_hip_enqueue) join one queue
// in call order and run only when the host waits (an event or stream
// synchronization, a synchronous copy, a free) or when a query of an event
// lets the "device" make some progress. A host write to a buffer that queued
// work has yet to read therefore shows up in what that work sees, and a read
// of results before the wait sees stale data, as it would on the device.
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <functional>
#include <map>

void (*fake_hip_on_copy)(void *dst, const void *src, size_t n) = nullptr;
void (*fake_hip_on_free)(void *p, size_t n) = nullptr;
size_t fake_hip_total_bytes = 288ull << 30;
size_t fake_hip_free_bytes = 280ull << 30;
int fake_hip_cus = 256;

namespace {
std::map<void *, size_t> g_dev;  // device allocations and their sizes
int g_events = 0;
std::deque<std::function<void()>> g_queue;  // the stream's work not yet run
uint64_t g_issued = 0, g_ran = 0;           // operations queued and run so far
std::map<hipEvent_t, uint64_t> g_marks;     // event -> operations before its record
uint64_t g_rng = 0x2545f4914f6cdd1dull;

void run_until(uint64_t n) {
  while (g_ran < n) {
    std::function<void()> f = std::move(g_queue.front());
    g_queue.pop_front();
    ++g_ran;
    f();
  }
}
void drain() { run_until(g_issued); }
}  // namespace

void fake_hip_enqueue(std::function<void()> f) {
  g_queue.push_back(std::move(f));
  ++g_issued;
}

extern "C" {

hipError_t hipGetDevice(int *deviceId) {
  *deviceId = 0;
  return hipSuccess;
}

hipError_t hipSetDevice(int deviceId) { return deviceId == 0 ? hipSuccess : hipErrorInvalidDevice; }

hipError_t hipDeviceGetAttribute(int *pi, hipDeviceAttribute_t attr, int deviceId) {
  if (deviceId != 0) return hipErrorInvalidDevice;
  *pi = attr == hipDeviceAttributeMultiprocessorCount ? fake_hip_cus : 0;
  return hipSuccess;
}

hipError_t hipMemGetInfo(size_t *free_b, size_t *total_b) {
  *free_b = fake_hip_free_bytes;
  *total_b = fake_hip_total_bytes;
  return hipSuccess;
}

hipError_t hipMalloc(void **ptr, size_t size) {
  const size_t n = (size + 255) & ~(size_t)255;
  if (n > fake_hip_free_bytes) return hipErrorOutOfMemory;
  void *p = aligned_alloc(256, n ? n : 256);
  if (!p) return hipErrorOutOfMemory;
  memset(p, 0xA5, n ? n : 256);  // device memory starts with garbage
  g_dev[p] = n;
  fake_hip_free_bytes -= n;
  *ptr = p;
  return hipSuccess;
}

hipError_t hipFree(void *ptr) {
  drain();  // frees wait for the device
  if (!ptr) return hipSuccess;
  auto it = g_dev.find(ptr);
  if (it == g_dev.end()) return hipErrorInvalidValue;
  fake_hip_free_bytes += it->second;
  if (fake_hip_on_free) fake_hip_on_free(ptr, it->second);
  g_dev.erase(it);
  free(ptr);
  return hipSuccess;
}

hipError_t hipHostMalloc(void **ptr, size_t size, unsigned int flags) {
  (void)flags;
  *ptr = malloc(size ? size : 1);
  return *ptr ? hipSuccess : hipErrorOutOfMemory;
}

hipError_t hipHostFree(void *ptr) {
  drain();
  free(ptr);
  return hipSuccess;
}

hipError_t hipMemcpy(void *dst, const void *src, size_t sizeBytes, hipMemcpyKind kind) {
  drain();
  if (kind == hipMemcpyDeviceToDevice && fake_hip_on_copy) fake_hip_on_copy(dst, src, sizeBytes);
  memcpy(dst, src, sizeBytes);
  return hipSuccess;
}

hipError_t hipMemcpyAsync(void *dst, const void *src, size_t sizeBytes, hipMemcpyKind kind,
                          hipStream_t stream) {
  (void)stream;
  fake_hip_enqueue([=] {  // reads src when it runs, not now
    if (kind == hipMemcpyDeviceToDevice && fake_hip_on_copy) fake_hip_on_copy(dst, src, sizeBytes);
    memcpy(dst, src, sizeBytes);
  });
  return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t stream) {
  (void)stream;
  drain();
  return hipSuccess;
}

hipError_t hipStreamIsCapturing(hipStream_t stream, hipStreamCaptureStatus *pCaptureStatus) {
  (void)stream;
  *pCaptureStatus = hipStreamCaptureStatusNone;
  return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t *event, unsigned flags) {
  (void)flags;
  *event = reinterpret_cast<hipEvent_t>(new int(++g_events));
  return hipSuccess;
}

hipError_t hipEventDestroy(hipEvent_t event) {
  g_marks.erase(event);
  delete reinterpret_cast<int *>(event);
  return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t event, hipStream_t stream) {
  (void)stream;
  g_marks[event] = g_issued;
  return hipSuccess;
}

hipError_t hipEventSynchronize(hipEvent_t event) {
  auto it = g_marks.find(event);
  if (it != g_marks.end()) run_until(it->second);
  return hipSuccess;
}

hipError_t hipEventQuery(hipEvent_t event) {
  // the device makes some progress meanwhile: up to two queued operations
  g_rng ^= g_rng << 13;
  g_rng ^= g_rng >> 7;
  g_rng ^= g_rng << 17;
  run_until(std::min<uint64_t>(g_issued, g_ran + g_rng % 3));
  auto it = g_marks.find(event);
  return it == g_marks.end() || g_ran >= it->second ? hipSuccess : hipErrorNotReady;
}

}  // extern "C"
