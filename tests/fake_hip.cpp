// A stand-in for the HIP runtime calls the library's host code makes, on
// host memory, for CPU tests of that code (tests/test_server_model.py).
// "Device" memory is host memory, copies are memcpy, streams run nothing of
// their own and events are always complete: a kernel stand-in called by the
// host code does its work at once, so call order is stream order.
#include <hip/hip_runtime_api.h>
#include <stdlib.h>
#include <string.h>

#include <map>

void (*fake_hip_on_copy)(void *dst, const void *src, size_t n) = nullptr;
size_t fake_hip_total_bytes = 288ull << 30;
size_t fake_hip_free_bytes = 280ull << 30;
int fake_hip_cus = 256;

namespace {
std::map<void *, size_t> g_dev;  // device allocations and their sizes
int g_events = 0;
}  // namespace

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
  if (!ptr) return hipSuccess;
  auto it = g_dev.find(ptr);
  if (it == g_dev.end()) return hipErrorInvalidValue;
  fake_hip_free_bytes += it->second;
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
  free(ptr);
  return hipSuccess;
}

hipError_t hipMemcpy(void *dst, const void *src, size_t sizeBytes, hipMemcpyKind kind) {
  if (kind == hipMemcpyDeviceToDevice && fake_hip_on_copy) fake_hip_on_copy(dst, src, sizeBytes);
  memcpy(dst, src, sizeBytes);
  return hipSuccess;
}

hipError_t hipMemcpyAsync(void *dst, const void *src, size_t sizeBytes, hipMemcpyKind kind,
                          hipStream_t stream) {
  (void)stream;
  return hipMemcpy(dst, src, sizeBytes, kind);
}

hipError_t hipStreamSynchronize(hipStream_t stream) {
  (void)stream;
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
  delete reinterpret_cast<int *>(event);
  return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t event, hipStream_t stream) {
  (void)event;
  (void)stream;
  return hipSuccess;
}

hipError_t hipEventSynchronize(hipEvent_t event) {
  (void)event;
  return hipSuccess;
}

hipError_t hipEventQuery(hipEvent_t event) {
  (void)event;
  return hipSuccess;
}

}  // extern "C"
