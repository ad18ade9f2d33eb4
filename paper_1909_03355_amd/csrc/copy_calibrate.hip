// Calibration program for the memory-traffic counters: copies 256 MiB three
// times (each copy reads 256 MiB and writes 256 MiB), so FETCH_SIZE and
// WRITE_SIZE per dispatch can be scaled to bytes.  Built beside the library.
#include <hip/hip_runtime.h>

#include <cstdio>

__global__ void copy_calibrate(const float4 *__restrict__ a, float4 *__restrict__ b, size_t n) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) b[i] = a[i];
}

int main() {
  const size_t bytes = 256ull << 20, n = bytes / sizeof(float4);
  float4 *a = nullptr, *b = nullptr;
  if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) return 1;
  if (hipMemset(a, 0, bytes) != hipSuccess || hipMemset(b, 0, bytes) != hipSuccess) return 1;
  for (int r = 0; r < 3; r++) hipLaunchKernelGGL(copy_calibrate, dim3(8192), dim3(256), 0, 0, a, b, n);
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) return 1;
  printf("copy_calibrate: 3 copies of %zu bytes (read + write)\n", bytes);
  hipFree(a);
  hipFree(b);
  return 0;
}
