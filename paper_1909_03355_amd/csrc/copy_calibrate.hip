// Memory-bandwidth reference program, built beside the library.
//
// Default (no argument): the calibration run of the memory-traffic counters,
// three copies of 256 MiB (each reads 256 MiB and writes 256 MiB), so
// FETCH_SIZE and WRITE_SIZE per dispatch can be scaled to bytes.
//
// `copy_calibrate time`: the measured ceiling the step kernels are quoted
// against besides the 8 TB/s vendor peak: warm copies (read + write; one
// block per 4 x 256 float4, and the grid-stride copy of the calibration run)
// and warm reads of buffers from 16 MiB to 4 GiB, each timed with HIP events
// over 20 dispatches after 3 untimed ones; prints one line per size and kind
// with the best and median rate in GB/s (bytes read + written per second).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

__global__ void copy_calibrate(const float4 *__restrict__ a, float4 *__restrict__ b, size_t n) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) b[i] = a[i];
}

// four 16-byte loads in flight per thread, then four stores
__global__ void copy4(const float4 *__restrict__ a, float4 *__restrict__ b, size_t n) {
  const size_t base = (blockIdx.x * (size_t)blockDim.x) * 4 + threadIdx.x;
  float4 v[4];
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const size_t i = base + (size_t)q * blockDim.x;
    if (i < n) v[q] = a[i];
  }
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const size_t i = base + (size_t)q * blockDim.x;
    if (i < n) b[i] = v[q];
  }
}

// reads only: four loads in flight, a sum per block written once
__global__ void read4(const float4 *__restrict__ a, float *__restrict__ out, size_t n) {
  const size_t base = (blockIdx.x * (size_t)blockDim.x) * 4 + threadIdx.x;
  float s = 0.f;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const size_t i = base + (size_t)q * blockDim.x;
    if (i < n) {
      const float4 v = a[i];
      s += (v.x + v.y) + (v.z + v.w);
    }
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) out[blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6)] = s;
}

static int calibrate() {
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

static int timed() {
  const size_t maxb = 4ull << 30;
  float4 *a = nullptr, *b = nullptr;
  float *part = nullptr;
  const int bs = 256;
  const size_t maxn = maxb / sizeof(float4), maxblocks = (maxn + 4 * bs - 1) / (4 * bs);
  if (hipMalloc(&a, maxb) != hipSuccess || hipMalloc(&b, maxb) != hipSuccess ||
      hipMalloc(&part, sizeof(float) * maxblocks * (bs / 64)) != hipSuccess)
    return 1;
  if (hipMemset(a, 0, maxb) != hipSuccess || hipMemset(b, 0, maxb) != hipSuccess) return 1;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
  printf("kind bytes_per_dispatch best_GBs median_GBs\n");
  for (size_t mb = 16; mb <= (maxb >> 20); mb *= 4) {
    const size_t bytes = mb << 20, n = bytes / sizeof(float4);
    const unsigned grid = (unsigned)((n + 4 * bs - 1) / (4 * bs));
    for (int kind = 0; kind < 3; kind++) {
      std::vector<float> us;
      for (int r = 0; r < 23; r++) {
        if (hipEventRecord(e0, 0) != hipSuccess) return 1;
        if (kind == 0) hipLaunchKernelGGL(copy4, dim3(grid), dim3(bs), 0, 0, a, b, n);
        else if (kind == 1) hipLaunchKernelGGL(read4, dim3(grid), dim3(bs), 0, 0, a, part, n);
        else hipLaunchKernelGGL(copy_calibrate, dim3(8192), dim3(256), 0, 0, a, b, n);
        if (hipEventRecord(e1, 0) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 1;
        float ms = 0;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 1;
        if (r >= 3) us.push_back(ms * 1e3f);
      }
      std::sort(us.begin(), us.end());
      const double moved = (kind == 1 ? 1.0 : 2.0) * (double)bytes;
      printf("%s %zu %.1f %.1f\n", kind == 0 ? "copy" : (kind == 1 ? "read" : "copy_stride"),
             (size_t)moved,
             moved / (us.front() * 1e-6) / 1e9, moved / (us[us.size() / 2] * 1e-6) / 1e9);
    }
  }
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) return 1;
  hipFree(a);
  hipFree(b);
  hipFree(part);
  return 0;
}

int main(int argc, char **argv) {
  if (argc > 1 && std::strcmp(argv[1], "time") == 0) return timed();
  return calibrate();
}
