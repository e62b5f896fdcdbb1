// Matrix-core calibration for the profiles: a kernel that keeps every SIMD's
// matrix unit busy with independent v_mfma_f64_16x16x4f64 (16 accumulators
// per wave, two waves per SIMD) for a known number of instructions.  Its
// achieved rate is the FP64 matrix peak measured on the device, and its
// SQ_VALU_MFMA_BUSY_CYCLES per unit of time (from a rocprofv3 counter run) is
// the reading of a fully busy device, which turns the same counter of any
// other kernel into a utilization fraction.
//
//   mfma_peak [iters]      prints one line per timed run and the rate
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

typedef double v4d __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256, 2) void k_mfma_peak(int iters, double* __restrict__ out) {
  const double a = 1.0 + 1e-9 * threadIdx.x, b = 1.0 - 1e-9 * blockIdx.x;
  v4d acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

#define CHECK(x)                                                               \
  do {                                                                         \
    hipError_t e = (x);                                                        \
    if (e != hipSuccess) {                                                     \
      fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e), __LINE__); \
      return 1;                                                                \
    }                                                                          \
  } while (0)

int main(int argc, char** argv) {
  const int iters = argc > 1 ? atoi(argv[1]) : 50000;
  int dev = 0, cus = 0;
  CHECK(hipGetDevice(&dev));
  CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int grid = 2 * cus, block = 256;
  double* out = nullptr;
  CHECK(hipMalloc(&out, sizeof(double) * grid * block));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  // per wave: iters x 16 MFMAs of 16 x 16 x 4 (2 * 16 * 16 * 4 flops each)
  const double flops = (double)grid * (block / 64) * iters * 16.0 * 2.0 * 16 * 16 * 4;
  hipLaunchKernelGGL(k_mfma_peak, dim3(grid), dim3(block), 0, 0, iters, out);   // warm-up
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  double best = 0.0;
  for (int r = 0; r < 3; ++r) {
    CHECK(hipEventRecord(e0, 0));
    hipLaunchKernelGGL(k_mfma_peak, dim3(grid), dim3(block), 0, 0, iters, out);
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    const double tf = flops / (ms * 1e-3) / 1e12;
    if (tf > best) best = tf;
    printf("k_mfma_peak: %d workgroups x %d threads, %d iterations, %.3f ms, %.2f TFLOP/s FP64\n", grid, block,
           iters, ms, tf);
  }
  printf("MFMA_PEAK_JSON: {\"kernel\": \"k_mfma_peak\", \"cus\": %d, \"flops_per_dispatch\": %.6e, "
         "\"best_tflops\": %.3f}\n", cus, flops, best);
  CHECK(hipFree(out));
  return 0;
}
