// Measured peaks of the device, for the roofline fractions the benchmark
// reports beside the published ones: a streaming copy (HBM bandwidth) and a
// loop of independent fused multiply-adds (vector FP64 / FP32 throughput).
// Measurement support only; not part of the potential.
//
// Included at the end of airebo.hip (one library, one HIP context).

namespace airebo {

// Streaming copy, 32 bytes per lane per iteration, grid-stride.
__global__ void k_peak_copy(const double4* __restrict__ src, double4* __restrict__ dst, int64_t n4) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n4; k += (int64_t)gridDim.x * blockDim.x)
    dst[k] = src[k];
}

// Eight independent FMA chains per lane, `iters` rounds; the sum is stored so
// that nothing is dead code.  2 * 8 * iters flops per lane.
template <typename T>
__global__ void k_peak_fma(T* __restrict__ out, int iters, T a, T b) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  T x0 = (T)(threadIdx.x & 7), x1 = x0 + (T)1, x2 = x0 + (T)2, x3 = x0 + (T)3;
  T x4 = x0 + (T)4, x5 = x0 + (T)5, x6 = x0 + (T)6, x7 = x0 + (T)7;
  for (int k = 0; k < iters; ++k) {
    x0 = fma(x0, a, b); x1 = fma(x1, a, b); x2 = fma(x2, a, b); x3 = fma(x3, a, b);
    x4 = fma(x4, a, b); x5 = fma(x5, a, b); x6 = fma(x6, a, b); x7 = fma(x7, a, b);
  }
  out[g] = ((x0 + x1) + (x2 + x3)) + ((x4 + x5) + (x6 + x7));
}

}  // namespace airebo

extern "C" {

int airebo_peak_copy(const void* src, void* dst, int64_t bytes, int32_t reps, double* gbs, void* stream) {
  if (!src || !dst || !gbs || bytes < 32 || reps < 1) return fail(AIREBO_E_ARG, "bad copy arguments");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n4 = bytes / 32;
  const int grid = (int)std::min<int64_t>((n4 + 255) / 256, 256 * 64);
  hipEvent_t a, b;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  hipLaunchKernelGGL(k_peak_copy, dim3(grid), dim3(256), 0, s, (const double4*)src, (double4*)dst, n4);   // warm
  (void)hipEventRecord(a, s);
  for (int r = 0; r < reps; ++r)
    hipLaunchKernelGGL(k_peak_copy, dim3(grid), dim3(256), 0, s, (const double4*)src, (double4*)dst, n4);
  (void)hipEventRecord(b, s);
  hipError_t e = hipEventSynchronize(b);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return fail(AIREBO_E_DEVICE, std::string("copy timing: ") + hipGetErrorString(e));
  *gbs = 2.0 * 32.0 * (double)n4 * reps / (1e-3 * ms) / 1e9;   // bytes read + written
  return 0;
}

int airebo_peak_fma(int32_t fp64, int32_t iters, double* tflops, void* stream) {
  if (!tflops || iters < 1) return fail(AIREBO_E_ARG, "bad FMA-loop arguments");
  hipStream_t s = (hipStream_t)stream;
  const int grid = 256 * 64, block = 256;   // 16 wavefronts per SIMD of every CU
  const int64_t lanes = (int64_t)grid * block;
  void* out = nullptr;
  HIPCHK(hipMalloc(&out, lanes * sizeof(double)));
  hipEvent_t a, b;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  auto launch = [&]() {
    if (fp64)
      hipLaunchKernelGGL(k_peak_fma<double>, dim3(grid), dim3(block), 0, s, (double*)out, iters, 0.9999999, 1e-7);
    else
      hipLaunchKernelGGL(k_peak_fma<float>, dim3(grid), dim3(block), 0, s, (float*)out, iters, 0.9999f, 1e-4f);
  };
  launch();   // warm
  (void)hipEventRecord(a, s);
  launch();
  (void)hipEventRecord(b, s);
  hipError_t e = hipEventSynchronize(b);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipFree(out);
  if (e != hipSuccess) return fail(AIREBO_E_DEVICE, std::string("FMA timing: ") + hipGetErrorString(e));
  *tflops = 2.0 * 8.0 * (double)iters * (double)lanes / (1e-3 * ms) / 1e12;
  return 0;
}

}  // extern "C"
