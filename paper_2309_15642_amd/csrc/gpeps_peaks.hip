// Peak-rate probes of the GPU the library runs on (libgpeps_peaks.so, used by the benchmark to
// quote measured peaks beside the datasheet ones): FP64 vector FMA throughput, FP64 matrix-core
// throughput (v_mfma_f64_16x16x4f64) and device-memory copy bandwidth; and one testing aid that
// fills the LDS of every CU with a chosen pattern.  Measurement and testing only; no step of the
// simple update runs here.
//
// Every entry point launches one kernel on the given stream and returns a hipError_t as int;
// the caller times the launch with events on that stream.  `out` receives one double per
// thread (FMA) or per lane (MFMA) so that the arithmetic cannot be removed; its contents carry
// no meaning.

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 16;  // independent FMA chains per thread (covers the FMA latency)

__global__ __launch_bounds__(256) void k_peak_fma(double* __restrict__ out, int iters, double a, double b) {
  double x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = 1e-3 * (threadIdx.x + c);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = fma(x[c], a, b);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_mfma(double* __restrict__ out, int iters, double a, double b) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int kAcc = 8;  // independent accumulators per wave
  d4 c[kAcc];
#pragma unroll
  for (int q = 0; q < kAcc; ++q) c[q] = (d4){0.0, 0.0, 0.0, 0.0};
  const double av = a * (1.0 + 1e-3 * threadIdx.x), bv = b;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int q = 0; q < kAcc; ++q) c[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, c[q], 0, 0, 0);
  }
  d4 s = c[0];
#pragma unroll
  for (int q = 1; q < kAcc; ++q) s += c[q];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s[0] + s[1] + s[2] + s[3];
}

// four 16-byte elements per thread in flight: the loads of a group of four, then their stores
__global__ __launch_bounds__(256) void k_peak_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                    int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const float4 v0 = src[i], v1 = src[i + stride], v2 = src[i + 2 * stride], v3 = src[i + 3 * stride];
    dst[i] = v0;
    dst[i + stride] = v1;
    dst[i + 2 * stride] = v2;
    dst[i + 3 * stride] = v3;
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

// Every workgroup writes `pattern` into each 64-bit word of its whole (dynamic) LDS allocation.
// LDS keeps what the last workgroup on a CU left there, so a later kernel that read LDS it had
// not written would see the pattern.  The stores are volatile: nothing reads them here.
__global__ __launch_bounds__(256) void k_fill_lds(unsigned long long pattern, int words) {
  extern __shared__ unsigned long long lds_fill[];
  volatile unsigned long long* p = lds_fill;
  for (int i = threadIdx.x; i < words; i += blockDim.x) p[i] = pattern;
}

}  // namespace

extern "C" {

// FP64 FMA probe: n_blocks x 256 threads, each kChains chains of `iters` fused multiply-adds
// (2 flops each).  out: n_blocks * 256 doubles of device memory.
int gpeps_peak_fma_f64(double* out, int n_blocks, int iters, void* stream) {
  if (!out || n_blocks < 1 || iters < 1) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_peak_fma, dim3(n_blocks), dim3(256), 0, (hipStream_t)stream, out, iters, 0.9999999,
                     1e-7);
  return (int)hipGetLastError();
}

// FP64 matrix-core probe: n_blocks x 256 threads (4 waves), each wave 8 x `iters`
// v_mfma_f64_16x16x4f64 (16 x 16 x 4 x 2 = 2048 flops each).  out: n_blocks * 256 doubles.
int gpeps_peak_mfma_f64(double* out, int n_blocks, int iters, void* stream) {
  if (!out || n_blocks < 1 || iters < 1) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_peak_mfma, dim3(n_blocks), dim3(256), 0, (hipStream_t)stream, out, iters, 1e-3, 1e-3);
  return (int)hipGetLastError();
}

// Copy probe: `bytes` (a multiple of 16) from src to dst, 16-byte loads and stores, grid-stride.
int gpeps_peak_copy(const void* src, void* dst, int64_t bytes, int n_blocks, void* stream) {
  if (!src || !dst || bytes < 16 || (bytes & 15) || n_blocks < 1) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_peak_copy, dim3(n_blocks), dim3(256), 0, (hipStream_t)stream, (const float4*)src,
                     (float4*)dst, bytes / 16);
  return (int)hipGetLastError();
}

// LDS fill (testing aid): n_blocks workgroups of 256 threads, each with `lds_bytes` (a multiple
// of 8, at most the device's per-workgroup LDS) of dynamic LDS filled with `pattern`.  Launch
// more workgroups than CUs (several per CU) to reach every CU.
int gpeps_probe_fill_lds(unsigned long long pattern, int lds_bytes, int n_blocks, void* stream) {
  if (lds_bytes < 8 || (lds_bytes & 7) || n_blocks < 1) return (int)hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute((const void*)k_fill_lds, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
  if (e != hipSuccess) return (int)e;
  hipLaunchKernelGGL(k_fill_lds, dim3(n_blocks), dim3(256), lds_bytes, (hipStream_t)stream, pattern, lds_bytes / 8);
  return (int)hipGetLastError();
}

}  // extern "C"
