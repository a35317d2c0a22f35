// Machine probes for the roofline denominators of the sweep: HBM copy rate,
// FP64 and FP32 vector FMA rates (packed FP32 forms are disabled at build
// time, so the FP32 figure is the non-packed rate the kernels can reach),
// and the latency of one hand-off between two waves of a work-group through
// an LDS counter (the protocol the pipelined sweep uses between levels).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "vef_sweep.h"

namespace {

__global__ void __launch_bounds__(256) k_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// Eight independent FMA chains per lane; the result is stored so nothing is
// removed.  a, b are kernel arguments so the chains cannot be folded.
template <typename T>
__global__ void __launch_bounds__(256) k_fma(T *__restrict__ out, int iters, T a, T b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  T x0 = T(i & 7) * T(1e-3), x1 = x0 + T(1), x2 = x0 + T(2), x3 = x0 + T(3);
  T x4 = x0 + T(4), x5 = x0 + T(5), x6 = x0 + T(6), x7 = x0 + T(7);
  for (int k = 0; k < iters; ++k) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      x0 = x0 * a + b;
      x1 = x1 * a + b;
      x2 = x2 * a + b;
      x3 = x3 * a + b;
      x4 = x4 * a + b;
      x5 = x5 * a + b;
      x6 = x6 * a + b;
      x7 = x7 * a + b;
    }
  }
  out[i] = ((x0 + x1) + (x2 + x3)) + ((x4 + x5) + (x6 + x7));
}

// Two waves hand a token back and forth through an LDS counter: wave w
// waits until the counter reaches r (r = w, w + 2, ...) and sets it to r + 1.
// Each wait is bounded; on expiry the wave sets *status and both leave.
__global__ void __launch_bounds__(128) k_handoff(int rounds, long long max_spins, int *status) {
  __shared__ int cnt, abort_flag;
  if (threadIdx.x == 0) {
    cnt = 0;
    abort_flag = 0;
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int r = w; r < 2 * rounds; r += 2) {
    long long spins = 0;
    while (__hip_atomic_load(&cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < r) {
      if ((++spins & 63) == 0) {
        if (__hip_atomic_load(&abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) return;
        if (spins > max_spins) {
          __hip_atomic_store(&abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          if (lane == 0) atomicOr(status, 1);
          return;
        }
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) __hip_atomic_store(&cnt, r + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s;
  explicit Timer(hipStream_t st) : s(st) {}
  hipError_t init() {
    hipError_t e = hipEventCreate(&a);
    return e == hipSuccess ? hipEventCreate(&b) : e;
  }
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

hipError_t elapsed_ms(Timer &t, float *ms) {
  hipError_t e = hipEventSynchronize(t.b);
  return e == hipSuccess ? hipEventElapsedTime(ms, t.a, t.b) : e;
}

}  // namespace

extern "C" int vef_probe_machine(vef_machine *out, void *stream) {
  if (!out) return VEF_ERR_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return VEF_ERR_HIP;
  *out = vef_machine{};
  out->compute_units = cus;
  Timer t(s);
  if (t.init() != hipSuccess) return VEF_ERR_HIP;
  float ms = 0.f;
  // HBM: copy 512 MiB (read + write), best of 3 after one warm-up
  const size_t bytes = (size_t)512 << 20, n = bytes / sizeof(uint4);
  void *src = nullptr, *dst = nullptr;
  if (hipMalloc(&src, bytes) != hipSuccess) return VEF_ERR_OOM;
  if (hipMalloc(&dst, bytes) != hipSuccess) {
    (void)hipFree(src);
    return VEF_ERR_OOM;
  }
  e = hipMemsetAsync(src, 0, bytes, s);
  double best = 1e30;
  for (int r = 0; r < 4 && e == hipSuccess; ++r) {
    if ((e = hipEventRecord(t.a, s)) != hipSuccess) break;
    hipLaunchKernelGGL(k_copy, dim3(cus * 16), dim3(256), 0, s, static_cast<const uint4 *>(src),
                       static_cast<uint4 *>(dst), n);
    if ((e = hipGetLastError()) != hipSuccess) break;
    if ((e = hipEventRecord(t.b, s)) != hipSuccess) break;
    if ((e = elapsed_ms(t, &ms)) != hipSuccess) break;
    if (r > 0 && ms < best) best = ms;
  }
  (void)hipFree(src);
  (void)hipFree(dst);
  if (e != hipSuccess) return VEF_ERR_HIP;
  out->hbm_copy_gbs = 2.0 * bytes / (best * 1e-3) / 1e9;
  // FMA rates: 8 chains x 8 unrolled x iters per lane, 2 flop each
  const int blocks = cus * 16, threads = blocks * 256, iters = 2048;
  void *buf = nullptr;
  if (hipMalloc(&buf, sizeof(double) * threads) != hipSuccess) return VEF_ERR_OOM;
  for (int prec = 0; prec < 2 && e == hipSuccess; ++prec) {
    best = 1e30;
    for (int r = 0; r < 3 && e == hipSuccess; ++r) {
      if ((e = hipEventRecord(t.a, s)) != hipSuccess) break;
      if (prec == 0)
        hipLaunchKernelGGL(k_fma<double>, dim3(blocks), dim3(256), 0, s, static_cast<double *>(buf), iters,
                           0.999999, 1e-7);
      else
        hipLaunchKernelGGL(k_fma<float>, dim3(blocks), dim3(256), 0, s, static_cast<float *>(buf), iters,
                           0.999999f, 1e-7f);
      if ((e = hipGetLastError()) != hipSuccess) break;
      if ((e = hipEventRecord(t.b, s)) != hipSuccess) break;
      if ((e = elapsed_ms(t, &ms)) != hipSuccess) break;
      if (r > 0 && ms < best) best = ms;
    }
    const double tf = 2.0 * 64.0 * iters * (double)threads / (best * 1e-3) / 1e12;
    if (prec == 0)
      out->fp64_fma_tflops = tf;
    else
      out->fp32_fma_tflops = tf;
  }
  (void)hipFree(buf);
  if (e != hipSuccess) return VEF_ERR_HIP;
  // LDS hand-off between two waves of one work-group
  int *status = nullptr;
  if (hipMalloc(&status, sizeof(int)) != hipSuccess) return VEF_ERR_OOM;
  const int rounds = 20000;
  e = hipMemsetAsync(status, 0, sizeof(int), s);
  best = 1e30;
  for (int r = 0; r < 3 && e == hipSuccess; ++r) {
    if ((e = hipEventRecord(t.a, s)) != hipSuccess) break;
    hipLaunchKernelGGL(k_handoff, dim3(1), dim3(128), 0, s, rounds, (long long)1 << 24, status);
    if ((e = hipGetLastError()) != hipSuccess) break;
    if ((e = hipEventRecord(t.b, s)) != hipSuccess) break;
    if ((e = elapsed_ms(t, &ms)) != hipSuccess) break;
    if (r > 0 && ms < best) best = ms;
  }
  int st = 0;
  if (e == hipSuccess) e = hipMemcpy(&st, status, sizeof(int), hipMemcpyDeviceToHost);
  (void)hipFree(status);
  if (e != hipSuccess) return VEF_ERR_HIP;
  if (st) return VEF_ERR_TIMEOUT;
  out->lds_handoff_ns = best * 1e6 / (2.0 * rounds);
  return VEF_OK;
}
