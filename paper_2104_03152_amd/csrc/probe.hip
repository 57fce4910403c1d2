// probe.hip -- issue-rate and bandwidth probes for the peaks the roofline
// uses (built as libckks_probe.so, run by `bench.py --probe`; not part of
// the library's ABI).
//
// Each rate kernel gives every thread eight independent dependency chains
// of one instruction kind, `iters` steps long, so the SIMDs issue
// back-to-back without waiting on a chain; the result is stored so that no
// chain is dead.  Rate = threads * iters * 8 / time (instructions of that
// kind per second, one per lane).
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef uint64_t u64;
typedef uint32_t u32;

namespace {

constexpr int CH = 8;

// v_mad_u64_u32: acc = a * b + acc (32 x 32 -> 64 plus a 64-bit addend)
__global__ void k_mad_u64(u64* out, int iters, u32 b) {
  u64 acc[CH];
  u32 a[CH];
#pragma unroll
  for (int c = 0; c < CH; c++) {
    acc[c] = threadIdx.x + c;
    a[c] = blockIdx.x * 7 + c;
  }
#pragma unroll 4
  for (int i = 0; i < iters; i++) {
    const u32 bi = b + (u32)i;  // a wave-uniform multiplier that changes every step
#pragma unroll
    for (int c = 0; c < CH; c++) {
      acc[c] = (u64)a[c] * bi + acc[c];
      asm volatile("" : "+v"(acc[c]));  // no closed form: a chain of v_mad_u64_u32
    }
  }
  u64 s = 0;
#pragma unroll
  for (int c = 0; c < CH; c++) s ^= acc[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// v_mul_lo_u32: x = x * m
__global__ void k_mul_lo(u64* out, int iters, u32 m) {
  u32 x[CH];
#pragma unroll
  for (int c = 0; c < CH; c++) x[c] = threadIdx.x * 2 + 1 + c;
#pragma unroll 4
  for (int i = 0; i < iters; i++)
#pragma unroll
    for (int c = 0; c < CH; c++) {
      x[c] = x[c] * m;
      asm volatile("" : "+v"(x[c]));  // no reassociation into powers of m
    }
  u32 s = 0;
#pragma unroll
  for (int c = 0; c < CH; c++) s ^= x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// v_mul_hi_u32: x = hi(x * m)
__global__ void k_mul_hi(u64* out, int iters, u32 m) {
  u32 x[CH];
#pragma unroll
  for (int c = 0; c < CH; c++) x[c] = 0xF0000000u + threadIdx.x + c;
#pragma unroll 4
  for (int i = 0; i < iters; i++)
#pragma unroll
    for (int c = 0; c < CH; c++) {
      x[c] = __umulhi(x[c], m);
      asm volatile("" : "+v"(x[c]));
    }
  u32 s = 0;
#pragma unroll
  for (int c = 0; c < CH; c++) s ^= x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// v_fma_f64: x = x * a + b
__global__ void k_fma_f64(u64* out, int iters, double a, double b) {
  double x[CH];
#pragma unroll
  for (int c = 0; c < CH; c++) x[c] = threadIdx.x + c;
#pragma unroll 4
  for (int i = 0; i < iters; i++)
#pragma unroll
    for (int c = 0; c < CH; c++) {
      x[c] = fma(x[c], a, b);
      asm volatile("" : "+v"(x[c]));
    }
  double s = 0;
#pragma unroll
  for (int c = 0; c < CH; c++) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = __double_as_longlong(s);
}

// v_add_u32 (the full-rate 32-bit integer reference): x = x + m
__global__ void k_add_u32(u64* out, int iters, u32 m) {
  u32 x[CH];
#pragma unroll
  for (int c = 0; c < CH; c++) x[c] = threadIdx.x + c;
#pragma unroll 4
  for (int i = 0; i < iters; i++)
#pragma unroll
    for (int c = 0; c < CH; c++) {
      x[c] = x[c] + m;
      asm volatile("" : "+v"(x[c]));  // no closed form: a chain of v_add_u32
    }
  u32 s = 0;
#pragma unroll
  for (int c = 0; c < CH; c++) s ^= x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// device copy, 16 bytes per lane per step, grid-stride
__global__ void k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, long long n16) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" {

// kind: 0 v_mad_u64_u32, 1 v_mul_lo_u32, 2 v_mul_hi_u32, 3 v_fma_f64,
// 4 v_add_u32.  Returns the kernel time
// in ms (HIP events) of one launch of blocks x 256 threads, `iters` steps
// of CH chains; out needs blocks * 256 words.  Negative on a HIP error.
double probe_rate(int kind, int blocks, int iters, u64* out) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1;
  (void)hipEventRecord(a, 0);
  switch (kind) {
    case 0: hipLaunchKernelGGL(k_mad_u64, dim3(blocks), dim3(256), 0, 0, out, iters, 0x9E3779B1u); break;
    case 1: hipLaunchKernelGGL(k_mul_lo, dim3(blocks), dim3(256), 0, 0, out, iters, 0x9E3779B1u); break;
    case 2: hipLaunchKernelGGL(k_mul_hi, dim3(blocks), dim3(256), 0, 0, out, iters, 0xFFFFFFFFu); break;
    case 3: hipLaunchKernelGGL(k_fma_f64, dim3(blocks), dim3(256), 0, 0, out, iters, 0.999999, 1e-9); break;
    case 4: hipLaunchKernelGGL(k_add_u32, dim3(blocks), dim3(256), 0, 0, out, iters, 0x9E3779B1u); break;
    default: return -2;
  }
  (void)hipEventRecord(b, 0);
  if (hipEventSynchronize(b) != hipSuccess) return -1;
  float ms = 0;
  (void)hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return hipGetLastError() == hipSuccess ? ms : -1;
}

// one copy of `bytes` (a multiple of 16) from src to dst; kernel time in ms
double probe_copy(const void* src, void* dst, long long bytes, int blocks) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1;
  (void)hipEventRecord(a, 0);
  hipLaunchKernelGGL(k_copy16, dim3(blocks), dim3(256), 0, 0, (const uint4*)src, (uint4*)dst, bytes / 16);
  (void)hipEventRecord(b, 0);
  if (hipEventSynchronize(b) != hipSuccess) return -1;
  float ms = 0;
  (void)hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return hipGetLastError() == hipSuccess ? ms : -1;
}

}  // extern "C"
