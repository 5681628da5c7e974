// HBM stream kernels for gfx950: the bandwidth plain streaming kernels reach
// on this device, the ceiling the round kernels' rates are set against.
// Three modes over one buffer of `bytes` (a multiple of 16): copy (read src,
// write dst), read (sum src), write (fill dst); three access variants, since
// the best one depends on the grid and the buffer: 0 grid-stride, one 16-byte
// vector per thread and pass; 1 grid-stride, eight vectors in flight per
// thread; 2 each workgroup streams one contiguous chunk, four vectors in
// flight per thread.  Stores are non-temporal, as in the round kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int THREADS = 256;
typedef float f4 __attribute__((ext_vector_type(4)));

// elements [b, e) of the workgroup, visited with stride st, U per pass
struct Span {
  long long b, e, st;
};

__device__ inline Span span_of(int variant, long long n) {
  Span s;
  if (variant == 2) {
    const long long chunk = (n + gridDim.x - 1) / gridDim.x;
    s.b = (long long)blockIdx.x * chunk + threadIdx.x;
    s.e = min((long long)(blockIdx.x + 1) * chunk, n);
    s.st = THREADS;
  } else {
    s.b = (long long)blockIdx.x * THREADS + threadIdx.x;
    s.e = n;
    s.st = (long long)gridDim.x * THREADS;
  }
  return s;
}

template <int U>
__device__ inline void copy_span(const f4* __restrict__ src, f4* __restrict__ dst, Span s) {
  long long i = s.b;
  for (; i + (U - 1) * s.st < s.e; i += U * s.st) {
    f4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = src[i + u * s.st];
#pragma unroll
    for (int u = 0; u < U; ++u) __builtin_nontemporal_store(v[u], &dst[i + u * s.st]);
  }
  for (; i < s.e; i += s.st) __builtin_nontemporal_store(src[i], &dst[i]);
}

template <int U>
__device__ inline float read_span(const f4* __restrict__ src, Span s) {
  float a = 0.f;
  long long i = s.b;
  for (; i + (U - 1) * s.st < s.e; i += U * s.st) {
    f4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = src[i + u * s.st];
#pragma unroll
    for (int u = 0; u < U; ++u) a += v[u].x + v[u].y + v[u].z + v[u].w;
  }
  for (; i < s.e; i += s.st) a += src[i].x + src[i].y + src[i].z + src[i].w;
  return a;
}

__global__ void __launch_bounds__(THREADS) k_copy(const f4* __restrict__ src, f4* __restrict__ dst, long long n,
                                                  int variant) {
  const Span s = span_of(variant, n);
  if (variant == 0) copy_span<1>(src, dst, s);
  else if (variant == 1) copy_span<8>(src, dst, s);
  else copy_span<4>(src, dst, s);
}

__global__ void __launch_bounds__(THREADS) k_read(const f4* __restrict__ src, float* __restrict__ out, long long n,
                                                  int variant) {
  const Span s = span_of(variant, n);
  const float a = variant == 0 ? read_span<1>(src, s) : variant == 1 ? read_span<8>(src, s) : read_span<4>(src, s);
  // one value per thread keeps the loads live; the buffer is tiny
  out[(long long)blockIdx.x * THREADS + threadIdx.x] = a;
}

__global__ void __launch_bounds__(THREADS) k_fill(f4* __restrict__ dst, long long n, float val, int variant) {
  const Span s = span_of(variant, n);
  const f4 v = {val, val, val, val};
  for (long long i = s.b; i < s.e; i += s.st) __builtin_nontemporal_store(v, &dst[i]);
}

}  // namespace

extern "C" {

// Runs `mode` (0 copy, 1 read, 2 write) in access `variant` (0, 1, 2 as
// above) `reps` times on the stream over `bytes` bytes (multiple of 16; src
// and dst device buffers of that size, 16-byte aligned; `out` a device buffer
// of blocks * 256 floats for the read mode), `blocks` workgroups of 256
// threads; writes the duration of each repetition (HIP events, ms) into
// ms[0..reps-1].  Returns 0, -1 on a bad argument, -3 on a HIP error.
int hbm_stream(int32_t mode, int32_t variant, const void* src, void* dst, void* out, int64_t bytes, int32_t blocks,
               int32_t reps, void* stream, float* ms) {
  if (mode < 0 || mode > 2 || variant < 0 || variant > 2 || bytes <= 0 || (bytes & 15) || blocks < 1 ||
      blocks > (1 << 20) || reps < 1 || !ms)
    return -1;
  if ((mode != 2 && !src) || (mode != 1 && !dst) || (mode == 1 && !out)) return -1;
  if (((uintptr_t)src & 15) || ((uintptr_t)dst & 15)) return -1;
  const long long n = bytes / 16;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return -3;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return -3;
  }
  int rc = 0;
  for (int r = 0; r < reps && rc == 0; ++r) {
    if (hipEventRecord(a, st) != hipSuccess) rc = -3;
    if (mode == 0)
      hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(THREADS), 0, st, (const f4*)src, (f4*)dst, n, variant);
    else if (mode == 1)
      hipLaunchKernelGGL(k_read, dim3(blocks), dim3(THREADS), 0, st, (const f4*)src, (float*)out, n, variant);
    else
      hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(THREADS), 0, st, (f4*)dst, n, (float)r, variant);
    if (hipGetLastError() != hipSuccess || hipEventRecord(b, st) != hipSuccess ||
        hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms[r], a, b) != hipSuccess)
      rc = -3;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return rc;
}

}  // extern "C"
