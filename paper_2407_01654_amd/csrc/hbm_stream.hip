// HBM stream kernels for gfx950: the bandwidth a plain streaming kernel
// reaches on this device, the ceiling the round kernels' rates are set against.
// Three modes over one buffer of `bytes` (a multiple of 16): copy (read src,
// write dst), read (sum src), write (fill dst).  Each thread moves 16-byte
// vectors in a grid-stride loop, four in flight at a time; stores are
// non-temporal, as in the round kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int THREADS = 256;
constexpr int UNROLL = 4;
typedef float f4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(THREADS) k_copy(const f4* __restrict__ src, f4* __restrict__ dst,
                                                  long long n) {
  const long long stride = (long long)gridDim.x * THREADS;
  long long i = (long long)blockIdx.x * THREADS + threadIdx.x;
  for (; i + (UNROLL - 1) * stride < n; i += UNROLL * stride) {
    f4 v[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) v[u] = src[i + u * stride];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) __builtin_nontemporal_store(v[u], &dst[i + u * stride]);
  }
  for (; i < n; i += stride) __builtin_nontemporal_store(src[i], &dst[i]);
}

__global__ void __launch_bounds__(THREADS) k_read(const f4* __restrict__ src, float* __restrict__ out,
                                                  long long n) {
  const long long stride = (long long)gridDim.x * THREADS;
  long long i = (long long)blockIdx.x * THREADS + threadIdx.x;
  float a = 0.f;
  for (; i + (UNROLL - 1) * stride < n; i += UNROLL * stride) {
    f4 v[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) v[u] = src[i + u * stride];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) a += v[u].x + v[u].y + v[u].z + v[u].w;
  }
  for (; i < n; i += stride) a += src[i].x + src[i].y + src[i].z + src[i].w;
  // one value per thread keeps the loads live; the buffer is tiny
  out[(long long)blockIdx.x * THREADS + threadIdx.x] = a;
}

__global__ void __launch_bounds__(THREADS) k_fill(f4* __restrict__ dst, long long n, float val) {
  const long long stride = (long long)gridDim.x * THREADS;
  const f4 v = {val, val, val, val};
  for (long long i = (long long)blockIdx.x * THREADS + threadIdx.x; i < n; i += stride)
    __builtin_nontemporal_store(v, &dst[i]);
}

}  // namespace

extern "C" {

// Runs `mode` (0 copy, 1 read, 2 write) `reps` times on the stream over
// `bytes` bytes (multiple of 16; src and dst device buffers of that size,
// 16-byte aligned; `out` a device buffer of blocks * 256 floats for the read
// mode), `blocks` workgroups of 256 threads; writes the duration of each
// repetition (HIP events, ms) into ms[0..reps-1].  Returns 0, -1 on a bad
// argument, -3 on a HIP error.
int hbm_stream(int32_t mode, const void* src, void* dst, void* out, int64_t bytes, int32_t blocks, int32_t reps,
               void* stream, float* ms) {
  if (mode < 0 || mode > 2 || bytes <= 0 || (bytes & 15) || blocks < 1 || reps < 1 || !ms) return -1;
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
      hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(THREADS), 0, st, (const f4*)src, (f4*)dst, n);
    else if (mode == 1)
      hipLaunchKernelGGL(k_read, dim3(blocks), dim3(THREADS), 0, st, (const f4*)src, (float*)out, n);
    else
      hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(THREADS), 0, st, (f4*)dst, n, (float)r);
    if (hipGetLastError() != hipSuccess || hipEventRecord(b, st) != hipSuccess ||
        hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms[r], a, b) != hipSuccess)
      rc = -3;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return rc;
}

}  // extern "C"
