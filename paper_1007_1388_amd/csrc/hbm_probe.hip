// hbm_probe.hip -- HBM bandwidth ceilings of plain access patterns on gfx950:
// read-only, write-only and copy streams of 16-byte accesses (grid-strided or
// in one contiguous chunk per workgroup), a two-read one-write triad, the
// sweep's 19-read 19-write stream pattern, and the runtime's own
// device-to-device copy and fill, with several independent accesses in
// flight per thread and streaming or ordinary loads/stores.  The sweep's
// bandwidth is read against these (the paper's attainable-bandwidth method,
// Sec. 3.1, extended from one copy kernel to several patterns).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/lbm.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ f4 ld(const f4* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT>
__device__ __forceinline__ void st(f4 v, f4* p) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// KIND 0: read a (a sum that the compiler cannot drop goes to b[0] only if
// it equals an impossible value); 1: write b; 2: copy a -> b.  Thread i
// touches i, i + S, ..., U at a time (S = all threads of the grid).
template <int KIND, int U, bool NT>
__global__ void __launch_bounds__(256) k_hbm(const f4* __restrict__ a, f4* __restrict__ b, long long n) {
  const long long S = (long long)gridDim.x * blockDim.x;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  const f4 w = {1.f, 2.f, 3.f, 4.f};
  for (; i + (U - 1) * S < n; i += U * S) {
    f4 v[U];
    if constexpr (KIND != 1) {
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = ld<NT>(a + i + u * S);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (KIND == 0) acc += v[u];
      if constexpr (KIND == 1) st<NT>(w, b + i + u * S);
      if constexpr (KIND == 2) st<NT>(v[u], b + i + u * S);
    }
  }
  for (; i < n; i += S) {
    if constexpr (KIND == 0) acc += a[i];
    if constexpr (KIND == 1) b[i] = w;
    if constexpr (KIND == 2) b[i] = a[i];
  }
  if constexpr (KIND == 0)
    if (acc[0] + acc[1] + acc[2] + acc[3] == -1.2345e-30f) b[0] = acc;
}

// KIND 3: copy a -> b in contiguous chunks, one chunk per workgroup (the
// workgroup's threads sweep it 16 bytes apart, U accesses in flight), so
// each workgroup streams one address range instead of interleaving with all
// others.
template <int U, bool NT>
__global__ void __launch_bounds__(256) k_hbm_chunk(const f4* __restrict__ a, f4* __restrict__ b, long long n) {
  const long long per = (n + gridDim.x - 1) / gridDim.x;
  const long long lo = (long long)blockIdx.x * per;
  const long long hi = lo + per < n ? lo + per : n;
  long long i = lo + threadIdx.x;
  const long long S = blockDim.x;
  for (; i + (U - 1) * S < hi; i += U * S) {
    f4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = ld<NT>(a + i + u * S);
#pragma unroll
    for (int u = 0; u < U; ++u) st<NT>(v[u], b + i + u * S);
  }
  for (; i < hi; i += S) b[i] = a[i];
}

// KIND 4: triad b = a0 + 3 a1 (two read streams, one write stream; a holds
// a0 then a1, each n vectors).
template <int U, bool NT>
__global__ void __launch_bounds__(256) k_hbm_triad(const f4* __restrict__ a, f4* __restrict__ b, long long n) {
  const long long S = (long long)gridDim.x * blockDim.x;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const f4* a1 = a + n;
  for (; i + (U - 1) * S < n; i += U * S) {
    f4 v[U], w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v[u] = ld<NT>(a + i + u * S);
      w[u] = ld<NT>(a1 + i + u * S);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) st<NT>(v[u] + 3.f * w[u], b + i + u * S);
  }
  for (; i < n; i += S) b[i] = a[i] + 3.f * a1[i];
}

// KIND 5: the stream-collide sweep's access pattern without its arithmetic:
// 19 source arrays and 19 destination arrays (starts staggered like the
// sweep's population arrays), each lane reading one W-byte word of all 19
// sources (all loads in flight) and writing it to the 19 destinations.
template <int W> struct Word;
template <> struct Word<4> { typedef float V; };
template <> struct Word<8> { typedef float V __attribute__((ext_vector_type(2))); };
template <> struct Word<16> { typedef float V __attribute__((ext_vector_type(4))); };

template <int W, bool NT>
__global__ void __launch_bounds__(256) k_hbm_q19(const char* __restrict__ a, char* __restrict__ b, long long m,
                                                 long long stride) {
  typedef typename Word<W>::V V;
  const long long S = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += S) {
    V v[19];
#pragma unroll
    for (int q = 0; q < 19; ++q) {
      const V* p = (const V*)(a + q * stride) + i;
      if constexpr (NT) v[q] = __builtin_nontemporal_load(p);
      else v[q] = *p;
    }
#pragma unroll
    for (int q = 0; q < 19; ++q) {
      V* p = (V*)(b + q * stride) + i;
      if constexpr (NT) __builtin_nontemporal_store(v[q], p);
      else *p = v[q];
    }
  }
}

using ProbeFn = void (*)(const f4*, f4*, long long, int, hipStream_t);

template <int KIND, int U, bool NT>
void launch(const f4* a, f4* b, long long n, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_hbm<KIND, U, NT>), dim3(grid), dim3(256), 0, s, a, b, n);
}

template <int KIND, bool NT>
ProbeFn pick_u(int u) {
  switch (u) {
    case 1: return launch<KIND, 1, NT>;
    case 2: return launch<KIND, 2, NT>;
    case 4: return launch<KIND, 4, NT>;
    default: return launch<KIND, 8, NT>;
  }
}

template <int KIND>
ProbeFn pick(int u, bool nt) { return nt ? pick_u<KIND, true>(u) : pick_u<KIND, false>(u); }

template <int U, bool NT>
void launch_chunk(const f4* a, f4* b, long long n, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_hbm_chunk<U, NT>), dim3(grid), dim3(256), 0, s, a, b, n);
}
template <int U, bool NT>
void launch_triad(const f4* a, f4* b, long long n, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_hbm_triad<U, NT>), dim3(grid), dim3(256), 0, s, a, b, n);
}
#define LBM_PICK_U(FN)                                                 \
  template <bool NT>                                                   \
  ProbeFn FN##_u(int u) {                                              \
    switch (u) {                                                       \
      case 1: return FN<1, NT>;                                        \
      case 2: return FN<2, NT>;                                        \
      case 4: return FN<4, NT>;                                        \
      default: return FN<8, NT>;                                       \
    }                                                                  \
  }
LBM_PICK_U(launch_chunk)
LBM_PICK_U(launch_triad)
#undef LBM_PICK_U

// 19-stream sweep pattern: `bytes` per side split into 19 arrays of m words
// of W = 4 * unroll bytes (unroll 1, 2 or 4), array starts 768 bytes past a
// 4 KiB multiple apart.
struct Q19 {
  long long m, stride;
};
Q19 q19_shape(size_t bytes, int w) {
  long long per = (long long)(bytes / 19) / 4096 * 4096;
  while (per > 0 && 19 * per + 18 * 768 > (long long)bytes) per -= 4096;
  return Q19{per / w, per + 768};
}
void launch_q19(int w, bool nt, const void* a, void* b, const Q19& q, int grid, hipStream_t s) {
  const char* ca = (const char*)a;
  char* cb = (char*)b;
#define LBM_Q19(W, N) hipLaunchKernelGGL((k_hbm_q19<W, N>), dim3(grid), dim3(256), 0, s, ca, cb, q.m, q.stride)
  if (w == 4) { if (nt) LBM_Q19(4, true); else LBM_Q19(4, false); }
  else if (w == 8) { if (nt) LBM_Q19(8, true); else LBM_Q19(8, false); }
  else { if (nt) LBM_Q19(16, true); else LBM_Q19(16, false); }
#undef LBM_Q19
}

}  // namespace

extern "C" lbm_status lbm_hbm_probe(int32_t kind, int32_t unroll, int32_t nontemporal, const void* a, void* b,
                                    size_t bytes, int32_t grid, int32_t reps, void* stream, double* ms) {
  const bool u_ok = kind == 5 ? (unroll == 1 || unroll == 2 || unroll == 4)
                              : (unroll == 1 || unroll == 2 || unroll == 4 || unroll == 8);
  if (kind < 0 || kind > 7 || !u_ok || !b || !ms || (kind != 1 && kind != 7 && !a) || bytes < 16 ||
      (bytes % 16) != 0 || reps < 1 || grid < 0 || grid > (1 << 22) || (kind == 5 && bytes < (size_t)19 * 8192))
    return LBM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (grid == 0) {
    int dev = 0, cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      cus = prop.multiProcessorCount;
    grid = 16 * cus;
  }
  const long long n = (long long)(bytes / 16);
  const bool nt = nontemporal != 0;
  ProbeFn fn = nullptr;
  switch (kind) {
    case 0: fn = pick<0>(unroll, nt); break;
    case 1: fn = pick<1>(unroll, nt); break;
    case 2: fn = pick<2>(unroll, nt); break;
    case 3: fn = nt ? launch_chunk_u<true>(unroll) : launch_chunk_u<false>(unroll); break;
    case 4: fn = nt ? launch_triad_u<true>(unroll) : launch_triad_u<false>(unroll); break;
    default: break;
  }
  const Q19 q = q19_shape(bytes, 4 * unroll);
  auto pass = [&]() -> hipError_t {
    if (fn) {
      fn((const f4*)a, (f4*)b, n, grid, s);
      return hipSuccess;
    }
    if (kind == 5) {
      launch_q19(4 * unroll, nt, a, b, q, grid, s);
      return hipSuccess;
    }
    if (kind == 6) return hipMemcpyAsync(b, a, bytes, hipMemcpyDeviceToDevice, s);
    return hipMemsetD32Async((hipDeviceptr_t)b, 0x3f800000u, bytes / 4, s);
  };
  if (pass() != hipSuccess) return LBM_EDEVICE;  // warm-up
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return LBM_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return LBM_EDEVICE;
  }
  bool ok = hipEventRecord(e0, s) == hipSuccess;
  for (int r = 0; r < reps && ok; ++r) ok = pass() == hipSuccess;
  ok = ok && hipEventRecord(e1, s) == hipSuccess;
  float t = 0.f;
  ok = ok && hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&t, e0, e1) == hipSuccess &&
       hipGetLastError() == hipSuccess;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!ok) return LBM_EDEVICE;
  *ms = t / reps;
  return LBM_OK;
}
