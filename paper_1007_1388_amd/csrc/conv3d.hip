// conv3d.hip -- gfx950 BF16 MFMA kernels of the learned warm start.
//
// Implicit-GEMM 3-D convolutions on channels-last BF16 tensors with FP32
// accumulation on the matrix cores (v_mfma_f32_16x16x32_bf16):
//   forward      C[voxel][co]      = sum_k  patch(x)[voxel][k] * w[co][k]
//   bwd-data     C[voxel_in][ci]   = sum_k  patch^T(dy)[voxel_in][k] * wt[ci][k]
//   bwd-weight   C[co][k]          = sum_v  dy[v][co] * patch(x)[v][k]      (split over voxels)
// with k = tap * Cin + ci.  A workgroup (4 waves) computes a 128 x BN tile;
// each wave owns 32 rows (two 16-row MFMA tiles) and all BN columns.  The
// operand tiles are staged through LDS with K fastest, so every MFMA operand
// is one 16-byte LDS read per lane.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbm_surrogate.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128;     // rows per workgroup tile
constexpr int BK = 32;      // K per MFMA step
constexpr int LDK = BK + 8; // LDS row length (bf16), padded against bank conflicts

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// round to nearest even by gfx950's conversion instruction
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

struct Geo {
  int n, d, h, w, c, ldc;
};

__device__ __forceinline__ long long vox(const Geo& g, int n, int d, int h, int w) {
  return (((long long)n * g.d + d) * g.h + h) * g.w + w;
}

// Decompose a voxel index of geometry g.
__device__ __forceinline__ void unvox(const Geo& g, long long m, int& n, int& d, int& h, int& w) {
  w = (int)(m % g.w);
  long long r = m / g.w;
  h = (int)(r % g.h);
  r /= g.h;
  d = (int)(r % g.d);
  n = (int)(r / g.d);
}

// ---------------------------------------------------------- fwd / bwd-data
// MODE 0: forward.  Row m = output voxel of y; k = tap*Cin + ci; A = x at
//         input position o*stride + tap - pad.
// MODE 1: input gradient.  Row m = input voxel of dx; k = tap*Cout + co;
//         A = dy at output position (i + pad - tap)/stride when integral.
template <int MODE, int BN>
__global__ void __launch_bounds__(256) k_conv_gemm(const uint16_t* __restrict__ src, Geo gs,  // gathered tensor
                                                  const uint16_t* __restrict__ wk, int kpad,   // [BNcols][kpad]
                                                  const float* __restrict__ bias, uint16_t* __restrict__ out,
                                                  Geo go,                                       // rows = voxels of go
                                                  const uint16_t* __restrict__ act, int act_ldc, int ksize,
                                                  int stride, int relu, int accumulate, int kin) {
  __shared__ __attribute__((aligned(16))) uint16_t As[BM * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN * LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long long M = (long long)go.n * go.d * go.h * go.w;
  const long long m0 = (long long)blockIdx.x * BM;
  const int n0 = blockIdx.y * BN;
  const int ncols = go.c;
  const int pad = ksize == 3 ? 1 : 0;
  const int taps = ksize * ksize * ksize;

  // A loads: BM rows x 4 chunks of 8 -> 512 chunks, 2 per thread
  int a_row[2], a_chk[2];
  int an[2], ad[2], ah[2], aw[2];
  bool a_ok[2];
  for (int q = 0; q < 2; ++q) {
    const int id = tid + q * 256;
    a_row[q] = id >> 2;
    a_chk[q] = id & 3;
    const long long m = m0 + a_row[q];
    a_ok[q] = m < M;
    unvox(go, a_ok[q] ? m : 0, an[q], ad[q], ah[q], aw[q]);
  }
  f32x4 acc[2][BN / 16];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < BN / 16; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < kpad; k0 += BK) {
    // ---- stage A
    for (int q = 0; q < 2; ++q) {
      const int k = k0 + a_chk[q] * 8;
      const int tap = k / kin, c0 = k - tap * kin;
      u32x4 v = u32x4{0u, 0u, 0u, 0u};
      if (a_ok[q] && tap < taps) {
        const int kd = tap / (ksize * ksize), kh = (tap / ksize) % ksize, kw = tap % ksize;
        int sd, sh, sw;
        bool ok;
        if (MODE == 0) {
          sd = ad[q] * stride + kd - pad;
          sh = ah[q] * stride + kh - pad;
          sw = aw[q] * stride + kw - pad;
          ok = sd >= 0 && sd < gs.d && sh >= 0 && sh < gs.h && sw >= 0 && sw < gs.w;
        } else {
          const int td = ad[q] + pad - kd, th = ah[q] + pad - kh, tw = aw[q] + pad - kw;
          ok = td >= 0 && th >= 0 && tw >= 0 && (td % stride) == 0 && (th % stride) == 0 && (tw % stride) == 0;
          sd = td / stride;
          sh = th / stride;
          sw = tw / stride;
          ok = ok && sd < gs.d && sh < gs.h && sw < gs.w;
        }
        if (ok) v = *(const u32x4*)(src + vox(gs, an[q], sd, sh, sw) * gs.ldc + c0);
      }
      *(u32x4*)(As + a_row[q] * LDK + a_chk[q] * 8) = v;
    }
    // ---- stage B: BN rows x 4 chunks
    for (int id = tid; id < BN * 4; id += 256) {
      const int r = id >> 2, ch = id & 3;
      u32x4 v = u32x4{0u, 0u, 0u, 0u};
      if (n0 + r < ncols) v = *(const u32x4*)(wk + (long long)(n0 + r) * kpad + k0 + ch * 8);
      *(u32x4*)(Bs + r * LDK + ch * 8) = v;
    }
    __syncthreads();
    const int row = lane & 15, kg = (lane >> 4) * 8;
    bf16x8 a0 = *(const bf16x8*)(As + (wave * 32 + row) * LDK + kg);
    bf16x8 a1 = *(const bf16x8*)(As + (wave * 32 + 16 + row) * LDK + kg);
#pragma unroll
    for (int j = 0; j < BN / 16; ++j) {
      bf16x8 b = *(const bf16x8*)(Bs + (j * 16 + row) * LDK + kg);
      acc[0][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b, acc[0][j], 0, 0, 0);
      acc[1][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b, acc[1][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // ---- epilogue: lane holds D[(lane/16)*4 + r][lane%16] of each 16x16 tile
  for (int i = 0; i < 2; ++i) {
    for (int r = 0; r < 4; ++r) {
      const long long m = m0 + wave * 32 + i * 16 + (lane >> 4) * 4 + r;
      if (m >= M) continue;
#pragma unroll
      for (int j = 0; j < BN / 16; ++j) {
        const int n = n0 + j * 16 + (lane & 15);
        if (n >= ncols) continue;
        float v = acc[i][j][r];
        if (bias) v += bias[n];
        if (relu) v = v > 0.f ? v : 0.f;
        const long long o = m * go.ldc + n;
        if (act && !(bf2f(act[m * act_ldc + n]) > 0.f)) v = 0.f;
        if (accumulate) v += bf2f(out[o]);
        out[o] = f2bf(v);
      }
    }
  }
}

// ------------------------------------------------------------- bwd-weight
// C[co][k] += sum over voxels v of dy[v][co] * patch(x)[v][k].  Rows = co
// (BM = 128 covers every Cout here in one or two tiles), columns = k
// (BN = 64), K loop over 32-voxel chunks of this workgroup's voxel range.
__global__ void __launch_bounds__(256) k_conv_wgrad(const uint16_t* __restrict__ x, Geo gx,
                                                    const uint16_t* __restrict__ dy, Geo gy, float* __restrict__ dw,
                                                    int kpad, int kin, int ksize, int stride, long long vox_per_wg) {
  constexpr int BN = 64;
  __shared__ __attribute__((aligned(16))) uint16_t As[BM * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN * LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int co0 = blockIdx.x * BM;
  const int k0c = blockIdx.y * BN;
  const long long V = (long long)gy.n * gy.d * gy.h * gy.w;
  const long long vbeg = (long long)blockIdx.z * vox_per_wg;
  const long long vend = vbeg + vox_per_wg < V ? vbeg + vox_per_wg : V;
  const int pad = ksize == 3 ? 1 : 0;
  const int taps = ksize * ksize * ksize;
  const int cout = gy.c;
  f32x4 acc[2][BN / 16];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < BN / 16; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (long long v0 = vbeg; v0 < vend; v0 += BK) {
    // A[co][vox]: 32 voxels x 128 co -> 512 chunks of 8 co, 2 per thread
    for (int q = 0; q < 2; ++q) {
      const int id = tid + q * 256;
      const int vv = id & 31, cc = id >> 5;  // 16 chunks of 8 co
      const long long v = v0 + vv;
      uint16_t e[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (v < vend && co0 + cc * 8 < cout) {
        const u32x4 t = *(const u32x4*)(dy + v * gy.ldc + co0 + cc * 8);
        e[0] = t[0] & 0xffff; e[1] = t[0] >> 16; e[2] = t[1] & 0xffff; e[3] = t[1] >> 16;
        e[4] = t[2] & 0xffff; e[5] = t[2] >> 16; e[6] = t[3] & 0xffff; e[7] = t[3] >> 16;
      }
      for (int j = 0; j < 8; ++j) As[(cc * 8 + j) * LDK + vv] = e[j];
    }
    // B[k][vox]: 32 voxels x 64 k -> 256 chunks of 8 k, 1 per thread
    {
      const int vv = tid & 31, kc = tid >> 5;  // 8 chunks of 8 k
      const long long v = v0 + vv;
      const int k = k0c + kc * 8;
      const int tap = k / kin, c0 = k - tap * kin;
      uint16_t e[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (v < vend && tap < taps) {
        int n, d, h, w;
        unvox(gy, v, n, d, h, w);
        const int kd = tap / (ksize * ksize), kh = (tap / ksize) % ksize, kw = tap % ksize;
        const int sd = d * stride + kd - pad, sh = h * stride + kh - pad, sw = w * stride + kw - pad;
        if (sd >= 0 && sd < gx.d && sh >= 0 && sh < gx.h && sw >= 0 && sw < gx.w) {
          const u32x4 t = *(const u32x4*)(x + vox(gx, n, sd, sh, sw) * gx.ldc + c0);
          e[0] = t[0] & 0xffff; e[1] = t[0] >> 16; e[2] = t[1] & 0xffff; e[3] = t[1] >> 16;
          e[4] = t[2] & 0xffff; e[5] = t[2] >> 16; e[6] = t[3] & 0xffff; e[7] = t[3] >> 16;
        }
      }
      for (int j = 0; j < 8; ++j) Bs[(kc * 8 + j) * LDK + vv] = e[j];
    }
    __syncthreads();
    const int row = lane & 15, kg = (lane >> 4) * 8;
    bf16x8 a0 = *(const bf16x8*)(As + (wave * 32 + row) * LDK + kg);
    bf16x8 a1 = *(const bf16x8*)(As + (wave * 32 + 16 + row) * LDK + kg);
#pragma unroll
    for (int j = 0; j < BN / 16; ++j) {
      bf16x8 b = *(const bf16x8*)(Bs + (j * 16 + row) * LDK + kg);
      acc[0][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b, acc[0][j], 0, 0, 0);
      acc[1][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b, acc[1][j], 0, 0, 0);
    }
    __syncthreads();
  }
  for (int i = 0; i < 2; ++i)
    for (int r = 0; r < 4; ++r) {
      const int co = co0 + wave * 32 + i * 16 + (lane >> 4) * 4 + r;
      if (co >= cout) continue;
#pragma unroll
      for (int j = 0; j < BN / 16; ++j) {
        const int k = k0c + j * 16 + (lane & 15);
        if (k < kpad) atomicAdd(dw + (long long)co * kpad + k, acc[i][j][r]);
      }
    }
}

// dbias[co] += sum_v dy[v][co]
__global__ void __launch_bounds__(256) k_bias_grad(const uint16_t* __restrict__ dy, Geo gy, float* __restrict__ db,
                                                   long long vox_per_wg) {
  const long long V = (long long)gy.n * gy.d * gy.h * gy.w;
  const long long vbeg = (long long)blockIdx.x * vox_per_wg;
  const long long vend = vbeg + vox_per_wg < V ? vbeg + vox_per_wg : V;
  for (int co = threadIdx.x; co < gy.c; co += blockDim.x) {
    float s = 0.f;
    for (long long v = vbeg; v < vend; ++v) s += bf2f(dy[v * gy.ldc + co]);
    atomicAdd(db + co, s);
  }
}

// w_bf16[co][t*cin+ci] = w[co][t*cin+ci]; wt[ci][t*cout+co] = w[co][t*cin+ci]
__global__ void __launch_bounds__(256) k_weight_t(const float* __restrict__ w, int taps, int cin, int cout,
                                                  int kpad_f, int kpad_t, uint16_t* __restrict__ wb,
                                                  uint16_t* __restrict__ wt) {
  const long long nf = (long long)cout * kpad_f;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < nf; q += (long long)gridDim.x * blockDim.x) {
    const int co = (int)(q / kpad_f), k = (int)(q % kpad_f);
    wb[q] = f2bf(w[q]);
    if (k < taps * cin) {
      const int t = k / cin, ci = k % cin;
      wt[(long long)ci * kpad_t + (long long)t * cout + co] = f2bf(w[q]);
    }
  }
  // zero the K padding of wt
  const long long nt = (long long)cin * kpad_t;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < nt; q += (long long)gridDim.x * blockDim.x)
    if ((int)(q % kpad_t) >= taps * cout) wt[q] = 0;
}

__global__ void __launch_bounds__(256) k_up2(const uint16_t* __restrict__ x, Geo gx, uint16_t* __restrict__ y,
                                             Geo gy) {
  const long long V = (long long)gy.n * gy.d * gy.h * gy.w;
  const int cv = gy.c / 8;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < V * cv; q += (long long)gridDim.x * blockDim.x) {
    const long long v = q / cv;
    const int c8 = (int)(q % cv) * 8;
    int n, d, h, w;
    unvox(gy, v, n, d, h, w);
    *(u32x4*)(y + v * gy.ldc + c8) = *(const u32x4*)(x + vox(gx, n, d >> 1, h >> 1, w >> 1) * gx.ldc + c8);
  }
}

__global__ void __launch_bounds__(256) k_up2_bwd(const uint16_t* __restrict__ dy, Geo gy, uint16_t* __restrict__ dx,
                                                 Geo gx, int accumulate) {
  const long long V = (long long)gx.n * gx.d * gx.h * gx.w;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < V * gx.c; q += (long long)gridDim.x * blockDim.x) {
    const long long v = q / gx.c;
    const int c = (int)(q % gx.c);
    int n, d, h, w;
    unvox(gx, v, n, d, h, w);
    float s = 0.f;
    for (int j = 0; j < 8; ++j) {
      const int dd = 2 * d + (j >> 2), hh = 2 * h + ((j >> 1) & 1), ww = 2 * w + (j & 1);
      if (dd < gy.d && hh < gy.h && ww < gy.w) s += bf2f(dy[vox(gy, n, dd, hh, ww) * gy.ldc + c]);
    }
    if (accumulate) s += bf2f(dx[v * gx.ldc + c]);
    dx[v * gx.ldc + c] = f2bf(s);
  }
}

__global__ void __launch_bounds__(256) k_mse(const uint16_t* __restrict__ pred, Geo gp, const float* __restrict__ t,
                                             const uint8_t* __restrict__ wgt, int nch, float inv_count,
                                             uint16_t* __restrict__ dp, int dp_ldc, float* __restrict__ loss) {
  const long long V = (long long)gp.n * gp.d * gp.h * gp.w;
  float s = 0.f;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x) {
    const bool on = wgt == nullptr || wgt[v] != 0;
    for (int c = 0; c < gp.c; ++c) {
      float g = 0.f;
      if (on && c < nch) {
        const float d = bf2f(pred[v * gp.ldc + c]) - t[v * nch + c];
        s += d * d;
        g = 2.f * d * inv_count;
      }
      dp[v * dp_ldc + c] = f2bf(g);
    }
  }
  __shared__ float red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, red[0] * inv_count);
}

__global__ void __launch_bounds__(256) k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, long long n, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.f - b1) * gq;
    const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    w[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
  }
}

__global__ void __launch_bounds__(256) k_sur_input(const uint8_t* __restrict__ solid, float gnorm, uint16_t* __restrict__ x,
                                                   Geo g) {
  const long long V = (long long)g.d * g.h * g.w;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x) {
    const int d = (int)(v / ((long long)g.h * g.w));
    const float zc = g.d > 1 ? 2.f * d / (g.d - 1) - 1.f : 0.f;
    uint16_t* o = x + v * g.ldc;
    o[0] = f2bf(solid[v] ? 1.f : 0.f);
    o[1] = f2bf(gnorm);
    o[2] = f2bf(1.f - zc * zc);
    for (int c = 3; c < g.c; ++c) o[c] = 0;
  }
}

__global__ void __launch_bounds__(256) k_sur_target(const double* __restrict__ rho, const double* __restrict__ u,
                                                    const uint8_t* __restrict__ solid, double rho0, double inv,
                                                    long long V, float* __restrict__ t, uint8_t* __restrict__ wgt) {
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x) {
    const bool s = solid && solid[v];
    t[v * 4 + 0] = s ? 0.f : (float)(u[v] * inv);
    t[v * 4 + 1] = s ? 0.f : (float)(u[V + v] * inv);
    t[v * 4 + 2] = s ? 0.f : (float)(u[2 * V + v] * inv);
    t[v * 4 + 3] = s ? 0.f : (float)((rho[v] - rho0) * inv);
    wgt[v] = s ? 0 : 1;
  }
}

__global__ void __launch_bounds__(256) k_sur_fields(const uint16_t* __restrict__ p, Geo g, const uint8_t* __restrict__ solid,
                                                    double rho0, double mul, double* __restrict__ rho,
                                                    double* __restrict__ u) {
  const long long V = (long long)g.d * g.h * g.w;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x) {
    const bool s = solid && solid[v];
    const uint16_t* q = p + v * g.ldc;
    u[v] = s ? 0.0 : bf2f(q[0]) * mul;
    u[V + v] = s ? 0.0 : bf2f(q[1]) * mul;
    u[2 * V + v] = s ? 0.0 : bf2f(q[2]) * mul;
    rho[v] = s ? rho0 : rho0 + bf2f(q[3]) * mul;
  }
}

// --------------------------------------------------------------- helpers
Geo geo_of(const lbm_tensor5* t) { return Geo{t->n, t->d, t->h, t->w, t->c, t->ldc}; }

bool tensor_ok(const lbm_tensor5* t) {
  return t && t->ptr && t->n > 0 && t->d > 0 && t->h > 0 && t->w > 0 && t->c > 0 && (t->c % 8) == 0 &&
         (t->ldc % 8) == 0 && t->ldc >= t->c && (((uintptr_t)t->ptr) & 15) == 0;
}

int outdim(int in, int stride) { return (in + stride - 1) / stride; }

int grid1(long long n) {
  long long g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  return (int)(g < 1 ? 1 : g);
}

}  // namespace

extern "C" {

int32_t lbm_conv_kpad(int32_t taps, int32_t cin) { return ((taps * cin + 31) / 32) * 32; }

lbm_status lbm_conv3d_fwd(const lbm_tensor5* x, const uint16_t* w, const float* bias, const lbm_tensor5* y,
                          int32_t ksize, int32_t stride, int32_t relu, void* stream) {
  if (!tensor_ok(x) || !tensor_ok(y) || !w || (ksize != 1 && ksize != 3) || (stride != 1 && stride != 2) ||
      (ksize == 1 && stride != 1))
    return LBM_EINVAL;
  if (y->n != x->n || y->d != outdim(x->d, stride) || y->h != outdim(x->h, stride) || y->w != outdim(x->w, stride))
    return LBM_EINVAL;
  const int taps = ksize * ksize * ksize;
  const int kpad = lbm_conv_kpad(taps, x->c);
  const long long M = (long long)y->n * y->d * y->h * y->w;
  hipStream_t s = (hipStream_t)stream;
  const Geo gs = geo_of(x), go = geo_of(y);
  const dim3 b(256);
  if (y->c <= 16) {
    dim3 g((unsigned)((M + BM - 1) / BM), (y->c + 15) / 16);
    hipLaunchKernelGGL((k_conv_gemm<0, 16>), g, b, 0, s, (const uint16_t*)x->ptr, gs, w, kpad, bias,
                       (uint16_t*)y->ptr, go, (const uint16_t*)nullptr, 0, ksize, stride, relu, 0, x->c);
  } else if (y->c <= 32) {
    dim3 g((unsigned)((M + BM - 1) / BM), 1);
    hipLaunchKernelGGL((k_conv_gemm<0, 32>), g, b, 0, s, (const uint16_t*)x->ptr, gs, w, kpad, bias,
                       (uint16_t*)y->ptr, go, (const uint16_t*)nullptr, 0, ksize, stride, relu, 0, x->c);
  } else {
    dim3 g((unsigned)((M + BM - 1) / BM), (y->c + 63) / 64);
    hipLaunchKernelGGL((k_conv_gemm<0, 64>), g, b, 0, s, (const uint16_t*)x->ptr, gs, w, kpad, bias,
                       (uint16_t*)y->ptr, go, (const uint16_t*)nullptr, 0, ksize, stride, relu, 0, x->c);
  }
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

lbm_status lbm_conv3d_bwd_data(const lbm_tensor5* dy, const uint16_t* w_t, const lbm_tensor5* dx,
                               const lbm_tensor5* act, int32_t ksize, int32_t stride, int32_t accumulate,
                               void* stream) {
  if (!tensor_ok(dy) || !tensor_ok(dx) || !w_t || (ksize != 1 && ksize != 3) || (stride != 1 && stride != 2) ||
      (ksize == 1 && stride != 1))
    return LBM_EINVAL;
  if (dy->n != dx->n || dy->d != outdim(dx->d, stride) || dy->h != outdim(dx->h, stride) ||
      dy->w != outdim(dx->w, stride))
    return LBM_EINVAL;
  if (act && (!tensor_ok(act) || act->n != dx->n || act->d != dx->d || act->h != dx->h || act->w != dx->w ||
              act->c < dx->c))
    return LBM_EINVAL;
  const int taps = ksize * ksize * ksize;
  const int kpad = lbm_conv_kpad(taps, dy->c);
  const long long M = (long long)dx->n * dx->d * dx->h * dx->w;
  hipStream_t s = (hipStream_t)stream;
  const Geo gs = geo_of(dy), go = geo_of(dx);
  const uint16_t* ap = act ? (const uint16_t*)act->ptr : nullptr;
  const int aldc = act ? act->ldc : 0;
  const dim3 b(256);
  if (dx->c <= 16) {
    dim3 g((unsigned)((M + BM - 1) / BM), (dx->c + 15) / 16);
    hipLaunchKernelGGL((k_conv_gemm<1, 16>), g, b, 0, s, (const uint16_t*)dy->ptr, gs, w_t, kpad,
                       (const float*)nullptr, (uint16_t*)dx->ptr, go, ap, aldc, ksize, stride, 0, accumulate, dy->c);
  } else if (dx->c <= 32) {
    dim3 g((unsigned)((M + BM - 1) / BM), 1);
    hipLaunchKernelGGL((k_conv_gemm<1, 32>), g, b, 0, s, (const uint16_t*)dy->ptr, gs, w_t, kpad,
                       (const float*)nullptr, (uint16_t*)dx->ptr, go, ap, aldc, ksize, stride, 0, accumulate, dy->c);
  } else {
    dim3 g((unsigned)((M + BM - 1) / BM), (dx->c + 63) / 64);
    hipLaunchKernelGGL((k_conv_gemm<1, 64>), g, b, 0, s, (const uint16_t*)dy->ptr, gs, w_t, kpad,
                       (const float*)nullptr, (uint16_t*)dx->ptr, go, ap, aldc, ksize, stride, 0, accumulate, dy->c);
  }
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

lbm_status lbm_conv3d_bwd_weight(const lbm_tensor5* x, const lbm_tensor5* dy, float* dw, float* dbias,
                                 int32_t ksize, int32_t stride, void* stream) {
  if (!tensor_ok(x) || !tensor_ok(dy) || !dw || (ksize != 1 && ksize != 3) || (stride != 1 && stride != 2) ||
      (ksize == 1 && stride != 1))
    return LBM_EINVAL;
  if (dy->n != x->n || dy->d != outdim(x->d, stride) || dy->h != outdim(x->h, stride) || dy->w != outdim(x->w, stride))
    return LBM_EINVAL;
  const int taps = ksize * ksize * ksize;
  const int kpad = lbm_conv_kpad(taps, x->c);
  const long long V = (long long)dy->n * dy->d * dy->h * dy->w;
  hipStream_t s = (hipStream_t)stream;
  const dim3 b(256);
  const int gm = (dy->c + BM - 1) / BM, gn = (kpad + 63) / 64;
  // split the voxel range so that the grid holds about 2048 workgroups
  long long splits = 2048 / (gm * gn);
  if (splits < 1) splits = 1;
  long long per = (V + splits - 1) / splits;
  per = ((per + BK - 1) / BK) * BK;
  splits = (V + per - 1) / per;
  dim3 g(gm, gn, (unsigned)splits);
  hipLaunchKernelGGL(k_conv_wgrad, g, b, 0, s, (const uint16_t*)x->ptr, geo_of(x), (const uint16_t*)dy->ptr,
                     geo_of(dy), dw, kpad, x->c, ksize, stride, per);
  if (dbias) {
    long long pb = 4096;
    hipLaunchKernelGGL(k_bias_grad, dim3((unsigned)((V + pb - 1) / pb)), b, 0, s, (const uint16_t*)dy->ptr,
                       geo_of(dy), dbias, pb);
  }
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

lbm_status lbm_conv3d_weight_t(const float* w_master, int32_t taps, int32_t cin, int32_t cout, uint16_t* w_bf16,
                               uint16_t* wt_bf16, void* stream) {
  if (!w_master || !w_bf16 || !wt_bf16 || (taps != 1 && taps != 27) || cin <= 0 || cout <= 0 || (cin % 8) ||
      (cout % 8))
    return LBM_EINVAL;
  const int kf = lbm_conv_kpad(taps, cin), kt = lbm_conv_kpad(taps, cout);
  const long long n = (long long)cout * kf > (long long)cin * kt ? (long long)cout * kf : (long long)cin * kt;
  hipLaunchKernelGGL(k_weight_t, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, w_master, taps, cin, cout, kf,
                     kt, w_bf16, wt_bf16);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

lbm_status lbm_upsample2(const lbm_tensor5* x, const lbm_tensor5* y, void* stream) {
  if (!tensor_ok(x) || !tensor_ok(y) || y->n != x->n || y->c != x->c || y->d != 2 * x->d || y->h != 2 * x->h ||
      y->w != 2 * x->w)
    return LBM_EINVAL;
  const long long n = (long long)y->n * y->d * y->h * y->w * (y->c / 8);
  hipLaunchKernelGGL(k_up2, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, (const uint16_t*)x->ptr, geo_of(x),
                     (uint16_t*)y->ptr, geo_of(y));
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

lbm_status lbm_upsample2_bwd(const lbm_tensor5* dy, const lbm_tensor5* dx, int32_t accumulate, void* stream) {
  if (!tensor_ok(dy) || !tensor_ok(dx) || dy->n != dx->n || dy->c != dx->c || dy->d != 2 * dx->d ||
      dy->h != 2 * dx->h || dy->w != 2 * dx->w)
    return LBM_EINVAL;
  const long long n = (long long)dx->n * dx->d * dx->h * dx->w * dx->c;
  hipLaunchKernelGGL(k_up2_bwd, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, (const uint16_t*)dy->ptr,
                     geo_of(dy), (uint16_t*)dx->ptr, geo_of(dx), accumulate);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

lbm_status lbm_mse_loss(const lbm_tensor5* pred, const float* target, const uint8_t* weight, int32_t nch,
                        float inv_count, const lbm_tensor5* dpred, float* loss, void* stream) {
  if (!tensor_ok(pred) || !tensor_ok(dpred) || !target || !loss || nch <= 0 || nch > pred->c ||
      dpred->c != pred->c || dpred->n != pred->n || dpred->d != pred->d || dpred->h != pred->h || dpred->w != pred->w)
    return LBM_EINVAL;
  const long long V = (long long)pred->n * pred->d * pred->h * pred->w;
  int g = grid1(V);
  if (g > 2048) g = 2048;
  hipLaunchKernelGGL(k_mse, dim3(g), dim3(256), 0, (hipStream_t)stream, (const uint16_t*)pred->ptr, geo_of(pred),
                     target, weight, nch, inv_count, (uint16_t*)dpred->ptr, dpred->ldc, loss);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

lbm_status lbm_adam_step(float* w, const float* g, float* m, float* v, int64_t n, float lr, float beta1, float beta2,
                         float eps, int32_t t, void* stream) {
  if (!w || !g || !m || !v || n <= 0 || t < 1) return LBM_EINVAL;
  const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, w, g, m, v, (long long)n, lr, beta1,
                     beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

lbm_status lbm_surrogate_input(const uint8_t* solid, double gx, const lbm_tensor5* x, void* stream) {
  if (!solid || !tensor_ok(x) || x->c < 8 || x->n != 1 || !(gx > 0)) return LBM_EINVAL;
  const float gnorm = (float)((log10(gx) + 5.8) / 0.5);
  const long long V = (long long)x->d * x->h * x->w;
  hipLaunchKernelGGL(k_sur_input, dim3(grid1(V)), dim3(256), 0, (hipStream_t)stream, solid, gnorm,
                     (uint16_t*)x->ptr, geo_of(x));
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

lbm_status lbm_surrogate_target(const double* rho, const double* u, const uint8_t* solid, double rho0, double gx,
                                double scale, int64_t voxels, float* target, uint8_t* weight, void* stream) {
  if (!rho || !u || !target || !weight || voxels <= 0 || !(gx > 0) || !(scale > 0)) return LBM_EINVAL;
  hipLaunchKernelGGL(k_sur_target, dim3(grid1(voxels)), dim3(256), 0, (hipStream_t)stream, rho, u, solid, rho0,
                     1.0 / (gx * scale), (long long)voxels, target, weight);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

lbm_status lbm_surrogate_fields(const lbm_tensor5* pred, const uint8_t* solid, double rho0, double gx, double scale,
                                double* rho, double* u, void* stream) {
  if (!tensor_ok(pred) || pred->n != 1 || !rho || !u || !(gx > 0) || !(scale > 0)) return LBM_EINVAL;
  const long long V = (long long)pred->d * pred->h * pred->w;
  hipLaunchKernelGGL(k_sur_fields, dim3(grid1(V)), dim3(256), 0, (hipStream_t)stream, (const uint16_t*)pred->ptr,
                     geo_of(pred), solid, rho0, gx * scale, rho, u);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

}  // extern "C"
