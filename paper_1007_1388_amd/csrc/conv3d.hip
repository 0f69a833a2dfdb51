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

// ------------------------------------------- fwd / bwd-data, tap-major
// The same products with the K loop ordered tap by tap (C gathered channels
// per tap, C a multiple of 32), for the shapes where that holds:
//  * each wave's A operand goes straight from memory into the MFMA registers
//    (lane = row l%16, K group l/16: one 16-byte load of 8 channels of the
//    tap's source voxel), through a raw buffer resource whose range check
//    returns zeros for taps outside the volume;
//  * every row's tap validity is a bit mask computed once, and the tap
//    offset is uniform per K step, so a K step costs each lane one add, one
//    select and one load per A fragment;
//  * the weight tile (shared by the four waves) is double-buffered in LDS,
//    one barrier per K step, and the next step's loads are in flight while
//    the current step's MFMAs run;
//  * the stride-2 input gradient runs per output parity class (grid.z): an
//    input voxel i receives only from taps k with k = i + 1 mod 2 on every
//    axis, so each class runs its 1, 2, 4 or 8 taps instead of 27.
// A wave owns FM 16-row fragments and all 16*FN columns of the tile.
struct DArgs {
  const uint16_t* src;
  Geo gs;
  unsigned src_bytes;  // range of the gathered view, for the buffer resource
  const uint16_t* wk;
  int kstride;         // weight row length
  unsigned wk_bytes;
  const float* bias;
  uint16_t* out;
  Geo go;
  const uint16_t* act;
  int act_ldc;
  int ksize, stride, relu, accumulate, C;
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)bytes, 0x00020000);
}

template <int MODE, bool CLS, int FM, int FN>
__global__ void __launch_bounds__(256) k_conv_tap(DArgs a) {
  constexpr int BN = 16 * FN, WM = 16 * FM, BMW = 4 * WM;
  constexpr int LDB = 40;  // padded weight-tile row (bf16)
  constexpr unsigned OOB = 0x80000000u;
  // weight chunks per thread (BN rows x 4 chunks of 8); rows past BN are
  // spare, so that every thread stores and the loop has no branch
  constexpr int NB = (BN * 4 + 255) / 256;
  constexpr int BROWS = NB * 64;
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BROWS * LDB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const Geo gs = a.gs, go = a.go;
  const int pad = a.ksize == 3 ? 1 : 0;
  // parity class and its row grid (CLS), else the whole output grid
  int pcl[3] = {0, 0, 0};
  int cd = go.d, ch = go.h, cw = go.w;
  if (CLS) {
    pcl[0] = blockIdx.z & 1;
    pcl[1] = (blockIdx.z >> 1) & 1;
    pcl[2] = (blockIdx.z >> 2) & 1;
    cd = (go.d - pcl[0] + 1) >> 1;
    ch = (go.h - pcl[1] + 1) >> 1;
    cw = (go.w - pcl[2] + 1) >> 1;
  }
  // per-axis tap lists: entry j has kernel index kk(j) and source shift dl(j)
  //   MODE 0:        kk = j, source = o*stride - pad + j
  //   MODE 1, s = 1: kk = j, source = i + pad - j
  //   MODE 1, s = 2: kk = p ? 2j : 1, source = (i + 1)/2 - j  (p = i mod 2)
  int na[3];
  for (int x = 0; x < 3; ++x) na[x] = CLS ? (pcl[x] ? 2 : 1) : a.ksize;
  const int Mrows = go.n * cd * ch * cw;
  const int m0 = blockIdx.x * BMW + wave * WM;

  int basef[FM], voxf[FM];
  unsigned mskf[FM];
#pragma unroll
  for (int f = 0; f < FM; ++f) {
    const int m = m0 + f * 16 + (lane & 15);
    const bool ok = m < Mrows;
    int r = ok ? m : 0;
    int c3[3];
    c3[2] = r % cw; r /= cw;
    c3[1] = r % ch; r /= ch;
    c3[0] = r % cd;
    const int n = r / cd;
    if (CLS)
      for (int x = 0; x < 3; ++x) c3[x] = 2 * c3[x] + pcl[x];
    voxf[f] = ok ? ((n * go.d + c3[0]) * go.h + c3[1]) * go.w + c3[2] : -1;
    const int ext[3] = {gs.d, gs.h, gs.w};
    int b3[3];
    unsigned v3[3];
    for (int x = 0; x < 3; ++x) {
      b3[x] = MODE == 0 ? c3[x] * a.stride - pad : (CLS ? (c3[x] + 1) >> 1 : c3[x] + pad);
      unsigned v = 0;
      for (int j = 0; j < na[x]; ++j) {
        const int sx = MODE == 0 ? b3[x] + j : b3[x] - j;
        if (sx >= 0 && sx < ext[x]) v |= 1u << j;
      }
      v3[x] = v;
    }
    unsigned mm = 0;
    for (int jd = 0; jd < na[0]; ++jd)
      for (int jh = 0; jh < na[1]; ++jh)
        for (int jw = 0; jw < na[2]; ++jw)
          if ((v3[0] >> jd) & (v3[1] >> jh) & (v3[2] >> jw) & 1u) mm |= 1u << ((jd * na[1] + jh) * na[2] + jw);
    mskf[f] = ok ? mm : 0u;
    basef[f] = (((n * gs.d + b3[0]) * gs.h + b3[1]) * gs.w + b3[2]) * gs.ldc + (lane >> 4) * 8;
  }

  const __amdgpu_buffer_rsrc_t rs = rsrc_of(a.src, a.src_bytes);
  const __amdgpu_buffer_rsrc_t rw = rsrc_of(a.wk, a.wk_bytes);
  const int n0 = blockIdx.y * BN;
  const int ncols = go.c;
  const int cpt = a.C >> 5;  // K steps per tap
  const int nsub = na[0] * na[1] * na[2] * cpt;

  // uniform K-step state: tap position (jd, jh, jw) and channel offset c0
  struct St {
    int jd, jh, jw, c0;
  };
  auto tap_of = [&](const St& q, int& off, int& bit, int& t) {
    int dd, dh, dw, kd, kh, kw;
    if (CLS) {
      dd = -q.jd; dh = -q.jh; dw = -q.jw;
      kd = pcl[0] ? 2 * q.jd : 1; kh = pcl[1] ? 2 * q.jh : 1; kw = pcl[2] ? 2 * q.jw : 1;
    } else {
      dd = MODE == 0 ? q.jd : -q.jd; dh = MODE == 0 ? q.jh : -q.jh; dw = MODE == 0 ? q.jw : -q.jw;
      kd = q.jd; kh = q.jh; kw = q.jw;
    }
    off = ((dd * gs.h + dh) * gs.w + dw) * gs.ldc + q.c0;
    bit = (q.jd * na[1] + q.jh) * na[2] + q.jw;
    t = (kd * a.ksize + kh) * a.ksize + kw;
  };
  // branch-free, so that the K loop stays one loop
  auto advance = [&](St& q) {
    q.c0 += 32;
    const int cw_ = q.c0 == a.C;
    q.c0 = cw_ ? 0 : q.c0;
    q.jw += cw_;
    const int ww = q.jw == na[2];
    q.jw = ww ? 0 : q.jw;
    q.jh += ww;
    const int hw = q.jh == na[1];
    q.jh = hw ? 0 : q.jh;
    q.jd += hw;
  };
  // An offset with the high bit set lies past the buffer's range, which
  // loads zeros without touching memory (proper offsets stay below 2^31).
  // `dead` is OOB for the step after the last, so every step issues the same
  // loads, with no branch, and the waits stay exact.
  auto load_a = [&](int off, int bit, unsigned dead, u32x4* dst) {
#pragma unroll
    for (int f = 0; f < FM; ++f) {
      const unsigned vo = (unsigned)(basef[f] + off) * 2u | ((~(mskf[f] >> bit) & 1u) << 31) | dead;
      dst[f] = __builtin_amdgcn_raw_buffer_load_b128(rs, vo, 0, 0);
    }
  };
  // per-thread weight offsets; the high bit sends a spare or missing row
  // out of range (offsets proper stay below 2^31)
  unsigned boff[NB], bpen[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int id = tid + i * 256;
    const int r = id >> 2, chk = id & 3;
    const bool ok = id < BN * 4 && n0 + r < ncols;
    boff[i] = (unsigned)((ok ? n0 + r : 0) * a.kstride + chk * 8) * 2u;
    bpen[i] = ok ? 0u : OOB;
  }
  auto load_b = [&](int t, int c0, unsigned dead, u32x4* dst) {
    const unsigned kb = (unsigned)(t * a.C + c0) * 2u;
#pragma unroll
    for (int i = 0; i < NB; ++i)
      dst[i] = __builtin_amdgcn_raw_buffer_load_b128(rw, (boff[i] + kb) | bpen[i] | dead, 0, 0);
  };
  auto store_b = [&](int buf, const u32x4* v) {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int id = tid + i * 256;
      *(u32x4*)(&Bs[buf][(id >> 2) * LDB + (id & 3) * 8]) = v[i];
    }
  };

  f32x4 acc[FM][FN];
#pragma unroll
  for (int f = 0; f < FM; ++f)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[f][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  St st{0, 0, 0, 0};
  u32x4 acur[FM], anxt[FM], breg[NB];
  {
    int off, bit, t;
    tap_of(st, off, bit, t);
    load_b(t, 0, 0u, breg);
    load_a(off, bit, 0u, acur);
  }
  store_b(0, breg);
  __syncthreads();
  // K step s: issue the loads of step s + 1 (weights first, so that staging
  // them waits for no A load), multiply step s (operands in acur, weights in
  // LDS buffer s & 1), then stage the next weights
  // two steps per iteration, the A registers alternating between acur and
  // anxt, so that a load is first waited for one step after its issue
#define LBM_CONV_KSTEP(S, CUR, NXT)                                                                          \
  {                                                                                                        \
    advance(st);                                                                                           \
    const unsigned dead = (unsigned)(nsub - 2 - (S)) & OOB; /* S + 1 == nsub */                            \
    int off, bit, t;                                                                                       \
    tap_of(st, off, bit, t);                                                                               \
    load_b(t, st.c0, dead, breg);                                                                          \
    load_a(off, bit, dead, NXT);                                                                           \
    __builtin_amdgcn_sched_barrier(0); /* the loads stay ahead of the MFMAs */                             \
    const uint16_t* B = Bs[(S) & 1];                                                                       \
    _Pragma("unroll") for (int j = 0; j < FN; ++j) {                                                       \
      const bf16x8 b = *(const bf16x8*)(B + (j * 16 + (lane & 15)) * LDB + (lane >> 4) * 8);               \
      _Pragma("unroll") for (int f = 0; f < FM; ++f) acc[f][j] =                                           \
          __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, CUR[f]), b, acc[f][j], 0, 0, 0); \
    }                                                                                                      \
    store_b(((S) + 1) & 1, breg);                                                                          \
    __syncthreads();                                                                                       \
  }
  int s = 0;
  for (; s + 1 < nsub; s += 2) {
    LBM_CONV_KSTEP(s, acur, anxt)
    LBM_CONV_KSTEP(s + 1, anxt, acur)
  }
  if (s < nsub) LBM_CONV_KSTEP(s, acur, anxt)
#undef LBM_CONV_KSTEP
  // ---- epilogue: lane holds D[(lane/16)*4 + r][lane%16] of each 16x16 tile;
  // the voxel of D row q is held by lane q (A layout row q)
#pragma unroll
  for (int f = 0; f < FM; ++f) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int vo = __shfl(voxf[f], (lane >> 4) * 4 + r);
      if (vo < 0) continue;
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int n = n0 + j * 16 + (lane & 15);
        if (n >= ncols) continue;
        float v = acc[f][j][r];
        if (a.bias) v += a.bias[n];
        if (a.relu) v = v > 0.f ? v : 0.f;
        const long long o = (long long)vo * go.ldc + n;
        if (a.act && !(bf2f(a.act[(long long)vo * a.act_ldc + n]) > 0.f)) v = 0.f;
        if (a.accumulate) v += bf2f(a.out[o]);
        a.out[o] = f2bf(v);
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

// ------------------------------------ fwd / bwd-data, stride 1, 3x3x3 halos
// The stride-1 3x3x3 products with 32 or 64 output columns (the
// full-resolution layers), where every gathered A element feeds only two or
// four MFMAs and the tap-major kernel runs at the L1/L2 gather rate.  A
// workgroup owns an 8 x 32 block of output voxels (rows h0.., columns w0..
// of one plane) and all output columns; per kernel plane kd and 32-channel
// chunk it stages in LDS
//   * the input halo  [10 rows][34 columns][32 channels] of source plane
//     d + kd - 1 (forward) or d + 1 - kd (input gradient), and
//   * the weights     [9 taps][columns][32 channels] of that plane and chunk,
// then runs the nine (kh, kw) taps on them: both MFMA operands are 16-byte
// LDS reads with channels as K, so each input value is fetched from memory
// once per (kd, chunk) instead of nine times.  The next stage's loads go to
// registers while the taps run and reach LDS after the next barrier.  Wave v owns output rows
// h0 + 2v and h0 + 2v + 1 (four 16-voxel fragments).  MODE 1 reads the taps
// mirrored (source i + 1 - k) with the transposed weights.
template <int MODE, int FN>
__global__ void __launch_bounds__(256) k_conv_halo(DArgs a) {
  constexpr int BN = 16 * FN;
  constexpr int HR = 10, HC = 34, PC = 40;  // halo rows, columns, cell pitch (bf16)
  constexpr int PW = 40;                    // weight row pitch (bf16)
  constexpr int NX = HR * HC * 4;           // halo chunks of 8 channels
  constexpr int NW = 9 * BN * 4;            // weight chunks
  constexpr unsigned OOB = 0x80000000u;
  __shared__ __attribute__((aligned(16))) uint16_t Xs[HR * HC * PC];
  __shared__ __attribute__((aligned(16))) uint16_t Ws[9 * BN * PW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const Geo gs = a.gs, go = a.go;
  // output block of this workgroup
  const int nwb = go.w / 32, nhb = (go.h + 7) / 8;
  int bx = blockIdx.x;
  const int wb = bx % nwb;
  bx /= nwb;
  const int hb = bx % nhb;
  bx /= nhb;
  const int d = bx % go.d, n = bx / go.d;
  const int h0 = hb * 8, w0 = wb * 32;
  const int C = a.C;
  const int ncols = go.c;
  const __amdgpu_buffer_rsrc_t rs = rsrc_of(a.src, a.src_bytes);
  const __amdgpu_buffer_rsrc_t rw = rsrc_of(a.wk, a.wk_bytes);

  f32x4 acc[4][FN];
#pragma unroll
  for (int f = 0; f < 4; ++f)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[f][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  // Per-thread staging slots.  Halo slot i covers cell (r, c) and 8
  // channels q; its offset within the source plane is fixed, the plane and
  // the chunk change per stage.  Weight slot j covers one column's 8
  // channels of one (kh, kw) tap.  A slot outside the tensor takes the
  // offset 2^30 elements, which lands past the buffer's range (real offsets
  // stay below 2^30 elements); a plane outside is sent there by the high bit.
  constexpr int SX = (NX + 255) / 256, SW = (NW + 255) / 256;
  constexpr int FAR = 1 << 30;
  int xoff[SX];
#pragma unroll
  for (int i = 0; i < SX; ++i) {
    const int id = tid + i * 256;
    const int cell = id >> 2, q = id & 3;
    const int r = cell / HC, c = cell - r * HC;
    const int hs = h0 - 1 + r, ws = w0 - 1 + c;
    const bool ok = id < NX && hs >= 0 && hs < gs.h && ws >= 0 && ws < gs.w;
    xoff[i] = ok ? (hs * gs.w + ws) * gs.ldc + q * 8 : FAR;
  }
  int woff[SW];
#pragma unroll
  for (int j = 0; j < SW; ++j) {
    const int id = tid + j * 256;
    const int t9 = id / (BN * 4), rem = id - t9 * (BN * 4);
    const int col = rem >> 2, q = rem & 3;
    woff[j] = id < NW && col < ncols ? col * a.kstride + t9 * C + q * 8 : FAR;
  }
  const int plane = gs.h * gs.w * gs.ldc;
  u32x4 xr[SX], wr[SW];
  // issue the loads of stage st = kd * (C / 32) + chunk into registers
  auto fetch = [&](int st) {
    const int cpk = C >> 5;
    const int kd = st / cpk, c0 = (st - kd * cpk) * 32;
    const int ds = MODE == 0 ? d + kd - 1 : d + 1 - kd;
    const unsigned dpen = ds >= 0 && ds < gs.d ? 0u : OOB;
    const int pb = (n * gs.d + ds) * plane + c0;
#pragma unroll
    for (int i = 0; i < SX; ++i)
      xr[i] = __builtin_amdgcn_raw_buffer_load_b128(rs, (unsigned)(pb + xoff[i]) * 2u | dpen, 0, 0);
    const int wb_ = kd * 9 * C + c0;
#pragma unroll
    for (int j = 0; j < SW; ++j)
      wr[j] = __builtin_amdgcn_raw_buffer_load_b128(rw, (unsigned)(woff[j] + wb_) * 2u, 0, 0);
  };
  // LDS homes of the slots
  auto xdst = [&](int i) {
    const int id = tid + i * 256;
    return (id >> 2) * PC + (id & 3) * 8;
  };
  auto wdst = [&](int j) {
    const int id = tid + j * 256;
    const int t9 = id / (BN * 4), rem = id - t9 * (BN * 4);
    return (t9 * BN + (rem >> 2)) * PW + (rem & 3) * 8;
  };

  const int L = lane & 15, g = lane >> 4;
  const int nst = 3 * (C >> 5);
  fetch(0);
  for (int st = 0; st < nst; ++st) {
    __syncthreads();  // the previous stage's readers are done
#pragma unroll
    for (int i = 0; i < SX; ++i)
      if (tid + i * 256 < NX) *(u32x4*)(&Xs[xdst(i)]) = xr[i];
#pragma unroll
    for (int j = 0; j < SW; ++j)
      if (tid + j * 256 < NW) *(u32x4*)(&Ws[wdst(j)]) = wr[j];
    __syncthreads();
    if (st + 1 < nst) fetch(st + 1);  // in flight while the taps run
#pragma unroll
    for (int kh = 0; kh < 3; ++kh)
#pragma unroll
      for (int kw = 0; kw < 3; ++kw) {
        // source offset of the tap in the halo: forward + (kh, kw),
        // input gradient + (2 - kh, 2 - kw)
        const int oh = MODE == 0 ? kh : 2 - kh, ow = MODE == 0 ? kw : 2 - kw;
        bf16x8 af[4];
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          const int r = 2 * wave + (f >> 1), c = (f & 1) * 16 + L;
          af[f] = *(const bf16x8*)(&Xs[((r + oh) * HC + c + ow) * PC + g * 8]);
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const bf16x8 bfr = *(const bf16x8*)(&Ws[((kh * 3 + kw) * BN + j * 16 + L) * PW + g * 8]);
#pragma unroll
          for (int f = 0; f < 4; ++f) acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[f], bfr, acc[f][j], 0, 0, 0);
        }
      }
  }
  // epilogue: lane holds D[(lane/16)*4 + q][lane%16] of each tile
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const int h = h0 + 2 * wave + (f >> 1);
    if (h >= go.h) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int w = w0 + (f & 1) * 16 + g * 4 + q;
      const long long vo = (((long long)n * go.d + d) * go.h + h) * go.w + w;
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int col = j * 16 + L;
        if (col >= ncols) continue;
        float v = acc[f][j][q];
        if (a.bias) v += a.bias[col];
        if (a.relu) v = v > 0.f ? v : 0.f;
        const long long o = vo * go.ldc + col;
        if (a.act && !(bf2f(a.act[vo * a.act_ldc + col]) > 0.f)) v = 0.f;
        if (a.accumulate) v += bf2f(a.out[o]);
        a.out[o] = f2bf(v);
      }
    }
  }
}

// ------------------------------------------------- bwd-weight, 3x3x3 halos
// dw[co][tap*Cin + ci] += sum_v dy[v][co] * x[src(v, tap)][ci] for 3x3x3
// kernels with Cin a multiple of 32, and (db given) db[co] += sum_v dy[v][co]
// from the dy tiles already in LDS, by the workgroups of kernel plane 0 and
// input-channel tile 0 (each dy tile once).  A workgroup owns one kernel plane kd,
// 32 input channels and BM output channels, i.e. a BM x (9 taps x 32) block
// of dw, and walks a range of 32-voxel steps of dy (R rows of W' voxels,
// W' = min(W, 32)).  Per step it stages, in their channels-last order,
//   * the dy tile  [32 voxels][BM channels] and
//   * the x halo   [(R-1)s+3 rows][(W'-1)s+3 columns][32 channels] of plane
//     z = d*s + kd - 1, which holds the sources of all nine (kh, kw) taps;
// both MFMA operands (voxels as K) are then read from LDS by the transposing
// read ds_read_b64_tr_b16 (a 16-lane group gives the addresses of four rows
// of four 16-bit values; lane l receives column l%16 of that 4 x 16 block),
// so the halo is staged once for nine taps and no lane transposes by hand.
// Tiles are double-buffered; out-of-range sources and voxels load zeros
// through the buffer range check.  Each wave keeps 9 x BM/32 accumulator
// tiles and adds them to dw once at the end (FP32 atomics).
struct WArgs {
  const uint16_t* x;
  Geo gx;
  unsigned x_bytes;
  const uint16_t* dy;
  Geo gy;
  unsigned dy_bytes;
  float* dw;
  float* db;            // bias gradient, or nullptr
  int kpad;
  int wp, r, nhb, nwb;  // step shape: R rows of W' voxels; steps per row block / plane
  int steps, per_wg;    // total steps, steps per workgroup
  int nco, nci;         // output / input channel tiles
};

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) bf16x4 lds_bf16x4;

__device__ __forceinline__ bf16x8 tr_load8(const uint16_t* p, int off_lo, int off_hi) {
  const __attribute__((address_space(3))) uint16_t* q = (const __attribute__((address_space(3))) uint16_t*)p;
  const bf16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf16x4*)(q + off_lo));
  const bf16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf16x4*)(q + off_hi));
  return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}

// VS = 64 or 128 (stride 1, rows of at least 32 voxels): steps of two or
// four 32-voxel rows, each tap's K chunks run on one staging of dy and of
// the halo of VS/32 + 2 rows, so a barrier and a staging round cover two or
// four times the MFMAs.
template <int S, int BM, int VS = 32>
__global__ void __launch_bounds__(256) k_conv_wgrad_halo(WArgs a) {
  constexpr int PA = BM + 8;                 // dy tile row pitch (bf16)
  constexpr int PC = 40;                     // halo cell pitch: 32 channels + 8
  // largest halo over the step shapes (VS >= 64: rows of 32 voxels only)
  constexpr int CELLS = VS >= 64 ? ((VS / 32 - 1) * S + 3) * (31 * S + 3) : (S == 1 ? 102 : 195);
  constexpr int NK = VS / 32;                // 32-voxel K chunks per step
  constexpr int NAC = VS * BM / 8;           // dy chunks of 8 channels
  constexpr int NAP = (NAC + 255) / 256;
  constexpr int NXP = (CELLS * 4 + 255) / 256;
  constexpr int NSUB = BM / 32;              // 16-row output tiles per wave
  constexpr unsigned OOB = 0x80000000u;
  __shared__ __attribute__((aligned(16))) uint16_t As[2][VS * PA];
  __shared__ __attribute__((aligned(16))) uint16_t Xs[2][CELLS * PC];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const Geo gx = a.gx, gy = a.gy;
  // Work index from the linear workgroup id, XCD-aware: workgroups are
  // dealt to the 8 XCDs in turn, so id L runs on XCD L % 8; consecutive
  // indices (the weight tiles of one step range, which read the same dy and
  // x data) are given to consecutive workgroups of one XCD and share its L2.
  // The tail past the last multiple of 8 keeps its own index.
  const int total = (int)gridDim.x, L8 = (int)blockIdx.x;
  const int q8 = total / 8 * 8;
  const int idx = L8 < q8 ? (L8 % 8) * (total / 8) + L8 / 8 : L8;
  const int ntiles = 3 * a.nci * a.nco;
  int by = idx % ntiles;
  const int split = idx / ntiles;
  const int co_t = by % a.nco;
  by /= a.nco;
  const int ci_t = by % a.nci;
  const int kd = by / a.nci;
  const int co0 = co_t * BM, ci0 = ci_t * 32;
  const int wp = a.wp, rr = a.r;
  const int hc = (wp - 1) * S + 3, ncell = ((rr - 1) * S + 3) * hc;

  // staging roles (fixed per thread): dy chunk (voxel, channel group)
  int a_v[NAP], a_q[NAP];
  bool a_on[NAP];
#pragma unroll
  for (int i = 0; i < NAP; ++i) {
    const int id = tid + i * 256;
    a_v[i] = id / (BM / 8);
    a_q[i] = id % (BM / 8);
    a_on[i] = id < NAC && co0 + a_q[i] * 8 < gy.c;
  }
  int a_r[NAP], a_c[NAP];
#pragma unroll
  for (int i = 0; i < NAP; ++i) {
    a_r[i] = (a_v[i] & (VS - 1)) / wp;
    a_c[i] = (a_v[i] & (VS - 1)) % wp;
  }
  // halo chunk (cell, channel group)
  int x_hr[NXP], x_hc[NXP], x_q[NXP];
  bool x_on[NXP];
#pragma unroll
  for (int i = 0; i < NXP; ++i) {
    const int id = tid + i * 256;
    const int cell = id >> 2;
    x_on[i] = cell < ncell;
    x_hr[i] = cell / hc;
    x_hc[i] = cell % hc;
    x_q[i] = id & 3;
  }
  // operand read offsets: 16-lane group g covers voxels 8g..8g+7, half h
  // the rows 8g+4h .. +3; lane L of the group addresses row L/4, columns
  // (L%4)*4 .. +3 of its 16-column block
  const int L = lane & 15, g = lane >> 4, jsub = wave & 1;
  int aoff[NSUB][2], xoff[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int v = 8 * g + 4 * h + (L >> 2);
#pragma unroll
    for (int i = 0; i < NSUB; ++i) aoff[i][h] = v * PA + ((wave >> 1) * NSUB + i) * 16 + (L & 3) * 4;
    xoff[h] = ((v / wp) * S * hc + (v % wp) * S) * PC + jsub * 16 + (L & 3) * 4;
  }

  const __amdgpu_buffer_rsrc_t rx = rsrc_of(a.x, a.x_bytes);
  const __amdgpu_buffer_rsrc_t rd = rsrc_of(a.dy, a.dy_bytes);
  const int s_begin = split * a.per_wg;
  const int s_end = s_begin + a.per_wg < a.steps ? s_begin + a.per_wg : a.steps;
  // uniform step coordinates, advanced without branches
  int st = s_begin;
  int wb = st % a.nwb, hb = (st / a.nwb) % a.nhb, pl = st / (a.nwb * a.nhb);
  int nn = pl / gy.d, dd = pl % gy.d;
  auto advance = [&]() {
    ++wb;
    const int c1 = wb == a.nwb;
    wb = c1 ? 0 : wb;
    hb += c1;
    const int c2 = hb == a.nhb;
    hb = c2 ? 0 : hb;
    dd += c2;
    const int c3 = dd == gy.d;
    dd = c3 ? 0 : dd;
    nn += c3;
  };
  u32x4 ar[NAP], xr[NXP];
  auto load_step = [&](unsigned dead) {
    const int h0 = hb * rr, w0 = wb * wp;
#pragma unroll
    for (int i = 0; i < NAP; ++i) {
      const int hh = h0 + a_r[i], ww = w0 + a_c[i];
      const bool ok = a_on[i] && hh < gy.h && ww < gy.w;
      const unsigned vo =
          (unsigned)((((nn * gy.d + dd) * gy.h + hh) * gy.w + ww) * gy.ldc + co0 + a_q[i] * 8) * 2u | (ok ? 0u : OOB);
      ar[i] = __builtin_amdgcn_raw_buffer_load_b128(rd, vo | dead, 0, 0);
    }
    const int zs = dd * S + kd - 1, ys0 = h0 * S - 1, xs0 = w0 * S - 1;
    const bool zok = zs >= 0 && zs < gx.d;
#pragma unroll
    for (int i = 0; i < NXP; ++i) {
      const int ys = ys0 + x_hr[i], xs = xs0 + x_hc[i];
      const bool ok = x_on[i] && zok && ys >= 0 && ys < gx.h && xs >= 0 && xs < gx.w;
      const unsigned vo =
          (unsigned)((((nn * gx.d + zs) * gx.h + ys) * gx.w + xs) * gx.ldc + ci0 + x_q[i] * 8) * 2u | (ok ? 0u : OOB);
      xr[i] = __builtin_amdgcn_raw_buffer_load_b128(rx, vo | dead, 0, 0);
    }
  };
  auto store_step = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NAP; ++i)
      if (tid + i * 256 < NAC) *(u32x4*)(&As[buf][(a_v[i] & (VS - 1)) * PA + a_q[i] * 8]) = ar[i];
#pragma unroll
    for (int i = 0; i < NXP; ++i)
      if (x_on[i]) *(u32x4*)(&Xs[buf][(x_hr[i] * hc + x_hc[i]) * PC + x_q[i] * 8]) = xr[i];
  };

  f32x4 acc[NSUB][9];
#pragma unroll
  for (int i = 0; i < NSUB; ++i)
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[i][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  // bias: thread sums channel b_ch over voxels b_v0 .. b_v0 + 32/BG - 1 of each step
  constexpr int BG = 256 / BM;
  const bool do_bias = a.db != nullptr && kd == 0 && ci_t == 0;
  const int b_ch = tid % BM, b_v0 = (tid / BM) * (VS / BG);
  float bsum = 0.f;

  if (s_begin < s_end) {
    load_step(0u);
    store_step(0);
    __syncthreads();
  }
  int buf = 0;
  for (; st < s_end; ++st) {
    advance();
    load_step(st + 1 < s_end ? 0u : OOB);
    __builtin_amdgcn_sched_barrier(0);  // the loads stay ahead of the MFMAs
    const uint16_t* A = As[buf];
    const uint16_t* X = Xs[buf];
    // K chunk c: voxels 32c..32c+31 of the step (with VS = 64 the second
    // 32-voxel row: dy rows +32, halo rows +1)
#pragma unroll
    for (int c = 0; c < NK; ++c) {
      bf16x8 af[NSUB];
#pragma unroll
      for (int i = 0; i < NSUB; ++i) af[i] = tr_load8(A, aoff[i][0] + c * 32 * PA, aoff[i][1] + c * 32 * PA);
#pragma unroll
      for (int kh = 0; kh < 3; ++kh)
#pragma unroll
        for (int kw = 0; kw < 3; ++kw) {
          const int to = (kh * hc + kw) * PC + c * S * hc * PC;
          const bf16x8 bfr = tr_load8(X, xoff[0] + to, xoff[1] + to);
#pragma unroll
          for (int i = 0; i < NSUB; ++i)
            acc[i][kh * 3 + kw] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr, acc[i][kh * 3 + kw], 0, 0, 0);
        }
    }
    if (do_bias) {
#pragma unroll
      for (int j = 0; j < VS / BG; ++j) bsum += __uint_as_float((unsigned)A[(b_v0 + j) * PA + b_ch] << 16);
    }
    store_step(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // lane holds D[(lane/16)*4 + q][lane%16] of each tile: rows co, columns ci
  const int cin = gx.c;
#pragma unroll
  for (int i = 0; i < NSUB; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int co = co0 + ((wave >> 1) * NSUB + i) * 16 + g * 4 + q;
      if (co >= gy.c) continue;
      const int ci = ci0 + jsub * 16 + L;
#pragma unroll
      for (int t = 0; t < 9; ++t) atomicAdd(a.dw + (long long)co * a.kpad + (kd * 9 + t) * cin + ci, acc[i][t][q]);
    }
  if (do_bias && co0 + b_ch < gy.c) atomicAdd(a.db + co0 + b_ch, bsum);
}

// --------------------------------- bwd-weight, 3x3x3, 8 input channels
// dw[co][tap*8 + ci] += sum_v dy[v][co] * x[src(v, tap)][ci] for the input
// layer (8 channels, stride 1): all 27 taps of a 32-output-channel tile in
// one workgroup, the 216 columns as 14 MFMA column tiles of two taps x 8
// channels (the last holds tap 26 and zeros).  Per 32-voxel step (R rows of
// W' voxels, as above) it stages the dy tile [32 voxels][32 channels] and the
// x halo of the three source planes [3][R+2 rows][W'+2 columns][8 channels];
// ds_read_b64_tr_b16 takes one address per lane, so each lane of a B
// fragment points at the tap of its half of the tile's columns, and both
// operands are transposing LDS reads.  Wave w owns output-channel tile w % 2
// and column tiles w/2, w/2 + 2, ..., w/2 + 12 (seven MFMA tiles).  With db
// given every workgroup also sums its dy tiles (each once per channel tile).
__global__ void __launch_bounds__(256) k_conv_wgrad_c8(WArgs a) {
  constexpr int BC = 32;                 // output channels per tile
  constexpr int PA = BC + 8;             // dy tile row pitch (bf16)
  constexpr int PC = 8;                  // halo cell: 8 channels
  constexpr int PLANE = 102;             // largest (R+2)(W'+2) over the step shapes
  constexpr int CELLS = 3 * PLANE;
  constexpr int ZERO = CELLS * PC;       // a cell of zeros (the missing 28th tap)
  constexpr int NXP = (CELLS + 255) / 256;
  constexpr unsigned OOB = 0x80000000u;
  __shared__ __attribute__((aligned(16))) uint16_t As[2][32 * PA];
  __shared__ __attribute__((aligned(16))) uint16_t Xs[2][(CELLS + 1) * PC];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const Geo gx = a.gx, gy = a.gy;
  // XCD-aware work index (see k_conv_wgrad_halo)
  const int total = (int)gridDim.x, L8 = (int)blockIdx.x;
  const int q8 = total / 8 * 8;
  const int idx = L8 < q8 ? (L8 % 8) * (total / 8) + L8 / 8 : L8;
  const int co_t = idx % a.nco, split = idx / a.nco;
  const int co0 = co_t * BC;
  const int wp = a.wp, rr = a.r;
  const int hc = wp + 2, hr = rr + 2, pcells = hr * hc, ncell = 3 * pcells;
  if (tid < 2 * PC / 8) *(u32x4*)(&Xs[tid][ZERO]) = u32x4{0u, 0u, 0u, 0u};

  // staging roles: dy chunk (voxel, 8-channel group), threads 0..127
  const bool a_act = tid < 32 * BC / 8;
  const int a_v = tid / (BC / 8), a_q = tid % (BC / 8);
  const bool a_on = a_act && co0 + a_q * 8 < gy.c;
  const int a_r = (a_v & 31) / wp, a_c = (a_v & 31) % wp;
  // halo cell (plane, row, column)
  int x_p[NXP], x_hr[NXP], x_hc[NXP];
  bool x_on[NXP];
#pragma unroll
  for (int i = 0; i < NXP; ++i) {
    const int cell = tid + i * 256;
    x_on[i] = cell < ncell;
    x_p[i] = cell / pcells;
    x_hr[i] = (cell % pcells) / hc;
    x_hc[i] = cell % hc;
  }
  // operand read offsets (16-lane group g covers voxels 8g..8g+7, half h the
  // rows 8g+4h..+3; lane L addresses row L/4, columns (L%4)*4..+3)
  const int L = lane & 15, g = lane >> 4;
  const int cot = wave & 1, kt0 = wave >> 1;
  const int hi = (L & 3) >> 1, cio = (L & 1) * 4;
  int aoff[2], xb[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int v = 8 * g + 4 * h + (L >> 2);
    aoff[h] = v * PA + cot * 16 + (L & 3) * 4;
    xb[h] = ((v / wp) * hc + (v % wp)) * PC + cio;
  }
  // per column tile j of this wave: the lane's tap and its halo offset
  int toff[7];
  bool tzero[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    const int t = 2 * (kt0 + 2 * j) + hi;
    tzero[j] = t >= 27;
    const int tt = tzero[j] ? 0 : t;
    toff[j] = ((tt / 9) * pcells + ((tt / 3) % 3) * hc + tt % 3) * PC;
  }

  const __amdgpu_buffer_rsrc_t rx = rsrc_of(a.x, a.x_bytes);
  const __amdgpu_buffer_rsrc_t rd = rsrc_of(a.dy, a.dy_bytes);
  const int s_begin = split * a.per_wg;
  const int s_end = s_begin + a.per_wg < a.steps ? s_begin + a.per_wg : a.steps;
  int st = s_begin;
  int wb = st % a.nwb, hb = (st / a.nwb) % a.nhb, pl = st / (a.nwb * a.nhb);
  int nn = pl / gy.d, dd = pl % gy.d;
  auto advance = [&]() {
    ++wb;
    const int c1 = wb == a.nwb;
    wb = c1 ? 0 : wb;
    hb += c1;
    const int c2 = hb == a.nhb;
    hb = c2 ? 0 : hb;
    dd += c2;
    const int c3 = dd == gy.d;
    dd = c3 ? 0 : dd;
    nn += c3;
  };
  u32x4 ar, xr[NXP];
  auto load_step = [&](unsigned dead) {
    const int h0 = hb * rr, w0 = wb * wp;
    {
      const int hh = h0 + a_r, ww = w0 + a_c;
      const bool ok = a_on && hh < gy.h && ww < gy.w;
      const unsigned vo =
          (unsigned)((((nn * gy.d + dd) * gy.h + hh) * gy.w + ww) * gy.ldc + co0 + a_q * 8) * 2u | (ok ? 0u : OOB);
      ar = __builtin_amdgcn_raw_buffer_load_b128(rd, vo | dead, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < NXP; ++i) {
      const int zs = dd + x_p[i] - 1, ys = h0 - 1 + x_hr[i], xs = w0 - 1 + x_hc[i];
      const bool ok = x_on[i] && zs >= 0 && zs < gx.d && ys >= 0 && ys < gx.h && xs >= 0 && xs < gx.w;
      const unsigned vo = (unsigned)((((nn * gx.d + zs) * gx.h + ys) * gx.w + xs) * gx.ldc) * 2u | (ok ? 0u : OOB);
      xr[i] = __builtin_amdgcn_raw_buffer_load_b128(rx, vo | dead, 0, 0);
    }
  };
  auto store_step = [&](int buf) {
    if (a_act) *(u32x4*)(&As[buf][(a_v & 31) * PA + a_q * 8]) = ar;
#pragma unroll
    for (int i = 0; i < NXP; ++i)
      if (x_on[i]) *(u32x4*)(&Xs[buf][(x_p[i] * pcells + x_hr[i] * hc + x_hc[i]) * PC]) = xr[i];
  };

  f32x4 acc[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bool do_bias = a.db != nullptr;
  const int b_ch = tid % BC, b_v0 = (tid / BC) * 4;
  float bsum = 0.f;

  if (s_begin < s_end) {
    load_step(0u);
    store_step(0);
    __syncthreads();
  }
  int buf = 0;
  for (; st < s_end; ++st) {
    advance();
    load_step(st + 1 < s_end ? 0u : OOB);
    __builtin_amdgcn_sched_barrier(0);  // the loads stay ahead of the MFMAs
    const uint16_t* A = As[buf];
    const uint16_t* X = Xs[buf];
    const bf16x8 af = tr_load8(A, aoff[0], aoff[1]);
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      const bf16x8 bfr = tr_load8(X, tzero[j] ? ZERO + cio : xb[0] + toff[j], tzero[j] ? ZERO + cio : xb[1] + toff[j]);
      acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr, acc[j], 0, 0, 0);
    }
    if (do_bias) {
#pragma unroll
      for (int j = 0; j < 4; ++j) bsum += __uint_as_float((unsigned)A[(b_v0 + j) * PA + b_ch] << 16);
    }
    store_step(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // lane holds D[(lane/16)*4 + q][lane%16] of each tile: rows co, columns k
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int co = co0 + cot * 16 + g * 4 + q;
    if (co >= gy.c) continue;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      const int k = (kt0 + 2 * j) * 16 + L;
      if (k < 216) atomicAdd(a.dw + (long long)co * a.kpad + k, acc[j][q]);
    }
  }
  if (do_bias && co0 + b_ch < gy.c) atomicAdd(a.db + co0 + b_ch, bsum);
}

// dbias[co] += sum_v dy[v][co]: a thread sums 8 channels (one 16-byte load
// per voxel) over every (256 / groups)-th voxel of the workgroup's range; the
// partial sums meet in LDS and each channel takes one atomic per workgroup.
__global__ void __launch_bounds__(256) k_bias_grad(const uint16_t* __restrict__ dy, Geo gy, float* __restrict__ db,
                                                   long long vox_per_wg) {
  __shared__ float part[256 * 8];
  const long long V = (long long)gy.n * gy.d * gy.h * gy.w;
  const long long vbeg = (long long)blockIdx.x * vox_per_wg;
  const long long vend = vbeg + vox_per_wg < V ? vbeg + vox_per_wg : V;
  const int groups = gy.c / 8;         // at most 256 (host check)
  const int vl = 256 / groups;         // voxel lanes
  const int tid = threadIdx.x, cg = tid % groups, vi = tid / groups;
  float s8[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (vi < vl)
    for (long long v = vbeg + vi; v < vend; v += vl) {
      const u32x4 t = *(const u32x4*)(dy + v * gy.ldc + cg * 8);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        s8[2 * j] += __uint_as_float(t[j] << 16);
        s8[2 * j + 1] += __uint_as_float(t[j] & 0xffff0000u);
      }
    }
#pragma unroll
  for (int j = 0; j < 8; ++j) part[tid * 8 + j] = s8[j];
  __syncthreads();
  for (int c = tid; c < gy.c; c += 256) {
    const int g = c / 8, j = c % 8;
    float t = 0.f;
    for (int k = 0; k < vl; ++k) t += part[(k * groups + g) * 8 + j];
    atomicAdd(db + c, t);
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

// bytes spanned by a channels-last view (last voxel's last channel included)
long long view_bytes(const lbm_tensor5* t) {
  return (((long long)t->n * t->d * t->h * t->w - 1) * t->ldc + t->c) * 2;
}

// the tap-major kernels index in 32 bits and address through buffer resources
bool tap_fits(const lbm_tensor5* t) { return view_bytes(t) < (1ll << 31); }

template <int MODE, bool CLS, int FM, int FN>
void launch_tap(const DArgs& a, long long rows, int nz, hipStream_t s) {
  constexpr int BMW = 64 * FM, BN = 16 * FN;
  const dim3 g((unsigned)((rows + BMW - 1) / BMW), (unsigned)((a.go.c + BN - 1) / BN), (unsigned)nz);
  hipLaunchKernelGGL((k_conv_tap<MODE, CLS, FM, FN>), g, dim3(256), 0, s, a);
}

// tile shape by output columns: 32 -> 64 rows x 32 per wave, 64 -> 32 x 64,
// more -> 32 x 128 per column tile, or 32 x 64 where 128-column tiles would
// leave the chip short of workgroups (fewer than two per compute unit: the
// 16x8x8 layers of 256 channels)
template <int MODE, bool CLS>
void launch_tap_cols(const DArgs& a, long long rows, int nz, hipStream_t s) {
  const long long wide = (rows + 127) / 128 * ((a.go.c + 127) / 128) * nz;
  if (a.go.c <= 32)
    launch_tap<MODE, CLS, 4, 2>(a, rows, nz, s);
  else if (a.go.c <= 64 || wide < 512)
    launch_tap<MODE, CLS, 2, 4>(a, rows, nz, s);
  else
    launch_tap<MODE, CLS, 2, 8>(a, rows, nz, s);
}

// the halo kernel: stride-1 3x3x3 products onto whole 32-column row pieces
// with at most 64 output columns
bool halo_fits(const lbm_tensor5* src, const lbm_tensor5* out, int ksize, int stride) {
  return ksize == 3 && stride == 1 && src->c % 32 == 0 && out->w % 32 == 0 && out->c <= 64;
}

template <int MODE>
void launch_halo(const DArgs& a, hipStream_t s) {
  const unsigned g = (unsigned)((a.go.w / 32) * ((a.go.h + 7) / 8) * a.go.d * a.go.n);
  if (a.go.c <= 32)
    hipLaunchKernelGGL((k_conv_halo<MODE, 2>), dim3(g), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_conv_halo<MODE, 4>), dim3(g), dim3(256), 0, s, a);
}

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
  if (x->c % 32 == 0 && tap_fits(x) && tap_fits(y)) {
    const DArgs a{(const uint16_t*)x->ptr, gs, (unsigned)view_bytes(x), w, kpad,
                  (unsigned)((long long)y->c * kpad * 2), bias, (uint16_t*)y->ptr, go, nullptr, 0, ksize, stride,
                  relu, 0, x->c};
    if (halo_fits(x, y, ksize, stride))
      launch_halo<0>(a, s);
    else
      launch_tap_cols<0, false>(a, M, 1, s);
  } else if (y->c <= 16) {
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
  if (dy->c % 32 == 0 && tap_fits(dy) && tap_fits(dx)) {
    const DArgs a{(const uint16_t*)dy->ptr, gs, (unsigned)view_bytes(dy), w_t, kpad,
                  (unsigned)((long long)dx->c * kpad * 2), nullptr, (uint16_t*)dx->ptr, go, ap, aldc, ksize, stride,
                  0, accumulate, dy->c};
    if (stride == 2) {
      // rows of the largest parity class; smaller classes mask their tail
      const long long rows = (long long)dx->n * ((dx->d + 1) / 2) * ((dx->h + 1) / 2) * ((dx->w + 1) / 2);
      launch_tap_cols<1, true>(a, rows, 8, s);
    } else if (halo_fits(dy, dx, ksize, stride)) {
      launch_halo<1>(a, s);
    } else {
      launch_tap_cols<1, false>(a, M, 1, s);
    }
  } else if (dx->c <= 16) {
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
  if (dbias && dy->c > 2048) return LBM_EINVAL;
  const int taps = ksize * ksize * ksize;
  const int kpad = lbm_conv_kpad(taps, x->c);
  const long long V = (long long)dy->n * dy->d * dy->h * dy->w;
  hipStream_t s = (hipStream_t)stream;
  const dim3 b(256);
  const bool wfit = dy->w >= 32 ? true : (32 % dy->w) == 0;
  if (ksize == 3 && x->c % 32 == 0 && wfit && tap_fits(x) && tap_fits(dy) && V < (1ll << 31)) {
    WArgs a{};
    a.x = (const uint16_t*)x->ptr;
    a.gx = geo_of(x);
    a.x_bytes = (unsigned)view_bytes(x);
    a.dy = (const uint16_t*)dy->ptr;
    a.gy = geo_of(dy);
    a.dy_bytes = (unsigned)view_bytes(dy);
    a.dw = dw;
    a.db = dbias;
    a.kpad = kpad;
    // steps of several 32-voxel rows with rows of 32 voxels or more
    const bool vs64 = dy->w >= 32;
    const int vs = !vs64 ? 32 : (stride == 2 ? 64 : 128);
    a.wp = dy->w >= 32 ? 32 : dy->w;
    a.r = vs / a.wp;
    a.nhb = (dy->h + a.r - 1) / a.r;
    a.nwb = (dy->w + a.wp - 1) / a.wp;
    const long long steps = (long long)dy->n * dy->d * a.nhb * a.nwb;
    const int bmw = dy->c <= 32 ? 32 : 64;
    a.nco = (dy->c + bmw - 1) / bmw;
    a.nci = x->c / 32;
    const long long tiles = 3ll * a.nci * a.nco;
    // About 2048 workgroups in all, and at least 48 voxel steps each: every
    // workgroup ends with BM x 288 FP32 atomics into dw, which dominate the
    // layers of few voxels when their work is split finer (measured on
    // gfx950, batch 8: 16x8x8 256->256 0.170 -> 0.115 ms, 32x16x16 128->128
    // 0.186 -> 0.158 ms; the full-resolution layers already take 96-384
    // steps per workgroup and lose with fewer workgroups).
    long long per = (steps * tiles + 2047) / 2048;
    if (per < 48 * 32 / vs) per = 48 * 32 / vs;
    const long long splits = (steps + per - 1) / per;
    a.steps = (int)steps;
    a.per_wg = (int)per;
    const dim3 g((unsigned)(splits * tiles));
    if (vs64 && stride == 1) {
      if (bmw == 32)
        hipLaunchKernelGGL((k_conv_wgrad_halo<1, 32, 128>), g, b, 0, s, a);
      else
        hipLaunchKernelGGL((k_conv_wgrad_halo<1, 64, 128>), g, b, 0, s, a);
    } else if (vs64) {
      if (bmw == 32)
        hipLaunchKernelGGL((k_conv_wgrad_halo<2, 32, 64>), g, b, 0, s, a);
      else
        hipLaunchKernelGGL((k_conv_wgrad_halo<2, 64, 64>), g, b, 0, s, a);
    } else if (stride == 1) {
      if (bmw == 32)
        hipLaunchKernelGGL((k_conv_wgrad_halo<1, 32>), g, b, 0, s, a);
      else
        hipLaunchKernelGGL((k_conv_wgrad_halo<1, 64>), g, b, 0, s, a);
    } else {
      if (bmw == 32)
        hipLaunchKernelGGL((k_conv_wgrad_halo<2, 32>), g, b, 0, s, a);
      else
        hipLaunchKernelGGL((k_conv_wgrad_halo<2, 64>), g, b, 0, s, a);
    }
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
  }
  if (ksize == 3 && stride == 1 && x->c == 8 && wfit && tap_fits(x) && tap_fits(dy) && V < (1ll << 31)) {
    WArgs a{};
    a.x = (const uint16_t*)x->ptr;
    a.gx = geo_of(x);
    a.x_bytes = (unsigned)view_bytes(x);
    a.dy = (const uint16_t*)dy->ptr;
    a.gy = geo_of(dy);
    a.dy_bytes = (unsigned)view_bytes(dy);
    a.dw = dw;
    a.db = dbias;
    a.kpad = kpad;
    a.wp = dy->w >= 32 ? 32 : dy->w;
    a.r = 32 / a.wp;
    a.nhb = (dy->h + a.r - 1) / a.r;
    a.nwb = (dy->w + a.wp - 1) / a.wp;
    const long long steps = (long long)dy->n * dy->d * a.nhb * a.nwb;
    a.nco = (dy->c + 31) / 32;
    a.nci = 1;
    // about 1024 workgroups, at least 48 steps each (each ends with 32 x 216
    // FP32 atomics)
    long long per = (steps * a.nco + 1023) / 1024;
    if (per < 48) per = 48;
    const long long splits = (steps + per - 1) / per;
    a.steps = (int)steps;
    a.per_wg = (int)per;
    hipLaunchKernelGGL(k_conv_wgrad_c8, dim3((unsigned)(splits * a.nco)), b, 0, s, a);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
  }
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
    const long long pb = 2048;
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
