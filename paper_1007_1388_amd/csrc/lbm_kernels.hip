// lbm_kernels.hip -- gfx950 kernels of the patch-and-block D3Q19 BGK solver.
//
// One thread updates one lattice cell (Sec. 3.2).  A workgroup takes a work
// item = a run of whole x-rows of one Block at one z, so a wave reads and
// writes 64 consecutive cells of a row: every one of the 19 pulled streams and
// the 19 stored streams is a coalesced, line-aligned access (SoA + pull,
// Sec. 3.2), and the x +- 1 pulls of a row stay inside the workgroup's lines.
// No LDS is needed for the sweep: every element is read exactly once per step.
//
// Precision variants (template PREC): 0 FP64, 1 FP32, 2 shifted FP16,
// 3 shifted BF16 (storage), arithmetic type C = double or float.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_internal.h"

// No implicit multiply-add contraction: every instantiation of a kernel must
// round exactly alike (schedules, exchange variants and Block tilings are
// bit-identical), so fused multiply-adds are written out where wanted.
#pragma clang fp contract(off)

namespace lbm {

// ------------------------------------------------------------------ lattice
// D3Q19 direction i -> e_i, opposite, and its slot among the five populations
// that cross an x face (x-ghost planes).  Sec. 2.1.
__host__ __device__ constexpr int EXd(int i) {
  constexpr int t[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  return t[i];
}
__host__ __device__ constexpr int EYd(int i) {
  constexpr int t[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  return t[i];
}
__host__ __device__ constexpr int EZd(int i) {
  constexpr int t[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  return t[i];
}
__host__ __device__ constexpr int OPPd(int i) {
  constexpr int t[kQ] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
  return t[i];
}
// slot of direction i in the x-lo ghost planes (e_x = +1) / x-hi planes (e_x = -1)
__host__ __device__ constexpr int KLOd(int i) {
  constexpr int t[kQ] = {-1, 0, -1, -1, -1, -1, -1, 1, -1, 2, -1, 3, -1, 4, -1, -1, -1, -1, -1};
  return t[i];
}
__host__ __device__ constexpr int KHId(int i) {
  constexpr int t[kQ] = {-1, -1, 0, -1, -1, -1, -1, -1, 1, -1, 2, -1, 3, -1, 4, -1, -1, -1, -1};
  return t[i];
}
// lattice weight times a factor, from |e_i|^2
__host__ __device__ constexpr double Wd(int i) {
  return (EXd(i) * EXd(i) + EYd(i) * EYd(i) + EZd(i) * EZd(i)) == 0   ? 1.0 / 3.0
         : (EXd(i) * EXd(i) + EYd(i) * EYd(i) + EZd(i) * EZd(i)) == 1 ? 1.0 / 18.0
                                                                      : 1.0 / 36.0;
}

// ---------------------------------------------------------------- storage
template <int PREC> struct Stor;
template <> struct Stor<0> { using T = double; };
template <> struct Stor<1> { using T = float; };
template <> struct Stor<2> { using T = uint16_t; };  // IEEE binary16 bits
template <> struct Stor<3> { using T = uint16_t; };  // bfloat16 bits

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// round-to-nearest-even float -> bfloat16 (NaN kept quiet)
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float f16_to_f32(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }
__device__ __forceinline__ uint16_t f32_to_f16(float f) { return __builtin_bit_cast(uint16_t, (_Float16)f); }

template <int PREC, typename C>
__device__ __forceinline__ C to_c(typename Stor<PREC>::T v) {
  if constexpr (PREC == 0 || PREC == 1) return (C)v;
  else if constexpr (PREC == 2) return (C)f16_to_f32(v);
  else return (C)bf16_to_f32(v);
}
template <int PREC, typename C>
__device__ __forceinline__ typename Stor<PREC>::T from_c(C v) {
  if constexpr (PREC == 0) return (double)v;
  else if constexpr (PREC == 1) return (float)v;
  else if constexpr (PREC == 2) return f32_to_f16((float)v);
  else return f32_to_bf16((float)v);
}

template <typename T, bool NT>
__device__ __forceinline__ T ld(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <typename T, bool NT>
__device__ __forceinline__ void st(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

__device__ __forceinline__ long long main_off(const BlockDev& B, int i, int x, int y, int z) {
  return B.base + (long long)i * B.Sf + (long long)(z + 1) * B.Sz + (long long)(y + 1) * B.Sx + x;
}

// ------------------------------------------------------------------- sweep
// One fluid cell: pull (Sec. 2.1, pull scheme), half-way bounce-back with
// wall velocity (Sec. 2.1, bounce-back rule), moments, BGK collision with the
// shifted incompressible equilibrium of Eq. (2) and the Guo force term,
// aligned store; with FUSED also the ghost-layer copy of the values that the
// neighbouring Blocks pull in the next step (Sec. 4.4 on-GPU copies, fused).
template <int PREC, typename C, bool MASK, bool FUSED, bool NT>
__device__ __forceinline__ void sweep_cell(const SweepArgs& A, const Phys<C>& ph, const BlockDev& B,
                                           int bid, int x, int y, int z) {
  using T = typename Stor<PREC>::T;
  const T* __restrict__ src = (const T*)A.src;
  T* __restrict__ dst = (T*)A.dst;
  const int a = B.dim[0], b = B.dim[1], c = B.dim[2];
  uint32_t m = 0;
  if constexpr (MASK) {
    m = A.mask[B.mask + ((long long)z * b + y) * a + x];
    if (m & kSolidBit) return;
  }
  const int gx = B.org[0] + x, gy = B.org[1] + y, gz = B.org[2] + z;
  const bool lox = A.geo.wall[0] && gx == 0, hix = A.geo.wall[0] && gx == A.geo.n[0] - 1;
  const bool loy = A.geo.wall[1] && gy == 0, hiy = A.geo.wall[1] && gy == A.geo.n[1] - 1;
  const bool loz = A.geo.wall[2] && gz == 0, hiz = A.geo.wall[2] && gz == A.geo.n[2] - 1;
  const long long cell = main_off(B, 0, x, y, z);
  const long long xrow = (long long)(z + 1) * B.Ry + (y + 1);

  C f[kQ];
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const int ex = EXd(i), ey = EYd(i), ez = EZd(i);
    if (i == 0) {
      f[0] = to_c<PREC, C>(ld<T, NT>(src + cell));
      continue;
    }
    // source beyond a wall face -> wall link
    bool bw = false;
    if (ex > 0) bw = bw || lox;
    if (ex < 0) bw = bw || hix;
    if (ey > 0) bw = bw || loy;
    if (ey < 0) bw = bw || hiy;
    if (ez > 0) bw = bw || loz;
    if (ez < 0) bw = bw || hiz;
    bool bb = bw;
    if constexpr (MASK) bb = bb || ((m >> i) & 1u);
    long long off = cell + (long long)i * B.Sf - (long long)ez * B.Sz - (long long)ey * B.Sx - ex;
    if (ex > 0 && x == 0) off = B.xg + (long long)KLOd(i) * B.P + xrow - (long long)ez * B.Ry - ey;
    if (ex < 0 && x == a - 1) off = B.xg + (long long)(5 + KHId(i)) * B.P + xrow - (long long)ez * B.Ry - ey;
    if (bb) off = cell + (long long)OPPd(i) * B.Sf;
    C v = to_c<PREC, C>(ld<T, NT>(src + off));
    if (bw) {
      // velocity of the first moving face, order -x,+x,-y,+y,-z,+z
      C cw = (C)0;
      if (ez != 0 && (ez > 0 ? loz : hiz) && A.geo.moving[ez > 0 ? 4 : 5]) cw = ph.corr[i][ez > 0 ? 4 : 5];
      if (ey != 0 && (ey > 0 ? loy : hiy) && A.geo.moving[ey > 0 ? 2 : 3]) cw = ph.corr[i][ey > 0 ? 2 : 3];
      if (ex != 0 && (ex > 0 ? lox : hix) && A.geo.moving[ex > 0 ? 0 : 1]) cw = ph.corr[i][ex > 0 ? 0 : 1];
      v += cw;
    }
    f[i] = v;
  }

  // moments (Sec. 2.1): drho = sum f~, rho0 u = sum e f~, plus half force
  C drho = (C)0, jx = (C)0, jy = (C)0, jz = (C)0;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    drho += f[i];
    if (EXd(i) > 0) jx += f[i];
    if (EXd(i) < 0) jx -= f[i];
    if (EYd(i) > 0) jy += f[i];
    if (EYd(i) < 0) jy -= f[i];
    if (EZd(i) > 0) jz += f[i];
    if (EZd(i) < 0) jz -= f[i];
  }
  const C ux = fma(jx, ph.inv_rho0, ph.hg[0]);
  const C uy = fma(jy, ph.inv_rho0, ph.hg[1]);
  const C uz = fma(jz, ph.inv_rho0, ph.hg[2]);
  const C uu15 = (C)1.5 * fma(ux, ux, fma(uy, uy, uz * uz));
  const C ug = fma(ux, ph.g[0], fma(uy, ph.g[1], uz * ph.g[2]));

  const bool edge = FUSED && ((x == 0) | (x == a - 1) | (y == 0) | (y == b - 1) | (z == 0) | (z == c - 1));
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const int ex = EXd(i), ey = EYd(i), ez = EZd(i);
    const C w = (C)Wd(i);
    C eu = (C)0, eg = (C)0;
    if (ex > 0) { eu += ux; eg += ph.g[0]; }
    if (ex < 0) { eu -= ux; eg -= ph.g[0]; }
    if (ey > 0) { eu += uy; eg += ph.g[1]; }
    if (ey < 0) { eu -= uy; eg -= ph.g[1]; }
    if (ez > 0) { eu += uz; eg += ph.g[2]; }
    if (ez < 0) { eu -= uz; eg -= ph.g[2]; }
    // feq~ = w [drho + rho0 (3 eu + 4.5 eu^2 - 1.5 u.u)],  F = w rho0 [3 (eg - ug) + 9 eu eg]
    const C feq = w * fma(ph.rho0, fma((C)4.5 * eu, eu, (C)3 * eu - uu15), drho);
    const C F = (w * ph.rho0) * fma((C)9 * eu, eg, (C)3 * (eg - ug));
    const C post = fma(ph.fcoef, F, fma(-ph.omega, f[i] - feq, f[i]));
    const T out = from_c<PREC, C>(post);
    st<T, NT>(dst + cell + (long long)i * B.Sf, out);
    if (FUSED && i > 0 && edge) {
      // x + e_i pulls f_i from x in the next step: outside this Block, the
      // value goes to the ghost layer of the Block that owns x + e_i
      const int cx = (ex > 0 && x == a - 1) ? 1 : ((ex < 0 && x == 0) ? -1 : 0);
      const int cy = (ey > 0 && y == b - 1) ? 1 : ((ey < 0 && y == 0) ? -1 : 0);
      const int cz = (ez > 0 && z == c - 1) ? 1 : ((ez < 0 && z == 0) ? -1 : 0);
      if ((cx | cy | cz) != 0) {
        const NbrDev nb = A.nbr[bid * 27 + 13 + cx + 3 * cy + 9 * cz];
        if (nb.id >= 0) {
          const BlockDev& M = A.blocks[nb.id];
          const int xm = x + nb.tx, ym = y + nb.ty, zm = z + nb.tz;
          long long o;
          if (ex > 0 && xm < 0)
            o = M.xg + (long long)KLOd(i) * M.P + (long long)(zm + 1) * M.Ry + (ym + 1);
          else if (ex < 0 && xm >= M.dim[0])
            o = M.xg + (long long)(5 + KHId(i)) * M.P + (long long)(zm + 1) * M.Ry + (ym + 1);
          else
            o = main_off(M, i, xm, ym, zm);
          dst[o] = out;
        }
      }
    }
  }
}

template <int PREC, typename C, bool MASK, bool FUSED, bool NT>
__global__ void __launch_bounds__(1024) k_sweep(const SweepArgs A, const Phys<C> ph) {
  for (int it = blockIdx.x; it < A.nitems; it += gridDim.x) {
    const ItemDev item = A.items[it];
    const BlockDev B = A.blocks[item.block];
    const int a = B.dim[0];
    const int ncell = item.nrows * a;
    for (int L = threadIdx.x; L < ncell; L += blockDim.x) {
      const int r = L / a;
      sweep_cell<PREC, C, MASK, FUSED, NT>(A, ph, B, item.block, L - r * a, item.y0 + r, item.z);
    }
  }
}

// --------------------------------------------------------- ghost exchange
// Separate (unfused) exchange: after the sweep, copy the boundary values of
// each neighbour Block straight into this Block's ghost layer (Sec. 4.3:
// process-local communication copies from the sending to the receiving
// Block).  One task = one (Block, neighbour offset, direction) triple.
template <typename T>
__global__ void __launch_bounds__(256) k_exchange(T* __restrict__ grid, const BlockDev* __restrict__ blocks,
                                                  const NbrDev* __restrict__ nbr,
                                                  const XchgTask* __restrict__ tasks, int ntasks) {
  for (int task = blockIdx.y; task < ntasks; task += gridDim.y) {
    const XchgTask t = tasks[task];
    const BlockDev M = blocks[t.dst];
    const NbrDev nb = nbr[t.dst * 27 + t.d];
    const BlockDev N = blocks[nb.id];
    const int i = t.i;
    const int ex = EXd(i), ey = EYd(i), ez = EZd(i);
    for (int L = blockIdx.x * blockDim.x + threadIdx.x; L < t.ncell; L += gridDim.x * blockDim.x) {
      const int q0 = L % t.ext[0];
      const int r = L / t.ext[0];
      const int q1 = r % t.ext[1];
      const int q2 = r / t.ext[1];
      const int gx = t.lo[0] + q0, gy = t.lo[1] + q1, gz = t.lo[2] + q2;
      // only slots whose puller (g + e_i) lies inside the receiving Block
      if (gx + ex < 0 || gx + ex >= M.dim[0] || gy + ey < 0 || gy + ey >= M.dim[1] || gz + ez < 0 ||
          gz + ez >= M.dim[2])
        continue;
      const long long so = main_off(N, i, gx + nb.tx, gy + nb.ty, gz + nb.tz);
      long long o;
      if (gx < 0)
        o = M.xg + (long long)KLOd(i) * M.P + (long long)(gz + 1) * M.Ry + (gy + 1);
      else if (gx >= M.dim[0])
        o = M.xg + (long long)(5 + KHId(i)) * M.P + (long long)(gz + 1) * M.Ry + (gy + 1);
      else
        o = main_off(M, i, gx, gy, gz);
      grid[o] = grid[so];
    }
  }
}

// ----------------------------------------------------- per-cell utilities
__device__ __forceinline__ long long gidx(const GridGeom& g, int x, int y, int z) {
  return ((long long)z * g.n[1] + y) * g.n[0] + x;
}

// Iterate the cells of the item list: f(B, block, x, y, z, solid).
template <typename Fn>
__device__ __forceinline__ void for_cells(const CellArgs& A, Fn&& fn) {
  for (int it = blockIdx.x; it < A.nitems; it += gridDim.x) {
    const ItemDev item = A.items[it];
    const BlockDev B = A.blocks[item.block];
    const int a = B.dim[0];
    const int ncell = item.nrows * a;
    for (int L = threadIdx.x; L < ncell; L += blockDim.x) {
      const int r = L / a;
      const int x = L - r * a, y = item.y0 + r, z = item.z;
      bool solid = false;
      if (A.has_mask) solid = (A.mask[B.mask + ((long long)z * B.dim[1] + y) * a + x] & kSolidBit) != 0;
      fn(B, x, y, z, solid);
    }
  }
}

// Link masks from the global solid mask (bounce-back at obstacles, Sec. 2.1).
__global__ void __launch_bounds__(256) k_linkmask(const uint8_t* __restrict__ solid, CellArgs A,
                                                  uint32_t* __restrict__ mask) {
  for (int it = blockIdx.x; it < A.nitems; it += gridDim.x) {
    const ItemDev item = A.items[it];
    const BlockDev B = A.blocks[item.block];
    const int a = B.dim[0];
    const int ncell = item.nrows * a;
    for (int L = threadIdx.x; L < ncell; L += blockDim.x) {
      const int r = L / a;
      const int x = L - r * a, y = item.y0 + r, z = item.z;
      const int p[3] = {B.org[0] + x, B.org[1] + y, B.org[2] + z};
      uint32_t m = 0;
      if (solid[gidx(A.geo, p[0], p[1], p[2])]) {
        m = kSolidBit;
      } else {
        for (int i = 1; i < kQ; ++i) {
          const int e[3] = {EXd(i), EYd(i), EZd(i)};
          int s[3];
          bool wall = false;
          for (int k = 0; k < 3; ++k) {
            s[k] = p[k] - e[k];
            if (s[k] < 0 || s[k] >= A.geo.n[k]) {
              if (A.geo.wall[k]) wall = true;
              else s[k] = (s[k] + A.geo.n[k]) % A.geo.n[k];
            }
          }
          if (!wall && solid[gidx(A.geo, s[0], s[1], s[2])]) m |= 1u << i;
        }
      }
      mask[B.mask + ((long long)z * B.dim[1] + y) * a + x] = m;
    }
  }
}

// f~ = feq~(rho - rho0, u) of Eq. (2) in FP64 (warm start), 0 in solid cells.
template <int PREC>
__global__ void __launch_bounds__(256) k_init_eq(void* grid_, CellArgs A, double rho0,
                                                 const double* __restrict__ rho,
                                                 const double* __restrict__ u, long long N) {
  using T = typename Stor<PREC>::T;
  T* grid = (T*)grid_;
  for_cells(A, [&](const BlockDev& B, int x, int y, int z, bool solid) {
    const long long g = gidx(A.geo, B.org[0] + x, B.org[1] + y, B.org[2] + z);
    const double ux = u[g], uy = u[N + g], uz = u[2 * N + g];
    const double drho = rho[g] - rho0;
    const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const double eu = EXd(i) * ux + EYd(i) * uy + EZd(i) * uz;
      const double v = Wd(i) * (drho + rho0 * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
      grid[main_off(B, i, x, y, z)] = solid ? from_c<PREC, double>(0.0) : from_c<PREC, double>(v);
    }
  });
}

// rho, u of the stored populations; hg = g/2 is subtracted for a
// post-collision state (the collision adds rho0 g to the momentum).
template <int PREC>
__global__ void __launch_bounds__(256) k_macro(const void* grid_, CellArgs A, double rho0, double hgx,
                                               double hgy, double hgz, double* __restrict__ rho,
                                               double* __restrict__ u, long long N) {
  using T = typename Stor<PREC>::T;
  const T* grid = (const T*)grid_;
  for_cells(A, [&](const BlockDev& B, int x, int y, int z, bool solid) {
    const long long g = gidx(A.geo, B.org[0] + x, B.org[1] + y, B.org[2] + z);
    if (solid) {
      rho[g] = rho0;
      u[g] = 0.0; u[N + g] = 0.0; u[2 * N + g] = 0.0;
      return;
    }
    double d = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const double v = to_c<PREC, double>(grid[main_off(B, i, x, y, z)]);
      d += v;
      jx += EXd(i) * v; jy += EYd(i) * v; jz += EZd(i) * v;
    }
    rho[g] = rho0 + d;
    u[g] = jx / rho0 - hgx;
    u[N + g] = jy / rho0 - hgy;
    u[2 * N + g] = jz / rho0 - hgz;
  });
}

// Global FP64 sums: [0] sum drho, [1..3] sum rho0 u, [4] sum |u - u_prev|^2,
// [5] sum |u|^2.  Per-workgroup partials; workgroup w always takes items w,
// w + G, ... so the result is deterministic.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int PREC>
__global__ void __launch_bounds__(256) k_reduce(const void* cur_, const void* prev_, CellArgs A, double rho0,
                                                double hcx, double hcy, double hcz, double hpx, double hpy,
                                                double hpz, int want_prev, double* __restrict__ partial) {
  using T = typename Stor<PREC>::T;
  const T* cur = (const T*)cur_;
  const T* prev = (const T*)prev_;
  double s[6] = {0, 0, 0, 0, 0, 0};
  for_cells(A, [&](const BlockDev& B, int x, int y, int z, bool solid) {
    if (solid) return;
    double d = 0, jx = 0, jy = 0, jz = 0, px = 0, py = 0, pz = 0;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const long long o = main_off(B, i, x, y, z);
      const double v = to_c<PREC, double>(cur[o]);
      d += v;
      jx += EXd(i) * v; jy += EYd(i) * v; jz += EZd(i) * v;
      if (want_prev) {
        const double w = to_c<PREC, double>(prev[o]);
        px += EXd(i) * w; py += EYd(i) * w; pz += EZd(i) * w;
      }
    }
    const double ux = jx / rho0 - hcx, uy = jy / rho0 - hcy, uz = jz / rho0 - hcz;
    s[0] += d;
    s[1] += rho0 * ux; s[2] += rho0 * uy; s[3] += rho0 * uz;
    if (want_prev) {
      const double dx = ux - (px / rho0 - hpx), dy = uy - (py / rho0 - hpy), dz = uz - (pz / rho0 - hpz);
      s[4] += dx * dx + dy * dy + dz * dz;
    }
    s[5] += ux * ux + uy * uy + uz * uz;
  });
  __shared__ double red[16][6];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double v = wave_sum(s[k]);
    if (lane == 0) red[wid][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double t = 0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) t += red[w][threadIdx.x];
    partial[blockIdx.x * 6 + threadIdx.x] = t;
  }
}

__global__ void __launch_bounds__(256) k_reduce_final(const double* __restrict__ partial, int nparts,
                                                      double* __restrict__ out) {
  __shared__ double red[4][6];
  double s[6] = {0, 0, 0, 0, 0, 0};
  for (int p = threadIdx.x; p < nparts; p += blockDim.x)
#pragma unroll
    for (int k = 0; k < 6; ++k) s[k] += partial[p * 6 + k];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double v = wave_sum(s[k]);
    if (lane == 0) red[wid][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 6) out[threadIdx.x] = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                                          red[3][threadIdx.x];
}

// Checkpoint gather/scatter between the Block grids and [i][z][y][x].
template <int PREC, bool F64>
__global__ void __launch_bounds__(256) k_get_state(const void* grid_, CellArgs A, void* out_, long long N) {
  using T = typename Stor<PREC>::T;
  const T* grid = (const T*)grid_;
  for_cells(A, [&](const BlockDev& B, int x, int y, int z, bool solid) {
    const long long g = gidx(A.geo, B.org[0] + x, B.org[1] + y, B.org[2] + z);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const T v = solid ? from_c<PREC, double>(0.0) : grid[main_off(B, i, x, y, z)];
      if constexpr (F64) ((double*)out_)[i * N + g] = to_c<PREC, double>(v);
      else ((T*)out_)[i * N + g] = v;
    }
  });
}

template <int PREC, bool F64>
__global__ void __launch_bounds__(256) k_set_state(void* grid_, CellArgs A, const void* in_, long long N) {
  using T = typename Stor<PREC>::T;
  T* grid = (T*)grid_;
  for_cells(A, [&](const BlockDev& B, int x, int y, int z, bool solid) {
    const long long g = gidx(A.geo, B.org[0] + x, B.org[1] + y, B.org[2] + z);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      T v;
      if constexpr (F64) v = from_c<PREC, double>(((const double*)in_)[i * N + g]);
      else v = ((const T*)in_)[i * N + g];
      grid[main_off(B, i, x, y, z)] = solid ? from_c<PREC, double>(0.0) : v;
    }
  });
}

// Attainable-bandwidth probe: 16-byte vector copy (Sec. 3.1 measures the
// device's copy bandwidth the same way).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_copy16(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                long long n) {
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + k), dst + k);
}

// ------------------------------------------------------------- launchers
using SweepFn = void (*)(SweepArgs, Phys<double>, Phys<float>, dim3, dim3, hipStream_t);

template <int PREC, typename C, bool MASK, bool FUSED, bool NT>
static void launch_sweep_t(SweepArgs a, Phys<double> pd, Phys<float> pf, dim3 g, dim3 b, hipStream_t s) {
  if constexpr (sizeof(C) == 8)
    hipLaunchKernelGGL((k_sweep<PREC, C, MASK, FUSED, NT>), g, b, 0, s, a, pd);
  else
    hipLaunchKernelGGL((k_sweep<PREC, C, MASK, FUSED, NT>), g, b, 0, s, a, pf);
}

template <int PREC, typename C>
static SweepFn pick3(bool mask, bool fused, bool nt) {
  if (mask) {
    if (fused) return nt ? launch_sweep_t<PREC, C, true, true, true> : launch_sweep_t<PREC, C, true, true, false>;
    return nt ? launch_sweep_t<PREC, C, true, false, true> : launch_sweep_t<PREC, C, true, false, false>;
  }
  if (fused) return nt ? launch_sweep_t<PREC, C, false, true, true> : launch_sweep_t<PREC, C, false, true, false>;
  return nt ? launch_sweep_t<PREC, C, false, false, true> : launch_sweep_t<PREC, C, false, false, false>;
}

void launch_sweep(int prec, bool f64math, bool mask, bool fused, bool nt, const SweepArgs& a,
                  const Phys<double>& pd, const Phys<float>& pf, dim3 grid, dim3 block, hipStream_t s) {
  SweepFn fn = nullptr;
  switch (prec) {
    case 0: fn = pick3<0, double>(mask, fused, nt); break;
    case 1: fn = f64math ? pick3<1, double>(mask, fused, nt) : pick3<1, float>(mask, fused, nt); break;
    case 2: fn = pick3<2, float>(mask, fused, nt); break;
    default: fn = pick3<3, float>(mask, fused, nt); break;
  }
  fn(a, pd, pf, grid, block, s);
}

void launch_exchange(int prec, void* grid, const BlockDev* blocks, const NbrDev* nbr, const XchgTask* tasks,
                     int ntasks, int max_cells, hipStream_t s) {
  if (ntasks <= 0) return;
  const int per = 256;
  int gx = (max_cells + per - 1) / per;
  if (gx > 64) gx = 64;
  if (gx < 1) gx = 1;
  dim3 g(gx, ntasks < 65535 ? ntasks : 65535), b(per);
  switch (prec) {
    case 0: hipLaunchKernelGGL(k_exchange<double>, g, b, 0, s, (double*)grid, blocks, nbr, tasks, ntasks); break;
    case 1: hipLaunchKernelGGL(k_exchange<float>, g, b, 0, s, (float*)grid, blocks, nbr, tasks, ntasks); break;
    default: hipLaunchKernelGGL(k_exchange<uint16_t>, g, b, 0, s, (uint16_t*)grid, blocks, nbr, tasks, ntasks); break;
  }
}

void launch_linkmask(const uint8_t* solid, const CellArgs& a, uint32_t* mask, hipStream_t s) {
  hipLaunchKernelGGL(k_linkmask, dim3(a.nitems), dim3(256), 0, s, solid, a, mask);
}

void launch_init_eq(int prec, void* grid, const CellArgs& a, double rho0, const double* rho, const double* u,
                    long long N, hipStream_t s) {
  dim3 g(a.nitems), b(256);
  switch (prec) {
    case 0: hipLaunchKernelGGL(k_init_eq<0>, g, b, 0, s, grid, a, rho0, rho, u, N); break;
    case 1: hipLaunchKernelGGL(k_init_eq<1>, g, b, 0, s, grid, a, rho0, rho, u, N); break;
    case 2: hipLaunchKernelGGL(k_init_eq<2>, g, b, 0, s, grid, a, rho0, rho, u, N); break;
    default: hipLaunchKernelGGL(k_init_eq<3>, g, b, 0, s, grid, a, rho0, rho, u, N); break;
  }
}

void launch_macro(int prec, const void* grid, const CellArgs& a, double rho0, const double hg[3], double* rho,
                  double* u, long long N, hipStream_t s) {
  dim3 g(a.nitems), b(256);
  switch (prec) {
    case 0: hipLaunchKernelGGL(k_macro<0>, g, b, 0, s, grid, a, rho0, hg[0], hg[1], hg[2], rho, u, N); break;
    case 1: hipLaunchKernelGGL(k_macro<1>, g, b, 0, s, grid, a, rho0, hg[0], hg[1], hg[2], rho, u, N); break;
    case 2: hipLaunchKernelGGL(k_macro<2>, g, b, 0, s, grid, a, rho0, hg[0], hg[1], hg[2], rho, u, N); break;
    default: hipLaunchKernelGGL(k_macro<3>, g, b, 0, s, grid, a, rho0, hg[0], hg[1], hg[2], rho, u, N); break;
  }
}

void launch_reduce(int prec, const void* cur, const void* prev, const CellArgs& a, double rho0, const double hc[3],
                   const double hp[3], int want_prev, double* partial, int nparts, double* out, hipStream_t s) {
  dim3 g(nparts), b(256);
  switch (prec) {
    case 0: hipLaunchKernelGGL(k_reduce<0>, g, b, 0, s, cur, prev, a, rho0, hc[0], hc[1], hc[2], hp[0], hp[1], hp[2], want_prev, partial); break;
    case 1: hipLaunchKernelGGL(k_reduce<1>, g, b, 0, s, cur, prev, a, rho0, hc[0], hc[1], hc[2], hp[0], hp[1], hp[2], want_prev, partial); break;
    case 2: hipLaunchKernelGGL(k_reduce<2>, g, b, 0, s, cur, prev, a, rho0, hc[0], hc[1], hc[2], hp[0], hp[1], hp[2], want_prev, partial); break;
    default: hipLaunchKernelGGL(k_reduce<3>, g, b, 0, s, cur, prev, a, rho0, hc[0], hc[1], hc[2], hp[0], hp[1], hp[2], want_prev, partial); break;
  }
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, partial, nparts, out);
}

void launch_get_state(int prec, bool f64, const void* grid, const CellArgs& a, void* out, long long N,
                      hipStream_t s) {
  dim3 g(a.nitems), b(256);
  switch (prec * 2 + (f64 ? 1 : 0)) {
    case 0: hipLaunchKernelGGL((k_get_state<0, false>), g, b, 0, s, grid, a, out, N); break;
    case 1: hipLaunchKernelGGL((k_get_state<0, true>), g, b, 0, s, grid, a, out, N); break;
    case 2: hipLaunchKernelGGL((k_get_state<1, false>), g, b, 0, s, grid, a, out, N); break;
    case 3: hipLaunchKernelGGL((k_get_state<1, true>), g, b, 0, s, grid, a, out, N); break;
    case 4: hipLaunchKernelGGL((k_get_state<2, false>), g, b, 0, s, grid, a, out, N); break;
    case 5: hipLaunchKernelGGL((k_get_state<2, true>), g, b, 0, s, grid, a, out, N); break;
    case 6: hipLaunchKernelGGL((k_get_state<3, false>), g, b, 0, s, grid, a, out, N); break;
    default: hipLaunchKernelGGL((k_get_state<3, true>), g, b, 0, s, grid, a, out, N); break;
  }
}

void launch_set_state(int prec, bool f64, void* grid, const CellArgs& a, const void* in, long long N,
                      hipStream_t s) {
  dim3 g(a.nitems), b(256);
  switch (prec * 2 + (f64 ? 1 : 0)) {
    case 0: hipLaunchKernelGGL((k_set_state<0, false>), g, b, 0, s, grid, a, in, N); break;
    case 1: hipLaunchKernelGGL((k_set_state<0, true>), g, b, 0, s, grid, a, in, N); break;
    case 2: hipLaunchKernelGGL((k_set_state<1, false>), g, b, 0, s, grid, a, in, N); break;
    case 3: hipLaunchKernelGGL((k_set_state<1, true>), g, b, 0, s, grid, a, in, N); break;
    case 4: hipLaunchKernelGGL((k_set_state<2, false>), g, b, 0, s, grid, a, in, N); break;
    case 5: hipLaunchKernelGGL((k_set_state<2, true>), g, b, 0, s, grid, a, in, N); break;
    case 6: hipLaunchKernelGGL((k_set_state<3, false>), g, b, 0, s, grid, a, in, N); break;
    default: hipLaunchKernelGGL((k_set_state<3, true>), g, b, 0, s, grid, a, in, N); break;
  }
}

void launch_copy16(const void* src, void* dst, long long n16, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, s, (const u32x4*)src, (u32x4*)dst, n16);
}

}  // namespace lbm
