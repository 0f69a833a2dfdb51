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
#include <hip/hip_cooperative_groups.h>
#include <stdint.h>
#include <climits>
#include <algorithm>

#include "lbm_internal.h"

// No implicit multiply-add contraction: every instantiation of a kernel must
// round exactly alike (schedules, exchange variants and Block tilings are
// bit-identical), so fused multiply-adds are written out where wanted.
#pragma clang fp contract(off)



namespace lbm {

// ------------------------------------------------------------------ lattice
// D3Q19 direction i -> e_i and its opposite.  Sec. 2.1.
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
// lattice weight times a factor, from |e_i|^2
// Representative index of the weight class of direction i (rest, face,
// edge): the per-direction constant tables hold equal values within a
// class, so reading one entry per class keeps the kernel's scalar
// registers for what differs.
__host__ __device__ constexpr int WCLS(int i) { return i == 0 ? 0 : (i < 7 ? 1 : 7); }

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
// float -> bfloat16, round to nearest even: gfx950's conversion instruction
// (two conversions of a lane pack into one v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t f32_to_bf16(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float f16_to_f32(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }
// float -> binary16, round to nearest even.  Written as the conversion
// instruction itself so the compiler cannot merge it with the preceding FMA
// into one mixed-precision operation (a single rounding where the other
// kernel variants round twice).
__device__ __forceinline__ uint16_t f32_to_f16(float f) {
  uint32_t r;
  asm("v_cvt_f16_f32 %0, %1" : "=v"(r) : "v"(f));
  return (uint16_t)(r & 0xffffu);
}

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

// Cache policy, measured on gfx950: population loads are ordinary (streaming
// loads lose 1-6 % on every workload but 32-wide Blocks), and the stores of
// whole row segments may stream (NT); values written one or a few per row
// (bounce-back at walls, x-ghost planes) are always ordinary stores, so
// that the L2 merges the parts of a line that different waves write
// before it goes to memory (streamed, each such part costs HBM a partial
// line: 7 % of the FP32 sweep on a 384^3 box with x walls).
template <typename T>
__device__ __forceinline__ T ld(const T* p) {
  return *p;
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
template <int BYTES> struct Raw;
template <> struct Raw<2> { typedef uint16_t V; };
template <> struct Raw<4> { typedef uint32_t V; };
template <> struct Raw<8> { typedef uint32_t V __attribute__((ext_vector_type(2))); };
template <> struct Raw<16> { typedef uint32_t V __attribute__((ext_vector_type(4))); };

// One value at a scalar base plus a 32-bit lane byte offset (one global
// instruction with the base in SGPRs).
template <typename T>
__device__ __forceinline__ T ldo(const T* base, uint32_t boff) {
  return ld<T>((const T*)((const char*)base + boff));
}
template <typename T, bool NT>
__device__ __forceinline__ void sto(T* base, uint32_t boff, T v) {
  st<T, NT>((T*)((char*)base + boff), v);
}
// VEC consecutive values at a scalar base plus a 32-bit lane byte offset.
template <typename T, int VEC>
__device__ __forceinline__ void vld(const T* base, uint32_t boff, T (&out)[VEC]) {
  typedef typename Raw<sizeof(T) * VEC>::V V;
  const V v = ld<V>((const V*)((const char*)base + boff));
  __builtin_memcpy(out, &v, sizeof(V));
}
// One value at base + boff (bytes) by a raw buffer store: the 64-bit base
// lives in the scalar descriptor, the lane supplies only the 32-bit offset.
template <typename T>
__device__ __forceinline__ void buf_store(T* base, uint32_t boff, T v) {
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, 0x7fffffff, 0x00020000);
  if constexpr (sizeof(T) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(unsigned int __attribute__((__vector_size__(8))), v),
                                          rs, boff, 0, 0);
  else if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rs, boff, 0, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), rs, boff, 0, 0);
}

// Addressing of the one-cell-per-lane sweep.  The 19 population arrays of a
// Block are covered by five buffer resources, one per group of arrays
// {0..4}, {5..8}, {9..12}, {13..16}, {17, 18} (a direction and its opposite
// share a group), each based two elements before its first array.  A
// pulled or stored value is then (resource, the lane's 32-bit offset, a
// 32-bit scalar offset of the direction's row, an immediate), so the 38
// streams of a row cost no per-direction 64-bit address arithmetic and the
// rows of an item share the lane offset.  Group offsets stay below
// 6 Sf elements (checked when the Block is created).
__host__ __device__ constexpr int GRP0(int i) { return i < 5 ? 0 : (i < 9 ? 5 : (i < 13 ? 9 : (i < 17 ? 13 : 17))); }
constexpr int kGroups = 5;
__host__ __device__ constexpr int GRPI(int i) { return i < 5 ? 0 : (i < 9 ? 1 : (i < 13 ? 2 : (i < 17 ? 3 : 4))); }
// Sector of a row's last line that the padding lanes of the sweep complete
// (measured on gfx950, FP32 periodic cubes: 32-byte sectors lift 255^3 from
// 31.3k to 35.0k MLUPS, 64-byte sectors 257^3 too, 31.6k -> 32.6k, and 200^3,
// 30.3k -> 32.0k; whole 128-byte lines add more write traffic than they save)
constexpr int kPadSector = 64;
constexpr uint32_t kRange = 0xFFFFFFF0u;  // records of a group resource; an offset of kRange reads zero
__device__ __forceinline__ __amdgpu_buffer_rsrc_t grp_rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)kRange, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T rs_load(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
  else if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(rs, voff, soff, 0));
}
template <typename T, bool NT>
__device__ __forceinline__ void rs_store(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, T v) {
  constexpr int aux = NT ? 2 : 0;  // streaming (nt)
  if constexpr (sizeof(T) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(unsigned int __attribute__((__vector_size__(8))), v),
                                          rs, voff, soff, aux);
  else if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rs, voff, soff, aux);
  else
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), rs, voff, soff, aux);
}

// VEC values loaded into whole 32-bit registers (a lone 16-bit value is
// zero-extended) and split later.
template <int BYTES> struct WideRaw { typedef typename Raw<BYTES>::V V; };
template <> struct WideRaw<2> { typedef uint32_t V; };
template <typename T, int VEC>
__device__ __forceinline__ typename WideRaw<sizeof(T) * VEC>::V ld_wide(const T* base, uint32_t boff) {
  typedef typename Raw<sizeof(T) * VEC>::V V;
  return (typename WideRaw<sizeof(T) * VEC>::V)ld<V>((const V*)((const char*)base + boff));
}
template <typename T, int VEC>
__device__ __forceinline__ void unpack_wide(typename WideRaw<sizeof(T) * VEC>::V w, T (&out)[VEC]) {
  typedef typename Raw<sizeof(T) * VEC>::V V;
  const V v = (V)w;
  __builtin_memcpy(out, &v, sizeof(V));
}
template <typename T, int VEC, bool NT>
__device__ __forceinline__ void vst(T* base, uint32_t boff, const T (&in)[VEC]) {
  typedef typename Raw<sizeof(T) * VEC>::V V;
  V v;
  __builtin_memcpy(&v, in, sizeof(V));
  st<V, NT>((V*)((char*)base + boff), v);
}
template <typename T>
__device__ __forceinline__ T sh_up(T v) {  // value of lane - 1
  if constexpr (sizeof(T) == 2) return (T)__shfl_up((int)v, 1, 64);
  else return __shfl_up(v, 1, 64);
}
template <typename T>
__device__ __forceinline__ T sh_down(T v) {  // value of lane + 1
  if constexpr (sizeof(T) == 2) return (T)__shfl_down((int)v, 1, 64);
  else return __shfl_down(v, 1, 64);
}

// A wave-uniform value moved into scalar registers behind an opaque point:
// what is computed from it stays after that point.
__device__ __forceinline__ int sgpr_launder(int v) {
  int r = __builtin_amdgcn_readfirstlane(v);
  asm volatile("" : "+s"(r));
  return r;
}
__device__ __forceinline__ long long sgpr_launder(long long v) {
  int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffLL));
  int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  asm volatile("" : "+s"(lo), "+s"(hi));
  return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Kernel arguments of the sweep read through the kernel-argument segment
// (address space 4: scalar loads): the SweepArgs first, the Phys<C> next at
// its natural alignment (the order and alignment of explicit kernel
// arguments).
#define KAS __attribute__((address_space(4)))
template <bool VIA_SEGMENT, typename C> struct ArgPtrs;
template <typename C>
struct ArgPtrs<true, C> {
  const SweepArgs KAS* a;
  const Phys<C> KAS* p;
  __device__ __forceinline__ static ArgPtrs at(const char KAS* k) {
    asm volatile("" : "+s"(k));
    constexpr size_t off = (sizeof(SweepArgs) + alignof(Phys<C>) - 1) / alignof(Phys<C>) * alignof(Phys<C>);
    return ArgPtrs{(const SweepArgs KAS*)k, (const Phys<C> KAS*)(k + off)};
  }
  __device__ __forceinline__ static ArgPtrs get(const SweepArgs&, const Phys<C>&) {
    return at((const char KAS*)__builtin_amdgcn_kernarg_segment_ptr());
  }
  __device__ __forceinline__ ArgPtrs again() const { return at((const char KAS*)a); }
};
// the plain form: the parameters themselves (the compiler keeps what it
// likes in registers)
template <typename C>
struct ArgPtrs<false, C> {
  const SweepArgs* a;
  const Phys<C>* p;
  __device__ __forceinline__ static ArgPtrs get(const SweepArgs& A, const Phys<C>& ph) { return ArgPtrs{&A, &ph}; }
  __device__ __forceinline__ ArgPtrs again() const { return *this; }
};

// Flags of the wall faces that the sources of a lane's cells lie beyond.
struct WallFlags {
  bool lox, hix, loy, hiy, loz, hiz;
};

// Wall link of direction i at element k of VEC: the source x - e_i lies
// beyond a wall face (x faces only concern the lane's first / last element).
template <int VEC>
__device__ __forceinline__ bool wall_link(const WallFlags& w, int i, int k) {
  const int ex = EXd(i), ey = EYd(i), ez = EZd(i);
  bool b = false;
  if (ex > 0 && k == 0) b = b || w.lox;
  if (ex < 0 && k == VEC - 1) b = b || w.hix;
  if (ey > 0) b = b || w.loy;
  if (ey < 0) b = b || w.hiy;
  if (ez > 0) b = b || w.loz;
  if (ez < 0) b = b || w.hiz;
  return b;
}

// 6 w_i rho0 (e_i . u_w) of the first moving face (order -x,+x,-y,+y,-z,+z)
// that the source of a wall link lies beyond (the half-way bounce-back rule
// with wall velocity, Sec. 2.1).
template <typename C, int VEC, typename AT, typename PT>
__device__ __forceinline__ C wall_corr(const AT& A, const PT& ph, const WallFlags& w, int i, int k) {
  const int ex = EXd(i), ey = EYd(i), ez = EZd(i);
  C cw = (C)0;
  if (ez > 0 && w.loz && A.geo.moving[4]) cw = ph.corr[i][4];
  if (ez < 0 && w.hiz && A.geo.moving[5]) cw = ph.corr[i][5];
  if (ey > 0 && w.loy && A.geo.moving[2]) cw = ph.corr[i][2];
  if (ey < 0 && w.hiy && A.geo.moving[3]) cw = ph.corr[i][3];
  if (ex > 0 && k == 0 && w.lox && A.geo.moving[0]) cw = ph.corr[i][0];
  if (ex < 0 && k == VEC - 1 && w.hix && A.geo.moving[1]) cw = ph.corr[i][1];
  return cw;
}

// Open x faces (non-equilibrium extrapolation, Guo, Zheng and Shi 2002): the
// boundary node beyond face `side`, next to a cell with moments (drho_f,
// u_f) and post-collision value f*_q, holds f*_q + feq~_q(drho_b, u_b) -
// feq~_q(drho_f, u_f).  VELOCITY: u_b prescribed, drho_b = drho_f, so
//   w_q rho0 [3 e.(u_b - u_f) + 4.5 ((e.u_b)^2 - (e.u_f)^2) - 1.5 (u_b^2 - u_f^2)];
// PRESSURE: drho_b prescribed, u_b = u_f, so w_q (drho_b - drho_f).
__device__ __forceinline__ double open_corr(const GridGeom& g, int side, int q, double rho0, double drho_f,
                                            double ufx, double ufy, double ufz) {
  const double w = Wd(q);
  if (g.open[side] == 2) return w * (g.ob_drho[side] - drho_f);
  const double* ub = g.ob_u[side];
  const double eb = EXd(q) * ub[0] + EYd(q) * ub[1] + EZd(q) * ub[2];
  const double ef = EXd(q) * ufx + EYd(q) * ufy + EZd(q) * ufz;
  const double bb = ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2];
  const double ff = ufx * ufx + ufy * ufy + ufz * ufz;
  return w * rho0 * (3.0 * (eb - ef) + 4.5 * (eb * eb - ef * ef) - 1.5 * (bb - ff));
}

// One wave updates a row segment: each lane owns VEC consecutive cells of a
// row, xw lanes per row (the smallest power of two covering the row, at most
// 64), 64/xw rows per wave, the segment's first cell at x = x0w; or (xw = 0,
// flat runs, one cell per lane) 64 consecutive cells of the plane, from cell
// x0w of row y0w on, across row ends.  Either way the plane z and the first
// row y0w are uniform and every stream is one access at a scalar base (SGPRs)
// plus a 32-bit lane offset.
//
// Pull phase (branch-free, all 19 streams in flight): every population comes
// from its source slot x - e_i -- inside the Block, from the ghost layer (the
// neighbour Block's value), or, across a wall, from a bounce-back slot written
// by this cell in the previous step (Sec. 2.1: pull scheme and half-way
// bounce-back).  Across an obstacle link the cell's own f*_ibar of the
// previous step replaces the pulled value (one more load per direction that
// has such a link in the wave).  With one cell per lane the x-shifted source
// is a shifted load; with two, the adjacent lane's value arrives by a lane
// shuffle.
//
// Update phase: moments, BGK collision with the shifted incompressible
// equilibrium of Eq. (2) and the Guo force term, evaluated per pair of
// opposite directions (even part of feq and F shared, odd part flips sign);
// aligned stores (zeros for solid cells, so that no cache line is written
// in part); bounce-back writes f*_ibar + 6 w_i rho0 e_i.u_w into the slot of
// every wall link; with FUSED the boundary values also go
// straight into the neighbours' ghost layers (the on-GPU copies of Sec. 4.4,
// fused into the sweep).
// FORCE = false (16-bit storage without a body force): the force terms,
// all zero, are left out of the collision (the storage formats' sweeps are
// bound by instruction issue, not bytes).
template <int PREC, typename C, bool MASK, int FX, bool NT, int VEC, bool OPEN, bool FORCE = true>
__device__ __forceinline__ void sweep_row(const SweepArgs& A_in, const Phys<C>& ph_in, const void* src_grid, void* dst_grid,
                                          const BlockDev& B_in, int bid, int z, int y0w, int x0w, int yend, int xw,
                                          const GhostTgt* gts) {
  // The kernel's arguments (this sweep's pointers, the geometry and the
  // physical constants) are read through the kernel-argument segment at the
  // point of use, here and again after the pull phase, instead of being
  // kept in scalar registers across the item and row loops (which spills
  // them into vector lanes): the pointer is laundered so that no load is
  // hoisted above these points.
  // Which of these help was measured per kernel variant on gfx950 (same
  // box, A/B): reading the arguments at the point of use pays for every
  // variant but the 16-bit ones without obstacles that apply a body force
  // (without one, 16-bit cavity sweep 0.835 -> 0.831 ms F16S, 0.841 ->
  // 0.833 ms BF16S); laundering the Block's layout values, for FP32 and
  // FP64 storage without obstacles (the force-free 16-bit sweeps lose 5 %
  // with it); the scalar-offset buffer addressing below, for the obstacle
  // variants (the porous channel's sweep 1.165 -> 1.108 ms; the others lose
  // 1-2 % with it).
  constexpr bool KARGS = !(PREC >= 2 && !MASK && FORCE);
  constexpr bool BLAUNDER = !MASK && PREC <= 1;
  constexpr bool ADDR = MASK && VEC == 1;
  auto ka = ArgPtrs<KARGS, C>::get(A_in, ph_in);
  auto pa = ka.a;
  auto pp = ka.p;
  // The Block's layout values, laundered likewise: what the row's addresses
  // derive from them is computed per row, not kept for the whole item.
  BlockDev B = B_in;
  if constexpr (BLAUNDER) {
    B.base = sgpr_launder(B.base);
    B.Sf = sgpr_launder(B.Sf);
    B.Sz = sgpr_launder(B.Sz);
    B.xgo = sgpr_launder(B.xgo);
    B.Sx = sgpr_launder(B.Sx);
    B.Ry = sgpr_launder(B.Ry);
  }
  using T = typename Stor<PREC>::T;
  const T* __restrict__ src = (const T*)src_grid;
  T* __restrict__ dst = (T*)dst_grid;
  const int lane = threadIdx.x & 63;
  const int a = B.dim[0], b = B.dim[1], c = B.dim[2];
  // row of the lane within the wave, its place in the row, its first cell
  const int r = xw ? lane / xw : (unsigned)(x0w + lane) / (unsigned)a;
  const int xl = xw ? lane - r * xw : 0;
  const int x0 = xw ? x0w + xl * VEC : x0w + lane - r * a;
  const int y = y0w + r;
  // Lanes of a live row all take part in the shuffles; a lane only reads a
  // neighbour lane of its own live row.
  // Padding lanes (one cell per lane, rows padded past a): the lanes past
  // the row's last cell up to the end of its last 64-byte sector store into
  // the row padding, so that the row's last line is not written in part
  // (the memory then merges the partial sector by a read-modify-write: a
  // row of 255 FP32 cells took 12 % longer than one of 256 with the same
  // traffic).  Their values go to the padding only, which no cell reads;
  // no wall, face or exchange rule applies to them, and with obstacles they
  // take the solid-cell path (no loads, zeros stored).  Otherwise their
  // pulls read slots next to their own (the row's last line, or slot Sx,
  // the next row's first), or, with 16-bit storage, their own slots
  // (measured per variant on gfx950: the select costs the FP32 sweep 0.7 %
  // and gains the F16S sweep 1.3 %).
  const int pend = VEC == 1 && xw != 0
                       ? min(B.Sx, (a * (int)sizeof(T) + kPadSector - 1) / kPadSector * kPadSector / (int)sizeof(T))
                       : a;
  if (x0 >= pend || y >= yend) return;
  const bool pad = x0 >= a;

  // The group resources and scalar row offsets of the one-cell-per-lane
  // addressing are rebuilt for every row from the Block's base and strides
  // (laundered here so that the compiler does not keep ten resources and
  // some forty offsets of an item live across its rows, which spills scalar
  // registers into vector lanes).
  long long gsrc = (long long)(uintptr_t)src_grid, gdst = (long long)(uintptr_t)dst_grid, gbase = B.base;
  if constexpr (VEC == 1 && BLAUNDER) {
    asm volatile("" : "+s"(gsrc), "+s"(gdst), "+s"(gbase));
  }
  const T* gsp = (const T*)(uintptr_t)gsrc;
  T* gdp = (T*)(uintptr_t)gdst;
  // Scalar bases address row starts; the lane offset carries the row within
  // the wave, the segment and the lane's cells (all non-negative).
  const long long rb = B.base + (long long)(z + 1) * B.Sz + (long long)(y0w + 1) * B.Sx;
  const uint32_t lo = (uint32_t)(r * B.Sx + x0);
  const uint32_t lob = lo * (uint32_t)sizeof(T);
  // axes on which the Block wraps onto itself (uniform; y only with one row
  // per wave, so y0w is every live lane's row)
  const bool wx = (B.wrap & 1) != 0, wy = (B.wrap & 2) != 0, wz = (B.wrap & 4) != 0;
  auto wrapc = [](int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); };
  // in-row sources past the x faces of a Block that wraps in x
  const uint32_t xwrap_lo = (uint32_t)((r * B.Sx + a) * (int)sizeof(T));  // x = -1 -> a - 1
  const uint32_t xwrap_hi = (uint32_t)((r * B.Sx + 1) * (int)sizeof(T));  // x = a  -> 0
  const bool xg_lo = x0 == 0;              // first cell pulls e_x = +1 from the x-ghost plane
  const bool xg_hi = x0 + VEC == a;         // last cell pulls e_x = -1 from the x-ghost plane
  const bool first = xl == 0;
  const bool last = (xl == xw - 1) || xg_hi;

  // Link masks first (obstacle links decide which sources are replaced
  // below); the pulls go out right behind this load.
  uint32_t m[VEC];
  bool solid[VEC];
#pragma unroll
  for (int k = 0; k < VEC; ++k) {
    m[k] = 0;
    solid[k] = false;
  }
  if constexpr (MASK) {
    const uint32_t* mp = pa->mask + B.mask + ((long long)z * b + y) * a + (pad ? 0 : x0);
#pragma unroll
    for (int k = 0; k < VEC; ++k) m[k] = mp[k];
    if (pad) m[0] = kSolidBit;
    if constexpr (VEC == 1) solid[0] = (m[0] & kSolidBit) != 0;
    __builtin_amdgcn_sched_barrier(0);
  }

  // ---- pull phase: W[i][k] = stored value that cell k receives along e_i
  T W[kQ][VEC];
  T sv[kQ];  // VEC > 1: the vector element the adjacent lane needs
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const int ex = EXd(i), ey = EYd(i), ez = EZd(i);
    // source row of direction i (wrapped on the Block's wrap axes)
    const int zs = wz ? wrapc(z - ez, c) : z - ez;
    const int ys = wy ? wrapc(y0w - ey, b) : y0w - ey;
    const long long row = B.base + (long long)i * B.Sf + (long long)(zs + 1) * B.Sz + (long long)(ys + 1) * B.Sx;
    // Scalar base one element before the row so that every lane offset is
    // non-negative (x - 1 of the first cell); the x-ghost slot of the lane's
    // source row, relative to the same base:
    const T* pr = src + (row - 1);
    const long long dxg = B.xgo + (long long)(zs + 1) * (B.Ry - B.Sz) + (long long)(ys + 1) * (1 - B.Sx) + 1;
    const uint32_t xgb = (uint32_t)((dxg + r) * (long long)sizeof(T));
    const uint32_t xlo = wx ? xwrap_lo : xgb, xhi = wx ? xwrap_hi : xgb;
    const uint32_t S1 = (uint32_t)sizeof(T);
    if constexpr (VEC == 1 && ADDR) {
      // group resource of direction i; scalar offset of its source row;
      // the lane offset (lob + s, shared by all directions) plus (1 - e_x) s
      const int g0 = GRP0(i);
      const __amdgpu_buffer_rsrc_t rs = grp_rsrc(gsp + (gbase + (long long)g0 * B.Sf - 2));
      const uint32_t so = (uint32_t)(((long long)(i - g0) * B.Sf + (long long)(zs + 1) * B.Sz +
                                      (long long)(ys + 1) * B.Sx) * (long long)sizeof(T));
      uint32_t vo = lob + (uint32_t)((2 - ex) * (int)sizeof(T));
      if (ex != 0) {
        // x-ghost slot of the source row (or, wrapping in x, the other end
        // of the row), as a lane offset against the same scalar offset
        const long long xg = B.xgo + (long long)(zs + 1) * (B.Ry - B.Sz) + (long long)(ys + 1) * (1 - B.Sx) + 2;
        const uint32_t xgv = (uint32_t)((xg + r) * (long long)sizeof(T));
        const uint32_t xwv = (uint32_t)((ex > 0 ? r * B.Sx + a + 1 : r * B.Sx + 2) * (int)sizeof(T));
        const uint32_t xv = wx ? xwv : xgv;
        if (ex > 0) vo = xg_lo ? xv : vo;
        if (ex < 0) vo = xg_hi ? xv : vo;
      }
      // one load per value: a lane with an obstacle link along e_i reads its
      // own slot of array ibar (same group) instead of the solid source, a
      // solid lane reads nothing (offset past the range)
      const uint32_t own = (uint32_t)(((long long)(OPPd(i) - g0) * B.Sf + (long long)(z + 1) * B.Sz +
                                       (long long)(y0w + 1) * B.Sx) * (long long)sizeof(T)) + lob + 2u * S1;
      uint32_t o = (i != 0 && ((m[0] >> i) & 1u)) ? own : so + vo;
      o = solid[0] ? kRange : o;
      W[i][0] = rs_load<T>(rs, o, 0u);
    } else if constexpr (VEC == 1) {
      uint32_t off = lob + (uint32_t)((1 - ex) * (int)sizeof(T));
      if (ex > 0) off = xg_lo ? xlo : off;
      if (ex < 0) off = xg_hi ? xhi : off;
      if constexpr (PREC >= 2) {
        if (ex != 0) off = pad ? lob + S1 : off;
      }
      W[i][0] = ldo<T>(pr, off);
    } else {
      T V[VEC];
      vld<T, VEC>(pr, lob + S1, V);
      // the element just outside the vector: x-ghost slot (or, wrapping, the
      // other end of the row), neighbouring segment, or (interior lanes,
      // replaced by the shuffle) the lane's own
      uint32_t off = lob + S1;
      if (ex > 0) off = first ? (xg_lo ? xlo : lob) : lob + S1;
      if (ex < 0) off = last ? (xg_hi ? xhi : lob + (uint32_t)(VEC + 1) * S1) : lob + S1;
      T e = V[0];
      if (ex != 0) e = ldo<T>(pr, off);
#pragma unroll
      for (int k = 0; k < VEC; ++k) W[i][k] = V[k];
      if (ex > 0) {
#pragma unroll
        for (int k = VEC - 1; k > 0; --k) W[i][k] = V[k - 1];
        W[i][0] = e;
        sv[i] = V[VEC - 1];
      } else if (ex < 0) {
#pragma unroll
        for (int k = 0; k < VEC - 1; ++k) W[i][k] = V[k + 1];
        W[i][VEC - 1] = e;
        sv[i] = V[0];
      }
    }
  }
  if constexpr (VEC > 1) {
    // x +- 1 from the adjacent lane (all loads are in flight by now)
#pragma unroll
    for (int i = 1; i < kQ; ++i) {
      const int ex = EXd(i);
      if (ex > 0) {
        const T v = sh_up(sv[i]);
        if (!first) W[i][0] = v;
      }
      if (ex < 0) {
        const T v = sh_down(sv[i]);
        if (!last) W[i][VEC - 1] = v;
      }
    }
  }

  if constexpr (MASK && VEC > 1) {
    // Half-way bounce-back at obstacles on the pull side: when x - e_i is
    // solid, cell x receives its own f*_ibar of the previous step, read from
    // its own slot of array ibar (one more load, only for directions where
    // some lane of the wave has such a link).
#pragma unroll
    for (int k = 0; k < VEC; ++k) solid[k] = (m[k] & kSolidBit) != 0;
    // All loads first, each into whole registers, and the substitutions
    // after them: a value merged into a shared register inside its branch
    // would make every load wait for all earlier ones.
    typedef typename WideRaw<sizeof(T) * VEC>::V RV;
    RV own[kQ];
#pragma unroll
    for (int i = 1; i < kQ; ++i) {
      bool any = false;
#pragma unroll
      for (int k = 0; k < VEC; ++k) any = any || ((m[k] >> i) & 1u);
      if (any) own[i] = ld_wide<T, VEC>(src + (rb + (long long)OPPd(i) * B.Sf), lob);
    }
#pragma unroll
    for (int i = 1; i < kQ; ++i) {
      T o[VEC];
      unpack_wide<T, VEC>(own[i], o);
#pragma unroll
      for (int k = 0; k < VEC; ++k)
        if ((m[k] >> i) & 1u) W[i][k] = o[k];
    }
  }

  // ---- update phase
  ka = ka.again();
  pa = ka.a;
  pp = ka.p;
  const int gx0 = B.org[0] + x0, gy = B.org[1] + y, gz = B.org[2] + z;
  WallFlags wf;
  wf.lox = pa->geo.fwall[0] && gx0 == 0;
  wf.hix = pa->geo.fwall[1] && gx0 + VEC - 1 == pa->geo.n[0] - 1;
  wf.loy = pa->geo.fwall[2] && gy == 0;
  wf.hiy = pa->geo.fwall[3] && gy == pa->geo.n[1] - 1;
  wf.loz = pa->geo.fwall[4] && gz == 0;
  wf.hiz = pa->geo.fwall[5] && gz == pa->geo.n[2] - 1;
  if (pad) wf.lox = wf.hix = wf.loy = wf.hiy = wf.loz = wf.hiz = false;
  const bool moving = pa->geo.moving[0] | pa->geo.moving[1] | pa->geo.moving[2] | pa->geo.moving[3] | pa->geo.moving[4] |
                      pa->geo.moving[5];

  // moments (Sec. 2.1): drho = sum f~, rho0 u = sum e f~, plus half force.
  // FP32 storage with FP32 arithmetic (HYB) keeps the velocity in FP64: the
  // half-force shift g/2 is far below the rounding unit of u in FP32.
  constexpr bool HYB = PREC == 1 && sizeof(C) == 4;
  C drho[VEC], ux[VEC], uy[VEC], uz[VEC], uu15[VEC], ug3[VEC];
  double dux[VEC], duy[VEC], duz[VEC];
#pragma unroll
  for (int k = 0; k < VEC; ++k) {
    C d = to_c<PREC, C>(W[0][k]), jx = (C)0, jy = (C)0, jz = (C)0;
#pragma unroll
    for (int i = 1; i < kQ; i += 2) {  // (i, i+1) are opposite directions
      const C fa = to_c<PREC, C>(W[i][k]), fb = to_c<PREC, C>(W[i + 1][k]);
      const C sp = fa + fb, dp = fa - fb;
      d += sp;
      if (EXd(i) > 0) jx += dp;
      if (EXd(i) < 0) jx -= dp;
      if (EYd(i) > 0) jy += dp;
      if (EYd(i) < 0) jy -= dp;
      if (EZd(i) > 0) jz += dp;
      if (EZd(i) < 0) jz -= dp;
    }
    drho[k] = d;
    if constexpr (HYB) {
      dux[k] = fma((double)jx, pp->dinv_rho0, pp->dhg[0]);
      duy[k] = fma((double)jy, pp->dinv_rho0, pp->dhg[1]);
      duz[k] = fma((double)jz, pp->dinv_rho0, pp->dhg[2]);
      ux[k] = (C)dux[k];
      uy[k] = (C)duy[k];
      uz[k] = (C)duz[k];
    } else {
      ux[k] = fma(jx, pp->inv_rho0, pp->hg[0]);
      uy[k] = fma(jy, pp->inv_rho0, pp->hg[1]);
      uz[k] = fma(jz, pp->inv_rho0, pp->hg[2]);
    }
    uu15[k] = (C)1.5 * fma(ux[k], ux[k], fma(uy[k], uy[k], uz[k] * uz[k]));
    if constexpr (FORCE)
      ug3[k] = pp->rho0x3 * fma(ux[k], pp->g[0], fma(uy[k], pp->g[1], uz[k] * pp->g[2]));
    else
      ug3[k] = (C)0;
  }

  // stores of direction i; solid cells store zero (no cell reads their
  // slots: obstacle links are bounced on the pull side), which keeps every
  // cache line whole (partial-line writes cost the memory a
  // read-modify-write)
  auto store_dir = [&](int i, const T (&o)[VEC]) {
    if constexpr (VEC == 1 && ADDR) {
      // group resource of direction i, scalar offset of the cell's row
      const int g0 = GRP0(i);
      const __amdgpu_buffer_rsrc_t rs = grp_rsrc(gdp + (gbase + (long long)g0 * B.Sf - 2));
      const uint32_t so = (uint32_t)(((long long)(i - g0) * B.Sf + (long long)(z + 1) * B.Sz +
                                      (long long)(y0w + 1) * B.Sx) * (long long)sizeof(T));
      T v = o[0];
      if constexpr (MASK) v = solid[0] ? from_c<PREC, double>(0.0) : v;
      rs_store<T, NT>(rs, lob + 2u * (uint32_t)sizeof(T), so, v);
      return;
    }
    T* base = dst + (rb + (long long)i * B.Sf);
    if constexpr (MASK) {
      T v[VEC];
#pragma unroll
      for (int k = 0; k < VEC; ++k) v[k] = solid[k] ? from_c<PREC, double>(0.0) : o[k];
      vst<T, VEC, NT>(base, lob, v);
    } else {
      vst<T, VEC, NT>(base, lob, o);
    }
  };
  // bounce-back writes at walls: cell k sends f*_q(x) (plus the moving-wall
  // term) to the slot (x + e_q, qbar) that it pulls along qbar next step
  // when x + e_q lies beyond a wall: its own slot in array qbar shifted by
  // e_q (a uniform offset from the stores' base, same lane offset), or, past
  // an x face of the Block, the x-ghost plane (rare, kept off the common path)
  auto bounce = [&](int q, const T (&o)[VEC]) {
    const int qb = OPPd(q);
    const int exq = EXd(q), eyq = EYd(q), ezq = EZd(q);
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      bool bb = wall_link<VEC>(wf, qb, k);
      if constexpr (MASK) bb = bb && !solid[k];
      if (bb) {
        T v = o[k];
        if (moving && wall_link<VEC>(wf, qb, k))
          v = from_c<PREC, C>(to_c<PREC, C>(o[k]) + wall_corr<C, VEC>(*pa, *pp, wf, qb, k));
        // shifted row of array qbar (wrapped like the pull that reads it),
        // one element early so that the lane offset stays non-negative
        const int zt = wz ? wrapc(z + ezq, c) : z + ezq;
        const int yt = wy ? wrapc(y0w + eyq, b) : y0w + eyq;
        const long long row = B.base + (long long)qb * B.Sf + (long long)(zt + 1) * B.Sz + (long long)(yt + 1) * B.Sx;
        const int j = k + exq;  // target element index relative to x0
        if (!((j < 0 && xg_lo) || (j >= VEC && xg_hi))) {
          sto<T, false>(dst + (row - 1), lob + (uint32_t)((j + 1) * (int)sizeof(T)), v);
        } else if (wx) {
          sto<T, false>(dst + (row - 1), j < 0 ? xwrap_lo : xwrap_hi, v);
        } else {
          const long long dxg = B.xgo + (long long)(zt + 1) * (B.Ry - B.Sz) + (long long)(yt + 1) * (1 - B.Sx) + 1;
          sto<T, false>(dst + (row - 1), (uint32_t)((dxg + r) * (long long)sizeof(T)), v);
        }
      }
    }
  };
  // fused exchange, generic case: neighbour (cx, cy, cz) of cell x0 + k
  // receives direction q when q leaves the Block through that face/edge/corner
  auto nbr_of = [&](int q, int k) {
    const int x = x0 + k;
    const int qx = EXd(q), qy = EYd(q), qz = EZd(q);
    // (crossing an axis the Block wraps on is no crossing)
    const int cx = wx ? 0 : ((qx > 0 && x == a - 1) ? 1 : ((qx < 0 && x == 0) ? -1 : 0));
    const int cy = wy ? 0 : ((qy > 0 && y == b - 1) ? 1 : ((qy < 0 && y == 0) ? -1 : 0));
    const int cz = wz ? 0 : ((qz > 0 && z == c - 1) ? 1 : ((qz < 0 && z == 0) ? -1 : 0));
    return (cx | cy | cz) != 0 ? 13 + cx + 3 * cy + 9 * cz : 13;
  };
  // Rows of this wave (y0w .. ylast, z fixed) off the y and z faces of the
  // Block only send from their first and last cell, to the two x-face
  // neighbours: their table entries are wave-uniform and read once.  Waves
  // with a row on a y or z face take the generic per-lane path.
  const int ylast = min(y0w + (xw ? 64 / xw : (x0w + 63) / a + 1), yend) - 1;
  const bool yz_face = (z == 0) | (z == c - 1) | (y0w == 0) | (ylast >= b - 1);
  constexpr bool FUSED = FX == 1;
  const bool edge = FUSED && yz_face && !pad &&
                    ((x0 == 0) | (x0 + VEC - 1 == a - 1) | (y == 0) | (y == b - 1) | (z == 0) | (z == c - 1));
  // x-ghost slot of row y for direction q: base + q * Sf (wave-uniform) plus
  // the lane's row offset within the wave
  long long xm0 = 0, xmf = 0, xp0 = 0, xpf = 0;
  bool xm_on = false, xp_on = false;
  // FX == 1: waves off the y/z faces (the rest takes the generic path);
  // FX == 2: every wave, lanes whose row is off the y/z faces (the exchange
  // kernel copies the rim rows)
  const bool xsend = FX == 1 ? !yz_face : FX == 2;
  if (xsend) {
    const GhostTgt& Gm = pa->ghost[bid * 27 + 12];
    const GhostTgt& Gp = pa->ghost[bid * 27 + 14];
    xm_on = Gm.kind != 0;
    xp_on = Gp.kind != 0;
    xm0 = Gm.xg0 + (long long)z * Gm.Ry + y0w;
    xp0 = Gp.xg0 + (long long)z * Gp.Ry + y0w;
    xmf = Gm.Sf;
    xpf = Gp.Sf;
  }
  const uint32_t roff = (uint32_t)(r * (int)sizeof(T));
  // open x faces (OPEN variants only): the cell on the face keeps its
  // moments and the populations that enter the domain through the face in a
  // compact buffer, one 128-byte line per face cell written whole (9 values
  // and zeros; a line written in part would cost the memory a
  // read-modify-write), from which k_openfill writes the boundary nodes after
  // the sweep: plain stores of values at hand, the boundary arithmetic stays
  // out of the sweep.  With open faces a lane holds one cell and nx >= 2, so
  // at most one face cell.
  double* sp = nullptr;
  int sdir = 0;  // e_x of the populations that enter through the lane's face
  if (OPEN && pa->side != nullptr && !pad) {
    const long long cell = (long long)gz * pa->geo.n[1] + gy;
    if (pa->geo.open[0] && gx0 == 0) {
      sp = pa->side + 16 * cell;
      sdir = 1;
    } else if (pa->geo.open[1] && gx0 + VEC - 1 == pa->geo.n[0] - 1) {
      sp = pa->side + 16 * ((long long)pa->geo.n[1] * pa->geo.n[2] + cell);
      sdir = -1;
    }
  }
  auto side_pop = [&](int q, const T (&o)[VEC]) {
    if (OPEN && sdir != 0 && EXd(q) == sdir) {
      const int slot = EXd(q) > 0 ? (q == 1 ? 0 : (q - 5) / 2) : (q == 2 ? 0 : (q - 6) / 2);
      sp[slot] = (double)to_c<PREC, C>(sdir > 0 ? o[0] : o[VEC - 1]);
    }
  };
  if (OPEN && sdir != 0) {
    const int k = sdir > 0 ? 0 : VEC - 1;
    sp[5] = (double)drho[k];
    if constexpr (HYB) {
      sp[6] = dux[k];
      sp[7] = duy[k];
      sp[8] = duz[k];
    } else {
      sp[6] = (double)ux[k];
      sp[7] = (double)uy[k];
      sp[8] = (double)uz[k];
    }
#pragma unroll
    for (int j = 9; j < 16; ++j) sp[j] = 0.0;
  }
  const bool rowok = FX != 2 || (y != 0 && y != b - 1 && z != 0 && z != c - 1);
  const bool send_lo = xm_on && x0 == 0 && rowok;
  const bool send_hi = xp_on && x0 + VEC - 1 == a - 1 && rowok;
  // (solid cells send the zeros they store; buffer stores keep the address
  // in scalar registers plus the one lane offset)
  auto xface = [&](int q, const T (&o)[VEC]) {
    const T zero = from_c<PREC, double>(0.0);
    if (EXd(q) < 0 && send_lo) buf_store<T>(dst + (xm0 + (long long)q * xmf), roff, solid[0] ? zero : o[0]);
    if (EXd(q) > 0 && send_hi) buf_store<T>(dst + (xp0 + (long long)q * xpf), roff, solid[VEC - 1] ? zero : o[VEC - 1]);
  };

  {
    T o[VEC];
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      // rest: feq~_0 = w0 (drho + rho0 (-1.5 u.u)), F_0 = w0 rho0 (-3 u.g)
      const C feq = pp->w[0] * fma(pp->rho0, -uu15[k], drho[k]);
      C even;
      if constexpr (FORCE) {
        const C F = -pp->w[0] * ug3[k];
        even = fma(pp->omega, feq, pp->fcoef * F);
      } else {
        even = pp->omega * feq;
      }
      if constexpr (HYB)
        o[k] = from_c<PREC, double>(fma(pp->domc, (double)to_c<PREC, C>(W[0][k]), (double)even));
      else
        o[k] = from_c<PREC, C>(fma(pp->omc, to_c<PREC, C>(W[0][k]), even));
    }
    store_dir(0, o);
  }
#pragma unroll
  for (int i = 1; i < kQ; i += 2) {
    T o0[VEC], o1[VEC];
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      C eu = (C)0;
      double deu = 0.0;
      if constexpr (HYB) {
        if (EXd(i) > 0) deu += dux[k];
        if (EXd(i) < 0) deu -= dux[k];
        if (EYd(i) > 0) deu += duy[k];
        if (EYd(i) < 0) deu -= duy[k];
        if (EZd(i) > 0) deu += duz[k];
        if (EZd(i) < 0) deu -= duz[k];
        eu = (C)deu;
      } else {
        if (EXd(i) > 0) eu += ux[k];
        if (EXd(i) < 0) eu -= ux[k];
        if (EYd(i) > 0) eu += uy[k];
        if (EYd(i) < 0) eu -= uy[k];
        if (EZd(i) > 0) eu += uz[k];
        if (EZd(i) < 0) eu -= uz[k];
      }
      // even part (shared by i and its opposite) and odd part (flips sign)
      const C sym = pp->w[WCLS(i)] * fma(pp->rho0, fma((C)4.5 * eu, eu, -uu15[k]), drho[k]);
      C even;
      if constexpr (FORCE) {
        const C Fs = fma(pp->c9g[i], eu, -pp->w[WCLS(i)] * ug3[k]);
        even = fma(pp->omega, sym, pp->fcoef * Fs);
      } else {
        even = pp->omega * sym;
      }
      if constexpr (HYB) {
        const double odd = fma(pp->domega, pp->dc3w[WCLS(i)] * deu, pp->dcfa[i]);
        const double ev = (double)even;
        o0[k] = from_c<PREC, double>(fma(pp->domc, (double)to_c<PREC, C>(W[i][k]), ev + odd));
        o1[k] = from_c<PREC, double>(fma(pp->domc, (double)to_c<PREC, C>(W[i + 1][k]), ev - odd));
      } else {
        const C odd = FORCE ? fma(pp->omega, pp->c3w[WCLS(i)] * eu, pp->cfa[i]) : pp->omega * (pp->c3w[WCLS(i)] * eu);
        o0[k] = from_c<PREC, C>(fma(pp->omc, to_c<PREC, C>(W[i][k]), even + odd));
        o1[k] = from_c<PREC, C>(fma(pp->omc, to_c<PREC, C>(W[i + 1][k]), even - odd));
      }
    }
    store_dir(i, o0);
    store_dir(i + 1, o1);
    bounce(i, o0);
    bounce(i + 1, o1);
    if (xsend) {
      xface(i, o0);
      xface(i + 1, o1);
    }
    if (OPEN && EXd(i) != 0) {
      side_pop(i, o0);
      side_pop(i + 1, o1);
    }
  }
  if constexpr (FUSED) {
    // Waves with a row on a y or z face: the lane re-reads the values it has
    // just stored (same-address order within a lane), all loads first, then
    // sends them to the neighbours' ghost layers through the Block's target
    // table staged in LDS.
    if (edge) {
      T v[kQ][VEC];
#pragma unroll
      for (int q = 1; q < kQ; ++q)
#pragma unroll
        for (int k = 0; k < VEC; ++k)
          if (nbr_of(q, k) != 13)
            v[q][k] = ldo<T>(dst + (rb + (long long)q * B.Sf), lob + (uint32_t)(k * sizeof(T)));
#pragma unroll
      for (int q = 1; q < kQ; ++q)
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
          const int d = nbr_of(q, k);
          if (d != 13) {
            const GhostTgt& G = gts[d];
            const int x = x0 + k;
            if (G.kind == 1)
              dst[G.main0 + (long long)q * G.Sf + (long long)z * G.Sz + (long long)y * G.Sx + x] = v[q][k];
            else if (G.kind == 2)
              dst[G.xg0 + (long long)q * G.Sf + (long long)z * G.Ry + y] = v[q][k];
          }
        }
    }
  }
}

// The work items of one sweep from src to dst, workgroup by workgroup
// (item w, w + grid, ...); the waves of a workgroup take an item's
// (row group, 64-lane segment) tasks in turn.
template <int PREC, typename C, bool MASK, int FX, bool NT, int VEC, bool OPEN, bool FORCE = true>
__device__ __forceinline__ void sweep_items(const SweepArgs& A, const Phys<C>& ph, const void* src, void* dst,
                                            GhostTgt* gts) {
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = blockDim.x >> 6;
  for (int it = blockIdx.x; it < A.nitems; it += gridDim.x) {
    const ItemDev item = A.items[it];
    if constexpr (FX == 1) {
      __syncthreads();  // the previous item's readers are done
      if (threadIdx.x < 27) gts[threadIdx.x] = A.ghost[item.block * 27 + threadIdx.x];
      __syncthreads();
    }
    const BlockDev B = A.blocks[item.block];
    const int a = B.dim[0];
    const int yend = item.y0 + item.nrows;
    if (VEC == 1 && flat_rows(B, VEC, (int)sizeof(typename Stor<PREC>::T)) && ((B.wrap & 2) == 0 || (item.y0 > 0 && yend < B.dim[1]))) {
      // flat runs: task t covers cells 64 t .. 64 t + 63 of the item
      const int ntask = (item.nrows * a + 63) >> 6;
      for (int t = wv; t < ntask; t += nw) {
        const int f = t * 64, ry = f / a;
        sweep_row<PREC, C, MASK, FX, NT, VEC, OPEN, FORCE>(A, ph, src, dst, B, item.block, item.z, item.y0 + ry,
                                                    f - ry * a, yend, 0, gts);
      }
      continue;
    }
    const int lanes = (a + VEC - 1) / VEC;  // lanes per row
    int xw = 64;
    while (xw > 1 && xw / 2 >= lanes) xw >>= 1;
    const int rpw = 64 / xw;                      // rows per wave
    const int nseg = (lanes + 63) >> 6;           // 64-lane segments per row
    const int ngroups = (item.nrows + rpw - 1) / rpw;
    const int ntask = ngroups * nseg;
    for (int t = wv; t < ntask; t += nw) {
      const int grp = t / nseg, seg = t - grp * nseg;
      sweep_row<PREC, C, MASK, FX, NT, VEC, OPEN, FORCE>(A, ph, src, dst, B, item.block, item.z, item.y0 + grp * rpw,
                                                  seg * 64 * VEC, yend, xw, gts);
    }
  }
}

// At least 4 (one cell per lane) or 3 (two cells per lane) waves per SIMD.
// OPEN: contexts with open x faces (one cell per lane).
template <int PREC, typename C, bool MASK, int FX, bool NT, int VEC, bool OPEN, bool FORCE = true>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(VEC > 1 ? 3 : 4)))
k_sweep(const SweepArgs A, const Phys<C> ph) {
  // ghost targets of the current item's Block (fused exchange)
  __shared__ GhostTgt gts[FX == 1 ? 27 : 1];
  sweep_items<PREC, C, MASK, FX, NT, VEC, OPEN, FORCE>(A, ph, A.src, A.dst, gts);
}

// Several steps in one launch: a persistent block-list kernel.  Every
// workgroup walks the item list once per step, the ghost exchange is fused
// into the sweep (every boundary value goes straight into the neighbours'
// ghost layers), the two grids swap roles from step to step, and a
// grid-wide barrier (agent-scope release and acquire, so the ghost values
// written on one XCD are seen on the others) separates the steps.  The
// launch is cooperative: every workgroup is resident, so the barrier never
// waits on one that has not started, and every workgroup passes every
// barrier (its item loop may be empty).
template <int PREC, typename C, bool MASK>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_sweep_steps(const SweepArgs A, const Phys<C> ph, int nsteps) {
  __shared__ GhostTgt gts[27];
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  for (int s = 0; s < nsteps; ++s) {
    const void* src = (s & 1) ? (const void*)A.dst : A.src;
    void* dst = (s & 1) ? const_cast<void*>(A.src) : A.dst;
    sweep_items<PREC, C, MASK, 1, true, 1, false>(A, ph, src, dst, gts);
    grid.sync();
  }
}

// --------------------------------------------------------- ghost exchange
__device__ __forceinline__ long long xg_off(const BlockDev& B, int i, int y, int z) {
  return B.base + (long long)i * B.Sf + B.xgo + (long long)(z + 1) * B.Ry + (y + 1);
}

// Lattice directions as tables for run-time indices (same order as EXd...).
__constant__ int kEx[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__constant__ int kEy[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__constant__ int kEz[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

// Separate (unfused) exchange: after the sweep, copy the boundary values of
// each neighbour Block straight into this Block's ghost layer (Sec. 4.3:
// process-local communication copies from the sending to the receiving
// Block).  One task = one (Block, neighbour offset) pair with the directions
// that cross.  Solid sources are copied too (as zeros): a cell never pulls
// across an obstacle link (its own value replaces it), and whole lines are
// cheaper.

//
// MODE 1 and 2 split the copy at an exchange buffer, for pairs of Blocks of
// which one lives on the host CPU (Sec. 4.5: both sides share the buffer's
// layout, value j of task cell l at bo + 5 (l - l0) + j): 1 packs the
// sending Block's values into buf, 2 writes buf into the ghost slots.
template <typename T, int MODE = 0>
__global__ void __launch_bounds__(256) k_exchange(T* __restrict__ grid, const BlockDev* __restrict__ blocks,
                                                  const NbrDev* __restrict__ nbr,
                                                  const XchgTask* __restrict__ tasks, int ntasks,
                                                  T* __restrict__ buf = nullptr) {
  // one workgroup per task; a thread copies every crossing direction of up
  // to kXU of the task's ghost cells (cells l, l + 256, ...), all loads
  // before the stores, so that up to 5 kXU loads per lane are in flight (a
  // task holds at most 1024 cells)
  constexpr int kXU = 4;
  for (int task = blockIdx.x; task < ntasks; task += gridDim.x) {
    const XchgTask t = tasks[task];
    const BlockDev M = blocks[t.dst];
    const NbrDev nb = nbr[t.dst * 27 + t.d];
    const BlockDev N = blocks[nb.id];
    const bool xplane = t.lo[0] < 0 || t.lo[0] >= M.dim[0];
    for (int L0 = t.l0 + threadIdx.x; L0 < t.l1; L0 += kXU * blockDim.x) {
      T v[kXU][5];
      bool ok[kXU][5];
      int g[kXU][3];
#pragma unroll
      for (int u = 0; u < kXU; ++u) {
        const int L = L0 + u * (int)blockDim.x;
        const bool live = L < t.l1;
        const int q0 = L % t.ext[0];
        const int r = L / t.ext[0];
        const int q1 = r % t.ext[1];
        const int q2 = r / t.ext[1];
        const int gx = t.lo[0] + q0, gy = t.lo[1] + q1, gz = t.lo[2] + q2;
        g[u][0] = gx;
        g[u][1] = gy;
        g[u][2] = gz;
        const int sx = gx + nb.tx, sy = gy + nb.ty, sz = gz + nb.tz;
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          const int i = (t.dirs >> (5 * j)) & 31;
          // only slots whose puller (g + e_i, folded on the axes the Block
          // wraps on) lies inside the receiving Block
          int px = gx + kEx[i], py = gy + kEy[i], pz = gz + kEz[i];
          if (M.wrap & 1) px = px < 0 ? px + M.dim[0] : (px >= M.dim[0] ? px - M.dim[0] : px);
          if (M.wrap & 2) py = py < 0 ? py + M.dim[1] : (py >= M.dim[1] ? py - M.dim[1] : py);
          if (M.wrap & 4) pz = pz < 0 ? pz + M.dim[2] : (pz >= M.dim[2] ? pz - M.dim[2] : pz);
          ok[u][j] = live && j < t.ndir && px >= 0 && px < M.dim[0] && py >= 0 && py < M.dim[1] && pz >= 0 &&
                     pz < M.dim[2];
          const long long bi = (long long)t.bo + 5ll * (L - t.l0) + j;
          if (ok[u][j]) v[u][j] = MODE == 2 ? buf[bi] : grid[main_off(N, i, sx, sy, sz)];
        }
      }
#pragma unroll
      for (int u = 0; u < kXU; ++u) {
        const int L = L0 + u * (int)blockDim.x;
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          const int i = (t.dirs >> (5 * j)) & 31;
          if (!ok[u][j]) continue;
          if (MODE == 1)
            buf[(long long)t.bo + 5ll * (L - t.l0) + j] = v[u][j];
          else
            grid[xplane ? xg_off(M, i, g[u][1], g[u][2]) : main_off(M, i, g[u][0], g[u][1], g[u][2])] = v[u][j];
        }
      }
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
      // link bits for fluid and solid cells alike (a solid cell's tell the
      // sweep which of its slots no fluid neighbour writes)
      uint32_t m = solid[gidx(A.geo, p[0], p[1], p[2])] ? kSolidBit : 0u;
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
      mask[B.mask + ((long long)z * B.dim[1] + y) * a + x] = m;
    }
  }
}

// Bounce-back slots of a state loaded from outside the sweep (rest state,
// warm start, checkpoint): for every wall link of a fluid cell x, slot
// (x - e_i, i) = f_ibar(x) + 6 w_i rho0 e_i.u_w, rounded as the sweep rounds
// it (arithmetic type C).  Obstacle links need nothing: the sweep reads the
// cell's own f_ibar for them.
template <int PREC, typename C>
__global__ void __launch_bounds__(256) k_bbfill(void* grid_, CellArgs A, const Phys<C> ph) {
  using T = typename Stor<PREC>::T;
  T* grid = (T*)grid_;
  SweepArgs sa{};
  sa.geo = A.geo;
  const bool moving = A.geo.moving[0] | A.geo.moving[1] | A.geo.moving[2] | A.geo.moving[3] | A.geo.moving[4] |
                      A.geo.moving[5];
  for_cells(A, [&](const BlockDev& B, int x, int y, int z, bool solid) {
    if (solid) return;
    const int gx = B.org[0] + x, gy = B.org[1] + y, gz = B.org[2] + z;
    WallFlags wf;
    wf.lox = A.geo.fwall[0] && gx == 0;
    wf.hix = A.geo.fwall[1] && gx == A.geo.n[0] - 1;
    wf.loy = A.geo.fwall[2] && gy == 0;
    wf.hiy = A.geo.fwall[3] && gy == A.geo.n[1] - 1;
    wf.loz = A.geo.fwall[4] && gz == 0;
    wf.hiz = A.geo.fwall[5] && gz == A.geo.n[2] - 1;
    for (int i = 1; i < kQ; ++i) {
      // walls only: obstacle links are bounced on the pull side of the sweep
      const bool bw = wall_link<1>(wf, i, 0);
      if (!bw) continue;
      // the slot the sweep pulls from (wrapped on the Block's wrap axes)
      int sx = x - EXd(i), sy = y - EYd(i), sz = z - EZd(i);
      if (B.wrap & 1) sx = sx < 0 ? sx + B.dim[0] : (sx >= B.dim[0] ? sx - B.dim[0] : sx);
      if (B.wrap & 2) sy = sy < 0 ? sy + B.dim[1] : (sy >= B.dim[1] ? sy - B.dim[1] : sy);
      if (B.wrap & 4) sz = sz < 0 ? sz + B.dim[2] : (sz >= B.dim[2] ? sz - B.dim[2] : sz);
      const long long o = (sx < 0 || sx >= B.dim[0]) ? xg_off(B, i, sy, sz) : main_off(B, i, sx, sy, sz);
      T v = grid[main_off(B, OPPd(i), x, y, z)];
      if (moving && bw) v = from_c<PREC, C>(to_c<PREC, C>(v) + wall_corr<C, 1>(sa, ph, wf, i, 0));
      grid[o] = v;
    }
  });
}

// Open faces (on one axis a; t1 < t2 the two other axes).  The side buffer
// holds, per face (low, high) and face cell (s1, s2) at [face][s2][s1], 16
// doubles: the post-collision populations of the five directions that enter
// the domain through the face (slot k: the k-th direction i in increasing
// order with e_a(i) = +1 on the low face, -1 on the high face), then
// drho, u_x, u_y, u_z of the cell's collision, then zeros (one 128-byte line
// per cell).
__device__ __forceinline__ int ecomp(int axis, int i) { return axis == 0 ? kEx[i] : (axis == 1 ? kEy[i] : kEz[i]); }
__device__ __forceinline__ int enter_dir(int axis, int sign, int slot) {
  int k = 0;
  for (int i = 1; i < kQ; ++i)
    if (ecomp(axis, i) == sign) {
      if (k == slot) return i;
      ++k;
    }
  return 0;
}
__device__ __forceinline__ void tangential(int a, int& t1, int& t2) {
  t1 = a == 0 ? 1 : 0;
  t2 = a == 2 ? 1 : 2;
}

// Once per step after the sweep (and after a state is loaded): the boundary
// nodes beyond the open faces from the face cells' entries in `side` (the
// moments of their collision, as the boundary rule asks).  A boundary node
// one cell beyond face f at tangential position (g1, g2) feeds the face
// cells around it, so its value goes into the ghost layer of every Block on
// that face whose ghost layer, tangential ghost cells included, covers it:
// the Block that owns the face cell, the face Blocks next to it, and on a
// periodic tangential axis the Blocks that hold its periodic image.  In a
// Block the node lies in the main arrays' ghost rows (y faces) or planes
// (z faces) or, for x faces and past a Block's x ends, in the x-ghost plane
// of the directions that pull from there.  One thread per node position
// (g1, g2) in [-1, n1] x [-1, n2] of each face; nodes beyond a wall are left
// to the sweep's bounce-back.  faceblk: per face the count of Blocks
// touching it, then their ids (stride 1 + nblocks).
template <int PREC>
__global__ void __launch_bounds__(256) k_openfill(void* grid_, const BlockDev* __restrict__ blocks, int nblocks,
                                                  const int* __restrict__ faceblk, GridGeom geo,
                                                  const double* __restrict__ side) {
  using T = typename Stor<PREC>::T;
  T* grid = (T*)grid_;
  const int a = geo.open_axis;
  int t1, t2;
  tangential(a, t1, t2);
  const int n1 = geo.n[t1], n2 = geo.n[t2];
  const int per_face = (n1 + 2) * (n2 + 2);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (a < 0 || t >= 2 * per_face) return;
  const int fs = t / per_face, r = t % per_face;
  const int f = 2 * a + fs;
  if (!geo.open[f]) return;
  const int g1 = r % (n1 + 2) - 1, g2 = r / (n1 + 2) - 1;
  if ((g1 < 0 || g1 >= n1) && geo.wall[t1]) return;
  if ((g2 < 0 || g2 >= n2) && geo.wall[t2]) return;
  const int s1 = g1 < 0 ? g1 + n1 : (g1 >= n1 ? g1 - n1 : g1);
  const int s2 = g2 < 0 ? g2 + n2 : (g2 >= n2 ? g2 - n2 : g2);
  const double* cs = side + 16 * ((long long)fs * n1 * n2 + (long long)s2 * n1 + s1);
  const double d = cs[5], ux = cs[6], uy = cs[7], uz = cs[8];
  const int sign = fs == 0 ? 1 : -1;
  T v[5];
  for (int slot = 0; slot < 5; ++slot) {
    const int q = enter_dir(a, sign, slot);
    v[slot] = from_c<PREC, double>(cs[slot] + open_corr(geo, f, q, geo.rho0, d, ux, uy, uz));
  }
  const int* list = faceblk + fs * (1 + nblocks);
  for (int k = 0; k < list[0]; ++k) {
    const BlockDev& M = blocks[list[1 + k]];
    int l[3];
    l[a] = fs == 0 ? -1 : M.dim[a];
    l[t1] = g1 - M.org[t1];
    l[t2] = g2 - M.org[t2];
    if (l[t1] < -1 || l[t1] > M.dim[t1] || l[t2] < -1 || l[t2] > M.dim[t2]) continue;
    for (int slot = 0; slot < 5; ++slot) {
      const int q = enter_dir(a, sign, slot);
      if (l[0] >= 0 && l[0] < M.dim[0])
        grid[main_off(M, q, l[0], l[1], l[2])] = v[slot];
      else if ((l[0] < 0 && kEx[q] == 1) || (l[0] >= M.dim[0] && kEx[q] == -1))
        grid[xg_off(M, q, l[1], l[2])] = v[slot];
    }
  }
}

// The face cells' entries of `side` rebuilt from their stored post-collision
// populations (drho = sum f~, u = sum e f~ / rho0 - g/2: the collision
// invariants, so the moments of their last collision up to rounding): after
// every sweep for y and z faces, after a state is loaded for x faces (whose
// entries the sweep writes itself).  One thread per face cell (FP64).
template <int PREC>
__global__ void __launch_bounds__(256) k_openside(const void* grid_, const BlockDev* __restrict__ blocks,
                                                  int nblocks, const int* __restrict__ faceblk, GridGeom geo,
                                                  double* __restrict__ side) {
  using T = typename Stor<PREC>::T;
  const T* grid = (const T*)grid_;
  const int a = geo.open_axis;
  int t1, t2;
  tangential(a, t1, t2);
  const int n1 = geo.n[t1], n2 = geo.n[t2];
  const int per_face = n1 * n2;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (a < 0 || t >= 2 * per_face) return;
  const int fs = t / per_face, r = t % per_face;
  if (!geo.open[2 * a + fs]) return;
  const int g1 = r % n1, g2 = r / n1;
  const int sign = fs == 0 ? 1 : -1;
  const int* list = faceblk + fs * (1 + nblocks);
  for (int k = 0; k < list[0]; ++k) {
    const BlockDev& B = blocks[list[1 + k]];
    int l[3];
    l[a] = fs == 0 ? 0 : B.dim[a] - 1;
    l[t1] = g1 - B.org[t1];
    l[t2] = g2 - B.org[t2];
    if (l[t1] < 0 || l[t1] >= B.dim[t1] || l[t2] < 0 || l[t2] >= B.dim[t2]) continue;
    double fi[kQ], dr = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int i = 0; i < kQ; ++i) {
      fi[i] = (double)to_c<PREC, double>(grid[main_off(B, i, l[0], l[1], l[2])]);
      dr += fi[i];
      jx += EXd(i) * fi[i];
      jy += EYd(i) * fi[i];
      jz += EZd(i) * fi[i];
    }
    double* cs = side + 16 * ((long long)fs * per_face + r);
    for (int slot = 0; slot < 5; ++slot) cs[slot] = fi[enter_dir(a, sign, slot)];
    cs[5] = dr;
    cs[6] = jx / geo.rho0 - geo.hg[0];
    cs[7] = jy / geo.rho0 - geo.hg[1];
    cs[8] = jz / geo.rho0 - geo.hg[2];
    for (int j = 9; j < 16; ++j) cs[j] = 0.0;
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
// [5] sum |u|^2, with u_prev from the other grid (want_prev 1) or from a
// stored FP64 velocity field um[3][N] (want_prev 2).  Per-workgroup
// partials; workgroup w always takes items w, w + G, ... so the result is
// deterministic.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int PREC>
__global__ void __launch_bounds__(256) k_reduce(const void* cur_, const void* prev_, CellArgs A, double rho0,
                                                double hcx, double hcy, double hcz, double hpx, double hpy,
                                                double hpz, int want_prev, const double* __restrict__ um,
                                                long long N, double* __restrict__ partial) {
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
      if (want_prev == 1) {
        const double w = to_c<PREC, double>(prev[o]);
        px += EXd(i) * w; py += EYd(i) * w; pz += EZd(i) * w;
      }
    }
    const double ux = jx / rho0 - hcx, uy = jy / rho0 - hcy, uz = jz / rho0 - hcz;
    s[0] += d;
    s[1] += rho0 * ux; s[2] += rho0 * uy; s[3] += rho0 * uz;
    if (want_prev == 1) {
      const double dx = ux - (px / rho0 - hpx), dy = uy - (py / rho0 - hpy), dz = uz - (pz / rho0 - hpz);
      s[4] += dx * dx + dy * dy + dz * dz;
    } else if (want_prev == 2) {
      const long long g = gidx(A.geo, B.org[0] + x, B.org[1] + y, B.org[2] + z);
      const double dx = ux - um[g], dy = uy - um[N + g], dz = uz - um[2 * N + g];
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

// Mean of the two grids' stored values, written into `cur` (every element:
// main arrays, ghost layers and slots; the caller rebuilds ghosts and slots
// from the mean).  Storage stays shifted (the mean of shifted values is the
// shifted mean); 16-bit values are averaged in FP32 and rounded once.
template <int PREC>
__global__ void __launch_bounds__(256) k_average(void* cur_, const void* prev_, long long n) {
  using T = typename Stor<PREC>::T;
  using A = typename std::conditional<PREC == 0, double, float>::type;
  T* cur = (T*)cur_;
  const T* prev = (const T*)prev_;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
    cur[k] = from_c<PREC, A>((to_c<PREC, A>(cur[k]) + to_c<PREC, A>(prev[k])) * (A)0.5);
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

template <int PREC, typename C, bool MASK, int FX, bool NT, int VEC, bool OPEN = false, bool FORCE = true>
static void launch_sweep_t(SweepArgs a, Phys<double> pd, Phys<float> pf, dim3 g, dim3 b, hipStream_t s) {
  if constexpr (sizeof(C) == 8)
    hipLaunchKernelGGL((k_sweep<PREC, C, MASK, FX, NT, VEC, OPEN, FORCE>), g, b, 0, s, a, pd);
  else
    hipLaunchKernelGGL((k_sweep<PREC, C, MASK, FX, NT, VEC, OPEN, FORCE>), g, b, 0, s, a, pf);
}

// Contexts with open faces: one cell per lane, non-temporal (the cache hint
// changes no result).
template <int PREC, typename C>
static SweepFn pick_open(bool mask, int fx) {
#define LBM_PICK(M, F) return launch_sweep_t<PREC, C, M, F, true, 1, true>
  if (mask) {
    if (fx == 1) LBM_PICK(true, 1);
    if (fx == 2) LBM_PICK(true, 2);
    LBM_PICK(true, 0);
  }
  if (fx == 1) LBM_PICK(false, 1);
  if (fx == 2) LBM_PICK(false, 2);
  LBM_PICK(false, 0);
#undef LBM_PICK
}

// force = false picks the force-free collision for 16-bit storage with
// streaming stores (measured on gfx950, 384^3 cavity: FP16S sweep 0.905 ->
// 0.851 ms; FP32 and FP64, bound by bytes, gain nothing)
template <int PREC, typename C, int VEC>
static SweepFn pick3(bool mask, int fx, bool nt, bool force) {
#define LBM_PICK(M, F)                                                                                    \
  return nt ? (PREC >= 2 && !force ? launch_sweep_t<PREC, C, M, F, true, VEC, false, PREC <= 1>          \
                                   : launch_sweep_t<PREC, C, M, F, true, VEC>)                            \
            : launch_sweep_t<PREC, C, M, F, false, VEC>
  if (mask) {
    if (fx == 1) LBM_PICK(true, 1);
    if (fx == 2) LBM_PICK(true, 2);
    LBM_PICK(true, 0);
  }
  if (fx == 1) LBM_PICK(false, 1);
  if (fx == 2) LBM_PICK(false, 2);
  LBM_PICK(false, 0);
#undef LBM_PICK
}

// Storage modes with a two-cells-per-lane sweep: 16-bit storage (four bytes
// per lane and stream, like FP32) and FP32 storage with FP64 arithmetic.
bool sweep_vec2_ok(int prec, bool f64math) { return prec >= 2 || (prec == 1 && f64math); }

void launch_sweep(int prec, bool f64math, bool mask, int fx, bool nt, bool force, int vec, const SweepArgs& a,
                  const Phys<double>& pd, const Phys<float>& pf, dim3 grid, dim3 block, hipStream_t s) {
  SweepFn fn = nullptr;
  const bool v = vec == 2 && sweep_vec2_ok(prec, f64math);
  if (a.side != nullptr) {
    switch (prec) {
      case 0: fn = pick_open<0, double>(mask, fx); break;
      case 1: fn = f64math ? pick_open<1, double>(mask, fx) : pick_open<1, float>(mask, fx); break;
      case 2: fn = pick_open<2, float>(mask, fx); break;
      default: fn = pick_open<3, float>(mask, fx); break;
    }
    fn(a, pd, pf, grid, block, s);
    return;
  }
  switch (prec) {
    case 0: fn = pick3<0, double, 1>(mask, fx, nt, force); break;
    case 1:
      if (f64math) fn = v ? pick3<1, double, 2>(mask, fx, nt, force) : pick3<1, double, 1>(mask, fx, nt, force);
      else fn = pick3<1, float, 1>(mask, fx, nt, force);
      break;
    case 2: fn = v ? pick3<2, float, 2>(mask, fx, nt, force) : pick3<2, float, 1>(mask, fx, nt, force); break;
    default: fn = v ? pick3<3, float, 2>(mask, fx, nt, force) : pick3<3, float, 1>(mask, fx, nt, force); break;
  }
  fn(a, pd, pf, grid, block, s);
}

// The persistent multi-step sweep: grid = the largest number of its
// workgroups the GPU holds at once (at most one per item), launched
// cooperatively.  Returns the HIP error of the launch.
template <int PREC, typename C, bool MASK>
static hipError_t launch_steps_t(const SweepArgs& a, const Phys<C>& ph, int nsteps, int cus, hipStream_t s) {
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_sweep_steps<PREC, C, MASK>, 256, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorCooperativeLaunchTooLarge;
  const int grid = std::max(1, std::min(a.nitems, per_cu * cus));
  SweepArgs aa = a;
  Phys<C> pp = ph;
  int n = nsteps;
  void* args[] = {&aa, &pp, &n};
  return hipLaunchCooperativeKernel((const void*)k_sweep_steps<PREC, C, MASK>, dim3(grid), dim3(256), args, 0, s);
}

hipError_t launch_sweep_steps(int prec, bool f64math, bool mask, const SweepArgs& a, const Phys<double>& pd,
                              const Phys<float>& pf, int nsteps, int cus, hipStream_t s) {
#define LBM_STEPS(P, CT, PH)                                                               \
  return mask ? launch_steps_t<P, CT, true>(a, PH, nsteps, cus, s) : launch_steps_t<P, CT, false>(a, PH, nsteps, cus, s)
  switch (prec) {
    case 0: LBM_STEPS(0, double, pd);
    case 1:
      if (f64math) LBM_STEPS(1, double, pd);
      LBM_STEPS(1, float, pf);
    case 2: LBM_STEPS(2, float, pf);
    default: LBM_STEPS(3, float, pf);
  }
#undef LBM_STEPS
}

void launch_exchange(int prec, void* grid, const BlockDev* blocks, const NbrDev* nbr, const XchgTask* tasks,
                     int ntasks, hipStream_t s) {
  if (ntasks <= 0) return;
  dim3 g(ntasks < (1 << 20) ? ntasks : (1 << 20)), b(256);
  switch (prec) {
    case 0: hipLaunchKernelGGL(k_exchange<double>, g, b, 0, s, (double*)grid, blocks, nbr, tasks, ntasks, nullptr); break;
    case 1: hipLaunchKernelGGL(k_exchange<float>, g, b, 0, s, (float*)grid, blocks, nbr, tasks, ntasks, nullptr); break;
    default:
      hipLaunchKernelGGL(k_exchange<uint16_t>, g, b, 0, s, (uint16_t*)grid, blocks, nbr, tasks, ntasks, nullptr);
      break;
  }
}

// mode 1: pack the senders' values into buf; 2: unpack buf into the ghosts
// (FP64 and FP32 storage)
void launch_exchange_buf(int prec, int mode, void* grid, const BlockDev* blocks, const NbrDev* nbr,
                         const XchgTask* tasks, int ntasks, void* buf, hipStream_t s) {
  if (ntasks <= 0) return;
  dim3 g(ntasks < (1 << 20) ? ntasks : (1 << 20)), b(256);
  if (prec == 0) {
    if (mode == 1)
      hipLaunchKernelGGL((k_exchange<double, 1>), g, b, 0, s, (double*)grid, blocks, nbr, tasks, ntasks, (double*)buf);
    else
      hipLaunchKernelGGL((k_exchange<double, 2>), g, b, 0, s, (double*)grid, blocks, nbr, tasks, ntasks, (double*)buf);
  } else {
    if (mode == 1)
      hipLaunchKernelGGL((k_exchange<float, 1>), g, b, 0, s, (float*)grid, blocks, nbr, tasks, ntasks, (float*)buf);
    else
      hipLaunchKernelGGL((k_exchange<float, 2>), g, b, 0, s, (float*)grid, blocks, nbr, tasks, ntasks, (float*)buf);
  }
}

void launch_bbfill(int prec, bool f64math, void* grid, const CellArgs& a, const Phys<double>& pd,
                   const Phys<float>& pf, hipStream_t s) {
  dim3 g(a.nitems), b(256);
  switch (prec) {
    case 0: hipLaunchKernelGGL((k_bbfill<0, double>), g, b, 0, s, grid, a, pd); break;
    case 1:
      if (f64math) hipLaunchKernelGGL((k_bbfill<1, double>), g, b, 0, s, grid, a, pd);
      else hipLaunchKernelGGL((k_bbfill<1, float>), g, b, 0, s, grid, a, pf);
      break;
    case 2: hipLaunchKernelGGL((k_bbfill<2, float>), g, b, 0, s, grid, a, pf); break;
    default: hipLaunchKernelGGL((k_bbfill<3, float>), g, b, 0, s, grid, a, pf); break;
  }
}

// node positions (openfill) or face cells (openside) of both open faces
static int open_threads(const GridGeom& geo, int ghost) {
  const int a = geo.open_axis;
  if (a < 0) return 0;
  const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
  return 2 * (geo.n[t1] + 2 * ghost) * (geo.n[t2] + 2 * ghost);
}

void launch_openfill(int prec, void* grid, const BlockDev* blocks, int nblocks, const int* faceblk,
                     const GridGeom& geo, const double* side, hipStream_t s) {
  const int n = open_threads(geo, 1);
  if (n == 0) return;
  const dim3 g((n + 255) / 256), b(256);
  switch (prec) {
    case 0: hipLaunchKernelGGL(k_openfill<0>, g, b, 0, s, grid, blocks, nblocks, faceblk, geo, side); break;
    case 1: hipLaunchKernelGGL(k_openfill<1>, g, b, 0, s, grid, blocks, nblocks, faceblk, geo, side); break;
    case 2: hipLaunchKernelGGL(k_openfill<2>, g, b, 0, s, grid, blocks, nblocks, faceblk, geo, side); break;
    default: hipLaunchKernelGGL(k_openfill<3>, g, b, 0, s, grid, blocks, nblocks, faceblk, geo, side); break;
  }
}

void launch_openside(int prec, const void* grid, const BlockDev* blocks, int nblocks, const int* faceblk,
                     const GridGeom& geo, double* side, hipStream_t s) {
  const int n = open_threads(geo, 0);
  if (n == 0) return;
  const dim3 g((n + 255) / 256), b(256);
  switch (prec) {
    case 0: hipLaunchKernelGGL(k_openside<0>, g, b, 0, s, grid, blocks, nblocks, faceblk, geo, side); break;
    case 1: hipLaunchKernelGGL(k_openside<1>, g, b, 0, s, grid, blocks, nblocks, faceblk, geo, side); break;
    case 2: hipLaunchKernelGGL(k_openside<2>, g, b, 0, s, grid, blocks, nblocks, faceblk, geo, side); break;
    default: hipLaunchKernelGGL(k_openside<3>, g, b, 0, s, grid, blocks, nblocks, faceblk, geo, side); break;
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
                   const double hp[3], int want_prev, const double* um, long long N, double* partial, int nparts,
                   double* out, hipStream_t s) {
  dim3 g(nparts), b(256);
  switch (prec) {
    case 0: hipLaunchKernelGGL(k_reduce<0>, g, b, 0, s, cur, prev, a, rho0, hc[0], hc[1], hc[2], hp[0], hp[1], hp[2], want_prev, um, N, partial); break;
    case 1: hipLaunchKernelGGL(k_reduce<1>, g, b, 0, s, cur, prev, a, rho0, hc[0], hc[1], hc[2], hp[0], hp[1], hp[2], want_prev, um, N, partial); break;
    case 2: hipLaunchKernelGGL(k_reduce<2>, g, b, 0, s, cur, prev, a, rho0, hc[0], hc[1], hc[2], hp[0], hp[1], hp[2], want_prev, um, N, partial); break;
    default: hipLaunchKernelGGL(k_reduce<3>, g, b, 0, s, cur, prev, a, rho0, hc[0], hc[1], hc[2], hp[0], hp[1], hp[2], want_prev, um, N, partial); break;
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

void launch_average(int prec, void* cur, const void* prev, long long n, hipStream_t s) {
  const long long blocks = std::min<long long>((n + 255) / 256, 8192);
  dim3 g((unsigned)std::max<long long>(1, blocks)), b(256);
  switch (prec) {
    case 0: hipLaunchKernelGGL(k_average<0>, g, b, 0, s, cur, prev, n); break;
    case 1: hipLaunchKernelGGL(k_average<1>, g, b, 0, s, cur, prev, n); break;
    case 2: hipLaunchKernelGGL(k_average<2>, g, b, 0, s, cur, prev, n); break;
    default: hipLaunchKernelGGL(k_average<3>, g, b, 0, s, cur, prev, n); break;
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
