// lbm_internal.h -- data layout shared by the gfx950 kernels and the host runtime.
//
// Per Block (interior a x b x c cells, Sec. 4.2) and per grid (two grids, pull
// scheme, Sec. 2.1) the populations are stored Structure-of-Arrays
// (Sec. 3.2): 19 arrays f_i[z][y][x] that include a one-cell ghost layer in y
// and z (rows y = -1, b and planes z = -1, c), with x-rows padded to a
// multiple of 128 bytes so every row starts on a cache line, or, for rows of
// an odd number of half lines, packed two rows to three lines (pack).  The ghost layer
// in x lives in one extra plane per array, placed right after it: for the five
// directions with e_x = +1 it holds x = -1, for the five with e_x = -1 it holds
// x = a (Sec. 4.4 counts 5 PDFs per face cell).  Keeping the x ghosts out of
// the rows keeps the interior aligned; keeping each plane next to its array
// lets one scalar base plus a 32-bit lane offset reach both.
//
//   main:    base + i*Sf + (z+1)*Sz + (y+1)*Sx + x          0 <= x < a
//   x ghost: base + i*Sf + xgo + (z+1)*Ry + (y+1)            x = -1 or a
//
// Bounce-back slots: a population that would be pulled from beyond a wall or
// from a solid cell is written there by the cell it bounces back to, so the
// ghost/halo/solid slot of (x - e_i, i) holds f*_ibar(x) + 6 w_i rho0 e_i.u_w.
//
// Offsets are in elements of the storage type, relative to the grid pool.
#pragma once
#include <stdint.h>

namespace lbm {

constexpr int kQ = 19;

struct BlockDev {
  int dim[3];       // a, b, c
  int org[3];       // global cell of the Block's (0,0,0)
  int Sx;           // x-row stride (elements)
  int Ry;           // b + 2: rows per plane of an x-ghost plane
  long long Sz;     // Sx * (b + 2)
  long long Sf;     // stride between the 19 population arrays (array + ghost plane)
  long long xgo;    // offset of a population's x-ghost plane from the array start
  long long base;   // element offset of main[0][z=-1][y=-1][x=0]
  long long mask;   // offset of the Block's link masks (a*b*c words), -1: none
  int wrap;         // bit k (x = 1, y = 2, z = 4): the Block is its own neighbour
                    // across both faces of axis k (periodic, one Block along k);
                    // the sweep then reads across that axis from the Block itself
                    // and no ghost value on that axis is used
  int pack;         // 1: rows packed (Sx = a; rows 2k, 2k + 1 share a line)
};

// Whether the one-cell-per-lane sweep runs the Block's planes as flat runs
// of cells: a wave takes 64 consecutive cells of a plane (rows in order,
// across row ends) instead of one row segment.  Only where that keeps every
// access on whole lines: rows stored back to back (Sx = a) in a whole
// number of half lines, neither a multiple of 64 cells nor a power of two
// (FP32 rows of 48, 80 or 96 cells; with packed rows, items of even row
// counts start on a line).  A 48-cell row segment leaves a quarter of the
// wave idle; measured on gfx950, 480 x 240 x 240 in 48^3 Blocks: sweep
// 0.919 -> 0.819 ms.  Where rows are padded (127, 129 or 200 cells), runs
// across row ends split accesses over more lines and lost 15-25 %: the sweep
// is bound by the lines its waves request as much as by bytes.  In a Block
// that wraps onto itself along y, rows 0 and b - 1 (whose source rows wrap)
// keep one row per wave: their items hold one row each.
__host__ __device__ inline bool flat_rows(const BlockDev& B, int vec, int sbytes) {
  const int a = B.dim[0];
  return vec == 1 && B.Sx == a && (a * sbytes) % 64 == 0 && (a & 63) != 0 && (a & (a - 1)) != 0;
}

// Neighbour entry of a Block for offset class d = 13 + dx + 3 dy + 9 dz:
// id of the Block that owns the cells across that face/edge/corner (-1 beyond
// a wall), and the translation from this Block's local coordinates to the
// neighbour's (periodic images included).
struct NbrDev {
  int id, tx, ty, tz;
};

// Work item: x-rows [y0, y0 + nrows) of plane z of one Block.
struct ItemDev {
  int block, z, y0, nrows;
};

// Plain ghost-exchange task: cells l0 .. l1-1 (x fastest) of a ghost region
// of Block `dst` in offset class d (extent ext[3] starting at lo[3], local
// coordinates of dst, -1 or dim on the offset axes) and the ndir population
// directions that cross into it (5 through a face, 1 through an edge), 5 bits
// each in dirs.  bo: where the task's values start in an exchange buffer
// (elements; value j of cell l at bo + 5 (l - l0) + j), for tasks whose two
// Blocks live in different memories (host-CPU Blocks).
struct XchgTask {
  int dst, d, ndir, dirs, l0, l1;
  int lo[3], ext[3];
  int bo, pad;
};

// Link-mask word of a cell: bit i (1..18) set when x - e_i is a solid cell
// (obstacle bounce-back link; set for solid cells too); bit 31 set when the
// cell itself is solid.
constexpr uint32_t kSolidBit = 0x80000000u;

struct GridGeom {
  int n[3];         // global nx, ny, nz
  int wall[3];      // 1: the axis is bounded (walls or open faces), 0: periodic
  int fwall[6];     // face is a bounce-back wall
  int moving[6];    // wall face with a nonzero wall velocity
  int open[6];      // face -x, +x, -y, +y, -z, +z: 0 not open, 1 VELOCITY, 2 PRESSURE
  int open_axis;    // axis of the open faces (they lie on one axis), -1: none
  double ob_u[6][3];  // prescribed velocity of an open face
  double ob_drho[6];  // prescribed rho - rho0 of an open face
  double rho0;        // reference density and g/2 (open faces rebuild the
  double hg[3];       // velocity of a post-collision state)
};

// Where a Block's boundary value of direction i goes when the fused
// exchange writes it into the ghost layer of neighbour M (one entry per
// Block and offset class d):
//   kind 1 (M's main arrays):    main0 + i*Sf + z*Sz + y*Sx + x
//   kind 2 (M's x-ghost planes): xg0 + i*Sf + z*Ry + y
// with (x, y, z) the sender's local cell; the translation into M's frame is
// folded into main0 / xg0.  kind 0: no neighbour (wall).
struct GhostTgt {
  long long main0;
  long long xg0;
  long long Sz;
  long long Sf;
  int Sx, Ry, kind, pad;
};

template <typename C>
struct Phys {
  C omega;          // 1/tau
  C omc;            // 1 - 1/tau
  C rho0;
  C inv_rho0;
  C fcoef;          // 1 - omega/2
  C rho0x3;         // 3 rho0
  C g[3];
  C hg[3];          // g/2
  C w[kQ];          // lattice weights
  C c3w[kQ];        // 3 w_i rho0
  C c9g[kQ];        // 9 w_i rho0 (e_i . g)
  C cfa[kQ];        // (1 - omega/2) 3 w_i rho0 (e_i . g)
  C corr[kQ][6];    // 6 w_i rho0 (e_i . u_w[face])
  // FP64 copies for the mixed arithmetic of FP32 storage (velocity, odd part
  // of the equilibrium and force, final update in FP64; even part in FP32)
  double dinv_rho0, dhg[3], domega, domc;
  double dc3w[kQ];
  double dcfa[kQ];
};

struct SweepArgs {
  const void* src;
  void* dst;
  const BlockDev* blocks;
  const NbrDev* nbr;
  const ItemDev* items;
  const uint32_t* mask;
  const GhostTgt* ghost;  // [block][27]
  double* side;           // open x faces: per face cell its 5 entering post-collision
                          // populations and drho, u, padded to 16 ([face][nz][ny][16]);
                          // NULL without
  int nitems;
  int pad;
  GridGeom geo;
};

// Arguments of the per-cell utility kernels (init, macroscopic, reductions,
// checkpoint, link masks): they walk the same item list as the sweep.
struct CellArgs {
  const BlockDev* blocks;
  const ItemDev* items;
  const uint32_t* mask;
  int nitems;
  int has_mask;
  GridGeom geo;
};

// ---- host-CPU Blocks (heterogeneous runs, Sec. 4.5) --------------------
// A Block on the CPU keeps its storage in host memory with the same layout
// as on the GPU (BlockDev offsets then count from a host pool), so the
// exchange buffers have one format for both sides.
struct HostPool;
HostPool* host_pool_create(int threads);
void host_pool_destroy(HostPool* p);
int host_pool_threads(const HostPool* p);

// One sweep (pull, bounce-back, collision, stores) of the listed Blocks
// from src to dst, rounding exactly as the GPU sweep of the same precision
// and arithmetic mode.  blocks: host-based table; ids: the Blocks to sweep;
// mask: host copy of the link masks (BlockDev::mask offsets into it), or
// NULL.  ph is Phys<double> for FP64 arithmetic, Phys<float> for FP32 storage
// with FP32 arithmetic.
void host_sweep(HostPool* p, int prec, bool f64math, const void* src, void* dst, const BlockDev* blocks,
                const int* ids, int nids, const uint32_t* mask, const GridGeom& geo, const Phys<double>& pd,
                const Phys<float>& pf);

// The host's share of an exchange over tasks (host-based Block table):
// mode 0 copies neighbour values into ghost slots (both Blocks on the host),
// 1 packs the sources into buf, 2 unpacks buf into the ghost slots.
void host_exchange(HostPool* p, int prec, int mode, void* grid, const BlockDev* blocks, const NbrDev* nbr,
                   const XchgTask* tasks, int ntasks, void* buf);

}  // namespace lbm
