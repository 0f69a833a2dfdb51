// lbm_runtime.hip -- host runtime behind include/lbm.h.
//
// Owns the Patch/Block management data (AABB, BlockID, neighbour table,
// Sec. 4.2), the device field data of every Block, the work-item list that
// the kernels walk, the captured HIP graphs of the time step and the
// schedule autotuner (the per-Block kernel selection of Sec. 4.1, done by
// measurement).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_internal.h"

namespace lbm {
void launch_sweep(int prec, bool f64math, bool mask, int fx, bool nt, bool force, int vec, const SweepArgs& a,
                  const Phys<double>& pd, const Phys<float>& pf, dim3 grid, dim3 block, hipStream_t s);
bool sweep_vec2_ok(int prec, bool f64math);
hipError_t launch_sweep_steps(int prec, bool f64math, bool mask, const SweepArgs& a, const Phys<double>& pd,
                              const Phys<float>& pf, int nsteps, int cus, hipStream_t s);
void launch_exchange(int prec, void* grid, const BlockDev* blocks, const NbrDev* nbr, const XchgTask* tasks,
                     int ntasks, hipStream_t s);
void launch_bbfill(int prec, bool f64math, void* grid, const CellArgs& a, const Phys<double>& pd,
                   const Phys<float>& pf, hipStream_t s);
void launch_linkmask(const uint8_t* solid, const CellArgs& a, uint32_t* mask, hipStream_t s);
void launch_openfill(int prec, void* grid, const BlockDev* blocks, int nblocks, const int* faceblk,
                     const GridGeom& geo, const double* side, hipStream_t s);
void launch_openside(int prec, const void* grid, const BlockDev* blocks, int nblocks, const int* faceblk,
                     const GridGeom& geo, double* side, hipStream_t s);
void launch_init_eq(int prec, void* grid, const CellArgs& a, double rho0, const double* rho, const double* u,
                    long long N, hipStream_t s);
void launch_macro(int prec, const void* grid, const CellArgs& a, double rho0, const double hg[3], double* rho,
                  double* u, long long N, hipStream_t s);
void launch_reduce(int prec, const void* cur, const void* prev, const CellArgs& a, double rho0, const double hc[3],
                   const double hp[3], int want_prev, const double* um, long long N, double* partial, int nparts,
                   double* out, hipStream_t s);
void launch_get_state(int prec, bool f64, const void* grid, const CellArgs& a, void* out, long long N,
                      hipStream_t s);
void launch_set_state(int prec, bool f64, void* grid, const CellArgs& a, const void* in, long long N,
                      hipStream_t s);
void launch_copy16(const void* src, void* dst, long long n16, int grid, hipStream_t s);
void launch_average(int prec, void* cur, const void* prev, long long n, hipStream_t s);
void launch_exchange_buf(int prec, int mode, void* grid, const BlockDev* blocks, const NbrDev* nbr,
                         const XchgTask* tasks, int ntasks, void* buf, hipStream_t s);
}  // namespace lbm

using namespace lbm;

namespace {

thread_local std::string g_last_error;

lbm_status fail(lbm_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define HIPCHK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(LBM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)

constexpr int E3[kQ][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
                           {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
                           {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

double weight(int i) {
  const int s = E3[i][0] * E3[i][0] + E3[i][1] * E3[i][1] + E3[i][2] * E3[i][2];
  return s == 0 ? 1.0 / 3.0 : (s == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

int storage_bytes(int prec) { return prec == 0 ? 8 : (prec == 1 ? 4 : 2); }

long long roundup(long long v, long long m) { return (v + m - 1) / m * m; }

}  // namespace

struct lbm_ctx {
  lbm_params p{};
  int prec = 1;
  bool f64math = false;
  int sbytes = 4;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  int device = 0;
  int cu_count = 256;

  std::vector<lbm_aabb> aabb;
  std::vector<BlockDev> bh;
  std::vector<NbrDev> nbh;
  std::vector<ItemDev> items_h;
  std::vector<XchgTask> tasks_h;   // every ghost slot
  std::vector<XchgTask> rim_h;     // the same, x faces cut to the rows on y/z faces
  GridGeom geo{};
  Phys<double> phd{};
  Phys<float> phf{};

  // device memory
  std::vector<std::pair<void*, size_t>> allocs;
  size_t held = 0;
  void* grid[2] = {nullptr, nullptr};
  size_t grid_elems = 0;
  BlockDev* d_blocks = nullptr;
  NbrDev* d_nbr = nullptr;
  GhostTgt* d_ghost = nullptr;
  ItemDev* d_items = nullptr;
  size_t items_cap = 0;
  XchgTask* d_tasks = nullptr;
  XchgTask* d_rim = nullptr;
  uint32_t* d_mask = nullptr;
  bool has_mask = false;
  bool x_even = false;   // every Block's x extent is even (two cells per lane possible)
  double* d_partial = nullptr;
  int nparts = 1024;
  double* d_red = nullptr;
  double* d_side = nullptr;  // open faces: [face][s2][s1][16] over the two other axes (see k_openfill)
  int* d_faceblk = nullptr;  // open faces: per face the count of Blocks touching it, then their ids
  void* d_stage = nullptr;
  double* d_umark = nullptr;   // [rho | u_x | u_y | u_z] snapshot, FP64, 4 N
  long long mark_steps = -1;   // step count of the snapshot, -1 = none
  long long set_steps = 0;     // step count when the state was last written from outside the sweep
  size_t stage_bytes = 0;

  int cur = 0;
  long long steps = 0;
  long long n_cells = 0;
  long long n_fluid = 0;
  lbm_schedule sched{};

  // captured graphs: [start parity] for 1 step and for graph_steps steps
  hipGraphExec_t g_one[2] = {nullptr, nullptr};
  hipGraphExec_t g_many[2] = {nullptr, nullptr};
  bool graphs_ok = false;

  // host-CPU Blocks (heterogeneous runs, Sec. 4.5).  Their state lives in
  // pinned host pools with the GPU layout (hbh: the Block table with host
  // offsets); their device storage holds a copy only after host_push.
  std::vector<char> on_host;
  std::vector<int> host_ids;
  HostPool* pool = nullptr;
  void* hgrid[2] = {nullptr, nullptr};
  std::vector<BlockDev> hbh;
  std::vector<uint32_t> hmask;
  std::vector<ItemDev> sweep_items_h;   // rows of the GPU Blocks
  ItemDev* d_sweep_items = nullptr;
  size_t sweep_items_cap = 0;
  // exchange tasks by (sender, receiver): GPU->GPU, GPU->host, host->GPU, host->host
  std::vector<XchgTask> t_dd, t_dh, t_hd, t_hh;
  std::vector<XchgTask> t_dd_rim;   // GPU->GPU rim tasks (x faces written by the sweep)
  XchgTask *d_t_dd = nullptr, *d_t_dh = nullptr, *d_t_hd = nullptr, *d_t_dd_rim = nullptr;
  void *d_xdn = nullptr, *d_xup = nullptr, *h_xdn = nullptr, *h_xup = nullptr;
  size_t xdn_elems = 0, xup_elems = 0;
  hipEvent_t x_done = nullptr;          // the step's down buffer has arrived
  std::vector<long long> bfluid;        // fluid cells per Block
};

namespace {

void* dalloc(lbm_ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* ptr = nullptr;
  if (c->p.dev_alloc) {
    ptr = c->p.dev_alloc(bytes, c->p.alloc_user);
  } else if (hipMalloc(&ptr, bytes) != hipSuccess) {
    ptr = nullptr;
  }
  if (ptr) {
    c->allocs.push_back({ptr, bytes});
    c->held += bytes;
  }
  return ptr;
}

void dfree(lbm_ctx* c, void* ptr) {
  if (!ptr) return;
  for (size_t k = 0; k < c->allocs.size(); ++k) {
    if (c->allocs[k].first == ptr) {
      c->held -= c->allocs[k].second;
      c->allocs.erase(c->allocs.begin() + k);
      break;
    }
  }
  if (c->p.dev_free) c->p.dev_free(ptr, c->p.alloc_user);
  else (void)hipFree(ptr);
}

void drop_graphs(lbm_ctx* c) {
  for (int k = 0; k < 2; ++k) {
    if (c->g_one[k]) (void)hipGraphExecDestroy(c->g_one[k]);
    if (c->g_many[k]) (void)hipGraphExecDestroy(c->g_many[k]);
    c->g_one[k] = c->g_many[k] = nullptr;
  }
  c->graphs_ok = false;
}

// some Blocks run on the host CPU
bool hetero(const lbm_ctx* c) { return !c->host_ids.empty(); }

CellArgs cell_args(const lbm_ctx* c) {
  CellArgs a;
  a.blocks = c->d_blocks;
  a.items = c->d_items;
  a.mask = c->d_mask;
  a.nitems = (int)c->items_h.size();
  a.has_mask = c->has_mask ? 1 : 0;
  a.geo = c->geo;
  return a;
}

// Validate the Block AABBs: exact, non-overlapping tiling of the Patch that
// forms a Cartesian grid.  Fills the per-axis cut lists and the
// (ix, iy, iz) -> BlockID map.
bool build_tiling(const int dims[3], const lbm_aabb* b, int n, std::vector<int> cuts[3], std::vector<int>& owner,
                  std::string& err) {
  for (int k = 0; k < 3; ++k) {
    cuts[k].clear();
    cuts[k].push_back(0);
    cuts[k].push_back(dims[k]);
  }
  for (int j = 0; j < n; ++j) {
    for (int k = 0; k < 3; ++k) {
      if (b[j].lo[k] < 0 || b[j].hi[k] > dims[k] || b[j].lo[k] >= b[j].hi[k]) {
        err = "block " + std::to_string(j) + ": empty or outside the domain";
        return false;
      }
      cuts[k].push_back(b[j].lo[k]);
      cuts[k].push_back(b[j].hi[k]);
    }
  }
  long long ncell = 1;
  for (int k = 0; k < 3; ++k) {
    std::sort(cuts[k].begin(), cuts[k].end());
    cuts[k].erase(std::unique(cuts[k].begin(), cuts[k].end()), cuts[k].end());
    ncell *= (long long)(cuts[k].size() - 1);
  }
  if (ncell != n) {
    err = "blocks do not form a Cartesian grid (" + std::to_string(n) + " blocks, " + std::to_string(ncell) +
          " grid slots)";
    return false;
  }
  const int nx = (int)cuts[0].size() - 1, ny = (int)cuts[1].size() - 1;
  owner.assign((size_t)ncell, -1);
  for (int j = 0; j < n; ++j) {
    int lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
      lo[k] = (int)(std::lower_bound(cuts[k].begin(), cuts[k].end(), b[j].lo[k]) - cuts[k].begin());
      hi[k] = (int)(std::lower_bound(cuts[k].begin(), cuts[k].end(), b[j].hi[k]) - cuts[k].begin());
      if (hi[k] != lo[k] + 1) {
        err = "block " + std::to_string(j) + " spans more than one grid slot";
        return false;
      }
    }
    const size_t s = ((size_t)lo[2] * ny + lo[1]) * nx + lo[0];
    if (owner[s] >= 0) {
      err = "blocks " + std::to_string(owner[s]) + " and " + std::to_string(j) + " overlap";
      return false;
    }
    owner[s] = j;
  }
  return true;
}

int slot_of(const std::vector<int>& cuts, int v) {
  return (int)(std::upper_bound(cuts.begin(), cuts.end(), v) - cuts.begin()) - 1;
}

int cells_per_lane(const lbm_ctx* c, const lbm_schedule& s);

// XCD-aware item order for many Blocks.  Workgroup w of a launch runs on
// XCD w % 8 (the dispatcher deals workgroups to the 8 XCDs in turn, each
// with its own L2), and the sweep gives item w to workgroup w (or w + k *
// grid with a persistent grid, a multiple of 8).  The sweep reads rows of
// the planes next to its own (pulls along z, the own-cell loads across
// obstacle links, ghost rows), which stay in an L2 only if the neighbouring
// planes' items run on the same XCD close in time.  So whole Blocks are
// dealt to 8 queues (largest first, to the shortest queue), each queue keeps
// its Blocks' items plane by plane, and the list interleaves the queues:
// item 8 s + x is the s-th of queue x.  Queues differ by at most one Block's
// items; past the shortest, the tail keeps the interleave of the rest.  With
// few Blocks (one Block walks its planes in order on all XCDs alike) the
// order is left as built.
void order_items_by_xcd(lbm_ctx* c) {
  constexpr int X = 8;
  const int nb = (int)c->bh.size();
  if (nb < 2 * X) return;
  std::vector<std::vector<ItemDev>> per_block(nb);
  for (const ItemDev& it : c->items_h) per_block[it.block].push_back(it);
  std::vector<int> order(nb);
  for (int j = 0; j < nb; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(),
                   [&](int u, int v) { return per_block[u].size() > per_block[v].size(); });
  std::vector<std::vector<ItemDev>> q(X);
  for (int j : order) {
    int best = 0;
    for (int x = 1; x < X; ++x)
      if (q[x].size() < q[best].size()) best = x;
    q[best].insert(q[best].end(), per_block[j].begin(), per_block[j].end());
  }
  c->items_h.clear();
  size_t longest = 0;
  for (const auto& v : q) longest = std::max(longest, v.size());
  for (size_t k = 0; k < longest; ++k)
    for (int x = 0; x < X; ++x)
      if (k < q[x].size()) c->items_h.push_back(q[x][k]);
}

void build_items(lbm_ctx* c) {
  c->items_h.clear();
  const int target = std::max(1, c->sched.item_cells);
  const int vec = cells_per_lane(c, c->sched), nw = std::max(1, c->sched.wg_size / 64);
  for (int j = 0; j < (int)c->bh.size(); ++j) {
    const BlockDev& B = c->bh[j];
    const int a = B.dim[0], b = B.dim[1], cz = B.dim[2];
    int rows = std::max(1, std::min(b, target / a));
    if (B.pack) rows = std::max(2, rows & ~1);  // pairs of packed rows share a line
    const bool flat = flat_rows(B, vec, (int)c->sbytes);
    if (flat) {
      // flat runs: whole waves per item where a few rows make a multiple of
      // 64 cells (48-cell rows: 4; packed rows' multiple is even)
      int m = 64;
      while (m > 1 && (a * (m / 2)) % 64 == 0) m /= 2;
      if (m <= b && m * a <= 2 * target) rows = std::max(m, rows / m * m);
    }
    // The sweep's waves take an item's (row group, 64-lane segment) tasks in
    // turn.  With 16-bit storage, round rows up so that their count is a
    // multiple of the waves per workgroup (a 384-cell row is 6 segments: one
    // row per item leaves half of a 4-wave workgroup idle in its second
    // round).  Measured on gfx950 (same box, 320^3 and 384^3 cavities):
    // +12-15 % for F16S, but -3-4 % for FP32 and FP64, whose sweeps gain
    // more from the larger number of smaller items.
    const int lanes = (a + vec - 1) / vec;
    int xw = 64;
    while (xw > 1 && xw / 2 >= lanes) xw >>= 1;
    const int rpw = 64 / xw, nseg = (lanes + 63) / 64;
    auto tasks = [&](int r) { return flat ? ((long long)r * a + 63) / 64 : (long long)((r + rpw - 1) / rpw) * nseg; };
    for (int r = rows; r <= b && c->prec >= 2; ++r) {
      if (tasks(r) % nw == 0 || r == b) {
        rows = r;
        break;
      }
    }
    // (flat runs in a Block that wraps along y: rows 0 and b - 1 alone, and
    // row 1 too with packed rows, so that the flat items start on even rows)
    const bool wy = flat && (B.wrap & 2) && b > 3;
    const int ylo = wy ? (B.pack ? 2 : 1) : 0, yhi = wy ? b - 1 : b;
    for (int z = 0; z < cz; ++z) {
      for (int y = 0; y < ylo; ++y) c->items_h.push_back({j, z, y, 1});
      for (int y = ylo; y < yhi; y += rows) c->items_h.push_back({j, z, y, std::min(rows, yhi - y)});
      if (wy) c->items_h.push_back({j, z, b - 1, 1});
    }
  }
  order_items_by_xcd(c);
  // the GPU sweep of a heterogeneous run covers the GPU Blocks only
  c->sweep_items_h.clear();
  if (hetero(c))
    for (const ItemDev& it : c->items_h)
      if (!c->on_host[it.block]) c->sweep_items_h.push_back(it);
}

lbm_status upload_list(lbm_ctx* c, const std::vector<ItemDev>& h, ItemDev** d, size_t* cap) {
  const size_t need = std::max<size_t>(1, h.size()) * sizeof(ItemDev);
  if (need > *cap) {
    if (*d) dfree(c, *d);
    *d = (ItemDev*)dalloc(c, need);
    *cap = *d ? need : 0;
    if (!*d) return fail(LBM_ENOMEM, "item list allocation failed");
  }
  if (!h.empty()) HIPCHK(hipMemcpy(*d, h.data(), h.size() * sizeof(ItemDev), hipMemcpyHostToDevice));
  return LBM_OK;
}

lbm_status upload_items(lbm_ctx* c) {
  lbm_status s = upload_list(c, c->items_h, &c->d_items, &c->items_cap);
  if (s == LBM_OK && hetero(c)) s = upload_list(c, c->sweep_items_h, &c->d_sweep_items, &c->sweep_items_cap);
  return s;
}

// Exchange tasks: per (Block, neighbour offset) the directions that cross,
// cut into chunks of at most kXchgChunk cells (one workgroup each).  The rim
// list serves the schedule whose sweep writes the x-face ghost planes of rows
// off the sender's y and z faces itself (fused_exchange = 2): its x-face
// tasks keep only the rows y = 0, b-1 and the planes z = 0, c-1 (x
// neighbours share their y and z extents in a Cartesian tiling).
constexpr int kXchgChunk = 1024;

void push_chunks(std::vector<XchgTask>& out, XchgTask t, int ncell) {
  for (int l0 = 0; l0 < ncell; l0 += kXchgChunk) {
    t.l0 = l0;
    t.l1 = std::min(ncell, l0 + kXchgChunk);
    out.push_back(t);
  }
}

void build_tasks(lbm_ctx* c) {
  c->tasks_h.clear();
  c->rim_h.clear();
  for (int j = 0; j < (int)c->bh.size(); ++j) {
    const BlockDev& M = c->bh[j];
    for (int d = 0; d < 27; ++d) {
      if (d == 13 || c->nbh[(size_t)j * 27 + d].id < 0) continue;
      const int off[3] = {d % 3 - 1, (d / 3) % 3 - 1, d / 9 - 1};
      // ghost slots across an axis the Block wraps on are never read
      if (((off[0] != 0) && (M.wrap & 1)) || ((off[1] != 0) && (M.wrap & 2)) || ((off[2] != 0) && (M.wrap & 4)))
        continue;
      XchgTask t{};
      t.dst = j;
      t.d = d;
      int ncell = 1;
      for (int k = 0; k < 3; ++k) {
        t.lo[k] = off[k] < 0 ? -1 : (off[k] > 0 ? M.dim[k] : 0);
        t.ext[k] = off[k] == 0 ? M.dim[k] : 1;
        ncell *= t.ext[k];
      }
      for (int i = 1; i < kQ; ++i) {
        bool ok = true, any = false;
        for (int k = 0; k < 3; ++k) {
          if (off[k] != 0) {
            any = true;
            if (E3[i][k] != -off[k]) ok = false;
          }
        }
        if (ok && any) t.dirs |= i << (5 * t.ndir++);
      }
      if (t.ndir == 0) continue;
      push_chunks(c->tasks_h, t, ncell);
      const bool xface = off[0] != 0 && off[1] == 0 && off[2] == 0;
      if (!xface) {
        push_chunks(c->rim_h, t, ncell);
        continue;
      }
      const int b = M.dim[1], cz = M.dim[2];
      auto part = [&](int y0, int ny, int z0, int nz) {
        if (ny <= 0 || nz <= 0) return;
        XchgTask r = t;
        r.lo[1] = y0;
        r.ext[1] = ny;
        r.lo[2] = z0;
        r.ext[2] = nz;
        push_chunks(c->rim_h, r, ny * nz);
      };
      part(0, b, 0, 1);                     // z = 0
      if (cz > 1) part(0, b, cz - 1, 1);    // z = c - 1
      part(0, 1, 1, cz - 2);                // y = 0, 0 < z < c - 1
      if (b > 1) part(b - 1, 1, 1, cz - 2); // y = b - 1
    }
  }
}

// --- step launches -------------------------------------------------------
SweepArgs sweep_args(const lbm_ctx* c, int from) {
  SweepArgs a{};
  a.src = c->grid[from];
  a.dst = c->grid[1 - from];
  a.blocks = c->d_blocks;
  a.nbr = c->d_nbr;
  a.items = c->d_items;
  a.mask = c->d_mask;
  a.ghost = c->d_ghost;
  // the sweep writes the side entries of open x faces itself (y and z faces:
  // k_openside after the sweep)
  a.side = c->geo.open_axis == 0 ? c->d_side : nullptr;
  a.nitems = (int)c->items_h.size();
  a.geo = c->geo;
  if (hetero(c)) {
    a.items = c->d_sweep_items;
    a.nitems = (int)c->sweep_items_h.size();
  }
  return a;
}

// Ghost-target table of the fused exchange: for Block j and offset class d,
// where the boundary values of j land in neighbour M (see GhostTgt).
std::vector<GhostTgt> build_ghost_table(const lbm_ctx* c) {
  const int nb = (int)c->bh.size();
  std::vector<GhostTgt> t((size_t)nb * 27);
  for (int j = 0; j < nb; ++j)
    for (int d = 0; d < 27; ++d) {
      GhostTgt& g = t[(size_t)j * 27 + d];
      std::memset(&g, 0, sizeof(g));
      const NbrDev& n = c->nbh[(size_t)j * 27 + d];
      if (d == 13 || n.id < 0) continue;
      const BlockDev& M = c->bh[n.id];
      const int cx = d % 3 - 1;
      g.Sz = M.Sz;
      g.Sf = M.Sf;
      g.Sx = M.Sx;
      g.Ry = M.Ry;
      g.main0 = M.base + (long long)(n.tz + 1) * M.Sz + (long long)(n.ty + 1) * M.Sx + n.tx;
      g.xg0 = M.base + M.xgo + (long long)(n.tz + 1) * M.Ry + (n.ty + 1);
      g.kind = cx == 0 ? 1 : 2;
      // the receiver never reads ghost slots across an axis it wraps on
      const int cy = (d / 3) % 3 - 1, cz = d / 9 - 1;
      if ((cx != 0 && (M.wrap & 1)) || (cy != 0 && (M.wrap & 2)) || (cz != 0 && (M.wrap & 4))) g.kind = 0;
    }
  return t;
}

void enqueue_exchange(lbm_ctx* c, int g, hipStream_t s, bool rim = false) {
  if (rim)
    launch_exchange(c->prec, c->grid[g], c->d_blocks, c->d_nbr, c->d_rim, (int)c->rim_h.size(), s);
  else
    launch_exchange(c->prec, c->grid[g], c->d_blocks, c->d_nbr, c->d_tasks, (int)c->tasks_h.size(), s);
}

bool has_open(const lbm_ctx* c);

// Bounce-back slots and the open faces' boundary nodes of a state written
// from outside the sweep (the nodes from the face cells' stored populations).
void enqueue_slots(lbm_ctx* c, int g, hipStream_t s) {
  launch_bbfill(c->prec, c->f64math, c->grid[g], cell_args(c), c->phd, c->phf, s);
  if (has_open(c)) {
    const int nb = (int)c->bh.size();
    launch_openside(c->prec, c->grid[g], c->d_blocks, nb, c->d_faceblk, c->geo, c->d_side, s);
    launch_openfill(c->prec, c->grid[g], c->d_blocks, nb, c->d_faceblk, c->geo, c->d_side, s);
  }
}

// Ghost layers and bounce-back slots of a state written from outside the sweep.
void enqueue_fill(lbm_ctx* c, int g, hipStream_t s) {
  enqueue_exchange(c, g, s);
  enqueue_slots(c, g, s);
}

// Cells per lane the sweep of schedule s runs with (0 = automatic = one: with
// a single cell per lane the sweep keeps more waves resident and measured
// faster for every storage mode on gfx950).
// Two cells per lane: F16S/BF16S or F32 with FP64 math, even x extents, and
// no open x faces (the sweep keeps one face cell per lane for them; open y
// or z faces leave the sweep untouched).
bool vec2_allowed(const lbm_ctx* c) {
  return c->x_even && sweep_vec2_ok(c->prec, c->f64math) && !c->geo.open[0] && !c->geo.open[1];
}

int cells_per_lane(const lbm_ctx* c, const lbm_schedule& s) { return s.cells_per_lane == 2 && vec2_allowed(c) ? 2 : 1; }

void enqueue_sweep(lbm_ctx* c, int from, hipStream_t s) {
  const SweepArgs a = sweep_args(c, from);
  const int nitems = a.nitems;
  if (nitems < 1) return;  // every Block on the host
  int grid = nitems;
  if (c->sched.persistent > 0) grid = std::min(nitems, c->sched.persistent * c->cu_count);
  if (grid < 1) grid = 1;
  const bool force = c->p.force[0] != 0.0 || c->p.force[1] != 0.0 || c->p.force[2] != 0.0;
  launch_sweep(c->prec, c->f64math, c->has_mask, c->sched.fused_exchange, c->sched.nontemporal != 0, force,
               cells_per_lane(c, c->sched), a, c->phd, c->phf, dim3(grid), dim3(c->sched.wg_size), s);
}

bool has_open(const lbm_ctx* c) { return c->geo.open_axis >= 0; }

// After the sweep into grid g: the ghost exchange (unless the sweep did it)
// and the boundary nodes of open faces.
void enqueue_post(lbm_ctx* c, int g, hipStream_t s) {
  if (c->sched.fused_exchange != 1) enqueue_exchange(c, g, s, c->sched.fused_exchange == 2);
  if (has_open(c)) {
    const int nb = (int)c->bh.size();
    if (c->geo.open_axis != 0)
      launch_openside(c->prec, c->grid[g], c->d_blocks, nb, c->d_faceblk, c->geo, c->d_side, s);
    launch_openfill(c->prec, c->grid[g], c->d_blocks, nb, c->d_faceblk, c->geo, c->d_side, s);
  }
}

void enqueue_step(lbm_ctx* c, int from, hipStream_t s) {
  enqueue_sweep(c, from, s);
  enqueue_post(c, 1 - from, s);
}

lbm_status capture(lbm_ctx* c, int from, int nsteps, hipGraphExec_t* out) {
  HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  int g = from;
  for (int k = 0; k < nsteps; ++k) {
    enqueue_step(c, g, c->cap_stream);
    g = 1 - g;
  }
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamEndCapture(c->cap_stream, &graph));
  hipError_t e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(LBM_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  return LBM_OK;
}

lbm_status ensure_graphs(lbm_ctx* c) {
  if (c->graphs_ok || c->sched.graph_steps <= 0) return LBM_OK;
  drop_graphs(c);
  for (int from = 0; from < 2; ++from) {
    lbm_status s = capture(c, from, 1, &c->g_one[from]);
    if (s != LBM_OK) return s;
    s = capture(c, from, c->sched.graph_steps, &c->g_many[from]);
    if (s != LBM_OK) return s;
  }
  c->graphs_ok = true;
  return LBM_OK;
}

// ---- host-CPU Blocks (heterogeneous runs, Sec. 4.5) ----------------------
size_t span_elems(const BlockDev& B) { return (size_t)kQ * (size_t)B.Sf; }

// Copy both grids of every host Block between its host pool slot and its
// device storage (to_device: host -> device).
lbm_status host_copy(lbm_ctx* c, bool to_device) {
  for (int g = 0; g < 2; ++g)
    for (int j : c->host_ids) {
      const size_t bytes = span_elems(c->bh[j]) * c->sbytes;
      char* dv = (char*)c->grid[g] + (size_t)c->bh[j].base * c->sbytes;
      char* hv = (char*)c->hgrid[g] + (size_t)c->hbh[j].base * c->sbytes;
      if (to_device)
        HIPCHK(hipMemcpyAsync(dv, hv, bytes, hipMemcpyHostToDevice, c->stream));
      else
        HIPCHK(hipMemcpyAsync(hv, dv, bytes, hipMemcpyDeviceToHost, c->stream));
    }
  HIPCHK(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

// Before a kernel reads the whole state (moments, sums, checkpoint): the
// host Blocks' current values into their device storage.
lbm_status host_push(lbm_ctx* c) { return hetero(c) ? host_copy(c, true) : LBM_OK; }

// After the device wrote the whole state (initialisation, geometry,
// checkpoint): link masks and state of the host Blocks to the host.
lbm_status host_pull(lbm_ctx* c) {
  if (!hetero(c)) return LBM_OK;
  c->hmask.clear();
  for (int j : c->host_ids) {
    BlockDev& H = c->hbh[j];
    const BlockDev& B = c->bh[j];
    H.mask = -1;
    if (c->has_mask && B.mask >= 0) {
      const size_t n = (size_t)B.dim[0] * B.dim[1] * B.dim[2];
      H.mask = (long long)c->hmask.size();
      c->hmask.resize(c->hmask.size() + n);
      HIPCHK(hipMemcpy(c->hmask.data() + H.mask, c->d_mask + B.mask, n * sizeof(uint32_t), hipMemcpyDeviceToHost));
    }
  }
  return host_copy(c, false);
}

// Free the heterogeneous set-up (state stays where it is: call host_push
// first to keep it).
void host_release(lbm_ctx* c) {
  if (c->pool) host_pool_destroy(c->pool);
  c->pool = nullptr;
  if (c->x_done) (void)hipEventDestroy(c->x_done);
  c->x_done = nullptr;
  for (void*& h : c->hgrid) {
    if (h) (void)hipHostFree(h);
    h = nullptr;
  }
  for (void** h : {&c->h_xdn, &c->h_xup}) {
    if (*h) (void)hipHostFree(*h);
    *h = nullptr;
  }
  for (void** d : {(void**)&c->d_t_dd, (void**)&c->d_t_dh, (void**)&c->d_t_hd, (void**)&c->d_t_dd_rim, &c->d_xdn,
                   &c->d_xup, (void**)&c->d_sweep_items}) {
    if (*d) dfree(c, *d);
    *d = nullptr;
  }
  c->sweep_items_cap = 0;
  c->host_ids.clear();
  c->on_host.assign(c->bh.size(), 0);
  c->hbh.clear();
  c->hmask.clear();
  c->sweep_items_h.clear();
  c->t_dd.clear();
  c->t_dd_rim.clear();
  c->t_dh.clear();
  c->t_hd.clear();
  c->t_hh.clear();
  c->xdn_elems = c->xup_elems = 0;
}

lbm_status upload_tasks(lbm_ctx* c, const std::vector<XchgTask>& h, XchgTask** d) {
  if (h.empty()) return LBM_OK;
  *d = (XchgTask*)dalloc(c, h.size() * sizeof(XchgTask));
  if (!*d) return fail(LBM_ENOMEM, "exchange task allocation failed");
  HIPCHK(hipMemcpy(*d, h.data(), h.size() * sizeof(XchgTask), hipMemcpyHostToDevice));
  return LBM_OK;
}

// Assign the Blocks in ids to the host CPU (state copied over) and build the
// exchange between the two memories.
lbm_status host_setup(lbm_ctx* c, const std::vector<int>& ids, int threads) {
  c->on_host.assign(c->bh.size(), 0);
  for (int j : ids) c->on_host[j] = 1;
  c->host_ids = ids;
  std::sort(c->host_ids.begin(), c->host_ids.end());
  // host pools: the Blocks' spans one after the other, page-aligned
  c->hbh = c->bh;
  long long hoff = 0;
  for (int j : c->host_ids) {
    c->hbh[j].base = hoff;
    hoff = roundup(hoff + (long long)span_elems(c->bh[j]), 4096 / c->sbytes);
  }
  for (void*& h : c->hgrid)
    if (hipHostMalloc(&h, (size_t)hoff * c->sbytes, hipHostMallocDefault) != hipSuccess) {
      h = nullptr;
      return fail(LBM_ENOMEM, "pinned host allocation for the host Blocks failed");
    }
  // exchange tasks by the sides of sender and receiver; the buffers hold
  // 5 values per task cell
  for (XchgTask t : c->tasks_h) {
    const bool hs = c->on_host[c->nbh[(size_t)t.dst * 27 + t.d].id] != 0, hr = c->on_host[t.dst] != 0;
    if (!hs && !hr) {
      c->t_dd.push_back(t);
    } else if (!hs && hr) {
      t.bo = (int)c->xdn_elems;
      c->xdn_elems += 5 * (size_t)(t.l1 - t.l0);
      c->t_dh.push_back(t);
    } else if (hs && !hr) {
      t.bo = (int)c->xup_elems;
      c->xup_elems += 5 * (size_t)(t.l1 - t.l0);
      c->t_hd.push_back(t);
    } else {
      c->t_hh.push_back(t);
    }
  }
  for (const XchgTask& t : c->rim_h)
    if (!c->on_host[c->nbh[(size_t)t.dst * 27 + t.d].id] && !c->on_host[t.dst]) c->t_dd_rim.push_back(t);
  if (c->xdn_elems + c->xup_elems >= (1ull << 31)) return fail(LBM_EINVAL, "exchange buffers too large");
  lbm_status st = upload_tasks(c, c->t_dd, &c->d_t_dd);
  if (st == LBM_OK) st = upload_tasks(c, c->t_dd_rim, &c->d_t_dd_rim);
  if (st == LBM_OK) st = upload_tasks(c, c->t_dh, &c->d_t_dh);
  if (st == LBM_OK) st = upload_tasks(c, c->t_hd, &c->d_t_hd);
  if (st != LBM_OK) return st;
  const size_t nd = std::max<size_t>(1, c->xdn_elems) * c->sbytes, nu = std::max<size_t>(1, c->xup_elems) * c->sbytes;
  c->d_xdn = dalloc(c, nd);
  c->d_xup = dalloc(c, nu);
  if (!c->d_xdn || !c->d_xup) return fail(LBM_ENOMEM, "exchange buffer allocation failed");
  if (hipHostMalloc(&c->h_xdn, nd, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(&c->h_xup, nu, hipHostMallocDefault) != hipSuccess)
    return fail(LBM_ENOMEM, "pinned exchange buffer allocation failed");
  build_items(c);
  st = upload_items(c);
  if (st != LBM_OK) return st;
  if (hipEventCreateWithFlags(&c->x_done, hipEventDisableTiming) != hipSuccess) {
    c->x_done = nullptr;
    return fail(LBM_EDEVICE, "hipEventCreate failed");
  }
  if (threads <= 0) threads = (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
  c->pool = host_pool_create(threads);
  return host_pull(c);
}

struct HostTimes {
  double gpu = 0.0, cpu = 0.0, xchg = 0.0, step = 0.0;
};

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// The exchange of a heterogeneous step into grid `to`, first half: host
// senders packed into the up buffer and host pairs copied on the host; on
// the stream the up buffer's copy and unpack, the GPU pairs as the schedule
// says (copy kernel for fused_exchange 0, its rim after the sweep's x faces
// for 2, nothing after the fully fused sweep), the GPU senders packed and
// copied to the host.  The sweep's writes into a host Block's device copy
// are never read.
lbm_status host_exchange_begin(lbm_ctx* c, int to) {
  host_exchange(c->pool, c->prec, 1, c->hgrid[to], c->hbh.data(), c->nbh.data(), c->t_hd.data(), (int)c->t_hd.size(),
                c->h_xup);
  host_exchange(c->pool, c->prec, 0, c->hgrid[to], c->hbh.data(), c->nbh.data(), c->t_hh.data(), (int)c->t_hh.size(),
                nullptr);
  if (!c->t_hd.empty()) {
    HIPCHK(hipMemcpyAsync(c->d_xup, c->h_xup, c->xup_elems * c->sbytes, hipMemcpyHostToDevice, c->stream));
    launch_exchange_buf(c->prec, 2, c->grid[to], c->d_blocks, c->d_nbr, c->d_t_hd, (int)c->t_hd.size(), c->d_xup,
                        c->stream);
  }
  if (c->sched.fused_exchange == 0)
    launch_exchange(c->prec, c->grid[to], c->d_blocks, c->d_nbr, c->d_t_dd, (int)c->t_dd.size(), c->stream);
  else if (c->sched.fused_exchange == 2)
    launch_exchange(c->prec, c->grid[to], c->d_blocks, c->d_nbr, c->d_t_dd_rim, (int)c->t_dd_rim.size(), c->stream);
  if (!c->t_dh.empty()) {
    launch_exchange_buf(c->prec, 1, c->grid[to], c->d_blocks, c->d_nbr, c->d_t_dh, (int)c->t_dh.size(), c->d_xdn,
                        c->stream);
    HIPCHK(hipMemcpyAsync(c->h_xdn, c->d_xdn, c->xdn_elems * c->sbytes, hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(hipGetLastError());
  return LBM_OK;
}

// Second half, once the down buffer has arrived: GPU senders into the host
// Blocks' ghost slots.
void host_exchange_end(lbm_ctx* c, int to) {
  host_exchange(c->pool, c->prec, 2, c->hgrid[to], c->hbh.data(), c->nbh.data(), c->t_dh.data(), (int)c->t_dh.size(),
                c->h_xdn);
}

// One time step of a heterogeneous run, its phases timed: the GPU sweeps
// its Blocks while the host threads sweep theirs; then the exchange.
// ev: two events for the GPU sweep time.
lbm_status host_step_timed(lbm_ctx* c, HostTimes* tm, hipEvent_t* ev) {
  const int from = c->cur, to = 1 - c->cur;
  const auto t0 = std::chrono::steady_clock::now();
  HIPCHK(hipEventRecord(ev[0], c->stream));
  enqueue_sweep(c, from, c->stream);
  HIPCHK(hipEventRecord(ev[1], c->stream));
  host_sweep(c->pool, c->prec, c->f64math, c->hgrid[from], c->hgrid[to], c->hbh.data(), c->host_ids.data(),
             (int)c->host_ids.size(), c->has_mask ? c->hmask.data() : nullptr, c->geo, c->phd, c->phf);
  tm->cpu += ms_since(t0);
  HIPCHK(hipEventSynchronize(ev[1]));
  const auto t1 = std::chrono::steady_clock::now();
  lbm_status st = host_exchange_begin(c, to);
  if (st != LBM_OK) return st;
  HIPCHK(hipStreamSynchronize(c->stream));
  host_exchange_end(c, to);
  float g = 0.f;
  HIPCHK(hipEventElapsedTime(&g, ev[0], ev[1]));
  tm->gpu += g;
  tm->xchg += ms_since(t1);
  tm->step += ms_since(t0);
  c->cur = to;
  c->steps += 1;
  return LBM_OK;
}

// n heterogeneous steps, pipelined: step k+1's GPU sweep is queued right
// behind step k's exchange, so the GPU does not wait for the host's
// unpack; the host unpacks and sweeps step k+1 while the GPU sweeps it.
lbm_status host_steps_pipelined(lbm_ctx* c, long long n) {
  if (n <= 0) return LBM_OK;
  enqueue_sweep(c, c->cur, c->stream);
  for (long long k = 0; k < n; ++k) {
    const int from = c->cur, to = 1 - c->cur;
    host_sweep(c->pool, c->prec, c->f64math, c->hgrid[from], c->hgrid[to], c->hbh.data(), c->host_ids.data(),
               (int)c->host_ids.size(), c->has_mask ? c->hmask.data() : nullptr, c->geo, c->phd, c->phf);
    lbm_status st = host_exchange_begin(c, to);
    if (st != LBM_OK) return st;
    HIPCHK(hipEventRecord(c->x_done, c->stream));
    if (k + 1 < n) enqueue_sweep(c, to, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventSynchronize(c->x_done));
    host_exchange_end(c, to);
    c->cur = to;
    c->steps += 1;
  }
  return LBM_OK;
}

lbm_status host_steps(lbm_ctx* c, long long n, HostTimes* tm) {
  if (!tm) return host_steps_pipelined(c, n);
  hipEvent_t ev[2] = {nullptr, nullptr};
  lbm_status st = LBM_OK;
  for (hipEvent_t& e : ev)
    if (hipEventCreate(&e) != hipSuccess) st = fail(LBM_EDEVICE, "hipEventCreate failed");
  for (long long k = 0; k < n && st == LBM_OK; ++k) st = host_step_timed(c, tm, ev);
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  return st;
}

lbm_status run_steps(lbm_ctx* c, long long n) {
  if (n <= 0) return LBM_OK;
  if (hetero(c)) return host_steps(c, n, nullptr);
  if (c->sched.graph_steps > 0) {
    lbm_status s = ensure_graphs(c);
    if (s != LBM_OK) return s;
    const long long G = c->sched.graph_steps;
    while (n >= G) {
      HIPCHK(hipGraphLaunch(c->g_many[c->cur], c->stream));
      if (G & 1) c->cur = 1 - c->cur;
      n -= G;
      c->steps += G;
    }
    while (n > 0) {
      HIPCHK(hipGraphLaunch(c->g_one[c->cur], c->stream));
      c->cur = 1 - c->cur;
      --n;
      c->steps += 1;
    }
    return LBM_OK;
  }
  for (long long k = 0; k < n; ++k) {
    enqueue_step(c, c->cur, c->stream);
    c->cur = 1 - c->cur;
    c->steps += 1;
  }
  HIPCHK(hipGetLastError());
  return LBM_OK;
}

lbm_status ensure_stage(lbm_ctx* c, size_t bytes) {
  if (bytes <= c->stage_bytes) return LBM_OK;
  if (c->d_stage) dfree(c, c->d_stage);
  c->d_stage = dalloc(c, bytes);
  if (!c->d_stage) {
    c->stage_bytes = 0;
    return fail(LBM_ENOMEM, "staging buffer allocation failed");
  }
  c->stage_bytes = bytes;
  return LBM_OK;
}

// g/2 correction of a grid: post-collision states carry rho0 g extra momentum.
void half_force(const lbm_ctx* c, bool post, double hg[3]) {
  for (int k = 0; k < 3; ++k) hg[k] = post ? 0.5 * c->p.force[k] : 0.0;
}

// want_prev: 0 sums only, 1 against the other grid (previous step), 2 against
// the velocity snapshot of lbm_residual_mark.
// Extra 128-byte lines appended to every x-row (lbm_params.row_pad).
long long row_pad_lines(const lbm_params& p, long long row_bytes) {
  if (p.row_pad < 0) return 0;
  if (p.row_pad > 0) return p.row_pad;
  (void)row_bytes;
  return 0;
}

// partials / red: the reduction's scratch (the context's own buffers, or
// the allocation-free entry point's device array with room for nparts_max
// workgroups)
lbm_status reduce(lbm_ctx* c, int want_prev, double out[6], double* partials = nullptr, double* red = nullptr,
                  int nparts_max = 0) {
  lbm_status hs = host_push(c);
  if (hs != LBM_OK) return hs;
  double hc[3], hp[3];
  half_force(c, c->steps >= 1, hc);
  half_force(c, c->steps >= 2, hp);
  const CellArgs a = cell_args(c);
  const int nparts = std::max(1, std::min(c->nparts, a.nitems));
  if (!partials) {
    partials = c->d_partial;
    red = c->d_red;
  } else if (nparts > nparts_max) {
    return fail(LBM_EINVAL, "reduction needs more workgroup partials than the scratch array holds");
  }
  launch_reduce(c->prec, c->grid[c->cur], c->grid[1 - c->cur], a, c->p.rho0, hc, hp, want_prev,
                want_prev == 2 ? c->d_umark + c->n_cells : nullptr, c->n_cells, partials, nparts, red, c->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(out, red, 6 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int k = 0; k < 6; ++k)
    if (!std::isfinite(out[k])) return fail(LBM_EUNSTABLE, "non-finite global sum");
  return LBM_OK;
}

// Scratch of the allocation-free reductions (lbm_sums_noalloc): the
// per-workgroup partials (6 doubles each, at most 1024 workgroups) and the
// six final sums, in one file-scope device array per GPU.  Host code never
// uses the array's name as an address: each device's address comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kScratchDoubles = 6 * 1024 + 8;
static __device__ __align__(256) double scratch[kScratchDoubles];
std::mutex g_scratch_mu;
double* g_scratch_dev[64] = {};

lbm_status scratch_ptr(int dev, double** out) {
  if (dev < 0 || dev >= 64) return fail(LBM_EDEVICE, "device index out of range for the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(LBM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = (double*)ptr;
  }
  *out = g_scratch_dev[dev];
  return LBM_OK;
}

lbm_status zero_grids(lbm_ctx* c) {
  for (int g = 0; g < 2; ++g)
    HIPCHK(hipMemsetAsync(c->grid[g], 0, c->grid_elems * c->sbytes, c->stream));
  return LBM_OK;
}

std::string sched_str(const lbm_schedule& s) {
  std::ostringstream o;
  o << s.fused_exchange << " " << s.item_cells << " " << s.wg_size << " " << s.persistent << " " << s.graph_steps
    << " " << s.nontemporal << " " << s.cells_per_lane;
  return o.str();
}

bool sched_valid(const lbm_schedule& s, std::string& err) {
  const int wg = s.wg_size;
  if (!(wg == 64 || wg == 128 || wg == 256)) {
    err = "wg_size must be 64, 128 or 256";
    return false;
  }
  if (s.item_cells < 1 || s.item_cells > (1 << 22)) {
    err = "item_cells out of range";
    return false;
  }
  if (s.persistent < 0 || s.persistent > 64 || s.graph_steps < 0 || s.graph_steps > 4096) {
    err = "persistent or graph_steps out of range";
    return false;
  }
  if (s.fused_exchange < 0 || s.fused_exchange > 2) {
    err = "fused_exchange must be 0, 1 or 2";
    return false;
  }
  if (s.cells_per_lane < 0 || s.cells_per_lane > 2) {
    err = "cells_per_lane must be 0, 1 or 2";
    return false;
  }
  return true;
}

}  // namespace

// =================================================================== ABI ==
extern "C" {

const char* lbm_strerror(lbm_status s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "out of memory";
    case LBM_EDEVICE: return "device error";
    case LBM_ESTATE: return "invalid state";
    case LBM_EUNSTABLE: return "simulation became unstable (non-finite values)";
  }
  return "unknown status";
}

const char* lbm_last_error(void) { return g_last_error.c_str(); }

lbm_status lbm_destroy(lbm_ctx* c) {
  if (!c) return LBM_OK;
  drop_graphs(c);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  host_release(c);
  while (!c->allocs.empty()) dfree(c, c->allocs.back().first);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
  return LBM_OK;
}

lbm_status lbm_create_blocks(const lbm_params* p, const lbm_aabb* blocks, int32_t nblocks, lbm_ctx** out) {
  g_last_error.clear();
  if (!p || !blocks || !out || nblocks <= 0) return fail(LBM_EINVAL, "NULL argument or no blocks");
  for (int k = 0; k < 3; ++k)
    if (p->dims[k] < 1) return fail(LBM_EINVAL, "dims must be >= 1");
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return fail(LBM_EINVAL, "tau must be > 0.5");
  if (!(p->rho0 > 0) || !std::isfinite(p->rho0)) return fail(LBM_EINVAL, "rho0 must be > 0");
  if (p->precision < LBM_F64 || p->precision > LBM_BF16S) return fail(LBM_EINVAL, "bad precision");
  if (p->row_pad < -1 || p->row_pad > 64) return fail(LBM_EINVAL, "row_pad must be in [-1, 64]");
  int open_axis = -1;
  for (int k = 0; k < 3; ++k) {
    if (!std::isfinite(p->force[k])) return fail(LBM_EINVAL, "force must be finite");
    const int f0 = p->face[2 * k], f1 = p->face[2 * k + 1];
    for (const int fk : {f0, f1}) {
      if (fk < LBM_PERIODIC || fk > LBM_PRESSURE) return fail(LBM_EINVAL, "bad face kind");
      if (fk == LBM_VELOCITY || fk == LBM_PRESSURE) {
        if (open_axis >= 0 && open_axis != k)
          return fail(LBM_EINVAL, "VELOCITY and PRESSURE faces lie on one axis");
        open_axis = k;
      }
    }
    if ((f0 == LBM_PERIODIC) != (f1 == LBM_PERIODIC))
      return fail(LBM_EINVAL, "PERIODIC faces come in opposite pairs");
  }
  for (int f = 0; f < 6; ++f) {
    const int axis = f / 2;
    for (int k = 0; k < 3; ++k) {
      const double v = p->wall_u[f][k];
      if (!std::isfinite(v)) return fail(LBM_EINVAL, "wall velocity must be finite");
      if (v != 0.0 && p->face[f] != LBM_VELOCITY && (k == axis || p->face[f] != LBM_WALL))
        return fail(LBM_EINVAL, "wall velocity must be tangential and only on WALL (or VELOCITY) faces");
    }
    if (p->face[f] == LBM_PRESSURE && !(p->face_rho[f] > 0 && std::isfinite(p->face_rho[f])))
      return fail(LBM_EINVAL, "a PRESSURE face needs a finite density > 0");
  }
  std::vector<int> cuts[3], owner;
  std::string err;
  if (!build_tiling(p->dims, blocks, nblocks, cuts, owner, err)) return fail(LBM_EINVAL, err);
  if (open_axis >= 0 && p->dims[open_axis] < 2)
    return fail(LBM_EINVAL, "open faces need at least two cells across them");

  lbm_ctx* c = new lbm_ctx();
  c->p = *p;
  c->prec = p->precision;
  c->f64math = (p->precision == LBM_F64) || (p->precision == LBM_F32 && p->fp64_math);
  c->sbytes = storage_bytes(c->prec);
  c->stream = (hipStream_t)p->stream;
  c->aabb.assign(blocks, blocks + nblocks);
  c->n_cells = (long long)p->dims[0] * p->dims[1] * p->dims[2];
  c->n_fluid = c->n_cells;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(LBM_EDEVICE, "no HIP device");
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess && prop.multiProcessorCount > 0)
    c->cu_count = prop.multiProcessorCount;
  if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return fail(LBM_EDEVICE, "stream creation failed");
  }

  // geometry and physics constants
  for (int k = 0; k < 3; ++k) {
    c->geo.n[k] = p->dims[k];
    c->geo.wall[k] = p->face[2 * k] != LBM_PERIODIC ? 1 : 0;
  }
  for (int f = 0; f < 6; ++f) {
    c->geo.fwall[f] = p->face[f] == LBM_WALL ? 1 : 0;
    c->geo.moving[f] = c->geo.fwall[f] &&
                       (p->wall_u[f][0] != 0.0 || p->wall_u[f][1] != 0.0 || p->wall_u[f][2] != 0.0);
  }
  c->geo.rho0 = p->rho0;
  for (int k = 0; k < 3; ++k) c->geo.hg[k] = 0.5 * p->force[k];
  c->geo.open_axis = open_axis;
  for (int s = 0; s < 6; ++s) {
    c->geo.open[s] = p->face[s] == LBM_VELOCITY ? 1 : (p->face[s] == LBM_PRESSURE ? 2 : 0);
    for (int k = 0; k < 3; ++k) c->geo.ob_u[s][k] = p->face[s] == LBM_VELOCITY ? p->wall_u[s][k] : 0.0;
    c->geo.ob_drho[s] = p->face[s] == LBM_PRESSURE ? p->face_rho[s] - p->rho0 : 0.0;
  }
  const double omega = 1.0 / p->tau;
  c->phd.omega = omega;
  c->phd.rho0 = p->rho0;
  c->phd.inv_rho0 = 1.0 / p->rho0;
  c->phd.fcoef = 1.0 - 0.5 * omega;
  for (int k = 0; k < 3; ++k) {
    c->phd.g[k] = p->force[k];
    c->phd.hg[k] = 0.5 * p->force[k];
  }
  for (int i = 0; i < kQ; ++i)
    for (int f = 0; f < 6; ++f) {
      const double eu = E3[i][0] * p->wall_u[f][0] + E3[i][1] * p->wall_u[f][1] + E3[i][2] * p->wall_u[f][2];
      c->phd.corr[i][f] = 6.0 * weight(i) * p->rho0 * eu;
    }
  c->phd.omc = 1.0 - omega;
  c->phd.rho0x3 = 3.0 * p->rho0;
  for (int i = 0; i < kQ; ++i) {
    const double eg = E3[i][0] * p->force[0] + E3[i][1] * p->force[1] + E3[i][2] * p->force[2];
    c->phd.w[i] = weight(i);
    c->phd.c3w[i] = 3.0 * weight(i) * p->rho0;
    c->phd.c9g[i] = 9.0 * weight(i) * p->rho0 * eg;
    c->phd.cfa[i] = c->phd.fcoef * 3.0 * weight(i) * p->rho0 * eg;
  }
  c->phf.omega = (float)c->phd.omega;
  c->phf.omc = (float)c->phd.omc;
  c->phf.rho0 = (float)c->phd.rho0;
  c->phf.inv_rho0 = (float)c->phd.inv_rho0;
  c->phf.fcoef = (float)c->phd.fcoef;
  c->phf.rho0x3 = (float)c->phd.rho0x3;
  for (int k = 0; k < 3; ++k) {
    c->phf.g[k] = (float)c->phd.g[k];
    c->phf.hg[k] = (float)c->phd.hg[k];
  }
  // FP32 constants chosen so that the discrete moment identities hold
  // exactly for the rounded values: sum_i w_i = 1 and sum_i 3 w_i e_i e_i = I
  // (edge constant rounded, face constant solved from it).  Plain rounding of
  // 1/18, 1/36 leaves a relative bias of ~3e-8 in every step's momentum
  // relaxation, which accumulates over thousands of steps.
  {
    const float we = (float)(1.0 / 36.0);
    const float wf = 2.0f * we;
    const float w0 = (float)(1.0 - 6.0 * (double)wf - 12.0 * (double)we);
    const float c3e = (float)(3.0 / 36.0 * p->rho0);
    const float c3f = (float)((p->rho0 - 8.0 * (double)c3e) / 2.0);
    for (int i = 0; i < kQ; ++i) {
      const int s2 = E3[i][0] * E3[i][0] + E3[i][1] * E3[i][1] + E3[i][2] * E3[i][2];
      const double eg = E3[i][0] * p->force[0] + E3[i][1] * p->force[1] + E3[i][2] * p->force[2];
      c->phf.w[i] = s2 == 0 ? w0 : (s2 == 1 ? wf : we);
      c->phf.c3w[i] = s2 == 0 ? 0.0f : (s2 == 1 ? c3f : c3e);
      c->phf.c9g[i] = (float)(3.0 * (double)c->phf.c3w[i] * eg);
      c->phf.cfa[i] = (float)(c->phd.fcoef * (double)c->phf.c3w[i] * eg);
      for (int f = 0; f < 6; ++f) c->phf.corr[i][f] = (float)c->phd.corr[i][f];
    }
  }
  {
    // FP64 part of the mixed arithmetic (same values in both instantiations)
    auto fill = [&](auto& ph) {
      ph.dinv_rho0 = 1.0 / p->rho0;
      ph.domega = omega;
      ph.domc = 1.0 - omega;
      for (int k = 0; k < 3; ++k) ph.dhg[k] = 0.5 * p->force[k];
      for (int i = 0; i < kQ; ++i) {
        const double eg = E3[i][0] * p->force[0] + E3[i][1] * p->force[1] + E3[i][2] * p->force[2];
        ph.dc3w[i] = 3.0 * weight(i) * p->rho0;
        ph.dcfa[i] = (1.0 - 0.5 * omega) * 3.0 * weight(i) * p->rho0 * eg;
      }
    };
    fill(c->phd);
    fill(c->phf);
  }

  // per-Block layout (see lbm_internal.h)
  const long long align = 128 / c->sbytes;  // elements per 128-byte line
  long long off = 0;
  c->bh.resize(nblocks);
  c->on_host.assign(nblocks, 0);
  c->bfluid.assign(nblocks, 0);
  for (int j = 0; j < nblocks; ++j) {
    BlockDev& B = c->bh[j];
    std::memset(&B, 0, sizeof(B));
    c->bfluid[j] = (long long)(blocks[j].hi[0] - blocks[j].lo[0]) * (blocks[j].hi[1] - blocks[j].lo[1]) *
                   (blocks[j].hi[2] - blocks[j].lo[2]);
    for (int k = 0; k < 3; ++k) {
      B.org[k] = blocks[j].lo[k];
      B.dim[k] = blocks[j].hi[k] - blocks[j].lo[k];
    }
    // A row of an odd number of half lines (FP32 rows of 48 cells: 1.5 lines)
    // padded to whole lines wastes a quarter of the line reads (HBM is read in
    // 128-byte lines): such rows are packed, two rows to three lines, with row
    // 0 of every plane on a line (the plane stride a whole number of lines,
    // the Block's base shifted by half a line); the sweep's items then hold
    // even numbers of rows, so the two halves of a shared line are written by
    // waves of one workgroup.  FP32/FP64 storage, even y extents, row_pad 0.
    B.pack = p->row_pad == 0 && c->prec <= 1 && (B.dim[0] * (long long)c->sbytes) % 128 == 64 && B.dim[1] % 2 == 0;
    B.Sx = B.pack ? B.dim[0]
                  : (int)(roundup(B.dim[0], align) + row_pad_lines(*p, B.dim[0] * (long long)c->sbytes) * align);
    B.Ry = B.dim[1] + 2;
    B.Sz = roundup((long long)B.Sx * (B.dim[1] + 2), align);
    // array (with y/z ghost layer), one spare row, then its x-ghost plane
    B.xgo = B.Sz * (B.dim[2] + 2) + B.Sx;
    const long long fmin = B.xgo + (long long)B.Ry * (B.dim[2] + 2);
    // stagger the 19 streams so they do not start on the same HBM channel
    B.Sf = roundup(fmin, 4096 / c->sbytes) + 768 / c->sbytes;
    B.base = B.pack ? off + (align - B.Sx % align) % align : off;
    off = roundup(B.base + (long long)kQ * B.Sf, 4096 / c->sbytes);
    B.mask = -1;
  }
  // The sweep addresses a row by a scalar base plus 32-bit offsets that
  // reach across one population array (its x-ghost plane included), so one
  // array of a Block must stay below 4 GiB; the obstacle variants' buffer
  // resources span six arrays (checked when obstacles are set).
  for (const auto& B : c->bh)
    if ((long long)B.Sf * c->sbytes >= 0xFFFFFFF0LL) {
      lbm_destroy(c);
      return fail(LBM_EINVAL, "Block too large: one population array of a Block (ghost layers included) "
                              "must stay below 4 GiB (about 530 M cells in FP64, 1070 M in FP32)");
    }
  c->grid_elems = (size_t)off;
  c->x_even = true;
  for (const auto& B : c->bh)
    if (B.dim[0] % 2) c->x_even = false;

  // neighbour table: Block across each face/edge/corner, with translation
  c->nbh.assign((size_t)nblocks * 27, NbrDev{-1, 0, 0, 0});
  const int gsz[3] = {(int)cuts[0].size() - 1, (int)cuts[1].size() - 1, (int)cuts[2].size() - 1};
  for (int j = 0; j < nblocks; ++j) {
    for (int d = 0; d < 27; ++d) {
      if (d == 13) continue;
      const int off3[3] = {d % 3 - 1, (d / 3) % 3 - 1, d / 9 - 1};
      int rep[3], q[3];
      bool ok = true;
      for (int k = 0; k < 3; ++k) {
        rep[k] = off3[k] < 0 ? blocks[j].lo[k] : (off3[k] > 0 ? blocks[j].hi[k] - 1 : blocks[j].lo[k]);
        q[k] = rep[k] + off3[k];
        if (q[k] < 0 || q[k] >= p->dims[k]) {
          if (c->geo.wall[k]) ok = false;
          else q[k] = (q[k] + p->dims[k]) % p->dims[k];
        }
      }
      if (!ok) continue;
      const int s0 = slot_of(cuts[0], q[0]), s1 = slot_of(cuts[1], q[1]), s2 = slot_of(cuts[2], q[2]);
      const int m = owner[((size_t)s2 * gsz[1] + s1) * gsz[0] + s0];
      NbrDev& nb = c->nbh[(size_t)j * 27 + d];
      nb.id = m;
      // rep in m's frame is q - org_m - off; in j's frame it is rep - org_j
      nb.tx = (q[0] - blocks[m].lo[0] - off3[0]) - (rep[0] - blocks[j].lo[0]);
      nb.ty = (q[1] - blocks[m].lo[1] - off3[1]) - (rep[1] - blocks[j].lo[1]);
      nb.tz = (q[2] - blocks[m].lo[2] - off3[2]) - (rep[2] - blocks[j].lo[2]);
    }
  }

  // Axes on which a Block is its own neighbour across both faces: the sweep
  // reads across them from the Block itself (no ghost values, no copies).
  // y only where every wave holds one row of the Block, so that the wrap is
  // uniform per wave: x extent > 64 (also with two cells per lane), or 64
  // where the storage mode never runs two cells per lane.
  const bool vec2_possible = sweep_vec2_ok(c->prec, c->f64math);
  for (int j = 0; j < nblocks; ++j) {
    BlockDev& B = c->bh[j];
    B.wrap = 0;
    const int st[3] = {1, 3, 9};
    for (int k = 0; k < 3; ++k) {
      const bool self = c->nbh[(size_t)j * 27 + 13 - st[k]].id == j && c->nbh[(size_t)j * 27 + 13 + st[k]].id == j;
      const bool one_row = B.dim[0] > 64 || (B.dim[0] == 64 && !vec2_possible);
      if (self && (k != 1 || one_row)) B.wrap |= 1 << k;
    }
  }

  // measured on gfx950: one Block exchanges cheapest with the copy kernel
  // alone; several Blocks with the x faces written by the sweep (mode 2),
  // whose rim leaves the copy kernel contiguous rows.  The fully fused
  // epilogue (mode 1) holds the sweep to fewer resident waves.
  c->sched.fused_exchange = nblocks > 1 ? 2 : 0;
  c->sched.item_cells = 512;
  c->sched.wg_size = 256;
  c->sched.persistent = 0;
  c->sched.graph_steps = 0;
  // streaming row stores, except for grids that the 256 MB memory-side
  // cache holds from one step to the next (measured on gfx950: the 128^3
  // FP32 grid of 159 MB 7 % faster with ordinary stores; 144^3, 227 MB,
  // 8 % slower)
  c->sched.nontemporal = c->grid_elems * c->sbytes > (192u << 20) ? 1 : 0;
  c->sched.cells_per_lane = 0;
  build_items(c);
  build_tasks(c);

  auto bail = [&](lbm_status s, const char* msg) {
    lbm_destroy(c);
    return fail(s, msg);
  };
  const size_t gbytes = c->grid_elems * c->sbytes;
  c->grid[0] = dalloc(c, gbytes);
  c->grid[1] = dalloc(c, gbytes);
  c->d_blocks = (BlockDev*)dalloc(c, sizeof(BlockDev) * nblocks);
  c->d_nbr = (NbrDev*)dalloc(c, sizeof(NbrDev) * c->nbh.size());
  c->d_ghost = (GhostTgt*)dalloc(c, sizeof(GhostTgt) * c->nbh.size());
  c->d_tasks = (XchgTask*)dalloc(c, sizeof(XchgTask) * std::max<size_t>(1, c->tasks_h.size()));
  c->d_rim = (XchgTask*)dalloc(c, sizeof(XchgTask) * std::max<size_t>(1, c->rim_h.size()));
  c->d_partial = (double*)dalloc(c, sizeof(double) * 6 * c->nparts);
  c->d_red = (double*)dalloc(c, sizeof(double) * 8);
  if (open_axis >= 0) {
    const int t1 = open_axis == 0 ? 1 : 0, t2 = open_axis == 2 ? 1 : 2;
    c->d_side = (double*)dalloc(c, sizeof(double) * 32 * (size_t)p->dims[t1] * p->dims[t2]);
  }
    c->d_faceblk = (int*)dalloc(c, sizeof(int) * 2 * (1 + (size_t)nblocks));
  if (!c->grid[0] || !c->grid[1] || !c->d_blocks || !c->d_nbr || !c->d_ghost || !c->d_tasks || !c->d_rim ||
      !c->d_partial || !c->d_red || (open_axis >= 0 && (!c->d_side || !c->d_faceblk)))
    return bail(LBM_ENOMEM, "device allocation failed");
  if (hipMemcpy(c->d_blocks, c->bh.data(), sizeof(BlockDev) * nblocks, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_nbr, c->nbh.data(), sizeof(NbrDev) * c->nbh.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_ghost, build_ghost_table(c).data(), sizeof(GhostTgt) * c->nbh.size(),
                hipMemcpyHostToDevice) != hipSuccess ||
      (!c->tasks_h.empty() && hipMemcpy(c->d_tasks, c->tasks_h.data(), sizeof(XchgTask) * c->tasks_h.size(),
                                        hipMemcpyHostToDevice) != hipSuccess) ||
      (!c->rim_h.empty() && hipMemcpy(c->d_rim, c->rim_h.data(), sizeof(XchgTask) * c->rim_h.size(),
                                      hipMemcpyHostToDevice) != hipSuccess))
    return bail(LBM_EDEVICE, "upload of block tables failed");
  if (c->d_faceblk) {
    // the Blocks touching each open face
    std::vector<int> fl((size_t)2 * (1 + nblocks), 0);
    const int a = open_axis;
    for (int f = 0; f < 2; ++f)
      for (int j = 0; j < nblocks; ++j) {
        const BlockDev& B = c->bh[j];
        if (f == 0 ? B.org[a] == 0 : B.org[a] + B.dim[a] == p->dims[a]) {
          int* list = fl.data() + (size_t)f * (1 + nblocks);
          list[1 + list[0]] = j;
          ++list[0];
        }
      }
    if (hipMemcpy(c->d_faceblk, fl.data(), sizeof(int) * fl.size(), hipMemcpyHostToDevice) != hipSuccess)
      return bail(LBM_EDEVICE, "upload of block tables failed");
  }
  if (upload_items(c) != LBM_OK) return bail(LBM_ENOMEM, "item list upload failed");
  if (zero_grids(c) != LBM_OK) return bail(LBM_EDEVICE, "grid initialisation failed");
  // rest state: bounce-back slots of moving walls carry the wall term
  enqueue_slots(c, 0, c->stream);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
    return bail(LBM_EDEVICE, "grid initialisation failed");
  *out = c;
  return LBM_OK;
}

lbm_status lbm_set_geometry(lbm_ctx* c, const uint8_t* solid) {
  if (!c) return fail(LBM_EINVAL, "NULL context");
  if (solid && has_open(c)) {
    // the boundary node of an open face extrapolates from a fluid cell
    const int a = c->geo.open_axis, nx = c->geo.n[0], ny = c->geo.n[1];
    for (long long k = 0; k < c->n_cells; ++k) {
      const int p[3] = {(int)(k % nx), (int)(k / nx % ny), (int)(k / ((long long)nx * ny))};
      if (solid[k] && ((c->geo.open[2 * a] && p[a] == 0) || (c->geo.open[2 * a + 1] && p[a] == c->geo.n[a] - 1)))
        return fail(LBM_EINVAL, "solid cell on an open face");
    }
  }
  bool any = false;
  long long nsolid = 0;
  if (solid) {
    for (long long k = 0; k < c->n_cells; ++k)
      if (solid[k]) ++nsolid;
    any = nsolid > 0;
  }
  if (any)
    for (const auto& B : c->bh)
      if (6LL * B.Sf * c->sbytes >= 0xFFFFFFF0LL)
        return fail(LBM_EINVAL, "Block too large for obstacles: six population arrays of a Block (ghost layers "
                                "included) must stay below 4 GiB (about 89 M cells in FP64, 178 M in FP32, "
                                "357 M in 16-bit storage)");
  drop_graphs(c);
  if (any) {
    if (!c->d_mask) {
      long long moff = 0;
      for (auto& B : c->bh) {
        B.mask = moff;
        moff += (long long)B.dim[0] * B.dim[1] * B.dim[2];
      }
      c->d_mask = (uint32_t*)dalloc(c, sizeof(uint32_t) * moff);
      if (!c->d_mask) {
        for (auto& B : c->bh) B.mask = -1;
        return fail(LBM_ENOMEM, "link-mask allocation failed");
      }
      HIPCHK(hipMemcpy(c->d_blocks, c->bh.data(), sizeof(BlockDev) * c->bh.size(), hipMemcpyHostToDevice));
    }
    lbm_status s = ensure_stage(c, (size_t)c->n_cells);
    if (s != LBM_OK) return s;
    HIPCHK(hipMemcpyAsync(c->d_stage, solid, (size_t)c->n_cells, hipMemcpyHostToDevice, c->stream));
    c->has_mask = true;
    CellArgs a = cell_args(c);
    a.has_mask = 0;
    launch_linkmask((const uint8_t*)c->d_stage, a, c->d_mask, c->stream);
    HIPCHK(hipGetLastError());
  } else {
    c->has_mask = false;
  }
  c->n_fluid = c->n_cells - nsolid;
  lbm_status s = zero_grids(c);
  if (s != LBM_OK) return s;
  enqueue_slots(c, 0, c->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  c->cur = 0;
  c->steps = 0;
  c->mark_steps = -1;
  c->set_steps = 0;
  // fluid cells per Block (static load balance)
  for (size_t j = 0; j < c->bh.size(); ++j) {
    const lbm_aabb& A = c->aabb[j];
    long long nf = (long long)(A.hi[0] - A.lo[0]) * (A.hi[1] - A.lo[1]) * (A.hi[2] - A.lo[2]);
    if (solid)
      for (int z = A.lo[2]; z < A.hi[2]; ++z)
        for (int y = A.lo[1]; y < A.hi[1]; ++y)
          for (int x = A.lo[0]; x < A.hi[0]; ++x)
            nf -= solid[((long long)z * c->geo.n[1] + y) * c->geo.n[0] + x] != 0;
    c->bfluid[j] = nf;
  }
  return host_pull(c);
}

lbm_status lbm_set_equilibrium(lbm_ctx* c, const double* rho, const double* u) {
  if (!c || !rho || !u) return fail(LBM_EINVAL, "NULL argument");
  const size_t N = (size_t)c->n_cells;
  lbm_status s = ensure_stage(c, 4 * N * sizeof(double));
  if (s != LBM_OK) return s;
  double* d = (double*)c->d_stage;
  HIPCHK(hipMemcpyAsync(d, rho, N * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(d + N, u, 3 * N * sizeof(double), hipMemcpyHostToDevice, c->stream));
  launch_init_eq(c->prec, c->grid[c->cur], cell_args(c), c->p.rho0, d, d + N, (long long)N, c->stream);
  enqueue_fill(c, c->cur, c->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  c->steps = 0;
  c->mark_steps = -1;
  c->set_steps = 0;
  return host_pull(c);
}

lbm_status lbm_step(lbm_ctx* c, int64_t n) {
  if (!c) return fail(LBM_EINVAL, "NULL context");
  if (n < 0) return fail(LBM_EINVAL, "negative step count");
  return run_steps(c, n);
}

lbm_status lbm_step_persistent(lbm_ctx* c, int64_t n, int32_t steps_per_launch) {
  if (!c || n < 0) return fail(LBM_EINVAL, "NULL context or negative step count");
  if (hetero(c)) return fail(LBM_EINVAL, "the persistent sweep runs every Block on the GPU");
  if (has_open(c)) return fail(LBM_EINVAL, "the persistent sweep has no pass for the boundary nodes of open faces");
  if (cells_per_lane(c, c->sched) != 1) return fail(LBM_EINVAL, "the persistent sweep takes one cell per lane");
  if (steps_per_launch < 1 || steps_per_launch > (1 << 20))
    return fail(LBM_EINVAL, "steps_per_launch must be in [1, 2^20]");
  while (n > 0) {
    const int k = (int)std::min<int64_t>(n, steps_per_launch);
    const SweepArgs a = sweep_args(c, c->cur);
    if (a.nitems > 0) {
      hipError_t e = launch_sweep_steps(c->prec, c->f64math, c->has_mask, a, c->phd, c->phf, k, c->cu_count,
                                        c->stream);
      if (e != hipSuccess)
        return fail(LBM_EDEVICE, std::string("cooperative launch of the persistent sweep: ") + hipGetErrorString(e));
    }
    if (k & 1) c->cur = 1 - c->cur;
    c->steps += k;
    n -= k;
  }
  HIPCHK(hipGetLastError());
  return LBM_OK;
}

lbm_status lbm_step_timed(lbm_ctx* c, int64_t n, double* sweep_ms, double* exchange_ms) {
  if (!c || !sweep_ms || !exchange_ms) return fail(LBM_EINVAL, "NULL argument");
  if (n < 1 || n > 100000) return fail(LBM_EINVAL, "step count must be in [1, 100000]");
  if (hetero(c)) {
    // wall-clock phases: both sweeps, then the exchange
    HostTimes tm;
    lbm_status st = host_steps(c, n, &tm);
    if (st != LBM_OK) return st;
    *sweep_ms = (tm.step - tm.xchg) / (double)n;
    *exchange_ms = tm.xchg / (double)n;
    return LBM_OK;
  }
  const bool ex = c->sched.fused_exchange != 1 || has_open(c);
  const size_t ne = (size_t)n * (ex ? 3 : 2);
  std::vector<hipEvent_t> ev(ne, nullptr);
  lbm_status st = LBM_OK;
  for (size_t k = 0; k < ne && st == LBM_OK; ++k)
    if (hipEventCreate(&ev[k]) != hipSuccess) st = fail(LBM_EDEVICE, "hipEventCreate failed");
  double ts = 0.0, te = 0.0;
  if (st == LBM_OK) {
    size_t k = 0;
    for (int64_t j = 0; j < n; ++j) {
      (void)hipEventRecord(ev[k++], c->stream);
      enqueue_sweep(c, c->cur, c->stream);
      (void)hipEventRecord(ev[k++], c->stream);
      if (ex) {
        enqueue_post(c, 1 - c->cur, c->stream);
        (void)hipEventRecord(ev[k++], c->stream);
      }
      c->cur = 1 - c->cur;
      c->steps += 1;
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
      st = fail(LBM_EDEVICE, "timed steps failed");
    for (size_t b = 0; st == LBM_OK && b < ne; b += ex ? 3 : 2) {
      float t0 = 0.f, t1 = 0.f;
      if (hipEventElapsedTime(&t0, ev[b], ev[b + 1]) != hipSuccess ||
          (ex && hipEventElapsedTime(&t1, ev[b + 1], ev[b + 2]) != hipSuccess))
        st = fail(LBM_EDEVICE, "hipEventElapsedTime failed");
      ts += t0;
      te += t1;
    }
  }
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  if (st != LBM_OK) return st;
  *sweep_ms = ts / (double)n;
  *exchange_ms = ex ? te / (double)n : 0.0;
  return LBM_OK;
}

lbm_status lbm_macroscopic(lbm_ctx* c, double* rho, double* u, int32_t dst_is_device) {
  if (!c || !rho || !u) return fail(LBM_EINVAL, "NULL argument");
  lbm_status hs = host_push(c);
  if (hs != LBM_OK) return hs;
  const size_t N = (size_t)c->n_cells;
  double hg[3];
  half_force(c, c->steps >= 1, hg);
  double *dr = rho, *du = u;
  if (!dst_is_device) {
    lbm_status s = ensure_stage(c, 4 * N * sizeof(double));
    if (s != LBM_OK) return s;
    dr = (double*)c->d_stage;
    du = dr + N;
  }
  launch_macro(c->prec, c->grid[c->cur], cell_args(c), c->p.rho0, hg, dr, du, (long long)N, c->stream);
  HIPCHK(hipGetLastError());
  if (!dst_is_device) {
    HIPCHK(hipMemcpyAsync(rho, dr, N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(u, du, 3 * N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_residual(lbm_ctx* c, double* r) {
  if (!c || !r) return fail(LBM_EINVAL, "NULL argument");
  if (c->steps < 2) return fail(LBM_ESTATE, "residual needs >= 2 steps since initialisation");
  if (c->steps == c->set_steps) return fail(LBM_ESTATE, "residual needs a step since the state was last set");
  double s[6];
  lbm_status st = reduce(c, 1, s);
  if (st != LBM_OK) return st;
  *r = std::sqrt(s[4]) / std::sqrt(s[5]);
  if (!std::isfinite(*r)) *r = s[4] == 0.0 ? 0.0 : INFINITY;
  return LBM_OK;
}

lbm_status lbm_residual_mark(lbm_ctx* c) {
  if (!c) return fail(LBM_EINVAL, "NULL context");
  if (!c->d_umark) {
    c->d_umark = (double*)dalloc(c, 4 * (size_t)c->n_cells * sizeof(double));
    if (!c->d_umark) return fail(LBM_ENOMEM, "velocity snapshot allocation failed");
  }
  lbm_status hs = host_push(c);
  if (hs != LBM_OK) return hs;
  double hg[3];
  half_force(c, c->steps >= 1, hg);
  launch_macro(c->prec, c->grid[c->cur], cell_args(c), c->p.rho0, hg, c->d_umark, c->d_umark + c->n_cells,
               c->n_cells, c->stream);
  HIPCHK(hipGetLastError());
  c->mark_steps = c->steps;
  return LBM_OK;
}

lbm_status lbm_residual_since_mark(lbm_ctx* c, double* r, int64_t* nsteps) {
  if (!c || !r) return fail(LBM_EINVAL, "NULL argument");
  if (c->mark_steps < 0) return fail(LBM_ESTATE, "no velocity snapshot since the last (re)initialisation");
  double s[6];
  lbm_status st = reduce(c, 2, s);
  if (st != LBM_OK) return st;
  *r = std::sqrt(s[4]) / std::sqrt(s[5]);
  if (!std::isfinite(*r)) *r = s[4] == 0.0 ? 0.0 : INFINITY;
  if (nsteps) *nsteps = c->steps - c->mark_steps;
  return LBM_OK;
}

lbm_status lbm_sums(lbm_ctx* c, double* mass, double mom[3]) {
  if (!c || !mass || !mom) return fail(LBM_EINVAL, "NULL argument");
  double s[6];
  lbm_status st = reduce(c, 0, s);
  if (st != LBM_OK) return st;
  *mass = (double)c->n_fluid * c->p.rho0 + s[0];
  mom[0] = s[1];
  mom[1] = s[2];
  mom[2] = s[3];
  return LBM_OK;
}

lbm_status lbm_sums_noalloc(lbm_ctx* c, double* mass, double mom[3]) {
  if (!c || !mass || !mom) return fail(LBM_EINVAL, "NULL argument");
  double* sp = nullptr;
  lbm_status st = scratch_ptr(c->device, &sp);
  if (st != LBM_OK) return st;
  constexpr int kMaxParts = (int)((kScratchDoubles - 8) / 6);
  double s[6];
  st = reduce(c, 0, s, sp, sp + 6 * kMaxParts, kMaxParts);
  if (st != LBM_OK) return st;
  *mass = (double)c->n_fluid * c->p.rho0 + s[0];
  mom[0] = s[1];
  mom[1] = s[2];
  mom[2] = s[3];
  return LBM_OK;
}

lbm_status lbm_get_state(lbm_ctx* c, void* f, int32_t as_fp64) {
  if (!c || !f) return fail(LBM_EINVAL, "NULL argument");
  lbm_status hs = host_push(c);
  if (hs != LBM_OK) return hs;
  const size_t N = (size_t)c->n_cells;
  const size_t bytes = (size_t)kQ * N * (as_fp64 ? sizeof(double) : c->sbytes);
  lbm_status s = ensure_stage(c, bytes);
  if (s != LBM_OK) return s;
  launch_get_state(c->prec, as_fp64 != 0, c->grid[c->cur], cell_args(c), c->d_stage, (long long)N, c->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(f, c->d_stage, bytes, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_set_state(lbm_ctx* c, const void* f, int32_t as_fp64) {
  if (!c || !f) return fail(LBM_EINVAL, "NULL argument");
  const size_t N = (size_t)c->n_cells;
  const size_t bytes = (size_t)kQ * N * (as_fp64 ? sizeof(double) : c->sbytes);
  lbm_status s = ensure_stage(c, bytes);
  if (s != LBM_OK) return s;
  HIPCHK(hipMemcpyAsync(c->d_stage, f, bytes, hipMemcpyHostToDevice, c->stream));
  launch_set_state(c->prec, as_fp64 != 0, c->grid[c->cur], cell_args(c), c->d_stage, (long long)N, c->stream);
  enqueue_fill(c, c->cur, c->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  c->steps = 1;
  c->mark_steps = -1;
  c->set_steps = 1;
  return host_pull(c);
}

lbm_status lbm_average_two_steps(lbm_ctx* c) {
  if (!c) return fail(LBM_EINVAL, "NULL context");
  if (hetero(c)) return fail(LBM_EINVAL, "averaging two steps needs every Block on the GPU");
  if (c->steps <= c->set_steps)
    return fail(LBM_ESTATE, "averaging two steps needs a step since the state was last set");
  launch_average(c->prec, c->grid[c->cur], c->grid[c->cur ^ 1], (long long)c->grid_elems, c->stream);
  enqueue_fill(c, c->cur, c->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  c->set_steps = c->steps;
  return LBM_OK;
}

lbm_status lbm_get_schedule(lbm_ctx* c, lbm_schedule* s) {
  if (!c || !s) return fail(LBM_EINVAL, "NULL argument");
  *s = c->sched;
  return LBM_OK;
}

lbm_status lbm_set_schedule(lbm_ctx* c, const lbm_schedule* s) {
  if (!c || !s) return fail(LBM_EINVAL, "NULL argument");
  std::string err;
  if (!sched_valid(*s, err)) return fail(LBM_EINVAL, err);
  if (s->cells_per_lane == 2 && !vec2_allowed(c))
    return fail(LBM_EINVAL,
                "two cells per lane need F16S/BF16S (or F32 with FP64 math), even x extents and no open x faces");
  HIPCHK(hipStreamSynchronize(c->stream));
  drop_graphs(c);
  const lbm_schedule old = c->sched;
  c->sched = *s;
  build_items(c);
  lbm_status st = upload_items(c);
  if (st != LBM_OK) {
    c->sched = old;
    build_items(c);
    (void)upload_items(c);
    return st;
  }
  return LBM_OK;
}

lbm_status lbm_info_get(lbm_ctx* c, lbm_info* info) {
  if (!c || !info) return fail(LBM_EINVAL, "NULL argument");
  HIPCHK(hipStreamSynchronize(c->stream));
  info->n_cells = c->n_cells;
  info->n_fluid = c->n_fluid;
  info->n_blocks = (int32_t)c->bh.size();
  info->n_items = (int32_t)c->items_h.size();
  info->steps = c->steps;
  info->device_bytes = (int64_t)c->held;
  info->storage_bytes = c->sbytes;
  info->has_obstacles = c->has_mask ? 1 : 0;
  info->bytes_per_update = 2.0 * kQ * c->sbytes;
  if (c->has_mask) info->bytes_per_update += 4.0 * (double)c->n_cells / (double)std::max(1LL, c->n_fluid);
  return LBM_OK;
}

lbm_status lbm_set_host_blocks(lbm_ctx* c, const int32_t* ids, int32_t n, int32_t threads) {
  if (!c) return fail(LBM_EINVAL, "NULL context");
  const int nb = (int)c->bh.size();
  if (n < 0 || n > nb || (n > 0 && !ids)) return fail(LBM_EINVAL, "host Block list: bad count or NULL list");
  if (threads < 0 || threads > 1024) return fail(LBM_EINVAL, "threads must be in [0, 1024]");
  std::vector<int> list(ids, ids + n);
  std::vector<char> seen(nb, 0);
  for (int j : list) {
    if (j < 0 || j >= nb || seen[j]) return fail(LBM_EINVAL, "host Block ids must be distinct BlockIDs");
    seen[j] = 1;
  }
  if (n > 0 && c->prec > 1) return fail(LBM_EINVAL, "host Blocks hold FP64 or FP32 storage");
  if (n > 0 && has_open(c)) return fail(LBM_EINVAL, "host Blocks need a lattice without open faces");
  HIPCHK(hipStreamSynchronize(c->stream));
  drop_graphs(c);
  // the whole state back on the device, then the new split
  lbm_status st = host_push(c);
  if (st != LBM_OK) return st;
  host_release(c);
  build_items(c);
  st = upload_items(c);
  if (st != LBM_OK || n == 0) return st;
  st = host_setup(c, list, threads);
  if (st != LBM_OK) {
    host_release(c);
    build_items(c);
    (void)upload_items(c);
  }
  return st;
}

lbm_status lbm_step_host_timed(lbm_ctx* c, int64_t n, double* gpu_sweep_ms, double* cpu_sweep_ms,
                               double* exchange_ms, double* step_ms) {
  if (!c || !gpu_sweep_ms || !cpu_sweep_ms || !exchange_ms || !step_ms) return fail(LBM_EINVAL, "NULL argument");
  if (n < 1 || n > 100000) return fail(LBM_EINVAL, "step count must be in [1, 100000]");
  if (!hetero(c)) return fail(LBM_ESTATE, "no Block runs on the host");
  HostTimes tm;
  lbm_status st = host_steps(c, n, &tm);
  if (st != LBM_OK) return st;
  *gpu_sweep_ms = tm.gpu / (double)n;
  *cpu_sweep_ms = tm.cpu / (double)n;
  *exchange_ms = tm.xchg / (double)n;
  *step_ms = tm.step / (double)n;
  return LBM_OK;
}

lbm_status lbm_balance_host_blocks(lbm_ctx* c, int32_t threads, int32_t trial_steps, int32_t* n_host,
                                   double* ms_gpu_only, double* ms_balanced) {
  if (!c || !n_host) return fail(LBM_EINVAL, "NULL argument");
  if (trial_steps < 1 || trial_steps > 10000) return fail(LBM_EINVAL, "trial_steps must be in [1, 10000]");
  if (threads < 0 || threads > 1024) return fail(LBM_EINVAL, "threads must be in [0, 1024]");
  if (c->prec > 1 || has_open(c)) return fail(LBM_EINVAL, "host Blocks need FP64/FP32 storage and no open faces");
  const int nb = (int)c->bh.size();
  auto wall = [&](double* ms) -> lbm_status {
    lbm_status s = run_steps(c, 2);
    if (s != LBM_OK) return s;
    HIPCHK(hipStreamSynchronize(c->stream));
    const auto t0 = std::chrono::steady_clock::now();
    s = run_steps(c, trial_steps);
    if (s != LBM_OK) return s;
    HIPCHK(hipStreamSynchronize(c->stream));
    *ms = ms_since(t0) / trial_steps;
    return LBM_OK;
  };
  // every Block on the GPU, and the state saved: the trials advance a copy
  // of the simulation
  lbm_status st = lbm_set_host_blocks(c, nullptr, 0, 0);
  if (st != LBM_OK) return st;
  const size_t gbytes = c->grid_elems * c->sbytes;
  void* save = dalloc(c, 2 * gbytes);
  if (!save) return fail(LBM_ENOMEM, "balance backup allocation failed");
  HIPCHK(hipMemcpyAsync(save, c->grid[0], gbytes, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync((char*)save + gbytes, c->grid[1], gbytes, hipMemcpyDeviceToDevice, c->stream));
  const int cur0 = c->cur;
  const long long steps0 = c->steps;
  double tg = 0.0, th = 0.0;
  int k = 0;
  st = wall(&tg);
  // the CPU's rate on the last Block of the list
  int32_t last = nb - 1;
  if (st == LBM_OK) st = lbm_set_host_blocks(c, &last, 1, threads);
  if (st == LBM_OK) st = run_steps(c, 2);
  double g = 0, cpu = 0, x = 0, sm = 0;
  if (st == LBM_OK) st = lbm_step_host_timed(c, trial_steps, &g, &cpu, &x, &sm);
  if (st == LBM_OK) {
    const double rate_c = (double)std::max(1LL, c->bfluid[last]) / std::max(cpu, 1e-6);
    const double rate_g = (double)std::max(1LL, c->n_fluid) / std::max(tg, 1e-6);
    // the last k Blocks of the list, k as large as keeps the CPU's sweep no
    // longer than the GPU's share (the Block counts per process of Sec. 5.3)
    long long fh = 0;
    while (k < nb - 1) {
      const long long f2 = fh + c->bfluid[nb - 1 - k];
      if ((double)f2 / rate_c > (double)(c->n_fluid - f2) / rate_g) break;
      fh = f2;
      ++k;
    }
    th = sm;  // k = 0: one Block on the host already outruns the GPU
    if (k > 0) {
      std::vector<int32_t> ids;
      for (int j = nb - k; j < nb; ++j) ids.push_back(j);
      st = lbm_set_host_blocks(c, ids.data(), k, threads);
      if (st == LBM_OK) st = wall(&th);
    }
    if (k > 0 && th >= tg) k = 0;
  }
  // restore the simulation, then apply the split
  lbm_status s2 = lbm_set_host_blocks(c, nullptr, 0, 0);
  (void)hipStreamSynchronize(c->stream);
  (void)hipMemcpyAsync(c->grid[0], save, gbytes, hipMemcpyDeviceToDevice, c->stream);
  (void)hipMemcpyAsync(c->grid[1], (char*)save + gbytes, gbytes, hipMemcpyDeviceToDevice, c->stream);
  (void)hipStreamSynchronize(c->stream);
  dfree(c, save);
  c->cur = cur0;
  c->steps = steps0;
  if (st == LBM_OK) st = s2;
  if (st != LBM_OK) return st;
  if (k > 0) {
    std::vector<int32_t> ids;
    for (int j = nb - k; j < nb; ++j) ids.push_back(j);
    st = lbm_set_host_blocks(c, ids.data(), k, threads);
    if (st != LBM_OK) return st;
  }
  *n_host = k;
  if (ms_gpu_only) *ms_gpu_only = tg;
  if (ms_balanced) *ms_balanced = th;
  return LBM_OK;
}

lbm_status lbm_autotune(lbm_ctx* c, const char* cache_path, int32_t trial_steps, lbm_schedule* chosen) {
  if (!c) return fail(LBM_EINVAL, "NULL context");
  if (hetero(c)) return fail(LBM_EINVAL, "the autotuner times schedules with every Block on the GPU");
  if (trial_steps < 1) trial_steps = 10;
  // problem signature
  std::ostringstream key;
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, c->device));
  key << prop.gcnArchName << "|p" << c->prec << "m" << c->f64math << "o" << c->has_mask << "|" << c->p.dims[0]
      << "x" << c->p.dims[1] << "x" << c->p.dims[2] << "|nb" << c->bh.size() << "|f";
  // face kinds (open faces restrict the sweep variants) and row padding
  for (int f = 0; f < 6; ++f) key << (int)c->p.face[f];
  key << "|r" << c->p.row_pad;
  {
    unsigned long long h = 1469598103934665603ULL;
    for (const auto& b : c->aabb)
      for (int k = 0; k < 3; ++k) {
        h = (h ^ (unsigned long long)b.lo[k]) * 1099511628211ULL;
        h = (h ^ (unsigned long long)b.hi[k]) * 1099511628211ULL;
      }
    key << "|h" << std::hex << h;
  }
  const std::string k = key.str();
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string kk;
      lbm_schedule s{};
      if (ls >> kk >> s.fused_exchange >> s.item_cells >> s.wg_size >> s.persistent >> s.graph_steps >>
          s.nontemporal >> s.cells_per_lane) {
        std::string err;
        // a cached schedule this context refuses (a hand-edited or foreign
        // line) is skipped, and the search runs
        if (kk == k && sched_valid(s, err) && (s.cells_per_lane != 2 || vec2_allowed(c))) {
          s.graph_steps = c->sched.graph_steps;
          lbm_status st = lbm_set_schedule(c, &s);
          if (st == LBM_OK) {
            if (chosen) *chosen = s;
            return st;
          }
        }
      }
    }
  }
  // save both grids; the trials advance a copy of the simulation
  HIPCHK(hipStreamSynchronize(c->stream));
  const size_t gbytes = c->grid_elems * c->sbytes;
  void* save = dalloc(c, 2 * gbytes);
  if (!save) return fail(LBM_ENOMEM, "autotune backup allocation failed");
  HIPCHK(hipMemcpyAsync(save, c->grid[0], gbytes, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync((char*)save + gbytes, c->grid[1], gbytes, hipMemcpyDeviceToDevice, c->stream));
  const int cur0 = c->cur;
  const long long steps0 = c->steps;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  auto timeit = [&](const lbm_schedule& s, double* ms) -> lbm_status {
    lbm_status st = lbm_set_schedule(c, &s);
    if (st != LBM_OK) return st;
    st = run_steps(c, 2);
    if (st != LBM_OK) return st;
    HIPCHK(hipEventRecord(e0, c->stream));
    st = run_steps(c, trial_steps);
    if (st != LBM_OK) return st;
    HIPCHK(hipEventRecord(e1, c->stream));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    *ms = t / trial_steps;
    return LBM_OK;
  };
  lbm_schedule best = c->sched;
  double best_ms = 1e30;
  lbm_status st = timeit(best, &best_ms);
  // coordinate descent over the schedule knobs
  const std::vector<int> cells = {128, 256, 512, 1024, 2048, 4096};
  const std::vector<int> wgs = {64, 128, 256};
  const std::vector<int> pers = {0, 2, 4, 8, 16};
  for (int pass = 0; pass < 2 && st == LBM_OK; ++pass) {
    for (int knob = 0; knob < 6 && st == LBM_OK; ++knob) {
      std::vector<lbm_schedule> cand;
      for (size_t q = 0;
           q < (knob == 0 ? cells.size() : knob == 1 ? wgs.size() : knob == 2 ? pers.size() : knob == 4 ? 3 : 2);
           ++q) {
        lbm_schedule s = best;
        if (knob == 0) s.item_cells = cells[q];
        if (knob == 1) s.wg_size = wgs[q];
        if (knob == 2) s.persistent = pers[q];
        if (knob == 3) s.nontemporal = (int)q;
        if (knob == 4) s.fused_exchange = (int)q;
        if (knob == 5) {
          if (!vec2_allowed(c)) continue;
          s.cells_per_lane = (int)q + 1;
        }
        cand.push_back(s);
      }
      for (const auto& s : cand) {
        double ms = 0;
        st = timeit(s, &ms);
        if (st != LBM_OK) break;
        if (ms < best_ms * 0.995) {
          best_ms = ms;
          best = s;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // restore the simulation
  (void)hipStreamSynchronize(c->stream);
  (void)hipMemcpyAsync(c->grid[0], save, gbytes, hipMemcpyDeviceToDevice, c->stream);
  (void)hipMemcpyAsync(c->grid[1], (char*)save + gbytes, gbytes, hipMemcpyDeviceToDevice, c->stream);
  (void)hipStreamSynchronize(c->stream);
  dfree(c, save);
  c->cur = cur0;
  c->steps = steps0;
  if (st != LBM_OK) return st;
  best.graph_steps = c->sched.graph_steps;
  st = lbm_set_schedule(c, &best);
  if (st != LBM_OK) return st;
  if (cache_path) {
    std::ofstream o(cache_path, std::ios::app);
    if (o) o << k << " " << sched_str(best) << "\n";
  }
  if (chosen) *chosen = best;
  return LBM_OK;
}

lbm_status lbm_bw_probe(void* dst, const void* src, size_t bytes, int32_t reps, void* stream, double* ms) {
  if (!dst || !src || !ms || bytes == 0 || (bytes % 16) != 0 || reps < 1)
    return fail(LBM_EINVAL, "bad probe arguments");
  hipStream_t s = (hipStream_t)stream;
  int dev = 0, cus = 256;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
  const long long n16 = (long long)(bytes / 16);
  const int grid = (int)std::min<long long>((n16 + 255) / 256, (long long)cus * 16);
  launch_copy16(src, dst, n16, grid, s);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r) launch_copy16(src, dst, n16, grid, s);
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float t = 0;
  HIPCHK(hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = t / reps;
  return LBM_OK;
}

}  // extern "C"
