// lbm_host.cpp -- the host-CPU side of heterogeneous runs (Sec. 4.5).
//
// Blocks assigned to the CPU run this sweep on host memory laid out exactly
// as on the GPU (SoA arrays with y/z ghost rows and x-ghost planes), and the
// exchange between a CPU Block and a GPU Block goes through buffers of one
// common format that both sides pack and unpack (the paper's extraction and
// insertion functions selected per hardware).  The arithmetic repeats the
// GPU sweep operation for operation, with fused multiply-adds only where the
// GPU writes them, so a CPU Block's values round exactly like a GPU Block's.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "lbm_internal.h"

#pragma clang fp contract(off)

namespace lbm {

namespace {

constexpr int kEx[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kEy[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kEz[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int kOpp[kQ] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
// representative of the weight class (rest, face, edge) of direction i
constexpr int wcls(int i) { return i == 0 ? 0 : (i < 7 ? 1 : 7); }

inline long long main_off(const BlockDev& B, int i, int x, int y, int z) {
  return B.base + (long long)i * B.Sf + (long long)(z + 1) * B.Sz + (long long)(y + 1) * B.Sx + x;
}
inline long long xg_off(const BlockDev& B, int i, int y, int z) {
  return B.base + (long long)i * B.Sf + B.xgo + (long long)(z + 1) * B.Ry + (y + 1);
}
inline int wrapc(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

}  // namespace

// ------------------------------------------------------------ thread pool
// Persistent workers: run(f) calls f(t) for t = 0 .. n-1, t = 0 on the
// calling thread, and returns when all have finished.
struct HostPool {
  int n = 1;
  std::vector<std::thread> th;
  std::mutex mu;
  std::condition_variable go, done;
  std::function<void(int)> job;
  long long gen = 0;
  int pending = 0;
  bool stop = false;

  explicit HostPool(int threads) : n(std::max(1, threads)) {
    for (int t = 1; t < n; ++t) th.emplace_back([this, t] { worker(t); });
  }
  ~HostPool() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    go.notify_all();
    for (auto& t : th) t.join();
  }
  void worker(int t) {
    long long seen = 0;
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      go.wait(lk, [&] { return stop || gen != seen; });
      if (stop) return;
      seen = gen;
      std::function<void(int)> f = job;
      lk.unlock();
      f(t);
      lk.lock();
      if (--pending == 0) done.notify_one();
    }
  }
  void run(const std::function<void(int)>& f) {
    if (n == 1) {
      f(0);
      return;
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      job = f;
      pending = n - 1;
      ++gen;
    }
    go.notify_all();
    f(0);
    std::unique_lock<std::mutex> lk(mu);
    done.wait(lk, [&] { return pending == 0; });
  }
};

HostPool* host_pool_create(int threads) { return new HostPool(threads); }
void host_pool_destroy(HostPool* p) { delete p; }
int host_pool_threads(const HostPool* p) { return p ? p->n : 0; }

namespace {

// ------------------------------------------------------------------ sweep
// One x-row (y, z) of Block B in three passes over row buffers, so that the
// collision runs as one branch-free loop over x that the compiler turns
// into SIMD code (element-wise, so each cell rounds exactly as alone):
//   pull:     W[i][x] = value cell x receives along e_i (shifted row copies;
//             the x-ghost slot or the wrapped row end at the row ends; the
//             cell's own f*_ibar across obstacle links),
//   collide:  O[i][x] from W (solid cells: zeros), stored to the dst rows,
//   bounce:   rows on a wall face only, f*_q to the slot (x + e_q, qbar).
// T: storage type; C: arithmetic type; HYB: FP32 storage with FP32
// arithmetic whose velocity and odd parts are kept in FP64 (the GPU's mixed
// mode).  W and O are per-thread buffers of kQ * a elements.
template <typename T, typename C, bool HYB>
void sweep_row(const T* __restrict__ src, T* __restrict__ dst, const BlockDev& B, const uint32_t* mask,
               const GridGeom& geo, const Phys<C>& ph, int y, int z, C* __restrict__ W, T* __restrict__ O,
               uint32_t* __restrict__ S) {
  const int a = B.dim[0], b = B.dim[1], c = B.dim[2];
  const bool wx = B.wrap & 1, wy = B.wrap & 2, wz = B.wrap & 4;
  const int gy = B.org[1] + y, gz = B.org[2] + z;
  const uint32_t* mrow = mask ? mask + B.mask + ((long long)z * b + y) * a : nullptr;

  // ---- pull
  for (int i = 0; i < kQ; ++i) {
    const int zs = wz ? wrapc(z - kEz[i], c) : z - kEz[i];
    const int ys = wy ? wrapc(y - kEy[i], b) : y - kEy[i];
    const T* __restrict__ sr = src + main_off(B, i, 0, ys, zs);
    C* __restrict__ w = W + (size_t)i * a;
    if (kEx[i] == 0) {
      for (int x = 0; x < a; ++x) w[x] = (C)sr[x];
    } else if (kEx[i] > 0) {  // source x - 1
      w[0] = (C)(wx ? sr[a - 1] : src[xg_off(B, i, ys, zs)]);
      for (int x = 1; x < a; ++x) w[x] = (C)sr[x - 1];
    } else {  // source x + 1
      for (int x = 0; x < a - 1; ++x) w[x] = (C)sr[x + 1];
      w[a - 1] = (C)(wx ? sr[0] : src[xg_off(B, i, ys, zs)]);
    }
  }
  // S[x]: all ones for a solid cell, else zero
  for (int x = 0; x < a; ++x) S[x] = mrow && (mrow[x] & kSolidBit) ? ~0u : 0u;
  if (mrow) {
    // obstacle links: the cell's own f*_ibar of the previous step
    for (int x = 0; x < a; ++x) {
      const uint32_t m = mrow[x];
      if (!(m & ~kSolidBit)) continue;
      for (int i = 1; i < kQ; ++i)
        if ((m >> i) & 1u) W[(size_t)i * a + x] = (C)src[main_off(B, kOpp[i], x, y, z)];
    }
  }

  // ---- collide
  const C omega = ph.omega, omc = ph.omc, fcoef = ph.fcoef, rho0 = ph.rho0, rho0x3 = ph.rho0x3;
  const C w0 = ph.w[0], w1 = ph.w[1], w7 = ph.w[7];
  const C inv_rho0 = ph.inv_rho0, hg0 = ph.hg[0], hg1 = ph.hg[1], hg2 = ph.hg[2];
  const C g0 = ph.g[0], g1 = ph.g[1], g2 = ph.g[2];
  const double dinv = ph.dinv_rho0, dhg0 = ph.dhg[0], dhg1 = ph.dhg[1], dhg2 = ph.dhg[2];
  const double domega = ph.domega, domc = ph.domc;
  C c9g[kQ], c3w[kQ], cfa[kQ];
  double dc3w[kQ], dcfa[kQ];
  for (int i = 0; i < kQ; ++i) {
    c9g[i] = ph.c9g[i];
    c3w[i] = ph.c3w[wcls(i)];
    cfa[i] = ph.cfa[i];
    dc3w[i] = ph.dc3w[wcls(i)];
    dcfa[i] = ph.dcfa[i];
  }
#pragma clang loop vectorize(enable)
  for (int x = 0; x < a; ++x) {
    C f[kQ];
    for (int i = 0; i < kQ; ++i) f[i] = W[(size_t)i * a + x];
    // moments: drho = sum f~, rho0 u = sum e f~, plus half force
    C d = f[0], jx = (C)0, jy = (C)0, jz = (C)0;
    for (int i = 1; i < kQ; i += 2) {
      const C sp = f[i] + f[i + 1], dp = f[i] - f[i + 1];
      d += sp;
      if (kEx[i] > 0) jx += dp;
      if (kEx[i] < 0) jx -= dp;
      if (kEy[i] > 0) jy += dp;
      if (kEy[i] < 0) jy -= dp;
      if (kEz[i] > 0) jz += dp;
      if (kEz[i] < 0) jz -= dp;
    }
    const C drho = d;
    C ux, uy, uz;
    double dux = 0.0, duy = 0.0, duz = 0.0;
    if constexpr (HYB) {
      dux = std::fma((double)jx, dinv, dhg0);
      duy = std::fma((double)jy, dinv, dhg1);
      duz = std::fma((double)jz, dinv, dhg2);
      ux = (C)dux;
      uy = (C)duy;
      uz = (C)duz;
    } else {
      ux = std::fma(jx, inv_rho0, hg0);
      uy = std::fma(jy, inv_rho0, hg1);
      uz = std::fma(jz, inv_rho0, hg2);
    }
    const C uu15 = (C)1.5 * std::fma(ux, ux, std::fma(uy, uy, uz * uz));
    const C ug3 = rho0x3 * std::fma(ux, g0, std::fma(uy, g1, uz * g2));
    const bool solid = S[x] != 0u;
    T o[kQ];
    {
      const C feq = w0 * std::fma(rho0, -uu15, drho);
      const C F = -w0 * ug3;
      const C even = std::fma(omega, feq, fcoef * F);
      if constexpr (HYB)
        o[0] = (T)std::fma(domc, (double)f[0], (double)even);
      else
        o[0] = (T)std::fma(omc, f[0], even);
    }
    for (int i = 1; i < kQ; i += 2) {
      const C wc = i < 7 ? w1 : w7;
      C eu = (C)0;
      double deu = 0.0;
      if constexpr (HYB) {
        if (kEx[i] > 0) deu += dux;
        if (kEx[i] < 0) deu -= dux;
        if (kEy[i] > 0) deu += duy;
        if (kEy[i] < 0) deu -= duy;
        if (kEz[i] > 0) deu += duz;
        if (kEz[i] < 0) deu -= duz;
        eu = (C)deu;
      } else {
        if (kEx[i] > 0) eu += ux;
        if (kEx[i] < 0) eu -= ux;
        if (kEy[i] > 0) eu += uy;
        if (kEy[i] < 0) eu -= uy;
        if (kEz[i] > 0) eu += uz;
        if (kEz[i] < 0) eu -= uz;
      }
      const C sym = wc * std::fma(rho0, std::fma((C)4.5 * eu, eu, -uu15), drho);
      const C Fs = std::fma(c9g[i], eu, -wc * ug3);
      const C even = std::fma(omega, sym, fcoef * Fs);
      if constexpr (HYB) {
        const double odd = std::fma(domega, dc3w[i] * deu, dcfa[i]);
        const double ev = (double)even;
        o[i] = (T)std::fma(domc, (double)f[i], ev + odd);
        o[i + 1] = (T)std::fma(domc, (double)f[i + 1], ev - odd);
      } else {
        const C odd = std::fma(omega, c3w[i] * eu, cfa[i]);
        o[i] = (T)std::fma(omc, f[i], even + odd);
        o[i + 1] = (T)std::fma(omc, f[i + 1], even - odd);
      }
    }
    // solid cells store zeros (the GPU keeps whole lines written)
    for (int i = 0; i < kQ; ++i) O[(size_t)i * a + x] = solid ? T(0) : o[i];
  }
  for (int i = 0; i < kQ; ++i) {
    T* __restrict__ dr = dst + main_off(B, i, 0, y, z);
    const T* __restrict__ orow = O + (size_t)i * a;
    for (int x = 0; x < a; ++x) dr[x] = orow[x];
  }

  // ---- bounce-back at walls: f*_q(x) (plus the moving-wall term) goes to
  // the slot (x + e_q, qbar) when x + e_q lies beyond a wall face
  const bool loy = geo.fwall[2] && gy == 0, hiy = geo.fwall[3] && gy == geo.n[1] - 1;
  const bool loz = geo.fwall[4] && gz == 0, hiz = geo.fwall[5] && gz == geo.n[2] - 1;
  const bool xwalls = (geo.fwall[0] && B.org[0] == 0) || (geo.fwall[1] && B.org[0] + a == geo.n[0]);
  if (!(loy | hiy | loz | hiz | xwalls)) return;
  const bool moving =
      geo.moving[0] | geo.moving[1] | geo.moving[2] | geo.moving[3] | geo.moving[4] | geo.moving[5];
  for (int x = 0; x < a; ++x) {
    if (mrow && (mrow[x] & kSolidBit)) continue;
    const int gx = B.org[0] + x;
    const bool lox = geo.fwall[0] && gx == 0, hix = geo.fwall[1] && gx == geo.n[0] - 1;
    if (!(lox | hix | loy | hiy | loz | hiz)) continue;
    for (int q = 1; q < kQ; ++q) {
      const int qb = kOpp[q];
      const int ex = kEx[qb], ey = kEy[qb], ez = kEz[qb];
      const bool link = (ex > 0 && lox) || (ex < 0 && hix) || (ey > 0 && loy) || (ey < 0 && hiy) ||
                        (ez > 0 && loz) || (ez < 0 && hiz);
      if (!link) continue;
      T v = O[(size_t)q * a + x];
      if (moving) {
        // the first moving face in the order -x, +x, -y, +y, -z, +z
        C cw = (C)0;
        if (ez > 0 && loz && geo.moving[4]) cw = ph.corr[qb][4];
        if (ez < 0 && hiz && geo.moving[5]) cw = ph.corr[qb][5];
        if (ey > 0 && loy && geo.moving[2]) cw = ph.corr[qb][2];
        if (ey < 0 && hiy && geo.moving[3]) cw = ph.corr[qb][3];
        if (ex > 0 && lox && geo.moving[0]) cw = ph.corr[qb][0];
        if (ex < 0 && hix && geo.moving[1]) cw = ph.corr[qb][1];
        v = (T)((C)v + cw);
      }
      const int zt = wz ? wrapc(z + kEz[q], c) : z + kEz[q];
      const int yt = wy ? wrapc(y + kEy[q], b) : y + kEy[q];
      const int xt = x + kEx[q];
      if (xt >= 0 && xt < a) dst[main_off(B, qb, xt, yt, zt)] = v;
      else if (wx) dst[main_off(B, qb, wrapc(xt, a), yt, zt)] = v;
      else dst[xg_off(B, qb, yt, zt)] = v;
    }
  }
}

template <typename T, typename C, bool HYB>
void sweep_all(HostPool* p, const T* src, T* dst, const BlockDev* blocks, const int* ids, int nids,
               const uint32_t* mask, const GridGeom& geo, const Phys<C>& ph) {
  // rows of all listed Blocks, handed out in small runs
  std::vector<long long> first(nids + 1, 0);
  for (int k = 0; k < nids; ++k)
    first[k + 1] = first[k] + (long long)blocks[ids[k]].dim[1] * blocks[ids[k]].dim[2];
  const long long nrows = first[nids];
  int amax = 1;
  for (int k = 0; k < nids; ++k) amax = std::max(amax, blocks[ids[k]].dim[0]);
  constexpr long long RUN = 4;
  std::atomic<long long> next(0);
  p->run([&](int) {
    std::vector<C> W((size_t)kQ * amax);
    std::vector<T> O((size_t)kQ * amax);
    std::vector<uint32_t> S(amax);
    for (;;) {
      const long long r0 = next.fetch_add(RUN);
      if (r0 >= nrows) return;
      const long long r1 = std::min(nrows, r0 + RUN);
      int k = (int)(std::upper_bound(first.begin(), first.end(), r0) - first.begin()) - 1;
      for (long long r = r0; r < r1; ++r) {
        while (r >= first[k + 1]) ++k;
        const BlockDev& B = blocks[ids[k]];
        const long long lr = r - first[k];
        sweep_row<T, C, HYB>(src, dst, B, mask, geo, ph, (int)(lr % B.dim[1]), (int)(lr / B.dim[1]), W.data(),
                             O.data(), S.data());
      }
    }
  });
}

template <typename T>
void exchange_tasks(HostPool* p, int mode, T* grid, const BlockDev* blocks, const NbrDev* nbr,
                    const XchgTask* tasks, int ntasks, T* buf) {
  std::atomic<int> next(0);
  auto work = [&](int) {
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= ntasks) return;
      const XchgTask& t = tasks[k];
      const BlockDev& M = blocks[t.dst];
      const NbrDev& nb = nbr[t.dst * 27 + t.d];
      const BlockDev& N = blocks[nb.id];
      const bool xplane = t.lo[0] < 0 || t.lo[0] >= M.dim[0];
      for (int L = t.l0; L < t.l1; ++L) {
        const int q0 = L % t.ext[0], r = L / t.ext[0];
        const int q1 = r % t.ext[1], q2 = r / t.ext[1];
        const int gx = t.lo[0] + q0, gy = t.lo[1] + q1, gz = t.lo[2] + q2;
        for (int j = 0; j < t.ndir; ++j) {
          const int i = (t.dirs >> (5 * j)) & 31;
          // only slots whose puller lies inside the receiving Block
          int px = gx + kEx[i], py = gy + kEy[i], pz = gz + kEz[i];
          if (M.wrap & 1) px = wrapc(px, M.dim[0]);
          if (M.wrap & 2) py = wrapc(py, M.dim[1]);
          if (M.wrap & 4) pz = wrapc(pz, M.dim[2]);
          if (px < 0 || px >= M.dim[0] || py < 0 || py >= M.dim[1] || pz < 0 || pz >= M.dim[2]) continue;
          const long long bi = (long long)t.bo + 5ll * (L - t.l0) + j;
          const long long to = xplane ? xg_off(M, i, gy, gz) : main_off(M, i, gx, gy, gz);
          if (mode == 2) {
            grid[to] = buf[bi];
          } else {
            const T v = grid[main_off(N, i, gx + nb.tx, gy + nb.ty, gz + nb.tz)];
            if (mode == 1) buf[bi] = v;
            else grid[to] = v;
          }
        }
      }
    }
  };
  // small exchanges stay on the calling thread (waking the pool costs more)
  long long cells = 0;
  for (int k = 0; k < ntasks; ++k) cells += tasks[k].l1 - tasks[k].l0;
  if (cells < 2048)
    work(0);
  else
    p->run(work);
}

}  // namespace

void host_sweep(HostPool* p, int prec, bool f64math, const void* src, void* dst, const BlockDev* blocks,
                const int* ids, int nids, const uint32_t* mask, const GridGeom& geo, const Phys<double>& pd,
                const Phys<float>& pf) {
  if (nids <= 0) return;
  if (prec == 0)
    sweep_all<double, double, false>(p, (const double*)src, (double*)dst, blocks, ids, nids, mask, geo, pd);
  else if (f64math)
    sweep_all<float, double, false>(p, (const float*)src, (float*)dst, blocks, ids, nids, mask, geo, pd);
  else
    sweep_all<float, float, true>(p, (const float*)src, (float*)dst, blocks, ids, nids, mask, geo, pf);
}

void host_exchange(HostPool* p, int prec, int mode, void* grid, const BlockDev* blocks, const NbrDev* nbr,
                   const XchgTask* tasks, int ntasks, void* buf) {
  if (ntasks <= 0) return;
  if (prec == 0)
    exchange_tasks<double>(p, mode, (double*)grid, blocks, nbr, tasks, ntasks, (double*)buf);
  else
    exchange_tasks<float>(p, mode, (float*)grid, blocks, nbr, tasks, ntasks, (float*)buf);
}

}  // namespace lbm
