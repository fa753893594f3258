// Many independent solves in one persistent launch per CG phase.
//
// A batch holds lattices of uneven size, each with its own links, kappa and
// number of right-hand sides (the N_f/2 pseudo-fermions of Section 2, for
// several gauge fields at once).  Every CG phase (D half, D^+ half with the
// vector update, search-direction update, reliable update) is one launch of a
// persistent kernel over a static work list of tiles (lattice, site tile,
// RHS group): a fixed grid walks the list grid-stride, so big and small
// lattices share the GPU without a launch per lattice.  Each lattice keeps its
// own per-RHS CG scalars; they sit in one contiguous array so that the host
// polls the whole batch with one copy.  The iterations are captured in a
// hipGraph and replayed.
#include <math.h>
#include <string.h>

#include <chrono>

#include "handle.h"
#include "hop_impl.h"

namespace mfq {

template <typename S, typename SX>
struct BatchLat {
  HopArgs<S, SX> d;             // t = D p               (inner precision)
  HopArgs<S, SX> cg;            // r -= alpha D^+ t, x += alpha p
  HopArgs<double, double> d64;  // t64 = D x64
  HopArgs<double, double> res;  // r64 = b - D^+ t64
  Field<S> r, p;
  Field<SX> x;
  Field<double> x64, r64, b64;
  CgScalars* sc;
  double* part[4];
  int nblk_both, nblk_full, nr, sb, n_rhs;  // tiles per RHS group: both-parity launches, vector kernels
};

struct Tile {
  int lat, tile, rgrp;
};

struct FinItem {
  CgScalars* sc;
  const double* pa;
  const double* pb;
  int nblk;
};

// Partial of v over one tile, one value per RHS row: a row is sb threads
// (a multiple of 64) of one RHS.
__device__ __forceinline__ void tile_partial(double v, double* part, int n_rhs, int r0, int sb, int tile,
                                             int nblk) {
  __shared__ double ws[8];
  const int tid = threadIdx.x;
  v = wave_sum(v);
  if ((tid & 63) == 0) ws[tid >> 6] = v;
  __syncthreads();
  if (tid % sb == 0) {
    const int row = tid / sb, wpr = sb >> 6;
    double s = 0.0;
    for (int k = 0; k < wpr; ++k) s += ws[row * wpr + k];
    if (r0 + row < n_rhs) part[(long)(r0 + row) * nblk + tile] = s;
  }
  __syncthreads();
}

enum : int { BM_D = 0, BM_CG = 1, BM_D64 = 2, BM_RES = 3 };
enum : int { BV_XPAY = 0, BV_FOLD = 1, BV_RESTART = 2, BV_INIT = 3 };

constexpr int kBatchThreads = 512;

// Both parities per launch: tile 2k and 2k+1 of a lattice cover the same
// half-index range at parity 0 and 1 (the D half reads only p, the D^+ half
// only t, so the parities are independent).
template <int MODE, typename S, typename SX>
__global__ __launch_bounds__(kBatchThreads) void batch_hop_kernel(const BatchLat<S, SX>* lats, const Tile* tiles,
                                                                  const int* n_tiles_dev, int slot, int mode) {
  const int n_tiles = *n_tiles_dev;
  for (int it = blockIdx.x; it < n_tiles; it += gridDim.x) {
    const Tile tl = tiles[it];
    const BatchLat<S, SX>& L = lats[tl.lat];
    const int row = wave_uniform(threadIdx.x / L.sb);  // L.sb is a multiple of 64
    const int par = tl.tile & 1;
    const int s = (tl.tile >> 1) * L.sb + (threadIdx.x - row * L.sb);
    const int r = tl.rgrp * L.nr + row;
    double red = 0.0;
    if constexpr (MODE == BM_D || MODE == BM_CG) {
      const HopArgs<S, SX>& a = MODE == BM_D ? L.d : L.cg;
      if (s < a.g.vh && r < a.n_rhs && a.sc[r].state < a.skip_state)
        red = hop_site<MODE == BM_D ? EPI_D : EPI_CGUPD>(a, par, s, r, a.sc[r].alpha);
    } else {
      const HopArgs<double, double>& a = MODE == BM_D64 ? L.d64 : L.res;
      if (s < a.g.vh && r < a.n_rhs && in_update(a.sc[r], mode))
        red = hop_site<MODE == BM_D64 ? EPI_D : EPI_RES>(a, par, s, r, 0.0);
    }
    if (slot >= 0) tile_partial(red, L.part[slot], L.n_rhs, tl.rgrp * L.nr, L.sb, tl.tile, L.nblk_both);
  }
}

// The inner-precision hopping phases with the directions of a site split
// over DS wavefronts (as the single-lattice direction-split kernel): the
// tile keeps its geometry (sb sites x nr RHS rows) and is walked in DS
// passes of 512 / DS (site, RHS) items, each pass's partial hopping terms
// meeting in LDS, where the first wavefront of each item group applies the
// epilogue.  Shorter dependent-load chains per thread, as in the tuned
// kernels of the one-by-one solves.  Per-row partial sums are added in a
// fixed order (pass, group).
template <int MODE, int DS, typename S, typename SX>
__global__ __launch_bounds__(kBatchThreads) void batch_hop_split_kernel(const BatchLat<S, SX>* lats,
                                                                        const Tile* tiles, const int* n_tiles_dev,
                                                                        int slot) {
  using T = typename Compute<S>::T;
  constexpr int G = kBatchThreads / 64 / DS;  // 64-item groups per pass
  constexpr int PER_PASS = kBatchThreads / DS;
  __shared__ T lds[G][DS - 1][24][64];
  __shared__ double wsum[DS][G];
  const int n_tiles = *n_tiles_dev;
  const int wave = wave_uniform(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int grp = wave / DS, d = wave - grp * DS;
  for (int it = blockIdx.x; it < n_tiles; it += gridDim.x) {
    const Tile tl = tiles[it];
    const BatchLat<S, SX>& L = lats[tl.lat];
    const HopArgs<S, SX>& a = MODE == BM_D ? L.d : L.cg;
    const int par = tl.tile & 1;
    for (int pass = 0; pass < DS; ++pass) {
      const int item = pass * PER_PASS + grp * 64 + lane;  // a 64-item group lies in one row (sb % 64 == 0)
      const int row = wave_uniform(item / L.sb);
      const int s = (tl.tile >> 1) * L.sb + (item - row * L.sb);
      const int r = tl.rgrp * L.nr + row;
      const bool active = s < a.g.vh && r < a.n_rhs && a.sc[r].state < a.skip_state;
      Spinor<T> acc;
      zero(acc);
      if (active) {
        const Coords c = site_coords(a.g, s, par);
        if constexpr (DS == 2) {
          if (d == 0) hop_dirs<0, 2>(a, par, s, c, r, acc);
          else hop_dirs<2, 4>(a, par, s, c, r, acc);
        } else {
          if (d == 0) hop_dirs<0, 1>(a, par, s, c, r, acc);
          else if (d == 1) hop_dirs<1, 2>(a, par, s, c, r, acc);
          else if (d == 2) hop_dirs<2, 3>(a, par, s, c, r, acc);
          else hop_dirs<3, 4>(a, par, s, c, r, acc);
        }
      }
      if (d > 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          lds[grp][d - 1][2 * k][lane] = acc.v[k].re;
          lds[grp][d - 1][2 * k + 1][lane] = acc.v[k].im;
        }
      }
      __syncthreads();
      if (d == 0) {
        double red = 0.0;
        if (active) {
#pragma unroll
          for (int q = 0; q < DS - 1; ++q)
#pragma unroll
            for (int k = 0; k < 12; ++k) {
              acc.v[k].re += lds[grp][q][2 * k][lane];
              acc.v[k].im += lds[grp][q][2 * k + 1][lane];
            }
          red = hop_epilogue<MODE == BM_D ? EPI_D : EPI_CGUPD>(a, par, s, r, a.sc[r].alpha, acc);
        }
        red = wave_sum(red);
        if (lane == 0) wsum[pass][grp] = red;
      }
      __syncthreads();  // the next pass reuses the LDS
    }
    if (slot >= 0) {
      if ((int)threadIdx.x < L.nr) {
        const int row = threadIdx.x;
        double t = 0.0;
        for (int pass = 0; pass < DS; ++pass)
          for (int g2 = 0; g2 < G; ++g2)
            if ((pass * PER_PASS + g2 * 64) / L.sb == row) t += wsum[pass][g2];
        const int r = tl.rgrp * L.nr + row;
        if (r < L.n_rhs) L.part[slot][(long)r * L.nblk_both + tl.tile] = t;
      }
      __syncthreads();
    }
  }
}

template <int MODE, typename S, typename SX>
__global__ __launch_bounds__(kBatchThreads) void batch_vec_kernel(const BatchLat<S, SX>* lats, const Tile* tiles,
                                                                  const int* n_tiles_dev, int mode) {
  const int n_tiles = *n_tiles_dev;
  using T = typename Compute<S>::T;
  using TX = typename Compute<SX>::T;
  for (int it = blockIdx.x; it < n_tiles; it += gridDim.x) {
    const Tile tl = tiles[it];
    const BatchLat<S, SX>& L = lats[tl.lat];
    const int row = threadIdx.x / L.sb;
    const int q = tl.tile * L.sb + (threadIdx.x - row * L.sb);
    const int r = tl.rgrp * L.nr + row;
    const int vh = L.d.g.vh;
    const bool valid = q < 2 * vh && r < L.n_rhs;
    const int par = q >= vh ? 1 : 0;
    const int s = q - par * vh;
    if constexpr (MODE == BV_XPAY) {
      if (valid && L.sc[r].state == ST_ACTIVE) {
        const T beta = (T)L.sc[r].beta;
        Spinor<T> rr, pp;
        load_spinor(L.r, r, par, s, rr);
        load_spinor(L.p, r, par, s, pp);
#pragma unroll
        for (int k = 0; k < 12; ++k) pp.v[k] = rr.v[k] + beta * pp.v[k];
        store_spinor(L.p, r, par, s, pp);
      }
    } else if constexpr (MODE == BV_FOLD) {
      if (valid && in_update(L.sc[r], mode)) {
        Spinor<TX> a;
        Spinor<double> b;
        load_spinor(L.x, r, par, s, a);
        load_spinor(L.x64, r, par, s, b);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          b.v[k].re += (double)a.v[k].re;
          b.v[k].im += (double)a.v[k].im;
          a.v[k] = {(TX)0, (TX)0};
        }
        store_spinor(L.x64, r, par, s, b);
        store_spinor(L.x, r, par, s, a);
      }
    } else if constexpr (MODE == BV_RESTART) {
      if (valid && L.sc[r].state == ST_ACTIVE && L.sc[r].fresh) {
        Spinor<double> a;
        load_spinor(L.r64, r, par, s, a);
        Spinor<T> b;
#pragma unroll
        for (int k = 0; k < 12; ++k) b.v[k] = {(T)a.v[k].re, (T)a.v[k].im};
        store_spinor(L.r, r, par, s, b);
        const int rp = L.sc[r].rp;
        if (rp == 2) {  // finish the paused step: p = r + beta p
          const T beta = (T)L.sc[r].beta;
          Spinor<T> pp;
          load_spinor(L.p, r, par, s, pp);
#pragma unroll
          for (int k = 0; k < 12; ++k) pp.v[k] = b.v[k] + beta * pp.v[k];
          store_spinor(L.p, r, par, s, pp);
        } else if (rp == 1) {
          store_spinor(L.p, r, par, s, b);
        }
      }
    } else {  // BV_INIT: r64 = b, partial |b|^2
      double v = 0.0;
      if (valid) {
        Spinor<double> a;
        load_spinor(L.b64, r, par, s, a);
        store_spinor(L.r64, r, par, s, a);
        v = snorm2(a);
      }
      tile_partial(v, L.part[0], L.n_rhs, tl.rgrp * L.nr, L.sb, tl.tile, L.nblk_full);
    }
  }
}

__global__ void batch_finish_kernel(const FinItem* items, int n_items, int fin, double tol2, double delta2) {
  const int w = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (w >= n_items) return;
  const FinItem it = items[w];
  double v = 0.0;
  for (int j = lane; j < it.nblk; j += 64) v += it.pa[j];
  if (it.pb)
    for (int j = lane; j < it.nblk; j += 64) v += it.pb[j];
  v = wave_sum(v);
  if (lane == 0) cg_scalar_update(fin, *it.sc, v, tol2, delta2);
}

}  // namespace mfq

using namespace mfq;

enum : int { FI_ALPHA = 0, FI_BETA = 1, FI_TRUE = 2, FI_INIT = 3 };

struct mfq_batch {
  std::vector<mfq_handle*> hs;
  std::vector<int> n_rhs, off;  // RHS count and offset of each lattice in the scalar array
  int prec = 0, total = 0;
  DevBuf lats, tiles_h, tiles_f, items[4], sc;
  int n_tiles_h = 0, n_tiles_f = 0, n_items[4] = {0, 0, 0, 0};
  // Tiles of each lattice, and the lattices still in the lists: lattices whose
  // RHS are all done are dropped from the launch lists between polls (the
  // kernels read the list lengths from device memory, so captured graphs stay
  // valid).
  std::vector<std::vector<Tile>> lat_th, lat_tf;
  std::vector<char> in_list;
  std::vector<Tile> host_th, host_tf;
  DevBuf counts;  // int[2]: current lengths of the two lists
  int grid = 512;
  int split = 0;  // the inner hopping phases split directions over wavefronts
  CgScalars* host_sc = nullptr;
  hipStream_t cap_stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::vector<GraphEntry> graphs;
  std::vector<int> host_bad;
  std::vector<uintptr_t> ws_ptrs;  // workspace pointers baked into the descriptors
};

namespace {

// RHS rows per tile: the largest power of two (<= 8) dividing n, so that no
// row of a 512-thread tile is idle (a tile is 512 / rows sites x rows RHS).
int rows_per_tile(int n) {
  int p = 1;
  while (p < 8 && n % (2 * p) == 0) p *= 2;
  return p;
}

template <typename S, typename SX>
struct Inner;
template <>
struct Inner<double, double> {
  static Field<double> r(mfq_handle* h) { return h->ws.rd.view(h->g); }
  static Field<double> p(mfq_handle* h) { return h->ws.pd.view(h->g); }
  static Field<double> t(mfq_handle* h) { return h->ws.td.view(h->g); }
  static Field<double> x(mfq_handle* h) { return h->ws.xd.view(h->g); }
  static Links<double> L(mfq_handle* h) { return links_d(h); }
  static hipError_t alloc(mfq_handle* h, int n) {
    hipError_t e;
    if ((e = h->ws.xd.alloc(h->g, n)) || (e = h->ws.rd.alloc(h->g, n)) || (e = h->ws.pd.alloc(h->g, n)) ||
        (e = h->ws.td.alloc(h->g, n)))
      return e;
    return hipSuccess;
  }
};
template <>
struct Inner<float, float> {
  static Field<float> r(mfq_handle* h) { return h->ws.rs.view(h->g); }
  static Field<float> p(mfq_handle* h) { return h->ws.ps.view(h->g); }
  static Field<float> t(mfq_handle* h) { return h->ws.ts.view(h->g); }
  static Field<float> x(mfq_handle* h) { return h->ws.xs.view(h->g); }
  static Links<float> L(mfq_handle* h) { return links_f(h); }
  static hipError_t alloc(mfq_handle* h, int n) {
    hipError_t e;
    if ((e = h->ws.xs.alloc(h->g, n)) || (e = h->ws.rs.alloc(h->g, n)) || (e = h->ws.ps.alloc(h->g, n)) ||
        (e = h->ws.ts.alloc(h->g, n)))
      return e;
    return hipSuccess;
  }
};
template <>
struct Inner<_Float16, float> {
  static Field<_Float16> r(mfq_handle* h) { return h->ws.rh.view(h->g); }
  static Field<_Float16> p(mfq_handle* h) { return h->ws.ph.view(h->g); }
  static Field<_Float16> t(mfq_handle* h) { return h->ws.th.view(h->g); }
  static Field<float> x(mfq_handle* h) { return h->ws.xs.view(h->g); }
  static Links<_Float16> L(mfq_handle* h) { return links_h(h); }
  static hipError_t alloc(mfq_handle* h, int n) {
    hipError_t e;
    if ((e = h->ws.xs.alloc(h->g, n)) || (e = h->ws.rh.alloc(h->g, n)) || (e = h->ws.ph.alloc(h->g, n)) ||
        (e = h->ws.th.alloc(h->g, n)))
      return e;
    return hipSuccess;
  }
};

// The device pointers a batch's descriptors hold; a solve refuses to run if
// any handle's workspace moved since (it was used for more RHS elsewhere).
std::vector<uintptr_t> workspace_pointers(mfq_batch* B) {
  std::vector<uintptr_t> v;
  for (mfq_handle* h : B->hs) {
    const Workspace& w = h->ws;
    for (const DevBuf* b : std::initializer_list<const DevBuf*>{&w.b64.data, &w.x64.data, &w.r64.data, &w.t64.data, &w.part, &w.xd.data, &w.rd.data,
                            &w.pd.data, &w.td.data, &w.xs.data, &w.rs.data, &w.ps.data, &w.ts.data, &w.rh.data,
                            &w.ph.data, &w.th.data, &w.rh.norm, &w.ph.norm, &w.th.norm, &h->links64,
                            &h->links32, &h->links16})
      v.push_back((uintptr_t)b->ptr);
    v.push_back((uintptr_t)h->links_su3);
  }
  return v;
}

template <typename S, typename SX>
int batch_setup(mfq_batch* B) {
  const int n_lat = (int)B->hs.size();
  std::vector<BatchLat<S, SX>> lats(n_lat);
  std::vector<Tile> th, tf;
  std::vector<FinItem> items[4];
  CgScalars* sc = (CgScalars*)B->sc.ptr;
  B->lat_th.assign(n_lat, {});
  B->lat_tf.assign(n_lat, {});
  for (int i = 0; i < n_lat; ++i) {
    mfq_handle* h = B->hs[i];
    const int n = B->n_rhs[i];
    int rc = need_su3(h, B->prec, MFQ_PC_NONE);
    if (rc) return rc;
    if ((rc = ensure_fp64_fields(h, n))) return rc;
    if (rc) return rc;
    HIPCHK(Inner<S, SX>::alloc(h, n));
    const Geom& g = h->g;
    BatchLat<S, SX>& L = lats[i];
    memset((void*)&L, 0, sizeof(L));
    L.n_rhs = n;
    L.nr = rows_per_tile(n);
    L.sb = kBatchThreads / L.nr;
    L.nblk_both = 2 * ((g.vh + L.sb - 1) / L.sb);
    L.nblk_full = (2 * g.vh + L.sb - 1) / L.sb;
    L.sc = sc + B->off[i];
    for (int q = 0; q < 4; ++q) L.part[q] = part_slot(h, q);
    L.r = Inner<S, SX>::r(h);
    L.p = Inner<S, SX>::p(h);
    L.x = Inner<S, SX>::x(h);
    L.x64 = h->ws.x64.view(g);
    L.r64 = h->ws.r64.view(g);
    L.b64 = h->ws.b64.view(g);
    const double mk = -h->lat.kappa;
    L.d = hop_args<S, SX>(h, Inner<S, SX>::L(h), n);
    L.d.sc = L.sc;
    L.d.coef = mk;
    L.d.skip_state = ST_WAIT;
    L.d.in = L.d.self = L.p;
    L.d.out = Inner<S, SX>::t(h);
    L.cg = L.d;
    L.cg.in = L.cg.self = Inner<S, SX>::t(h);
    L.cg.out = L.r;
    L.cg.x = L.x;
    L.cg.p = L.p;
    L.cg.dagger = 1;
    L.d64 = hop_args<double, double>(h, links_d(h), n);
    L.d64.sc = L.sc;
    L.d64.coef = mk;
    L.d64.skip_state = ST_DONE;
    L.d64.in = L.d64.self = L.x64;
    L.d64.out = h->ws.t64.view(g);
    L.res = L.d64;
    L.res.in = L.res.self = h->ws.t64.view(g);
    L.res.bvec = L.b64;
    L.res.r64 = L.r64;
    L.res.dagger = 1;
    const int ng = (n + L.nr - 1) / L.nr;
    B->lat_th[i].clear();
    B->lat_tf[i].clear();
    for (int rg = 0; rg < ng; ++rg) {
      for (int t = 0; t < L.nblk_both; ++t) B->lat_th[i].push_back({i, t, rg});
      for (int t = 0; t < L.nblk_full; ++t) B->lat_tf[i].push_back({i, t, rg});
    }
    th.insert(th.end(), B->lat_th[i].begin(), B->lat_th[i].end());
    tf.insert(tf.end(), B->lat_tf[i].begin(), B->lat_tf[i].end());
    for (int r = 0; r < n; ++r) {
      const size_t ro = (size_t)r;
      items[FI_ALPHA].push_back({L.sc + r, L.part[0] + ro * L.nblk_both, nullptr, L.nblk_both});
      items[FI_BETA].push_back({L.sc + r, L.part[2] + ro * L.nblk_both, nullptr, L.nblk_both});
      items[FI_TRUE].push_back({L.sc + r, L.part[0] + ro * L.nblk_both, nullptr, L.nblk_both});
      items[FI_INIT].push_back({L.sc + r, L.part[0] + ro * L.nblk_full, nullptr, L.nblk_full});
    }
  }
  HIPCHK(ensure(B->lats, sizeof(BatchLat<S, SX>) * n_lat));
  HIPCHK(hipMemcpy(B->lats.ptr, lats.data(), sizeof(BatchLat<S, SX>) * n_lat, hipMemcpyHostToDevice));
  HIPCHK(ensure(B->tiles_h, sizeof(Tile) * th.size()));
  HIPCHK(hipMemcpy(B->tiles_h.ptr, th.data(), sizeof(Tile) * th.size(), hipMemcpyHostToDevice));
  HIPCHK(ensure(B->tiles_f, sizeof(Tile) * tf.size()));
  HIPCHK(hipMemcpy(B->tiles_f.ptr, tf.data(), sizeof(Tile) * tf.size(), hipMemcpyHostToDevice));
  B->n_tiles_h = (int)th.size();
  B->n_tiles_f = (int)tf.size();
  HIPCHK(ensure(B->counts, 2 * sizeof(int)));
  const int cnt[2] = {B->n_tiles_h, B->n_tiles_f};
  HIPCHK(hipMemcpy(B->counts.ptr, cnt, sizeof(cnt), hipMemcpyHostToDevice));
  B->in_list.assign(n_lat, 1);
  for (int k = 0; k < 4; ++k) {
    HIPCHK(ensure(B->items[k], sizeof(FinItem) * items[k].size()));
    HIPCHK(hipMemcpy(B->items[k].ptr, items[k].data(), sizeof(FinItem) * items[k].size(), hipMemcpyHostToDevice));
    B->n_items[k] = (int)items[k].size();
  }
  B->ws_ptrs = workspace_pointers(B);
  return MFQ_OK;
}

template <typename S, typename SX>
hipError_t bhop(mfq_batch* B, int mode, int slot, hipStream_t st, int upd_mode = UPD_ALL) {
  const BatchLat<S, SX>* L = (const BatchLat<S, SX>*)B->lats.ptr;
  const Tile* t = (const Tile*)B->tiles_h.ptr;
  const int grid = B->grid < B->n_tiles_h ? B->grid : B->n_tiles_h;
  const int* nt = (const int*)B->counts.ptr;
  constexpr int DS = sizeof(typename Compute<S>::T) == 8 ? 2 : 4;  // LDS: 48 KB (FP64) / 36 KB (FP32)
  if (B->split && (mode == BM_D || mode == BM_CG)) {
    if (mode == BM_D)
      hipLaunchKernelGGL((batch_hop_split_kernel<BM_D, DS, S, SX>), grid, kBatchThreads, 0, st, L, t, nt, slot);
    else
      hipLaunchKernelGGL((batch_hop_split_kernel<BM_CG, DS, S, SX>), grid, kBatchThreads, 0, st, L, t, nt, slot);
    return hipGetLastError();
  }
  switch (mode) {
    case BM_D: hipLaunchKernelGGL((batch_hop_kernel<BM_D, S, SX>), grid, kBatchThreads, 0, st, L, t, nt, slot, upd_mode); break;
    case BM_CG: hipLaunchKernelGGL((batch_hop_kernel<BM_CG, S, SX>), grid, kBatchThreads, 0, st, L, t, nt, slot, upd_mode); break;
    case BM_D64: hipLaunchKernelGGL((batch_hop_kernel<BM_D64, S, SX>), grid, kBatchThreads, 0, st, L, t, nt, slot, upd_mode); break;
    default: hipLaunchKernelGGL((batch_hop_kernel<BM_RES, S, SX>), grid, kBatchThreads, 0, st, L, t, nt, slot, upd_mode); break;
  }
  return hipGetLastError();
}

template <typename S, typename SX>
hipError_t bvec(mfq_batch* B, int mode, int arg, hipStream_t st) {
  const BatchLat<S, SX>* L = (const BatchLat<S, SX>*)B->lats.ptr;
  const Tile* t = (const Tile*)B->tiles_f.ptr;
  const int grid = B->grid < B->n_tiles_f ? B->grid : B->n_tiles_f;
  const int* nt = (const int*)B->counts.ptr + 1;
  switch (mode) {
    case BV_XPAY: hipLaunchKernelGGL((batch_vec_kernel<BV_XPAY, S, SX>), grid, kBatchThreads, 0, st, L, t, nt, arg); break;
    case BV_FOLD: hipLaunchKernelGGL((batch_vec_kernel<BV_FOLD, S, SX>), grid, kBatchThreads, 0, st, L, t, nt, arg); break;
    case BV_RESTART: hipLaunchKernelGGL((batch_vec_kernel<BV_RESTART, S, SX>), grid, kBatchThreads, 0, st, L, t, nt, arg); break;
    default: hipLaunchKernelGGL((batch_vec_kernel<BV_INIT, S, SX>), grid, kBatchThreads, 0, st, L, t, nt, arg); break;
  }
  return hipGetLastError();
}

hipError_t bfin(mfq_batch* B, int which, int fin, double tol2, double delta2, hipStream_t st) {
  const int n = B->n_items[which];
  const int blocks = (n + 3) / 4;
  hipLaunchKernelGGL(batch_finish_kernel, blocks, 256, 0, st, (const FinItem*)B->items[which].ptr, n, fin, tol2,
                     delta2);
  return hipGetLastError();
}

template <typename S, typename SX>
int batch_tune(mfq_batch* B, hipStream_t st) {
  // persistent grid size (a few multiples of the 256 CUs) and whether the
  // inner hopping phases split directions over wavefronts
  int best_grid = 512, best_split = 0;
  float best = 1e30f;
  const int cands[4] = {256, 512, 1024, 2048};
  for (int c = 0; c < 8; ++c) {
    B->grid = cands[c & 3];
    B->split = c >> 2;
    for (int i = 0; i < 2; ++i) HIPCHK(bhop<S, SX>(B, BM_D, -1, st));
    HIPCHK(hipEventRecord(B->ev0, st));
    for (int i = 0; i < 5; ++i) HIPCHK(bhop<S, SX>(B, BM_D, -1, st));
    HIPCHK(hipEventRecord(B->ev1, st));
    HIPCHK(hipEventSynchronize(B->ev1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, B->ev0, B->ev1));
    // the timing covers one phase with every tile live; a larger grid must
    // win it by 10 % (by 3 % at an equal or smaller grid), since the tail of
    // a batch, where few lattices are left, favours fewer workgroups
    // (64-lattice workload: 2186 ms at 256 and 512 workgroups, 2248 ms at
    // 1024, which had won this timing by more than 3 %)
    const float margin = cands[c & 3] > best_grid ? 0.90f : 0.97f;
    if (ms < best * margin) {
      best = ms;
      best_grid = cands[c & 3];
      best_split = c >> 2;
    }
  }
  B->grid = best_grid;
  B->split = best_split;
  return MFQ_OK;
}

void batch_drop_graphs(mfq_batch* B) {
  for (auto& e : B->graphs) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.graph) (void)hipGraphDestroy(e.graph);
  }
  B->graphs.clear();
}

// Drop the lattices whose RHS are all done (host_sc holds the last poll) from
// the launch lists, or restore all (every = true).  The copies run on the
// solve stream before the next launches; the host lists stay alive in the
// batch until the next rebuild, which happens only after a stream sync.
int batch_relist(mfq_batch* B, bool every, hipStream_t st) {
  const int n_lat = (int)B->hs.size();
  bool changed = false;
  for (int i = 0; i < n_lat; ++i) {
    bool live = every;
    for (int r = 0; r < B->n_rhs[i] && !live; ++r) live = B->host_sc[B->off[i] + r].state != ST_DONE;
    if ((char)live != B->in_list[i]) {
      B->in_list[i] = live;
      changed = true;
    }
  }
  if (!changed) return MFQ_OK;
  B->host_th.clear();
  B->host_tf.clear();
  for (int i = 0; i < n_lat; ++i)
    if (B->in_list[i]) {
      B->host_th.insert(B->host_th.end(), B->lat_th[i].begin(), B->lat_th[i].end());
      B->host_tf.insert(B->host_tf.end(), B->lat_tf[i].begin(), B->lat_tf[i].end());
    }
  static thread_local int cnt[2];
  cnt[0] = (int)B->host_th.size();
  cnt[1] = (int)B->host_tf.size();
  if (cnt[0]) HIPCHK(hipMemcpyAsync(B->tiles_h.ptr, B->host_th.data(), sizeof(Tile) * cnt[0], hipMemcpyHostToDevice, st));
  if (cnt[1]) HIPCHK(hipMemcpyAsync(B->tiles_f.ptr, B->host_tf.data(), sizeof(Tile) * cnt[1], hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(B->counts.ptr, cnt, sizeof(cnt), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return MFQ_OK;
}

template <typename S, typename SX>
int batch_run(mfq_batch* B, const mfq_solve_params* P, hipStream_t st, mfq_solve_stats* stats) {
  const double tol2 = P->tol * P->tol;
  const double delta = P->prec == MFQ_PREC_FP64 ? 0.0 : (P->reliable_delta > 0.0 ? P->reliable_delta : 0.1);
  const double delta2 = delta * delta;
  const int n_lat = (int)B->hs.size();
  CgScalars* sc = (CgScalars*)B->sc.ptr;
  if (int rl = batch_relist(B, true, st)) return rl;

  // x = 0, r = b, p = r
  for (int i = 0; i < n_lat; ++i) {
    mfq_handle* h = B->hs[i];
    const int n = B->n_rhs[i];
    HIPCHK(hipMemsetAsync(h->ws.x64.data.ptr, 0, field_chunks<double>(h->g, n) * sizeof(d2), st));
    Field<SX> x = Inner<S, SX>::x(h);
    HIPCHK(hipMemsetAsync(x.data, 0, field_chunks<SX>(h->g, n) * sizeof(typename Store<SX>::chunk), st));
  }
  HIPCHK(bvec<S, SX>(B, BV_INIT, 0, st));
  HIPCHK(bfin(B, FI_INIT, FIN_INIT, tol2, delta2, st));
  HIPCHK(bvec<S, SX>(B, BV_RESTART, 0, st));

  auto iteration = [&](hipStream_t s) -> int {
    HIPCHK(bhop<S, SX>(B, BM_D, 0, s));
    HIPCHK(bfin(B, FI_ALPHA, FIN_ALPHA, tol2, delta2, s));
    HIPCHK(bhop<S, SX>(B, BM_CG, 2, s));
    HIPCHK(bfin(B, FI_BETA, FIN_BETA, tol2, delta2, s));
    HIPCHK(bvec<S, SX>(B, BV_XPAY, 0, s));
    return MFQ_OK;
  };
  // per-RHS reliable update over the RHS the mode covers
  auto reliable_update = [&](int mode) -> int {
    HIPCHK(bvec<S, SX>(B, BV_FOLD, mode, st));
    HIPCHK(bhop<S, SX>(B, BM_D64, -1, st, mode));
    HIPCHK(bhop<S, SX>(B, BM_RES, 0, st, mode));
    HIPCHK(bfin(B, FI_TRUE, mode == UPD_ALL ? FIN_TRUE : FIN_TRUE_FLAGGED, tol2, delta2, st));
    HIPCHK(bvec<S, SX>(B, BV_RESTART, 0, st));
    return MFQ_OK;
  };
  auto run_iters = [&](int k) -> int {
    if (!P->use_graph) {
      for (int i = 0; i < k; ++i) {
        int rc = iteration(st);
        if (rc) return rc;
      }
      return MFQ_OK;
    }
    std::vector<uintptr_t> key = {(uintptr_t)k, bits(tol2), bits(delta2), (uintptr_t)B->grid, (uintptr_t)B->split};
    GraphEntry* hit = nullptr;
    for (auto& e : B->graphs)
      if (e.key == key) hit = &e;
    if (!hit) {
      if (B->graphs.size() >= 24) batch_drop_graphs(B);
      GraphEntry e;
      e.key = key;
      HIPCHK(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal));
      int rc2 = MFQ_OK;
      for (int i = 0; i < k && rc2 == MFQ_OK; ++i) rc2 = iteration(B->cap_stream);
      hipError_t ec = hipStreamEndCapture(B->cap_stream, &e.graph);
      if (rc2) return rc2;
      HIPCHK(ec);
      HIPCHK(hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0));
      B->graphs.push_back(e);
      hit = &B->graphs.back();
    }
    HIPCHK(hipGraphLaunch(hit->exec, st));
    return MFQ_OK;
  };

  const int max_k = P->check_every > 0 ? P->check_every : 64;
  const int min_k = max_k < 4 ? max_k : 4;
  int k = min_k, total = 0, rc;
  // every reliable update follows at least one iteration of some RHS, except
  // right after a restart: bound them so that the loop always ends
  int n_updates = 0;
  const int max_updates = 2 * P->max_iter + 16;
  std::vector<double> rho_prev(B->total, 0.0);
  for (;;) {
    HIPCHK(hipMemcpyAsync(B->host_sc, sc, sizeof(CgScalars) * B->total, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    bool all_done = true, need_update = false, have = false;
    int max_it = 0;
    double want = 1e30;
    for (int r = 0; r < B->total; ++r) {
      const CgScalars& s = B->host_sc[r];
      all_done = all_done && s.state == ST_DONE;
      need_update = need_update || in_update(s, UPD_FLAGGED);
      if (s.state != ST_DONE && s.iters > max_it) max_it = s.iters;
      if (s.state == ST_ACTIVE && rho_prev[r] > 0.0 && s.rho < rho_prev[r] && total > 0) {
        const double rate = log(s.rho / rho_prev[r]) / k;
        double target = tol2 * s.bnorm2;
        if (delta2 > 0.0 && delta2 * s.rho_ru > target) target = delta2 * s.rho_ru;
        const double it = log(target / s.rho) / rate;
        if (it < want) want = it;
        have = true;
      }
      rho_prev[r] = s.state == ST_ACTIVE ? s.rho : 0.0;
    }
    if (all_done) break;
    if (int rl = batch_relist(B, false, st)) return rl;
    if (need_update && ++n_updates > max_updates) {
      // reliable updates without iteration progress: stop (bounded loop)
      HIPCHK(hipMemcpyAsync(B->host_sc, sc, sizeof(CgScalars) * B->total, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      break;
    }
    if (need_update) {
      if ((rc = reliable_update(UPD_FLAGGED))) return rc;
      for (int r = 0; r < B->total; ++r)
        if (in_update(B->host_sc[r], UPD_FLAGGED)) rho_prev[r] = 0.0;
      k = min_k;
      continue;
    }
    if (max_it >= P->max_iter) {
      if ((rc = reliable_update(UPD_ALL))) return rc;
      HIPCHK(hipMemcpyAsync(B->host_sc, sc, sizeof(CgScalars) * B->total, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      break;
    }
    if (have) {
      int kk = min_k;
      while (kk < max_k && kk * 2 <= (int)(fmin(want, (double)max_k) + 1.0)) kk *= 2;
      k = kk;
    }
    if (k > P->max_iter - max_it) k = P->max_iter - max_it;
    if ((rc = run_iters(k))) return rc;
    total += k;
  }
  int status = MFQ_OK;
  for (int r = 0; r < B->total; ++r) {
    const CgScalars& s = B->host_sc[r];
    if (stats) {
      stats[r].iters = s.iters;
      stats[r].reliable_updates = s.n_true;
      stats[r].true_rel_resid = s.bnorm2 > 0 ? sqrt(s.rtrue2 / s.bnorm2) : 0.0;
      stats[r].status = s.state == ST_DONE ? MFQ_OK : MFQ_NOT_CONVERGED;
    }
    if (s.state != ST_DONE) status = MFQ_NOT_CONVERGED;
  }
  return status;
}

}  // namespace

extern "C" {

void mfq_batch_destroy(mfq_batch* B) {
  if (!B) return;
  batch_drop_graphs(B);
  release(B->lats);
  release(B->tiles_h);
  release(B->tiles_f);
  release(B->counts);
  for (int k = 0; k < 4; ++k) release(B->items[k]);
  release(B->sc);
  if (B->host_sc) (void)hipHostFree(B->host_sc);
  if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
  if (B->ev0) (void)hipEventDestroy(B->ev0);
  if (B->ev1) (void)hipEventDestroy(B->ev1);
  delete B;
}

int mfq_batch_create(mfq_handle** hs, int n_lat, const int* n_rhs, int prec, void* stream, mfq_batch** out) {
  if (!out) return fail(MFQ_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!hs || !n_rhs || n_lat < 1) return fail(MFQ_ERR_ARG, "empty batch");
  if (prec < MFQ_PREC_FP64 || prec > MFQ_PREC_FP16_REFINE) return fail(MFQ_ERR_ARG, "unknown precision");
  for (int i = 0; i < n_lat; ++i) {
    if (!hs[i]) return fail(MFQ_ERR_ARG, "NULL handle in batch");
    if (n_rhs[i] < 1 || n_rhs[i] > 64) return fail(MFQ_ERR_ARG, "n_rhs must be in [1, 64]");
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(MFQ_ERR_ARG, "a handle appears twice in the batch");
  }
  mfq_batch* B = new mfq_batch();
  B->hs.assign(hs, hs + n_lat);
  B->n_rhs.assign(n_rhs, n_rhs + n_lat);
  B->prec = prec;
  for (int i = 0; i < n_lat; ++i) {
    B->off.push_back(B->total);
    B->total += n_rhs[i];
  }
  hipStream_t st = (hipStream_t)stream;
  int rc = MFQ_OK;
  hipError_t e;
  if ((e = ensure(B->sc, sizeof(CgScalars) * B->total)) != hipSuccess ||
      (e = hipHostMalloc((void**)&B->host_sc, sizeof(CgScalars) * B->total, hipHostMallocDefault)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreate(&B->ev0)) != hipSuccess || (e = hipEventCreate(&B->ev1)) != hipSuccess) {
    rc = fail_hip(e, "batch setup");
  } else if (prec == MFQ_PREC_FP64) {
    if (!(rc = batch_setup<double, double>(B))) rc = batch_tune<double, double>(B, st);
  } else if (prec == MFQ_PREC_FP32_RELIABLE) {
    if (!(rc = batch_setup<float, float>(B))) rc = batch_tune<float, float>(B, st);
  } else {
    if (!(rc = batch_setup<_Float16, float>(B))) rc = batch_tune<_Float16, float>(B, st);
  }
  if (rc) {
    mfq_batch_destroy(B);
    return rc;
  }
  *out = B;
  return MFQ_OK;
}

int mfq_batch_solve(mfq_batch* B, const double* const* b_dev, double* const* x_dev,
                    const mfq_solve_params* params, mfq_solve_stats* stats_host, void* stream) {
  auto t0 = std::chrono::steady_clock::now();
  if (!B || !b_dev || !x_dev) return fail(MFQ_ERR_ARG, "NULL argument");
  int rc = check_params(params);
  if (rc) return rc;
  if (params->prec != B->prec) return fail(MFQ_ERR_STATE, "params.prec differs from the batch's precision");
  if (workspace_pointers(B) != B->ws_ptrs)
    return fail(MFQ_ERR_STATE, "a handle's workspace was reallocated since the batch was created");
  hipStream_t st = (hipStream_t)stream;
  const int n_lat = (int)B->hs.size();
  for (int i = 0; i < n_lat; ++i) {
    mfq_handle* h = B->hs[i];
    if (!b_dev[i] || !x_dev[i]) return fail(MFQ_ERR_ARG, "NULL spinor in batch");
    HIPCHK(hipMemsetAsync(h->ws.bad.ptr, 0, sizeof(int), st));
    HIPCHK(launch_pack_spinor<double>(h->g, b_dev[i], h->ws.b64.view(h->g), B->n_rhs[i], 0, (int*)h->ws.bad.ptr, st));
  }
  B->host_bad.assign(n_lat, 0);
  for (int i = 0; i < n_lat; ++i)
    HIPCHK(hipMemcpyAsync(&B->host_bad[i], B->hs[i]->ws.bad.ptr, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int i = 0; i < n_lat; ++i)
    if (B->host_bad[i]) return fail(MFQ_ERR_ARG, "input spinor holds NaN or Inf");
  if (B->prec == MFQ_PREC_FP64)
    rc = batch_run<double, double>(B, params, st, stats_host);
  else if (B->prec == MFQ_PREC_FP32_RELIABLE)
    rc = batch_run<float, float>(B, params, st, stats_host);
  else
    rc = batch_run<_Float16, float>(B, params, st, stats_host);
  if (rc < 0) return rc;
  for (int i = 0; i < n_lat; ++i)
    HIPCHK(launch_unpack_spinor(B->hs[i]->g, B->hs[i]->ws.x64.view(B->hs[i]->g), x_dev[i], B->n_rhs[i], st));
  HIPCHK(hipStreamSynchronize(st));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats_host)
    for (int r = 0; r < B->total; ++r) stats_host[r].seconds = secs;
  return rc;
}

int mfq_solve_batch(mfq_handle** hs, int n_lat, const double* const* b_dev, double* const* x_dev, const int* n_rhs,
                    const mfq_solve_params* params, mfq_solve_stats* stats_host, void* stream) {
  int rc = check_params(params);
  if (rc) return rc;
  mfq_batch* B = nullptr;
  if ((rc = mfq_batch_create(hs, n_lat, n_rhs, params->prec, stream, &B))) return rc;
  rc = mfq_batch_solve(B, b_dev, x_dev, params, stats_host, stream);
  mfq_batch_destroy(B);
  return rc;
}

int mfq_batch_grid(mfq_batch* B) { return B ? B->grid : -1; }

int mfq_batch_set_shape(mfq_batch* B, int grid, int split) {
  if (!B) return fail(MFQ_ERR_ARG, "NULL batch");
  if (grid < 1 || grid > 65536 || (split != 0 && split != 1))
    return fail(MFQ_ERR_ARG, "grid must be in 1..65536 and split 0 or 1");
  B->grid = grid;
  B->split = split;
  batch_drop_graphs(B);
  return MFQ_OK;
}

int mfq_batch_split(mfq_batch* B) { return B ? B->split : -1; }

}  // extern "C"
