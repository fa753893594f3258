// Device implementation of the Wilson hopping term and its fused epilogues,
// shared by the single-lattice kernels and the multi-lattice persistent
// kernels.
//
// H psi(n) = sum_mu [ (1 - g_mu) U_mu(n) psi(n+mu) + (1 + g_mu) U_mu(n-mu)^+ psi(n-mu) ]
// and its adjoint (projector signs swapped); D = 1 - kappa H.
#pragma once

#include "internal.h"

namespace mfq {

template <typename S>
struct Compute {
  using T = float;
};
template <>
struct Compute<double> {
  using T = double;
};

template <typename T>
__device__ __forceinline__ void zero(Spinor<T>& a) {
#pragma unroll
  for (int c = 0; c < 12; ++c) a.v[c] = {(T)0, (T)0};
}

template <typename T>
__device__ __forceinline__ double snorm2(const Spinor<T>& a) {
  T s = 0;
#pragma unroll
  for (int c = 0; c < 12; ++c) s += norm2(a.v[c]);
  return (double)s;
}

// Partial sum of v over the sites of this workgroup, one value per RHS row
// (row = threadIdx.y, RHS r = r0 + row), stored at part[r * nblk + tile].
// A wavefront holds one RHS (blockDim.x is a multiple of 64).
__device__ __forceinline__ void block_partial(double v, double* part, int n_rhs, int r0, int tile, int nblk) {
  __shared__ double ws[16];
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  v = wave_sum(v);
  if ((tid & 63) == 0) ws[tid >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int wpr = blockDim.x >> 6;
    double s = 0.0;
    for (int k = 0; k < wpr; ++k) s += ws[threadIdx.y * wpr + k];
    const int r = r0 + threadIdx.y;
    if (r < n_rhs) part[(long)r * nblk + tile] = s;
  }
  __syncthreads();
}

// Where the hopping term reads its input spinors.
template <typename S, typename T>
struct PlainSrc {
  Field<S> f;
  __device__ __forceinline__ void load(int r, int par, int s, Spinor<T>& o) const { load_spinor(f, r, par, s, o); }
};

// Where the hopping term reads its links: the global arrays, or an LDS tile
// holding, for each site of the workgroup's tile, its 4 forward links U_mu(n)
// and 4 backward links U_mu(n - mu) (two-row FP32 / FP16 storage), filled
// once per workgroup and read by every RHS row.
template <typename S>
struct GlobalLinks {
  Links<S> L;
  template <int MU, typename T>
  __device__ __forceinline__ void fwd(int par, int s, cpx<T> u[9]) const { load_link(L, par, MU, s, u); }
  template <int MU, typename T>
  __device__ __forceinline__ void bwd(int po, int sbk, cpx<T> u[9]) const { load_link(L, po, MU, sbk, u); }
};

template <typename S>
struct LinkChunk;
template <>
struct LinkChunk<float> {
  using type = f4;
};
template <>
struct LinkChunk<_Float16> {
  using type = h4;
};

template <typename S>
struct LdsLinks {
  const typename LinkChunk<S>::type* tile;  // [slot 0..7][3 chunks][sb]: slot mu forward, 4 + mu backward
  int sb, lane;
  template <int SLOT, typename T>
  __device__ __forceinline__ void get(cpx<T> u[9]) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const auto q = tile[(SLOT * 3 + k) * sb + lane];
      u[2 * k] = {(T)(float)q.x, (T)(float)q.y};
      u[2 * k + 1] = {(T)(float)q.z, (T)(float)q.w};
    }
    third_row(u);
  }
  template <int MU, typename T>
  __device__ __forceinline__ void fwd(int, int, cpx<T> u[9]) const { get<MU>(u); }
  template <int MU, typename T>
  __device__ __forceinline__ void bwd(int, int, cpx<T> u[9]) const { get<4 + MU>(u); }
};

// The backward neighbour of coordinates c in direction MU (half-lattice
// index, always inside the lattice; the boundary factor is not needed here).
template <int MU>
__device__ __forceinline__ int back_neighbour(const Geom& g, const Coords& c) {
  int x = c.x, y = c.y, z = c.z, t = c.t;
  if constexpr (MU == 0) t = c.t == 0 ? g.td - 1 : c.t - 1;
  else if constexpr (MU == 1) x = c.x == 0 ? g.lx - 1 : c.x - 1;
  else if constexpr (MU == 2) y = c.y == 0 ? g.ly - 1 : c.y - 1;
  else z = c.z == 0 ? g.lz - 1 : c.z - 1;
  return half_index(g, x, y, z, t);
}

// One direction mu of the hopping term: forward hop from n+mu through U_mu(n),
// backward hop from n-mu through U_mu(n-mu)^+.  sgf / sgb are the projector
// signs (-1 / +1 for H, +1 / -1 for H^+).  The time boundary is folded into a
// factor (0 across a Schroedinger-functional boundary, -1 across an
// antiperiodic wrap) on a neighbour index that always stays inside the
// lattice, so the loads of every direction are unconditional and can be
// issued together.
template <int MU, typename S, typename SX, typename T, typename Src, typename LS>
__device__ __forceinline__ void hop_dir(const HopArgs<S, SX>& a, const Src& src, const LS& lk, int par,
                                        const Coords& c, int s, int r, T sgf, T sgb, Spinor<T>& acc) {
  const Geom& g = a.g;
  const int po = 1 - par;
  int xf = c.x, yf = c.y, zf = c.z, tf = c.t;
  int xb = c.x, yb = c.y, zb = c.z, tb = c.t;
  T wf = (T)1, wb = (T)1;
  if constexpr (MU == 0) {
    const T wrap = g.bc == BC_SF ? (T)0 : (g.bc == BC_ANTIPERIODIC ? (T)-1 : (T)1);
    tf = c.t + 1;
    if (tf == g.td) {
      tf = 0;
      wf = wrap;
    }
    tb = c.t - 1;
    if (tb < 0) {
      tb = g.td - 1;
      wb = wrap;
    }
  } else if constexpr (MU == 1) {
    xf = (c.x + 1 == g.lx) ? 0 : c.x + 1;
    xb = (c.x == 0) ? g.lx - 1 : c.x - 1;
  } else if constexpr (MU == 2) {
    yf = (c.y + 1 == g.ly) ? 0 : c.y + 1;
    yb = (c.y == 0) ? g.ly - 1 : c.y - 1;
  } else {
    zf = (c.z + 1 == g.lz) ? 0 : c.z + 1;
    zb = (c.z == 0) ? g.lz - 1 : c.z - 1;
  }
  const int sf = half_index(g, xf, yf, zf, tf);
  const int sbk = half_index(g, xb, yb, zb, tb);
  Spinor<T> nf, nb;
  cpx<T> uf[9], ub[9];
  src.load(r, po, sf, nf);
  lk.template fwd<MU>(par, s, uf);
  src.load(r, po, sbk, nb);
  lk.template bwd<MU>(po, sbk, ub);
  {  // forward
    cpx<T> h0[3], h1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) project<MU>(nf, sgf, k, h0[k], h1[k]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cpx<T> g0 = cmul(uf[3 * i], h0[0]) + cmul(uf[3 * i + 1], h0[1]) + cmul(uf[3 * i + 2], h0[2]);
      cpx<T> g1 = cmul(uf[3 * i], h1[0]) + cmul(uf[3 * i + 1], h1[1]) + cmul(uf[3 * i + 2], h1[2]);
      reconstruct<MU>(acc, sgf, i, wf * g0, wf * g1);
    }
  }
  {  // backward: (U^+)_{ik} = conj(U_{ki})
    cpx<T> h0[3], h1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) project<MU>(nb, sgb, k, h0[k], h1[k]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cpx<T> g0 = cjmul(ub[i], h0[0]) + cjmul(ub[3 + i], h0[1]) + cjmul(ub[6 + i], h0[2]);
      cpx<T> g1 = cjmul(ub[i], h1[0]) + cjmul(ub[3 + i], h1[1]) + cjmul(ub[6 + i], h1[2]);
      reconstruct<MU>(acc, sgb, i, wb * g0, wb * g1);
    }
  }
}

// The per-RHS CG scalar recursion, applied once the reduction `sum` of the
// partials of one kernel pair is known (see the FIN_* codes).
__device__ __forceinline__ void cg_scalar_update(int fin, CgScalars& s, double sum, double tol2, double delta2) {
  const bool finite = isfinite(sum);
  switch (fin) {
    case FIN_ALPHA:
      s.rp = 0;
      s.fresh = 0;
      s.pap = sum;
      if (s.state == ST_ACTIVE && finite && sum > 0.0) {
        s.alpha = s.rho / sum;
      } else {
        if (s.state == ST_ACTIVE) s.state = ST_CHECK;  // breakdown: re-check truth
        s.alpha = 0.0;
      }
      break;
    case FIN_BETA:
      s.rp = 0;
      s.fresh = 0;
      if (s.state == ST_ACTIVE) {
        s.beta = sum / s.rho;
        s.rho = sum;
        s.iters += 1;
        if (!finite || sum <= tol2 * s.bnorm2)
          s.state = ST_CHECK;
        else if (sum < delta2 * s.rho_ru)
          s.state = ST_WAIT;  // keeps beta for p = r + beta p after the update
      }
      break;
    case FIN_TRUE:
    case FIN_TRUE_FLAGGED:
      if (in_update(s, fin == FIN_TRUE ? UPD_ALL : UPD_FLAGGED)) {
        // continue from the true residual: a paused RHS finishes its step
        // with p = r + beta p, one that claimed convergence (or broke down)
        // restarts with p = r, one interrupted mid-recursion keeps p
        const int was = s.state;
        s.rtrue2 = sum;
        s.n_true += 1;
        if (sum <= tol2 * s.bnorm2) {
          s.state = ST_DONE;
        } else {
          s.state = ST_ACTIVE;
          s.rho = sum;
          s.rho_ru = sum;
          s.rp = was == ST_CHECK ? 1 : (was == ST_WAIT ? 2 : 0);
          s.fresh = 1;
        }
      }
      break;
    case FIN_INIT:
      s.bnorm2 = sum;
      s.rho = s.rho_ru = s.rtrue2 = sum;
      s.alpha = s.beta = s.pap = 0.0;
      s.iters = s.n_true = 0;
      s.rp = 1;
      s.fresh = 1;
      s.state = sum > 0.0 ? ST_ACTIVE : ST_DONE;
      break;
  }
}


// Directions [MU0, MU1) of the hopping term at output site s, accumulated into acc.
template <int MU0, int MU1, typename S, typename SX, typename T, typename LS>
__device__ __forceinline__ void hop_dirs_with(const HopArgs<S, SX>& a, const LS& lk, int par, int s,
                                              const Coords& c, int r, Spinor<T>& acc) {
  const T sgf = a.dagger ? (T)1 : (T)-1;
  const T sgb = -sgf;
  PlainSrc<S, T> src{a.in};
  if constexpr (MU0 <= 0 && 0 < MU1) hop_dir<0>(a, src, lk, par, c, s, r, sgf, sgb, acc);
  if constexpr (MU0 <= 1 && 1 < MU1) hop_dir<1>(a, src, lk, par, c, s, r, sgf, sgb, acc);
  if constexpr (MU0 <= 2 && 2 < MU1) hop_dir<2>(a, src, lk, par, c, s, r, sgf, sgb, acc);
  if constexpr (MU0 <= 3 && 3 < MU1) hop_dir<3>(a, src, lk, par, c, s, r, sgf, sgb, acc);
}

template <int MU0, int MU1, typename S, typename SX, typename T>
__device__ __forceinline__ void hop_dirs(const HopArgs<S, SX>& a, int par, int s, const Coords& c, int r,
                                         Spinor<T>& acc) {
  hop_dirs_with<MU0, MU1>(a, GlobalLinks<S>{a.links}, par, s, c, r, acc);
}

// The epilogue applied to the complete hopping term acc at output site s;
// returns the value this site contributes to the partial sum.
template <int EPI, typename S, typename SX, typename T>
__device__ __forceinline__ double hop_epilogue(const HopArgs<S, SX>& a, int par, int s, int r, double al,
                                               Spinor<T>& acc) {
  double red = 0.0;
  const T b = (T)a.coef;
  if constexpr (EPI == EPI_HOP) {
#pragma unroll
    for (int k = 0; k < 12; ++k) acc.v[k] = b * acc.v[k];
    store_spinor(a.out, r, par, s, acc);
  } else if constexpr (EPI == EPI_D) {
    Spinor<T> self;
    load_spinor(a.self, r, par, s, self);
#pragma unroll
    for (int k = 0; k < 12; ++k) acc.v[k] = self.v[k] + b * acc.v[k];
    store_spinor(a.out, r, par, s, acc);
    red = snorm2(acc);
  } else if constexpr (EPI == EPI_CGUPD) {
    using TX = typename Compute<SX>::T;
    Spinor<T> self, rr, pp;
    Spinor<TX> xx;
    load_spinor(a.self, r, par, s, self);
    load_spinor(a.out, r, par, s, rr);
    load_spinor(a.p, r, par, s, pp);
    load_spinor(a.x, r, par, s, xx);
    const T alpha = (T)al;
    const TX alx = (TX)al;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const cpx<T> ap = self.v[k] + b * acc.v[k];
      rr.v[k] = rr.v[k] - alpha * ap;
      xx.v[k] = xx.v[k] + alx * cpx<TX>{(TX)pp.v[k].re, (TX)pp.v[k].im};
    }
    store_spinor(a.out, r, par, s, rr);
    store_spinor(a.x, r, par, s, xx);
    red = snorm2(rr);
  } else {  // EPI_RES (FP64)
    Spinor<double> self, bb;
    load_spinor(a.self, r, par, s, self);
    load_spinor(a.bvec, r, par, s, bb);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const cpx<double> ap = {(double)self.v[k].re + (double)b * (double)acc.v[k].re,
                              (double)self.v[k].im + (double)b * (double)acc.v[k].im};
      bb.v[k] = bb.v[k] - ap;
    }
    store_spinor(a.r64, r, par, s, bb);
    red = snorm2(bb);
  }
  return red;
}

// The hopping term at output site s of parity par for RHS r, followed by the
// epilogue (alpha is the CG step length, used by EPI_CGUPD).
template <int EPI, typename S, typename SX>
__device__ __forceinline__ double hop_site(const HopArgs<S, SX>& a, int par, int s, const Coords& c, int r,
                                           double al) {
  using T = typename Compute<S>::T;
  Spinor<T> acc;
  zero(acc);
  hop_dirs<0, 4>(a, par, s, c, r, acc);
  return hop_epilogue<EPI>(a, par, s, r, al, acc);
}

template <int EPI, typename S, typename SX>
__device__ __forceinline__ double hop_site(const HopArgs<S, SX>& a, int par, int s, int r, double al) {
  return hop_site<EPI>(a, par, s, site_coords(a.g, s, par), r, al);
}

}  // namespace mfq
